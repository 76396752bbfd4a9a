/*
 * hoqri_gather.h — C ABI of libhoqri_gather.so, a measurement aid for the
 * TTMcTC passes (not part of the HOQRI computation, not used by libhoqri).
 *
 * The TTMcTC pass of mode n reads, for every nonzero of X in the mode-n sorted
 * order, one row of each other mode's factor (the gathers that build y_i from
 * the Kronecker product of those rows, §4.1). hoqri_gather_only reads exactly
 * those rows for two other modes and nothing else: a plain, pipelined pass of
 * the gathers alone on the same index streams, with no products into y_i, no
 * slice ends and no stores beyond one float per thread. It is a reference
 * point, not a lower bound: a pass that reuses rows or orders its loads better
 * can take less time.
 */
#ifndef HOQRI_GATHER_H
#define HOQRI_GATHER_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reads row i1[e] of d_U1 and row i2[e] of d_U2 for e = 0..nnz-1 and sums
 * their dot products per thread into d_out.
 *  - d_U1, d_U2: device tables of rows of 64 bytes each, read as 16 float32
 *    (rows of 16 float32 factors, or of 32 bfloat16 ones, move the same bytes).
 *  - d_i1, d_i2: device int32 row numbers, nnz of each, in the order the pass
 *    reads them; the caller guarantees 0 <= value < its table's row count
 *    (not checked: the tables' sizes are not arguments).
 *  - nnz: a positive multiple of 16 (one 16-nonzero block per wave step).
 *  - wide: 0 = one 4-byte load per lane (lane l reads quarter l/16 of the row
 *    of nonzero l%16, as the passes' operand layout does), 1 = one 16-byte load
 *    per lane (lane l reads quarter l%4 of the row of nonzero l/4).
 *  - d_out: grid*256 float32 per-thread sums (written, never read); grid >= 1
 *    workgroups of 256 threads, each wave taking one contiguous range of blocks.
 * Asynchronous on `stream`. Returns 0, 1 for an argument error (no launch), or
 * the hipError_t of the launch.
 */
int hoqri_gather_only(const float* d_U1, const float* d_U2, const int32_t* d_i1, const int32_t* d_i2, int64_t nnz,
                       int32_t wide, float* d_out, int32_t grid, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HOQRI_GATHER_H */
