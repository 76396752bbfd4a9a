// Gather-only pass (include/hoqri_gather.h): the factor rows of two other
// modes per nonzero, in the TTMcTC pass's order, with nothing else.
#include "hoqri_gather.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int kG = 4;  // 16-nonzero blocks per group

// Row numbers of the kG blocks from block g on (blocks past the range's last
// block re-read that block: in bounds, and never summed).
__device__ inline void load_rows_of(const int32_t* __restrict__ i1, const int32_t* __restrict__ i2, int64_t g,
                                    int64_t last, int eo, int32_t (&c1)[kG], int32_t (&c2)[kG]) {
#pragma unroll
  for (int j = 0; j < kG; ++j) {
    const int64_t e = (g + j < last ? g + j : last) * 16 + eo;
    c1[j] = i1[e];
    c2[j] = i2[e];
  }
}

// Four entries of each of the two rows a lane reads per block.
// WIDE: lane l reads entries 4(l%4)..4(l%4)+3 of the rows of nonzero l/4, in
// one 16-byte load per row. Otherwise lane l reads entry l%16 of the rows of
// nonzeros l/16, 4 + l/16, 8 + l/16, 12 + l/16, in four 4-byte loads per
// row: each load instruction covers four whole rows (16 lanes x 4 bytes
// each), the coalesced operand layout of a 16x16x4 matrix product. The lane
// holding a row number (lane e%16 for nonzero e) hands it over by a lane
// shuffle.
template <bool WIDE>
__device__ inline void gather(const float* __restrict__ U1, const float* __restrict__ U2, const int32_t (&c1)[kG],
                              const int32_t (&c2)[kG], int lane, float (&u)[kG][4], float (&v)[kG][4]) {
#pragma unroll
  for (int j = 0; j < kG; ++j) {
    if constexpr (WIDE) {
      const int q = (lane & 3) * 4;
      // unsigned row numbers: widening them needs nothing from the loaded
      // value, so the compiler does not wait for the row-number loads there
      const float4 a = *reinterpret_cast<const float4*>(U1 + (uint64_t)(uint32_t)c1[j] * 16u + q);
      const float4 b = *reinterpret_cast<const float4*>(U2 + (uint64_t)(uint32_t)c2[j] * 16u + q);
      u[j][0] = a.x, u[j][1] = a.y, u[j][2] = a.z, u[j][3] = a.w;
      v[j][0] = b.x, v[j][1] = b.y, v[j][2] = b.z, v[j][3] = b.w;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int src = 4 * t + (lane >> 4);
        const uint32_t r1 = (uint32_t)__shfl(c1[j], src);
        const uint32_t r2 = (uint32_t)__shfl(c2[j], src);
        u[j][t] = U1[(uint64_t)r1 * 16u + (lane & 15)];
        v[j][t] = U2[(uint64_t)r2 * 16u + (lane & 15)];
      }
    }
  }
}

__device__ inline float use(const float (&u)[kG][4], const float (&v)[kG][4], int64_t g, int64_t b1, float acc) {
#pragma unroll
  for (int j = 0; j < kG; ++j)
    if (g + j < b1) acc += u[j][0] * v[j][0] + u[j][1] * v[j][1] + u[j][2] * v[j][2] + u[j][3] * v[j][3];
  return acc;
}

// One wave per contiguous range of 16-nonzero blocks, in groups of kG
// blocks, with two groups of rows in flight: while the rows of group k are
// used, those of group k+1 are loading and the row numbers of group k+2 have
// been requested before them (vector loads return in order, so the wait for
// group k's rows never covers the newer loads). Two row buffers alternate
// (the loop body covers two groups) so no register copy waits on a load.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_gather_only(const float* __restrict__ U1, const float* __restrict__ U2,
                                                      const int32_t* __restrict__ i1,
                                                      const int32_t* __restrict__ i2, int64_t nblk, int64_t per,
                                                      float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int eo = WIDE ? (lane >> 2) : (lane & 15);  // this lane's nonzero in a block
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b0 = wave * per;
  const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  float acc = 0.f;
  if (b0 < b1) {
    const int64_t last = b1 - 1;
    int32_t c1[kG], c2[kG], n1[kG], n2[kG], f1[kG], f2[kG];
    float ua[kG][4], va[kG][4], ub[kG][4], vb[kG][4];
    // the loop's order at its head: the next group's row numbers, then the
    // current group's rows (so the waits there are the same on entry)
    load_rows_of(i1, i2, b0, last, eo, c1, c2);
    load_rows_of(i1, i2, b0 + kG, last, eo, n1, n2);
    __builtin_amdgcn_sched_barrier(0);
    gather<WIDE>(U1, U2, c1, c2, lane, ua, va);
    __builtin_amdgcn_sched_barrier(0);
    for (int64_t g = b0; g < b1; g += 2 * kG) {
      load_rows_of(i1, i2, g + 2 * kG, last, eo, f1, f2);
      __builtin_amdgcn_sched_barrier(0);
      gather<WIDE>(U1, U2, n1, n2, lane, ub, vb);
      __builtin_amdgcn_sched_barrier(0);
      acc = use(ua, va, g, b1, acc);
      load_rows_of(i1, i2, g + 3 * kG, last, eo, n1, n2);
      __builtin_amdgcn_sched_barrier(0);
      gather<WIDE>(U1, U2, f1, f2, lane, ua, va);
      __builtin_amdgcn_sched_barrier(0);
      acc = use(ub, vb, g + kG, b1, acc);
    }
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

extern "C" int hoqri_gather_only(const float* d_U1, const float* d_U2, const int32_t* d_i1, const int32_t* d_i2,
                                  int64_t nnz, int32_t wide, float* d_out, int32_t grid, hipStream_t stream) {
  if (!d_U1 || !d_U2 || !d_i1 || !d_i2 || !d_out || nnz <= 0 || nnz % 16 != 0 || grid < 1 ||
      (wide != 0 && wide != 1))
    return 1;
  const int64_t nblk = nnz / 16;
  const int64_t waves = (int64_t)grid * 4;
  const int64_t per = (nblk + waves - 1) / waves;
  if (wide)
    hipLaunchKernelGGL(k_gather_only<true>, dim3(grid), dim3(256), 0, stream, d_U1, d_U2, d_i1, d_i2, nblk, per,
                       d_out);
  else
    hipLaunchKernelGGL(k_gather_only<false>, dim3(grid), dim3(256), 0, stream, d_U1, d_U2, d_i1, d_i2, nblk, per,
                       d_out);
  return (int)hipGetLastError();
}
