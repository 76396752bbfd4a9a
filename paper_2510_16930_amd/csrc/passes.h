// Launch descriptors of the segment-pass and CholeskyQR2 kernels.
//
// Every kernel of a mode step (core pass, TTMcTC pass, QR) is written as a
// device body that takes its descriptor and a block index. The single-plan
// entry points launch each body once per plan; the request server launches
// each body once per engine step for all active requests together: the
// launch's blocks are split among the requests by a prefix table, and every
// block reads its request's descriptor from a per-step table in device memory.
// A request gets the same blocks, ranges and summation order either way, so
// its results do not depend on what else is in the batch.
#pragma once

#include <cstring>
#include <vector>

#include "common.h"

namespace hoqri {

struct SegArgs {
  const int32_t* rec;       // mode-sorted block records (ModeData::rec)
  const int32_t* seg_off;   // [R+1]
  const int32_t* seg_row;   // [R]
  int32_t R;
  int32_t nnz;
  int32_t nnz_pad;          // nnz rounded up to 16 (the stored length)
  int32_t W;                // ranges
  int32_t B, RB, CB;        // y_i blocks (16x16) per range, as RB x CB
  int32_t RPW;              // ranges per workgroup
  const void* U[3];         // factors of the other modes (float32 or 16-bit copies), ascending
  uint32_t Ubytes[3];
  float ascale;             // FP16: power of two applied to x * (row factors) before rounding
  float yscale;             // 16-bit forms: exact unscale of y
  int32_t K1;               // rank of the second other mode (row split for N = 4)
  int32_t K0, K2;           // ranks of the first and third other modes (N = 4, c-tile 16-bit pass)
  // TTMcTC
  const float* gtop;        // stage-two operand [B][KN2][64][64]
  float* A;
  int32_t Kn;
  float* carry;             // [W][2][32]
  int32_t* meta;            // [W][4]
  const int32_t* out_map;   // null: A rows in label order; else row r goes to out_map[r]
  float* yrow;              // non-null: the TTMcTC pass also stores every y_i, [R][B * 256] by label
  float* ycarry;            // with yrow: partial rows of split slices [W][2][B * 256]
  int32_t* fault;           // set to 1 if a wait of the 2 x 2-block pass's slice pool timed out
  // core
  const float* Uc;          // factor of the pass mode
  int32_t Kc;
  float* gpart;             // [groups][B][16*KN2][256]
};

struct PrepArgs {
  const float* G;
  float* gtop;
  int32_t B, CB, KN2, krow, kcol, Kn, mode, N, nm1;
  int32_t om[kMaxOrder - 1];  // other modes ascending
  int32_t Ko[kMaxOrder - 1];  // their ranks
  int64_t gstride[kMaxOrder];  // C-order strides of G
  int32_t nblk;           // blocks of this launch (grid-stride loop)
  int32_t wide16;         // bfloat16 operand of the one-wave 16-bit passes: 1 c-tile layout, 2 2x2-block layout
  int32_t pair;           // block (rb, cb) of y_i holds entries (2r + rb, 2c + cb) instead of (16 rb + r, 16 cb + c)
};

struct FixArgs {
  const int32_t* meta;
  const float* carry;
  const int32_t* seg_row;
  const int32_t* seg_off;
  int32_t W, nnz, Kn;
  const int32_t* out_map;
  float* A;
};

struct CoreRedArgs {
  const float* gpart;
  int32_t groups, B, CB, KN2, krow, kcol, Kc, mode, nm1;
  int32_t om[kMaxOrder - 1], Ko[kMaxOrder - 1];
  int64_t gstride[kMaxOrder];
  float* G;
  double* fpart;
  int32_t pair;  // the rows are in the paired order of the 2 x 2-block pass (see PrepArgs)
};

// Core product of the row-writing core pass: partial[chunk][b][kc][j'] =
// sum over the chunk's rows v of U^(c)(label(v), kc) * row_v[b][j'], where the
// rows are the complete slice rows ybuf[0..R) followed by the split-slice
// partials ycarry[w][head / tail] (valid ones only, per ymeta).
struct CoreGemmArgs {
  const float* ybuf;
  const float* ycarry;
  const int32_t* ymeta;
  const int32_t* seg_row;
  const float* Uc;
  int32_t Kc, KC, R, W, B;
  int32_t nchunk;  // partials: chunk c takes the 16-row groups c, c + nchunk, ...
  int32_t split;   // 1: products in split bfloat16 (hi + lo, three per product; 16-bit forms)
  int32_t yb16;    // 1: the rows are bfloat16 (stored by the 2 x 2-block BF16 pass; implies split)
  float* gpart;
};

// A from stored slice rows: A(row) = y_row G_(n)^T for the rows of Y_(n) a
// TTMcTC pass stored (complete rows into A by label, split-slice partials into
// carry like the pass itself, for the fix-up).
struct RowsAArgs {
  const float* ybuf;
  const float* ycarry;
  const int32_t* ymeta;
  const float* gtop;
  int32_t R, W, B, KN2, Kn;
  int32_t yb16;    // 1: the rows are bfloat16
  const int32_t* out_map;  // null: A rows by label; else label r goes to row out_map[r]
  int64_t groups;  // 16-row groups over the R + 2W rows
  float* A;
  float* carry;
};

struct SumArgs {
  const double* part;
  int32_t n;
  double* out;
};

// Item of a batched launch that owns block b: first[r] <= b < first[r+1].
__device__ inline int batch_item(const int32_t* first, int count, int b) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Kernel instance of a segment pass: tensor order, rank blocks, precision.
inline int seg_key(int nm1, int kn2, int prec) { return nm1 * 100 + kn2 * 10 + prec; }

struct TtmJob {
  int key, threads;
  size_t shmem;
  PrepArgs prep;
  int prep_blocks;
  SegArgs seg;
  int seg_blocks;
  FixArgs fix;
  int fix_blocks;
};

struct CoreJob {
  int key, threads;  // key >= 1000: row-writing core pass (+ 1000, or the c-tile key)
  size_t shmem;
  SegArgs seg;
  int seg_blocks;
  CoreGemmArgs gemm;  // row-writing path only
  int gemm_blocks;
  CoreRedArgs red;
  int red_blocks;
  SumArgs sum;
};

// Core from the slice rows a TTMcTC pass stored (G_(n) = U^(n)T Y_(n) with the
// updated factor U^(n)): product over chunks of rows, fixed-order reduction.
struct YCoreJob {
  CoreGemmArgs gemm;
  int gemm_blocks;
  CoreRedArgs red;
  int red_blocks;
  SumArgs sum;
};

// Fills a job for one plan (no device work). G: the core the TTMcTC pass
// multiplies by; A: its output (rows in label order when out_map is null);
// rows: the pass also stores Y_(n) for prepare_ycore.
hoqri_status prepare_ttm(hoqri_plan* p, int mode, const Operands& op, const float* G, float* A,
                         const int32_t* out_map, TtmJob* job, bool rows = false);
hoqri_status prepare_core(hoqri_plan* p, const Operands& op, float* G, double* f_out, CoreJob* job);
// After the TTMcTC pass of `mode` with rows and the update of U^(mode) (float32, label order).
// yb16: the pass stored the rows in bfloat16 (ttm_rows_bf16).
hoqri_status prepare_ycore(hoqri_plan* p, int mode, float* G, double* f_out, YCoreJob* job, bool split = false,
                           bool yb16 = false);


struct GramArgs {
  const float* A;
  int64_t rows;
  int32_t K;
  const double* M;  // null: Gram of A; else Gram of A M (M = R1^-1, upper triangular)
  double* part;     // [K*K][nb]
  int32_t nb;
};
struct GRedArgs {
  const double* part;
  int32_t nb;
  double* W;
};
struct CholArgs {
  const double* W;
  int32_t K;
  const double* M1;  // second step: R1^-1 of the first (null: this is the first step)
  const double* R1;  // second step: R1
  double* Mout;
  double* Rout;
  int32_t* flag;
  int32_t* status;
  int32_t sticky;
  int32_t* skipped;  // null: breakdown sets *status; else counts kept factors
};
struct ApplyArgs {
  const float* A;
  int64_t rows;
  int32_t K;
  const double* M;
  float* U;
  const int32_t* flag;
  int32_t nblk;
  int64_t zero_to;  // rows [rows, zero_to) of U are zeroed with the update
  uint16_t* Uh;       // non-null: the 16-bit copy of rows [0, rows) of U, written with them
  int32_t prec16;     // its form (OP_BF16, OP_FP16: as k_cast16)
  int32_t* range_flag;  // FP16: set when an entry has magnitude >= 1.5 (as k_cast16)
};
struct OrthJob {
  GramArgs g1, g2;  // Gram of A; Gram of Q1 = A R1^-1
  GRedArgs r1, r2;
  CholArgs c1, c;   // R1 = chol(W1); R2 = chol(W2) and the combined factors
  ApplyArgs ap;
  int gram_blocks, red_blocks, apply_blocks;
};
hoqri_status prepare_orth(int64_t rows, int32_t K, const float* A, float* U, double* R, int32_t* status, void* ws,
                          size_t ws_bytes, bool sticky, OrthJob* job, int32_t* skipped = nullptr,
                          int64_t zero_to = 0);

// ---------------------------------------------------------------------------
// Per-step descriptor tables: written on the host into pinned memory, copied
// to device memory with one asynchronous copy, read by the batched kernels.
// ---------------------------------------------------------------------------
struct Staging {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0;
  size_t off = 0;
  size_t mark = 0;
  void bind(char* h, char* d, size_t c) {
    host = h;
    dev = d;
    cap = c;
    off = mark = 0;
  }
  // Copies n items into the table; returns their device address (null: full).
  template <class T>
  const T* put(const T* items, size_t n) {
    const size_t start = align_up(off, 64);
    const size_t bytes = n * sizeof(T);
    if (start + bytes > cap) return nullptr;
    std::memcpy(host + start, items, bytes);
    off = start + bytes;
    return reinterpret_cast<const T*>(dev + start);
  }
  hipError_t upload(hipStream_t s) {
    hipError_t e = hipSuccess;
    if (off > mark) e = hipMemcpyAsync(dev + mark, host + mark, off - mark, hipMemcpyHostToDevice, s);
    mark = off;
    return e;
  }
};

// A batched launch: `count` items, item r owns blocks [first[r], first[r+1]).
struct BatchTable {
  const void* descs;
  const int32_t* first;
  int32_t count;
  int32_t blocks;
};

// Stages descs[0..n) with their block counts; false when the table is full.
template <class T>
bool stage_table(Staging& st, const T* descs, const int32_t* nblocks, int n, BatchTable* out) {
  if (n < 1 || n > 1024) return false;
  std::vector<int32_t> first((size_t)n + 1);
  first[0] = 0;
  for (int i = 0; i < n; ++i) first[i + 1] = first[i] + nblocks[i];
  out->descs = st.put(descs, (size_t)n);
  out->first = st.put(first.data(), (size_t)n + 1);
  out->count = n;
  out->blocks = first[n];
  return out->descs && out->first;
}

struct TtmGroup {
  int key, threads;
  size_t shmem;
  BatchTable prep, seg, fix;
};
struct CoreGroup {
  int key, threads;
  size_t shmem;
  BatchTable seg, gemm, red, sum;
};
struct OrthGroup {
  BatchTable g1, r1, c1, g2, r2, c, ap;
};
struct YCoreGroup {
  BatchTable gemm, red, sum;
};

// Jobs of one group must share key, threads and shmem.
bool stage_ttm_group(const TtmJob* const* jobs, int n, Staging& st, TtmGroup* g);
bool stage_core_group(const CoreJob* const* jobs, int n, Staging& st, CoreGroup* g);
bool stage_orth_group(const OrthJob* const* jobs, int n, Staging& st, OrthGroup* g);
bool stage_ycore_group(const YCoreJob* const* jobs, int n, Staging& st, YCoreGroup* g);
hoqri_status launch_ttm_group(const TtmGroup& g, hipStream_t s);
hoqri_status launch_core_group(const CoreGroup& g, hipStream_t s);
hoqri_status launch_orth_group(const OrthGroup& g, hipStream_t s);
hoqri_status launch_ycore_group(const YCoreGroup& g, hipStream_t s);

}  // namespace hoqri
