// QR step of HOQRI (Alg. 2): an orthonormal basis of A (I x K, K <= 32) by
// CholeskyQR2 in float64:
//   W1 = A^T A, R1 = chol(W1), Q1 = A R1^-1, W2 = Q1^T Q1, R2 = chol(W2),
//   U = A (R2 R1)^-1 = A M with M = R1^-1 R2^-1.
// W1 is formed from the float32 A with float64 products on the float64
// matrix cores (v_mfma_f64_16x16x4_f64). Q1 is never stored: a second pass
// over A forms each 16-row tile of A R1^-1 on the same matrix cores and adds
// its Gram to W2 at once, so W2 is the Gram of the float64 Q1 itself and the
// loss of orthonormality of U is that of CholeskyQR2 (about u64 times a
// modest factor while kappa(A)^2 u64 < 1, then the float32 rounding of U),
// not kappa(A)^2 times the rounding of W1. Both Cholesky factors have a
// positive diagonal, so U is the thin QR factor with diag(R) > 0 (the basis
// the paper leaves free, made unique).
// A Cholesky pivot <= 1e-13 * trace(W) (or not finite) in either step flags
// breakdown: A is numerically rank deficient; U is then left untouched.
//
// Only the diagonal 16 x 16 blocks and the block above them are formed (the
// factorisation reads nothing below the diagonal): three float64 products
// per step instead of four, on matrix cores whose float64 rate is the
// vector rate.
// Memory traffic: two reads of A for the Gram matrices and one read + one
// write for the final product; the K x K work runs in single waves.
#include "passes.h"

#include <mutex>
#include <vector>

namespace hoqri {
namespace {

constexpr int kT = 256;
static_assert(kMaxRank == 32, "rank blocks are at most 32 wide");
constexpr int kChunk = 32;    // rows staged per step
constexpr double kBreakRel = 1e-13;

// Gram blocks: one per 1024 rows, at most kGramBlocks (several per CU, each
// streaming its rows; more, shorter blocks spend their time on start-up and
// on writing their K x K partials)
constexpr int kGramBlocks = 1024;
int gram_blocks(int64_t rows) {
  int64_t nb = (rows + 1023) / 1024;
  if (nb < 1) nb = 1;
  if (nb > kGramBlocks) nb = kGramBlocks;
  return (int)nb;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Adds the 4 waves' Gram tiles in wave order and stores the block's partial:
// tile (pb, qb) holds entry (16 pb + 4 v + gg, 16 qb + q) in D[pb][qb][v]
// (the float64 16x16 result layout); part[e * nb + blk] for entry e = p*K + q.
// Only tiles (0,0), (0,1) and (1,1) are formed (the block below the diagonal
// blocks is zero), so LDS holds three tiles per wave.
__device__ inline void gram_store(const d4 (&D)[2][2], const GramArgs& g, const int blk) {
  __shared__ double red[kT / 64][3][256];
  const int K = g.K;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane & 15, gg = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int pos = (4 * v + gg) * 16 + q;
    red[wv][0][pos] = D[0][0][v];
    red[wv][1][pos] = D[0][1][v];
    red[wv][2][pos] = D[1][1][v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * K; e += kT) {
    const int p = e / K, c = e - p * K;
    const int pb = p >> 4, qb = c >> 4;
    double t = 0.0;
    if (pb <= qb) {
      const int tile = pb + qb, pos = (p & 15) * 16 + (c & 15);
      t = red[0][tile][pos];
      for (int w = 1; w < kT / 64; ++w) t += red[w][tile][pos];
    }
    g.part[(size_t)e * g.nb + blk] = t;
  }
}

// Partial Gram of the rows [r0, r1) of block blk, on the float64 matrix cores:
// each wave takes 4 rows at a time (lane group g: row 4s + g, lane q: columns
// 16 pb + q), W tile (pb, qb) += A_rows^T A_rows; the 4 waves' tiles are added
// in order. part[e * nb + blk] for entry e = p*K + q.
__device__ inline void gram_body(const GramArgs& g, const int blk) {
  const float* A = g.A;
  const int64_t rows = g.rows;
  const int K = g.K;
  const int nb = g.nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane & 15, gg = lane >> 4;
  const int64_t per = (rows + nb - 1) / nb;
  const int64_t r0 = blk * per;
  int64_t r1 = r0 + per;
  if (r1 > rows) r1 = rows;
  d4 D[2][2];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) D[pb][qb] = d4{0.0, 0.0, 0.0, 0.0};
  const bool two = K > 16;
  // groups of 8 steps of 4 rows: loads go to clamped (valid) addresses, and
  // the next group's loads are issued before a group's products; rows past r1
  // and columns past K are masked afterwards
  constexpr int NS = 8;
  constexpr int64_t kStride = 4 * NS * (kT / 64);
  const int q0 = q < K ? q : 0, q1 = 16 + q < K ? 16 + q : 0;
  float x0[NS], x1[NS], y0[NS], y1[NS];
  auto fetch = [&](int64_t base, float* a0, float* a1) {
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int64_t row = base + st * 4 * (kT / 64) + gg;
      const int64_t rr = row < r1 ? row : r0;
      a0[st] = A[rr * K + q0];
      a1[st] = A[rr * K + q1];  // (same line as a0; used only when K > 16)
    }
  };
  if (r0 + 4 * wv < r1) fetch(r0 + 4 * wv, x0, x1);
  for (int64_t base = r0 + 4 * wv; base < r1; base += kStride) {
    fetch(base + kStride < r1 ? base + kStride : base, y0, y1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const bool ok = base + st * 4 * (kT / 64) + gg < r1;
      const double a0 = (ok && q < K) ? (double)x0[st] : 0.0;
      D[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, D[0][0], 0, 0, 0);
      if (two) {
        const double a1 = (ok && 16 + q < K) ? (double)x1[st] : 0.0;
        D[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, D[0][1], 0, 0, 0);
        D[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, D[1][1], 0, 0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      x0[st] = y0[st];
      x1[st] = y1[st];
    }
  }
  gram_store(D, g, blk);
}


// Partial Gram of Q1 = A M (M = R1^-1, upper triangular) over the rows
// [r0, r1) of block blk. Each wave takes 16-row tiles of A (staged in its
// own LDS rows), forms the tile of Q1 on the float64 matrix cores (lane
// (gg, q) supplies A(row q, 4s + gg) and M(4s + gg, 16 ct + q), and receives
// Q1(4 r + gg, 16 ct + q) in D[ct][r]), and multiplies it into its Gram
// tiles at once: that output layout is the operand layout of the Gram
// product (step r: rows 4 r + gg of the tile, lane column q). Rows past r1
// and columns past K are zero and add nothing.
__device__ inline void gramq_body(const GramArgs& g, const int blk) {
  __shared__ float tile[kT / 64][16][kMaxRank + 1];
  const float* A = g.A;
  const int64_t rows = g.rows;
  const int K = g.K;
  const int nb = g.nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane & 15, gg = lane >> 4;
  const int KT = (K + 15) >> 4;
  const int64_t per = (rows + nb - 1) / nb;
  const int64_t r0 = blk * per;
  int64_t r1 = r0 + per;
  if (r1 > rows) r1 = rows;
  double mb[8][2];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int kk = 4 * s + gg, cc = 16 * ct + q;
      mb[s][ct] = (kk < K && cc < K) ? g.M[kk * K + cc] : 0.0;
    }
  d4 W[2][2];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) W[pb][qb] = d4{0.0, 0.0, 0.0, 0.0};
  // a tile's nr * K floats are contiguous in A; the next tile's are loaded
  // into registers before this tile's products
  float cur[8], nxt[8];
  auto fetch = [&](int64_t base, float* x) {
    const int nr = (int)((r1 - base) < 16 ? (r1 - base) : 16);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = lane + 64 * i;
      x[i] = t < nr * K ? A[base * K + t] : 0.f;
    }
  };
  if (r0 + 16 * wv < r1) fetch(r0 + 16 * wv, cur);
  for (int64_t base = r0 + 16 * wv; base < r1; base += 16 * (kT / 64)) {
    const int nr = (int)((r1 - base) < 16 ? (r1 - base) : 16);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = lane + 64 * i;
      if (t < nr * K) tile[wv][t / K][t % K] = cur[i];
    }
    if (base + 16 * (kT / 64) < r1) fetch(base + 16 * (kT / 64), nxt);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    d4 D[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s >= 4 * KT) break;
      const int kk = 4 * s + gg;
      const double av = (q < nr && kk < K) ? (double)tile[wv][q][kk] : 0.0;
      D[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, mb[s][0], D[0], 0, 0, 0);
      if (KT > 1) D[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, mb[s][1], D[1], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      W[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[0][r], D[0][r], W[0][0], 0, 0, 0);
      if (KT > 1) {
        W[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[0][r], D[1][r], W[0][1], 0, 0, 0);
        W[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[1][r], D[1][r], W[1][1], 0, 0, 0);
      }
    }
    // the next tile overwrites this wave's LDS rows after every lane read them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 8; ++i) cur[i] = nxt[i];
  }
  gram_store(W, g, blk);
}

__global__ __launch_bounds__(kT) void k_gram(GramArgs g) {
  if (g.M) gramq_body(g, blockIdx.x);
  else gram_body(g, blockIdx.x);
}

__global__ __launch_bounds__(kT) void k_gram_b(const GramArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  if (d[r].M) gramq_body(d[r], blockIdx.x - first[r]);
  else gram_body(d[r], blockIdx.x - first[r]);
}

// W[e] = sum over blocks of part[e * nb + b], fixed tree order.
__device__ inline void gred_body(const GRedArgs& g, const int e) {
  __shared__ double sh[kT];
  const double* part = g.part;
  const int nb = g.nb;
  double* W = g.W;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kT) s += part[(size_t)e * nb + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) W[e] = sh[0];
}

__global__ __launch_bounds__(kT) void k_gram_reduce(GRedArgs g) { gred_body(g, blockIdx.x); }

__global__ __launch_bounds__(kT) void k_gram_reduce_b(const GRedArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  gred_body(d[r], blockIdx.x - first[r]);
}

// The two Cholesky steps, each in one wave: lane j < 32 holds column j of
// the working matrix in registers (the K x K matrix padded to 32 x 32 with
// the identity, which the factorisation leaves unchanged), and lane 32 + c
// column c of the identity appended to it: the row operations that turn W
// into R turn that identity into R^-T (each step divides row k by the pivot's
// square root and subtracts R(k, i) times it from rows i > k, so
// [W | I] -> [R | L] with L W = R, L = R W^-1 = R^-T), and R^-1 comes out of
// the same loop with no back substitution. Each finished row of [R | R^-T]
// and each next pivot is shared through LDS, where every lane reads the same
// address; there is no workgroup barrier. Operations and their order per
// entry are those of the textbook right-looking factorisation; zero terms of
// the triangular factors added after the last nonzero one change nothing. The
// step loop is serial (float64 square roots, divisions and dependent LDS
// reads).
// Stage 1 (c.M1 == null): R1 = chol(W1); Mout = R1^-1, Rout = R1;
//   *flag = breakdown (a pivot <= 1e-13 * trace(W) or not finite).
// Stage 2: R2 = chol(W2) with W2 the Gram of Q1 = A R1^-1; Mout = M1 R2^-1
//   (= R1^-1 R2^-1), Rout = R2 R1 (optional). Breakdown in either stage:
//   *skipped += 1 when a counter is given (the factor is left as it was), else
//   *status = HOQRI_ERR_BREAKDOWN; without breakdown *status = 0 unless
//   `sticky` (then an earlier breakdown recorded in *status is kept).
//   *flag = breakdown (read by the apply kernel).
constexpr int kCholT = 64;
constexpr int kCholLd = 2 * kMaxRank + 1;  // LDS row of [R | R^-T] (odd: rows fall on different banks)

// orders this wave's LDS writes before its later LDS reads
__device__ inline void lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void chol_body(const CholArgs& c) {
  __shared__ double Rr[kMaxRank][kCholLd];    // input W, then the rows of [R | R^-T]
  __shared__ double Mr[kMaxRank][kMaxRank];   // rows of M1 (stage 2)
  __shared__ double R1s[kMaxRank][kMaxRank];  // R1 (stage 2)
  const int K = c.K;
  const int t = threadIdx.x;
  const int j = t & (kMaxRank - 1);  // column of W (t < 32) or of the appended identity (t >= 32)
  const bool aug = t >= kMaxRank;
  const bool mine = t < K;           // lanes writing a column of the K x K result
  const bool second = c.M1 != nullptr;
  // W padded with the identity
  for (int e = t; e < kMaxRank * kMaxRank; e += kCholT) {
    const int i = e >> 5, k = e & 31;
    Rr[i][k] = (i < K && k < K) ? c.W[i * K + k] : (i == k ? 1.0 : 0.0);
    if (second) {
      Mr[i][k] = (i < K && k < K) ? c.M1[i * K + k] : 0.0;
      R1s[i][k] = (i < K && k < K) ? c.R1[i * K + k] : 0.0;
    }
  }
  lds_order();
  double w[kMaxRank];
#pragma unroll
  for (int i = 0; i < kMaxRank; ++i) w[i] = aug ? (i == j ? 1.0 : 0.0) : Rr[i][j];
  double dj = Rr[j][j];  // this column's diagonal entry, updated with w[j]
  // trace(W), summed in index order
  double tr = 0.0;
#pragma unroll 1
  for (int k = 0; k < K; ++k) tr += Rr[k][k];
  int bad = second ? *c.flag : 0;
  lds_order();
  // Right-looking factorisation: row k of [R | R^-T] is row k of the working
  // [W | I] divided by sqrt(W(k, k)), then row i -= R(k, i) row k for i > k.
  // The step loop runs from the instruction cache (a fully unrolled kernel
  // runs once and is bound by instruction fetch); register indices stay
  // compile-time through selects. (Steps k >= K would leave the identity
  // padding as it is.)
#pragma unroll 1
  for (int k = 0; k < K; ++k) {
    const double piv = Rr[k][k];  // lane k's dj after step k - 1
    if (!(piv > kBreakRel * tr) || !(piv < 1e300)) bad = 1;
    const double d = sqrt(piv > 0.0 ? piv : 1.0);
    double wk = w[0];
#pragma unroll
    for (int i = 1; i < kMaxRank; ++i) wk = i == k ? w[i] : wk;
    // (R: zero left of the diagonal; R^-T: its zeros right of the diagonal
    // come out of the elimination exactly)
    const double rk = (aug || j > k) ? wk / d : (j == k ? d : 0.0);
    lds_order();
    Rr[k][t] = rk;
    lds_order();
    // entries i < k (R(k, i) = 0) keep their value; i = k and those below
    // the diagonal change but are never read again
#pragma unroll
    for (int i = 0; i < kMaxRank; ++i) w[i] -= Rr[k][i] * rk;
    // the same operation on the diagonal copy (Rr(k, j) = rk on this lane)
    if (j > k) dj = dj - rk * rk;
    if (!aug && j > k) Rr[j][j] = dj;  // next pivots
    lds_order();
  }
  if (!second) {
    // Mout = R^-1 = (R^-T)^T, Rout = R, stored row by row
    for (int e = t; e < K * K; e += kCholT) {
      const int i = e / K, q = e - i * K;
      c.Mout[e] = Rr[q][kMaxRank + i];
      c.Rout[e] = Rr[i][q];
    }
    if (t == 0) *c.flag = bad;
    return;
  }
  // M = M1 R2^-1 and R = R2 R1, k ascending (rows i of M1 and R2 are zero left
  // of the diagonal: the sums start with exact zeros, as if they began at k = i);
  // lane j < 32 takes column j: R2^-1(k, j) = R2^-T(j, k)
  double ri[kMaxRank], r1[kMaxRank];
#pragma unroll
  for (int k = 0; k < kMaxRank; ++k) {
    ri[k] = k < K ? Rr[j][kMaxRank + k] : 0.0;
    r1[k] = R1s[k][j];
  }
#pragma unroll 1
  for (int i = 0; i < K; ++i) {
    double m = 0.0, r = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxRank; ++k) {
      m += Mr[i][k] * ri[k];
      r += Rr[i][k] * r1[k];
    }
    if (mine) {
      c.Mout[i * K + j] = j >= i ? m : 0.0;
      if (c.Rout) c.Rout[i * K + j] = j >= i ? r : 0.0;
    }
  }
  if (t == 0) {
    *c.flag = bad;
    if (bad) {
      if (c.skipped) *c.skipped += 1;  // the caller keeps its previous factor
      else *c.status = HOQRI_ERR_BREAKDOWN;
    } else if (!c.sticky) {
      *c.status = 0;
    }
  }
}

__global__ __launch_bounds__(kCholT) void k_chol(CholArgs c) { chol_body(c); }

__global__ __launch_bounds__(kCholT) void k_chol_b(const CholArgs* d, const int32_t* first, int count) {
  chol_body(d[batch_item(first, count, blockIdx.x)]);
}

// U = A M (M upper triangular), rows staged in LDS so U may alias A, then
// rows [rows, zero_to) of U set to zero. Skipped entirely when this
// factorisation broke down (*flag != 0): U keeps its previous contents.
// With a.Uh, every updated entry of U is also written to the 16-bit copy the
// 16-bit passes read, rounded as k_cast16 rounds it (bfloat16, or float16 of
// u 2^15 with the range flag), so no separate cast pass re-reads U.
// Each 64-row tile is multiplied on the float64 matrix cores: wave w takes
// rows 16w .. 16w+15, lane (gg, q) supplies A(row q, 4s + gg) (from LDS) and
// M(4s + gg, 16 ct + q) (kept in registers), and receives U entries
// (4v + gg, 16 ct + q).
__device__ inline void apply_body(const ApplyArgs& a, const int blk) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ float tile[64][kMaxRank + 1];
  const float* A = a.A;
  const int64_t rows = a.rows;
  const int K = a.K;
  const double* M = a.M;
  float* U = a.U;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gg = lane >> 4, q = lane & 15;
  const int KT = (K + 15) >> 4;  // 16-column tiles (1 or 2)
  const int64_t last = rows * K - 1;
  // a tile's loads go to clamped (valid) addresses, all issued together; the
  // next tile's loads are in flight while a tile is multiplied (its rows are
  // other rows, so U may still alias A)
  float v[8];
  auto load_tile = [&](int64_t base) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t e = base * K + threadIdx.x + i * kT;
      v[i] = A[e < last ? e : last];
    }
  };
  const int64_t step = (int64_t)a.nblk * 64;
  int64_t base = blk * (int64_t)64;
  if (base < rows) load_tile(base);
  if (*a.flag != 0) return;
  bool bad = false;
  double mb[8][2];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int kk = 4 * s + gg, cc = 16 * ct + q;
      mb[s][ct] = (kk < K && cc < K) ? M[kk * K + cc] : 0.0;
    }
  for (; base < rows; base += step) {
    const int nr = (int)((rows - base) < 64 ? (rows - base) : 64);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = threadIdx.x + i * kT;
      if (t < nr * K) tile[t / K][t % K] = v[i];
    }
    __syncthreads();
    if (base + step < rows) load_tile(base + step);
    __builtin_amdgcn_sched_barrier(0);
    const int rw = 16 * wv;  // this wave's rows in the tile
    if (rw < nr) {
      d4 D[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (s >= 4 * KT) break;
        const int kk = 4 * s + gg;
        const double av = (rw + q < nr && kk < K) ? (double)tile[rw + q][kk] : 0.0;
        D[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, mb[s][0], D[0], 0, 0, 0);
        if (KT > 1) D[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, mb[s][1], D[1], 0, 0, 0);
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        if (ct >= KT) break;
        const int cc = 16 * ct + q;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rw + 4 * r + gg;
          if (row < nr && cc < K) {
            const float uf = (float)D[ct][r];
            const int64_t at = (base + row) * K + cc;
            U[at] = uf;
            if (a.Uh) {
              if (a.prec16 == OP_BF16) {
                a.Uh[at] = __builtin_bit_cast(uint16_t, (__bf16)uf);
              } else {
                bad |= !(__builtin_fabsf(uf) < 1.5f);
                a.Uh[at] = __builtin_bit_cast(uint16_t, (_Float16)(uf * 32768.f));
              }
            }
          }
        }
      }
    }
  }
  if (bad && a.range_flag) *a.range_flag = 1;
  // rows [rows, zero_to) of U (rows of empty slices) become zero with the update
  const int64_t ztot = (a.zero_to - rows) * K;
  for (int64_t t = blk * (int64_t)kT + threadIdx.x; t < ztot; t += (int64_t)a.nblk * kT) U[rows * K + t] = 0.f;
}

__global__ __launch_bounds__(kT) void k_apply(ApplyArgs a) { apply_body(a, blockIdx.x); }

__global__ __launch_bounds__(kT) void k_apply_b(const ApplyArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  apply_body(d[r], blockIdx.x - first[r]);
}

// ||W - I||_F of a symmetric Gram from its upper triangle (the Gram kernels
// leave the block below the diagonal blocks zero)
__global__ void k_orth_err(const double* W, int K, double* out) {
  __shared__ double sh[kT];
  double s = 0.0;
  for (int e = threadIdx.x; e < K * K; e += kT) {
    const int p = e / K, q = e % K;
    if (p > q) continue;
    const double d = W[e] - (p == q ? 1.0 : 0.0);
    s += (p == q ? 1.0 : 2.0) * (d * d);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0]);
}

struct OrthWs {
  int32_t* flag;
  double* part;
  double* W;
  double* M1;
  double* R1;
  double* M;
  double* R;
};

OrthWs carve(void* ws, int64_t rows, int K) {
  const int nb = gram_blocks(rows);
  char* p = (char*)ws;
  OrthWs o;
  size_t off = 0;
  o.flag = (int32_t*)(p + off);
  off = align_up(off + 64);
  o.part = (double*)(p + off);
  off = align_up(off + (size_t)nb * kMaxRank * kMaxRank * 8);
  o.W = (double*)(p + off);
  off = align_up(off + kMaxRank * kMaxRank * 8);
  o.M1 = (double*)(p + off);
  off = align_up(off + kMaxRank * kMaxRank * 8);
  o.R1 = (double*)(p + off);
  off = align_up(off + kMaxRank * kMaxRank * 8);
  o.M = (double*)(p + off);
  off = align_up(off + kMaxRank * kMaxRank * 8);
  o.R = (double*)(p + off);
  return o;
}

}  // namespace

size_t orth_ws_bytes(int64_t rows, int32_t cols) {
  (void)cols;
  const int nb = gram_blocks(rows);
  return align_up(64) + align_up((size_t)nb * kMaxRank * kMaxRank * 8) + 5 * align_up(kMaxRank * kMaxRank * 8);
}

hoqri_status prepare_orth(int64_t rows, int32_t K, const float* A, float* U, double* R, int32_t* status, void* ws,
                          size_t ws_bytes, bool sticky, OrthJob* job, int32_t* skipped, int64_t zero_to) {
  if (rows < 1 || K < 1 || K > kMaxRank || K > rows || !A || !U || !status || !ws) return HOQRI_ERR_ARG;
  if (ws_bytes < orth_ws_bytes(rows, K)) return HOQRI_ERR_NOMEM;
  OrthWs o = carve(ws, rows, K);
  const int nb = gram_blocks(rows);
  *job = OrthJob{};
  job->g1 = GramArgs{A, rows, K, nullptr, o.part, nb};
  job->r1 = GRedArgs{o.part, nb, o.W};
  job->c1 = CholArgs{o.W, K, nullptr, nullptr, o.M1, o.R1, o.flag, status, (int32_t)sticky, skipped};
  job->g2 = GramArgs{A, rows, K, o.M1, o.part, nb};
  job->r2 = GRedArgs{o.part, nb, o.W};
  job->c = CholArgs{o.W, K, o.M1, o.R1, o.M, R ? R : o.R, o.flag, status, (int32_t)sticky, skipped};
  int64_t ab = (rows + 63) / 64;
  if (ab > 4096) ab = 4096;
  job->ap = ApplyArgs{A, rows, K, o.M, U, o.flag, (int32_t)ab, zero_to > rows ? zero_to : rows};
  job->gram_blocks = nb;
  job->red_blocks = K * K;
  job->apply_blocks = (int)ab;
  return HOQRI_OK;
}

hoqri_status launch_orth(int64_t rows, int32_t K, const float* A, float* U, double* R, int32_t* status, void* ws,
                         size_t ws_bytes, hipStream_t s, bool sticky, int32_t* skipped, int64_t zero_to, uint16_t* Uh,
                         int prec16, int32_t* range_flag) {
  OrthJob j;
  HOQRI_TRY(prepare_orth(rows, K, A, U, R, status, ws, ws_bytes, sticky, &j, skipped, zero_to));
  if (Uh && (prec16 == OP_BF16 || prec16 == OP_FP16)) {
    j.ap.Uh = Uh;
    j.ap.prec16 = prec16;
    j.ap.range_flag = range_flag;
  }
  hipLaunchKernelGGL(k_gram, dim3(j.gram_blocks), dim3(kT), 0, s, j.g1);
  hipLaunchKernelGGL(k_gram_reduce, dim3(j.red_blocks), dim3(kT), 0, s, j.r1);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholT), 0, s, j.c1);
  hipLaunchKernelGGL(k_gram, dim3(j.gram_blocks), dim3(kT), 0, s, j.g2);
  hipLaunchKernelGGL(k_gram_reduce, dim3(j.red_blocks), dim3(kT), 0, s, j.r2);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholT), 0, s, j.c);
  hipLaunchKernelGGL(k_apply, dim3(j.apply_blocks), dim3(kT), 0, s, j.ap);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

bool stage_orth_group(const OrthJob* const* jobs, int n, Staging& st, OrthGroup* g) {
  if (n < 1 || n > 1024) return false;
  std::vector<GramArgs> g1(n), g2(n);
  std::vector<GRedArgs> r1(n), r2(n);
  std::vector<CholArgs> c1(n), c(n);
  std::vector<ApplyArgs> ap(n);
  std::vector<int32_t> nb_g(n), nb_r(n), ones(n), nb_a(n);
  for (int i = 0; i < n; ++i) {
    g1[i] = jobs[i]->g1;
    r1[i] = jobs[i]->r1;
    c1[i] = jobs[i]->c1;
    g2[i] = jobs[i]->g2;
    r2[i] = jobs[i]->r2;
    c[i] = jobs[i]->c;
    ap[i] = jobs[i]->ap;
    nb_g[i] = jobs[i]->gram_blocks;
    nb_r[i] = jobs[i]->red_blocks;
    ones[i] = 1;
    nb_a[i] = jobs[i]->apply_blocks;
  }
  return stage_table(st, g1.data(), nb_g.data(), n, &g->g1) && stage_table(st, r1.data(), nb_r.data(), n, &g->r1) &&
         stage_table(st, c1.data(), ones.data(), n, &g->c1) && stage_table(st, g2.data(), nb_g.data(), n, &g->g2) &&
         stage_table(st, r2.data(), nb_r.data(), n, &g->r2) && stage_table(st, c.data(), ones.data(), n, &g->c) &&
         stage_table(st, ap.data(), nb_a.data(), n, &g->ap);
}

hoqri_status launch_orth_group(const OrthGroup& g, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_b, dim3(g.g1.blocks), dim3(kT), 0, s, (const GramArgs*)g.g1.descs, g.g1.first, g.g1.count);
  hipLaunchKernelGGL(k_gram_reduce_b, dim3(g.r1.blocks), dim3(kT), 0, s, (const GRedArgs*)g.r1.descs, g.r1.first,
                     g.r1.count);
  hipLaunchKernelGGL(k_chol_b, dim3(g.c1.blocks), dim3(kCholT), 0, s, (const CholArgs*)g.c1.descs, g.c1.first,
                     g.c1.count);
  hipLaunchKernelGGL(k_gram_b, dim3(g.g2.blocks), dim3(kT), 0, s, (const GramArgs*)g.g2.descs, g.g2.first, g.g2.count);
  hipLaunchKernelGGL(k_gram_reduce_b, dim3(g.r2.blocks), dim3(kT), 0, s, (const GRedArgs*)g.r2.descs, g.r2.first,
                     g.r2.count);
  hipLaunchKernelGGL(k_chol_b, dim3(g.c.blocks), dim3(kCholT), 0, s, (const CholArgs*)g.c.descs, g.c.first, g.c.count);
  hipLaunchKernelGGL(k_apply_b, dim3(g.ap.blocks), dim3(kT), 0, s, (const ApplyArgs*)g.ap.descs, g.ap.first,
                     g.ap.count);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_orth_err(int64_t rows, int32_t K, const float* U, double* err_out, void* ws, size_t ws_bytes,
                             hipStream_t s) {
  if (ws_bytes < orth_ws_bytes(rows, K)) return HOQRI_ERR_NOMEM;
  OrthWs o = carve(ws, rows, K);
  const int nb = gram_blocks(rows);
  hipLaunchKernelGGL(k_gram, dim3(nb), dim3(kT), 0, s, GramArgs{U, rows, K, nullptr, o.part, nb});
  hipLaunchKernelGGL(k_gram_reduce, dim3(K * K), dim3(kT), 0, s, GRedArgs{o.part, nb, o.W});
  hipLaunchKernelGGL(k_orth_err, dim3(1), dim3(kT), 0, s, o.W, K, err_out);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

}  // namespace hoqri

using namespace hoqri;

extern "C" size_t hoqri_orth_workspace_size(int64_t rows, int32_t cols) { return orth_ws_bytes(rows, cols); }

extern "C" hoqri_status hoqri_orth(int64_t rows, int32_t cols, const float* d_A, float* d_U, double* d_R,
                                   int32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return launch_orth(rows, cols, d_A, d_U, d_R, d_status, d_ws, ws_bytes, stream, false);
}

// ---------------------------------------------------------------------------
// The QR step without a caller workspace, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops): its scratch
// (Gram partials, the K x K matrices and the breakdown flag) lives in a
// file-scope device array, one per GPU, held until the process ends. Every
// piece of it is written before it is read within one call, so nothing has to
// be cleared between calls; calls that overlap on one GPU share the array and
// race.
// ---------------------------------------------------------------------------
namespace hoqri {
namespace {
// the largest workspace hoqri_orth needs: at most kGramBlocks Gram blocks of
// 32 x 32 float64 partials, plus the flag and five 32 x 32 float64 matrices
constexpr size_t kNoAllocScratchBytes =
    256 + (size_t)kGramBlocks * kMaxRank * kMaxRank * 8 + 5 * (size_t)kMaxRank * kMaxRank * 8;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's name is a host-side stand-in, not a
// device address, so host code only ever passes this pointer on).
hoqri_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HOQRI_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HOQRI_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return HOQRI_OK;
}
}  // namespace hoqri

extern "C" size_t hoqri_orth_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

extern "C" hoqri_status hoqri_orth_noalloc(int64_t rows, int32_t cols, const float* d_A, float* d_U, double* d_R,
                                           int32_t* d_status, hipStream_t stream) {
  if (rows < 1 || cols < 1 || cols > kMaxRank || cols > rows || !d_A || !d_U || !d_status) return HOQRI_ERR_ARG;
  if (orth_ws_bytes(rows, cols) > kNoAllocScratchBytes) return HOQRI_ERR_UNSUPPORTED;
  void* ws = nullptr;
  HOQRI_TRY(noalloc_scratch(&ws));
  return launch_orth(rows, cols, d_A, d_U, d_R, d_status, ws, kNoAllocScratchBytes, stream, false);
}
