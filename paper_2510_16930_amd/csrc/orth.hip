// QR step of HOQRI (Alg. 2): an orthonormal basis of A (I x K, K <= 32) by
// CholeskyQR2 with float64 Gram matrices and Cholesky factors:
//   W1 = A^T A, R1 = chol(W1), Q1 = A R1^-1 (never stored), W2 = Q1^T Q1,
//   R2 = chol(W2), U = A (R2 R1)^-1 = A M with M = R1^-1 R2^-1.
// Both Cholesky factors have a positive diagonal, so U is the thin QR factor
// with diag(R) > 0 (the basis the paper leaves free, made unique).
// A Cholesky pivot <= 1e-13 * trace(W) (or not finite) flags breakdown: A is
// numerically rank deficient; U is then left untouched.
//
// Memory traffic: two reads of A for the Grams and one read + one write for
// the final product; the K x K work runs in a single workgroup.
#include "passes.h"

#include <vector>

namespace hoqri {
namespace {

constexpr int kT = 256;
constexpr int kChunk = 32;    // rows staged per step
constexpr double kBreakRel = 1e-13;

int gram_blocks(int64_t rows) {
  int64_t nb = (rows + 1023) / 1024;
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return (int)nb;
}

// Partial Gram of rows [r0, r1): part[e * nb + block] for entry e = p*K + q.
// With M != null the rows are first multiplied by the upper-triangular M
// (float64), i.e. the Gram of A M.
__device__ inline int batch_item(const int32_t* first, int count, int b) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ inline void gram_body(const GramArgs& g, const int blk) {
  __shared__ double rowsd[kChunk][kMaxRank + 1];
  __shared__ double Ms[kMaxRank][kMaxRank];
  const float* A = g.A;
  const int64_t rows = g.rows;
  const int K = g.K;
  const double* M = g.M;
  double* part = g.part;
  const int nb = g.nb;
  const int64_t per = (rows + nb - 1) / nb;
  const int64_t r0 = blk * per;
  int64_t r1 = r0 + per;
  if (r1 > rows) r1 = rows;
  if (M)
    for (int t = threadIdx.x; t < K * K; t += kT) Ms[t / K][t % K] = M[t];
  const int KK = K * K;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  for (int64_t base = r0; base < r1; base += kChunk) {
    const int nr = (int)((r1 - base) < kChunk ? (r1 - base) : kChunk);
    // stage rows (coalesced), optionally times M
    for (int t = threadIdx.x; t < kChunk * K; t += kT) {
      const int r = t / K, c = t - (t / K) * K;
      double v = 0.0;
      if (r < nr) {
        if (M) {
          const float* ar = A + (base + r) * K;
          for (int k = 0; k <= c; ++k) v += (double)ar[k] * Ms[k][c];
        } else {
          v = (double)A[(base + r) * K + c];
        }
      }
      rowsd[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = threadIdx.x + j * kT;
      if (e < KK) {
        const int p = e / K, q = e - (e / K) * K;
        double s = 0.0;
        for (int r = 0; r < nr; ++r) s += rowsd[r][p] * rowsd[r][q];
        acc[j] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = threadIdx.x + j * kT;
    if (e < KK) part[(size_t)e * nb + blk] = acc[j];
  }
}

__global__ __launch_bounds__(kT) void k_gram(GramArgs g) { gram_body(g, blockIdx.x); }

__global__ __launch_bounds__(kT) void k_gram_b(const GramArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  gram_body(d[r], blockIdx.x - first[r]);
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

// Cholesky W = R^T R (R upper, positive diagonal) and Rinv = R^-1, in one
// workgroup. First pass (Mprev null): Mout = Rinv, Rout = R, *flag = breakdown.
// Second pass: Mout = Mprev * Rinv, Rout = R * Rprev, *flag |= breakdown, and
// on breakdown either *skipped += 1 (when a counter is given: the factor is
// left as it was) or *status = HOQRI_ERR_BREAKDOWN; without breakdown *status
// = 0 unless `sticky` (then an earlier breakdown recorded in *status is kept).
__device__ inline void chol_body(const CholArgs& c) {
  const double* W = c.W;
  const int K = c.K;
  const double* Mprev = c.Mprev;
  const double* Rprev = c.Rprev;
  double* Mout = c.Mout;
  double* Rout = c.Rout;
  int32_t* flag = c.flag;
  int32_t* status = c.status;
  const int sticky = c.sticky;
  int32_t* skipped = c.skipped;
  __shared__ double L[kMaxRank][kMaxRank + 1];   // holds R (upper)
  __shared__ double Ri[kMaxRank][kMaxRank + 1];  // R^-1
  __shared__ double tr;
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int e = t; e < K * K; e += kT) {
    L[e / K][e % K] = W[e];
    Ri[e / K][e % K] = 0.0;
  }
  if (t == 0) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += W[k * K + k];
    tr = s;
    bad = (Mprev && *flag != 0) ? 1 : 0;
  }
  __syncthreads();
  // right-looking Cholesky on the upper triangle: row k of R
  for (int k = 0; k < K; ++k) {
    if (t == 0) {
      const double piv = L[k][k];
      if (!(piv > kBreakRel * tr) || !(piv < 1e300)) bad = 1;
      L[k][k] = sqrt(piv > 0.0 ? piv : 1.0);
    }
    __syncthreads();
    const double d = L[k][k];
    for (int j = k + 1 + t; j < K; j += kT) L[k][j] /= d;
    __syncthreads();
    for (int e = t; e < K * K; e += kT) {
      const int i = e / K, j = e % K;
      if (i > k && j >= i) L[i][j] -= L[k][i] * L[k][j];
    }
    __syncthreads();
  }
  // inverse of the upper-triangular R, one column per thread
  for (int j = t; j < K; j += kT) {
    for (int i = j; i >= 0; --i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) s -= L[i][k] * Ri[k][j];
      Ri[i][j] = s / L[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < K * K; e += kT) {
    const int i = e / K, j = e % K;
    double m = 0.0, r = 0.0;
    if (Mprev) {
      // (Mprev * Rinv)[i][j], both upper triangular
      for (int k = i; k <= j; ++k) m += Mprev[i * K + k] * Ri[k][j];
      if (Rout && Rprev)
        for (int k = i; k <= j; ++k) r += L[i][k] * Rprev[k * K + j];
    } else {
      m = (j >= i) ? Ri[i][j] : 0.0;
      r = (j >= i) ? L[i][j] : 0.0;
    }
    if (j < i) m = r = 0.0;
    Mout[e] = m;
    if (Rout) Rout[e] = r;
  }
  if (t == 0) {
    *flag = bad;
    if (Mprev) {
      if (bad) {
        if (skipped) *skipped += 1;  // the caller keeps its previous factor
        else *status = HOQRI_ERR_BREAKDOWN;
      } else if (!sticky) {
        *status = 0;
      }
    }
  }
}

__global__ __launch_bounds__(kT) void k_chol(CholArgs c) { chol_body(c); }

__global__ __launch_bounds__(kT) void k_chol_b(const CholArgs* d, const int32_t* first, int count) {
  chol_body(d[batch_item(first, count, blockIdx.x)]);
}

// U = A M (M upper triangular), rows staged in LDS so U may alias A, then
// rows [rows, zero_to) of U set to zero. Skipped entirely when this
// factorisation broke down (*flag != 0): U keeps its previous contents.
__device__ inline void apply_body(const ApplyArgs& a, const int blk) {
  __shared__ float tile[64][kMaxRank + 1];
  __shared__ double Ms[kMaxRank][kMaxRank];
  const float* A = a.A;
  const int64_t rows = a.rows;
  const int K = a.K;
  const double* M = a.M;
  float* U = a.U;
  if (*a.flag != 0) return;
  for (int t = threadIdx.x; t < K * K; t += kT) Ms[t / K][t % K] = M[t];
  for (int64_t base = blk * (int64_t)64; base < rows; base += (int64_t)a.nblk * 64) {
    const int nr = (int)((rows - base) < 64 ? (rows - base) : 64);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * K; t += kT) tile[t / K][t % K] = A[base * K + t];
    __syncthreads();
    for (int t = threadIdx.x; t < nr * K; t += kT) {
      const int r = t / K, c = t - (t / K) * K;
      double v = 0.0;
      for (int k = 0; k <= c; ++k) v += (double)tile[r][k] * Ms[k][c];
      U[base * K + t] = (float)v;
    }
  }
  // rows [rows, zero_to) of U (rows of empty slices) become zero with the update
  const int64_t ztot = (a.zero_to - rows) * K;
  for (int64_t t = blk * (int64_t)kT + threadIdx.x; t < ztot; t += (int64_t)a.nblk * kT) U[rows * K + t] = 0.f;
}

__global__ __launch_bounds__(kT) void k_apply(ApplyArgs a) { apply_body(a, blockIdx.x); }

__global__ __launch_bounds__(kT) void k_apply_b(const ApplyArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  apply_body(d[r], blockIdx.x - first[r]);
}

__global__ void k_orth_err(const double* W, int K, double* out) {
  __shared__ double sh[kT];
  double s = 0.0;
  for (int e = threadIdx.x; e < K * K; e += kT) {
    const double d = W[e] - ((e / K) == (e % K) ? 1.0 : 0.0);
    s += d * d;
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
  job->c2 = CholArgs{o.W, K, o.M1, o.R1, o.M, R ? R : o.R, o.flag, status, (int32_t)sticky, skipped};
  int64_t ab = (rows + 63) / 64;
  if (ab > 4096) ab = 4096;
  job->ap = ApplyArgs{A, rows, K, o.M, U, o.flag, (int32_t)ab, zero_to > rows ? zero_to : rows};
  job->gram_blocks = nb;
  job->red_blocks = K * K;
  job->apply_blocks = (int)ab;
  return HOQRI_OK;
}

hoqri_status launch_orth(int64_t rows, int32_t K, const float* A, float* U, double* R, int32_t* status, void* ws,
                         size_t ws_bytes, hipStream_t s, bool sticky, int32_t* skipped, int64_t zero_to) {
  OrthJob j;
  HOQRI_TRY(prepare_orth(rows, K, A, U, R, status, ws, ws_bytes, sticky, &j, skipped, zero_to));
  hipLaunchKernelGGL(k_gram, dim3(j.gram_blocks), dim3(kT), 0, s, j.g1);
  hipLaunchKernelGGL(k_gram_reduce, dim3(j.red_blocks), dim3(kT), 0, s, j.r1);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kT), 0, s, j.c1);
  hipLaunchKernelGGL(k_gram, dim3(j.gram_blocks), dim3(kT), 0, s, j.g2);
  hipLaunchKernelGGL(k_gram_reduce, dim3(j.red_blocks), dim3(kT), 0, s, j.r2);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kT), 0, s, j.c2);
  hipLaunchKernelGGL(k_apply, dim3(j.apply_blocks), dim3(kT), 0, s, j.ap);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

bool stage_orth_group(const OrthJob* const* jobs, int n, Staging& st, OrthGroup* g) {
  if (n < 1 || n > 1024) return false;
  std::vector<GramArgs> g1(n), g2(n);
  std::vector<GRedArgs> r1(n), r2(n);
  std::vector<CholArgs> c1(n), c2(n);
  std::vector<ApplyArgs> ap(n);
  std::vector<int32_t> nb_g(n), nb_r(n), ones(n), nb_a(n);
  for (int i = 0; i < n; ++i) {
    g1[i] = jobs[i]->g1;
    g2[i] = jobs[i]->g2;
    r1[i] = jobs[i]->r1;
    r2[i] = jobs[i]->r2;
    c1[i] = jobs[i]->c1;
    c2[i] = jobs[i]->c2;
    ap[i] = jobs[i]->ap;
    nb_g[i] = jobs[i]->gram_blocks;
    nb_r[i] = jobs[i]->red_blocks;
    ones[i] = 1;
    nb_a[i] = jobs[i]->apply_blocks;
  }
  return stage_table(st, g1.data(), nb_g.data(), n, &g->g1) && stage_table(st, r1.data(), nb_r.data(), n, &g->r1) &&
         stage_table(st, c1.data(), ones.data(), n, &g->c1) && stage_table(st, g2.data(), nb_g.data(), n, &g->g2) &&
         stage_table(st, r2.data(), nb_r.data(), n, &g->r2) && stage_table(st, c2.data(), ones.data(), n, &g->c2) &&
         stage_table(st, ap.data(), nb_a.data(), n, &g->ap);
}

hoqri_status launch_orth_group(const OrthGroup& g, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_b, dim3(g.g1.blocks), dim3(kT), 0, s, (const GramArgs*)g.g1.descs, g.g1.first, g.g1.count);
  hipLaunchKernelGGL(k_gram_reduce_b, dim3(g.r1.blocks), dim3(kT), 0, s, (const GRedArgs*)g.r1.descs, g.r1.first,
                     g.r1.count);
  hipLaunchKernelGGL(k_chol_b, dim3(g.c1.blocks), dim3(kT), 0, s, (const CholArgs*)g.c1.descs, g.c1.first, g.c1.count);
  hipLaunchKernelGGL(k_gram_b, dim3(g.g2.blocks), dim3(kT), 0, s, (const GramArgs*)g.g2.descs, g.g2.first, g.g2.count);
  hipLaunchKernelGGL(k_gram_reduce_b, dim3(g.r2.blocks), dim3(kT), 0, s, (const GRedArgs*)g.r2.descs, g.r2.first,
                     g.r2.count);
  hipLaunchKernelGGL(k_chol_b, dim3(g.c2.blocks), dim3(kT), 0, s, (const CholArgs*)g.c2.descs, g.c2.first, g.c2.count);
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
