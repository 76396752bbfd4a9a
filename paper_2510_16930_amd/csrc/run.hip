// Public entry points for the core, TTMcTC and the HOQRI loop (Alg. 2).
//
// One sweep = one HOQRI iteration: for n = 1..N, the core G from the current
// factors (the core Alg. 3 forms first), A^(n) = TTMcTC(X, {U}, n), U^(n) = an
// orthonormal basis of A^(n). Factors updated earlier in the sweep are used by
// later modes (the single-mode update rule of §5). The core computed after the
// last mode of a sweep is reused as the first core of the next sweep, so f
// after every sweep is known without an extra pass, and the core returned at
// the end belongs to the returned factors (last line of Alg. 2).
#include <cmath>
#include <cstring>

#include "common.h"

namespace hoqri {
namespace {

__global__ void k_fill_i32(int32_t* x, int n, int32_t v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = v;
}

// hist[t * N + 0] = fsweep[t] for t < T (the first mode of each sweep sees the
// core of the previous sweep's end).
__global__ void k_hist_first(const double* fsweep, int T, int N, double* hist) {
  for (int t = threadIdx.x; t < T; t += blockDim.x) hist[(size_t)t * N] = fsweep[t];
}

hoqri_status check_plan(const hoqri_plan* p) {
  if (!p) return HOQRI_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HOQRI_ERR_HIP;
  if (dev != p->device) return HOQRI_ERR_ARG;
  return HOQRI_OK;
}

// Up[r, :] = U[inv[r], :] (rows into the plan's label order)
__global__ void k_rows_to_labels(const float* U, const int32_t* inv, int64_t I, int32_t K, float* Up) {
  const int64_t total = I * K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / K;
    Up[t] = U[(size_t)inv[r] * K + (t - r * K)];
  }
}

// U[inv[r], :] = Up[r, :] (rows back to the caller's order)
__global__ void k_rows_from_labels(const float* Up, const int32_t* inv, int64_t I, int32_t K, float* U) {
  const int64_t total = I * K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / K;
    U[(size_t)inv[r] * K + (t - r * K)] = Up[t];
  }
}

__global__ void k_fill_f32(float* x, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// GG[p][q] = sum over the other indices of G(p, .) G(q, .) in mode n (float64).
struct Ranks {
  int32_t K[kMaxOrder];
};
__global__ __launch_bounds__(256) void k_ggt(const float* G, int N, int mode, Ranks R, double* GG) {
  const int32_t* Kd = R.K;
  const int Kn = Kd[mode];
  int64_t stride = 1, other = 1;
  for (int m = N - 1; m > mode; --m) stride *= Kd[m];
  for (int m = 0; m < N; ++m)
    if (m != mode) other *= Kd[m];
  // element (p, o) of the unfolding: o = hi * stride + lo with lo < stride
  for (int e = threadIdx.x; e < Kn * Kn; e += blockDim.x) {
    const int pr = e / Kn, pc = e - (e / Kn) * Kn;
    double acc = 0.0;
    for (int64_t o = 0; o < other; ++o) {
      const int64_t hi = o / stride, lo = o - hi * stride;
      const int64_t base = hi * stride * Kn + lo;
      acc += (double)G[base + (int64_t)pr * stride] * (double)G[base + (int64_t)pc * stride];
    }
    GG[e] = acc;
  }
}

// Per-block partial of ||A - U GG||_F^2 over rows x K elements (float64).
__global__ __launch_bounds__(256) void k_grad_rows(const float* A, const float* U, const double* GG, int64_t rows,
                                                   int32_t K, double* part) {
  __shared__ double gg[32 * 32];
  __shared__ double sh[256];
  for (int e = threadIdx.x; e < K * K; e += 256) gg[e] = GG[e];
  __syncthreads();
  const int64_t total = rows * K;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int64_t r = t / K;
    const int c = (int)(t - r * K);
    double v = (double)A[t];
    for (int k = 0; k < K; ++k) v -= (double)U[r * K + k] * gg[k * K + c];
    acc += v * v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out = 4 * (sum of the partials), in order
__global__ void k_grad_final(const double* part, int n, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 4.0 * sh[0];
}

// sum of the N values of row t of the history
__global__ void k_grad_sweep(const double* hist, int t, int N, double* out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += hist[(size_t)t * N + n];
    out[0] = s;
  }
}

int grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}


hoqri_status check_prec(hoqri_prec prec, int* op) {
  if (prec == HOQRI_FP32) *op = OP_FP32;
  else if (prec == HOQRI_BF16) *op = OP_BF16;
  else if (prec == HOQRI_FP16) *op = OP_FP16;
  else return HOQRI_ERR_ARG;
  return HOQRI_OK;
}

// Operands of the segment passes: the plan's label-order factors and, for the
// 16-bit forms, their copies refreshed from rows [0, R_m) (only rows of
// nonempty slices are ever gathered).
Operands plan_operands(hoqri_plan* p, int op) {
  Operands o;
  o.prec = op;
  o.U32 = p->sc.Up;
  o.U16 = p->sc.Uh;
  return o;
}

// status[2]: an FP16 factor copy met an entry of magnitude >= 1.5 (see k_cast16)
hoqri_status refresh16(hoqri_plan* p, int op, int mode, hipStream_t s) {
  if (op == OP_FP32) return HOQRI_OK;
  return launch_cast16(p->sc.Up[mode], p->md[mode].R, p->K[mode], p->sc.Uh[mode], op, s, p->sc.status + 2);
}

// FP16 form: the caller's factors must have entries of magnitude below 1.5
// (orthonormal columns give at most 1) so their scaled float16 copies stay in
// range. Clears the flag, casts, and reads it back (one synchronisation) before
// any pass runs; HOQRI_ERR_ARG otherwise.
hoqri_status refresh16_checked(hoqri_plan* p, int op, int skip_mode, hipStream_t s) {
  if (op != OP_FP16) {
    for (int n = 0; n < p->N; ++n)
      if (n != skip_mode) HOQRI_TRY(refresh16(p, op, n, s));
    return HOQRI_OK;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p->sc.status + 2, 1, 0);
  for (int n = 0; n < p->N; ++n)
    if (n != skip_mode) HOQRI_TRY(refresh16(p, op, n, s));
  int32_t flag = 0;
  HOQRI_HIP_TRY(hipMemcpyAsync(&flag, p->sc.status + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HOQRI_HIP_TRY(hipStreamSynchronize(s));
  return flag ? HOQRI_ERR_ARG : HOQRI_OK;
}

}  // namespace

hoqri_status to_labels(hoqri_plan* p, const float* const* U, hipStream_t s) {
  for (int n = 0; n < p->N; ++n) {
    const int64_t I = p->dims[n];
    hipLaunchKernelGGL(k_rows_to_labels, dim3(grid_of(I * p->K[n])), dim3(256), 0, s, U[n], p->md[n].inv, I, p->K[n],
                       p->sc.Up[n]);
  }
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status from_labels(hoqri_plan* p, float* const* U, hipStream_t s) {
  for (int n = 0; n < p->N; ++n)
    hipLaunchKernelGGL(k_rows_from_labels, dim3(grid_of(p->dims[n] * p->K[n])), dim3(256), 0, s, p->sc.Up[n],
                       p->md[n].inv, p->dims[n], p->K[n], U[n]);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status zero_empty_rows(hoqri_plan* p, int n, hipStream_t s) {
  const int64_t Rn = p->md[n].R;
  if (p->dims[n] > Rn) {
    const int64_t ne = (p->dims[n] - Rn) * p->K[n];
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(ne)), dim3(256), 0, s, p->sc.Up[n] + Rn * p->K[n], ne, 0.f);
    HOQRI_HIP_TRY(hipGetLastError());
  }
  return HOQRI_OK;
}

hoqri_status launch_grad(hoqri_plan* p, int mode, const float* A, const float* U, const float* G, double* out,
                         hipStream_t s) {
  double* GG = p->sc.gscr;
  double* part = p->sc.gscr + kMaxRank * kMaxRank;
  Ranks Kd{};
  for (int m = 0; m < p->N; ++m) Kd.K[m] = p->K[m];
  hipLaunchKernelGGL(k_ggt, dim3(1), dim3(256), 0, s, G, p->N, mode, Kd, GG);
  const int64_t total = p->dims[mode] * p->K[mode];
  int64_t nb = (total + 255) / 256;
  if (nb > kGradParts) nb = kGradParts;
  hipLaunchKernelGGL(k_grad_rows, dim3((unsigned)nb), dim3(256), 0, s, A, U, (const double*)GG, p->dims[mode],
                     p->K[mode], part);
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), 0, s, (const double*)part, (int)nb, out);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status fill_i32(int32_t* x, int n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, x, n, v);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

}  // namespace hoqri

using namespace hoqri;

extern "C" hoqri_status hoqri_core(hoqri_plan* p, const float* const* d_U, float* d_G, double* d_f, hoqri_prec prec,
                                   hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  if (!d_U || !d_G) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!d_U[n]) return HOQRI_ERR_ARG;
  int op = 0;
  HOQRI_TRY(check_prec(prec, &op));
  HOQRI_TRY(to_labels(p, d_U, stream));
  HOQRI_TRY(refresh16_checked(p, op, -1, stream));
  return launch_core(p, plan_operands(p, op), d_G, d_f, stream);
}

extern "C" hoqri_status hoqri_ttmctc(hoqri_plan* p, int32_t mode, const float* const* d_U, const float* d_G,
                                     float* d_A, hoqri_prec prec, hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  if (mode < 0 || mode >= p->N || !d_U || !d_G || !d_A) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!d_U[n]) return HOQRI_ERR_ARG;
  int op = 0;
  HOQRI_TRY(check_prec(prec, &op));
  HOQRI_TRY(to_labels(p, d_U, stream));
  HOQRI_TRY(refresh16_checked(p, op, mode, stream));
  return launch_ttmctc(p, mode, plan_operands(p, op), d_G, d_A, p->md[mode].inv, stream);
}

extern "C" hoqri_status hoqri_core_rows(hoqri_plan* p, int32_t mode, const float* const* d_U,
                                        const float* d_G_stage, float* d_G, double* d_f, hoqri_prec prec,
                                        hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  if (mode < 0 || mode >= p->N || !d_U || !d_G_stage || !d_G) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!d_U[n]) return HOQRI_ERR_ARG;
  int op = 0;
  HOQRI_TRY(check_prec(prec, &op));
  if (!p->yfuse) return HOQRI_ERR_UNSUPPORTED;
  if (!segpass_supported(p, mode) && !(generic_supported(p) && (op == OP_FP32 || op == OP_BF16)))
    return HOQRI_ERR_UNSUPPORTED;
  HOQRI_TRY(to_labels(p, d_U, stream));
  HOQRI_TRY(refresh16_checked(p, op, -1, stream));
  const Operands ops = plan_operands(p, op);
  HOQRI_TRY(launch_ttmctc(p, mode, ops, d_G_stage, p->sc.A, nullptr, stream, true));
  return launch_ycore(p, mode, d_G, d_f ? d_f : p->sc.f_dev, stream, op != OP_FP32, ttm_rows_bf16(p, mode, op));
}

extern "C" hoqri_status hoqri_sketch_start(hoqri_plan* p, const float* const* d_Omega, const float* d_Gamma,
                                          float* const* d_U_out, hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  if (!d_Omega || !d_Gamma || !d_U_out) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!d_Omega[n] || !d_U_out[n]) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!segpass_supported(p, n) && !generic_supported(p)) return HOQRI_ERR_UNSUPPORTED;
  for (int n = 0; n < p->N; ++n)
    if (p->md[n].R < p->K[n]) return HOQRI_ERR_BREAKDOWN;
  // the random factors in label order (the pass reads them there)
  HOQRI_TRY(to_labels(p, d_Omega, stream));
  const Operands ops = plan_operands(p, OP_FP32);
  int32_t* status = p->sc.status;
  HOQRI_TRY(fill_i32(status, 4, 0, stream));
  for (int n = 0; n < p->N; ++n) {
    // sketch of mode n (label-order rows), its basis in place, rows of empty slices zeroed
    HOQRI_TRY(launch_ttmctc(p, n, ops, d_Gamma, p->sc.A, nullptr, stream));
    HOQRI_TRY(launch_orth(p->md[n].R, p->K[n], p->sc.A, p->sc.A, nullptr, status, p->sc.orth_ws,
                          p->sc.orth_ws_bytes, stream, true, nullptr, p->dims[n]));
    hipLaunchKernelGGL(k_rows_from_labels, dim3(grid_of(p->dims[n] * p->K[n])), dim3(256), 0, stream, p->sc.A,
                       p->md[n].inv, p->dims[n], p->K[n], d_U_out[n]);
    HOQRI_HIP_TRY(hipGetLastError());
  }
  int32_t st = 0;
  HOQRI_HIP_TRY(hipMemcpyAsync(&st, status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipStreamSynchronize(stream));
  return st != 0 ? HOQRI_ERR_BREAKDOWN : HOQRI_OK;
}

extern "C" hoqri_status hoqri_run(hoqri_plan* p, float* const* d_U_inout, float* d_G_out, double* d_f_hist,
                                  const hoqri_run_opts* opts, hoqri_run_stats* stats, hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  if (!d_U_inout || !d_G_out || !opts || !stats) return HOQRI_ERR_ARG;
  for (int n = 0; n < p->N; ++n)
    if (!d_U_inout[n]) return HOQRI_ERR_ARG;
  if (opts->max_sweeps < 0 || opts->max_sweeps > kMaxSweeps || opts->check_every < 1 || !(opts->tol >= 0.0))
    return HOQRI_ERR_ARG;
  int op = 0;
  HOQRI_TRY(check_prec(opts->prec, &op));
  // modes beyond the segment passes: float32, and bfloat16 where the split-Kronecker pass stores rows
  for (int n = 0; n < p->N; ++n)
    if (!segpass_supported(p, n) &&
        (!generic_supported(p) || !(op == OP_FP32 || (op == OP_BF16 && p->yfuse))))
      return HOQRI_ERR_UNSUPPORTED;
  if (opts->method != HOQRI_METHOD_HOQRI && opts->method != HOQRI_METHOD_HOOI) return HOQRI_ERR_ARG;
  if (opts->inner_iters < 0 || opts->inner_iters > 1000) return HOQRI_ERR_ARG;
  if (opts->stop_rule != HOQRI_STOP_REL_F && opts->stop_rule != HOQRI_STOP_ERR_CHANGE) return HOQRI_ERR_ARG;
  const bool hooi = opts->method == HOQRI_METHOD_HOOI;
  const int inner = hooi && opts->inner_iters > 1 ? opts->inner_iters : 1;
  if (hooi && !p->yfuse) return HOQRI_ERR_UNSUPPORTED;
  if (op == OP_FP16) {
    float as, ys;
    if (!fp16_scales(p, p->N - 1, &as, &ys)) return HOQRI_ERR_UNSUPPORTED;
  }

  const int N = p->N;
  int32_t* status = p->sc.status;
  double* fsw = p->sc.fsweep;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, status, 4, 0);
  HOQRI_HIP_TRY(hipGetLastError());

  if (opts->orthonormalize_input) {
    for (int n = 0; n < N; ++n)
      HOQRI_TRY(launch_orth(p->dims[n], p->K[n], d_U_inout[n], d_U_inout[n], nullptr, status, p->sc.orth_ws,
                            p->sc.orth_ws_bytes, stream, true));
  }
  // the loop works on row-relabelled copies of the factors (label order)
  for (int n = 0; n < N; ++n)
    if (p->md[n].R < p->K[n]) return HOQRI_ERR_BREAKDOWN;  // fewer nonempty slices than K_n
  HOQRI_TRY(to_labels(p, d_U_inout, stream));
  float* const* Up = p->sc.Up;
  const Operands ops = plan_operands(p, op);
  HOQRI_TRY(refresh16_checked(p, op, -1, stream));
  // core of the starting factors
  HOQRI_TRY(launch_core(p, ops, d_G_out, fsw + 0, stream));

  int T = 0;
  double f_last = 0.0, f_prev = 0.0, rel = 0.0;
  bool have_prev = false;
  // relative approximation error sqrt(max(||X||^2 - f, 0) / ||X||^2) (§2.2: for
  // orthonormal factors and the optimal core the squared error is ||X||^2 - f)
  const auto rel_err = [&](double f) { return std::sqrt(std::fmax(p->normx2 - f, 0.0) / p->normx2); };

  if (!(opts->grad_tol >= 0.0)) return HOQRI_ERR_ARG;
  const bool grad_on = opts->d_grad_hist != nullptr || opts->grad_tol > 0.0;
  double* ghist = p->sc.gscr + kMaxRank * kMaxRank + kGradParts;  // [kMaxSweeps][N]
  // With stored rows, the pass of mode n keeps Y_(n) (which does not involve
  // U^(n)), and the core of the updated factors is U^(n)T Y_(n): no separate
  // core pass between mode updates.
  const bool fuse = p->yfuse != 0;
  for (int t = 0; t < opts->max_sweeps; ++t) {
    for (int n = 0; n < N; ++n) {
      if (n > 0 && !fuse) {
        double* fdst = d_f_hist ? d_f_hist + (size_t)t * N + n : p->sc.f_dev;
        HOQRI_TRY(launch_core(p, ops, d_G_out, fdst, stream));
      }
      HOQRI_TRY(launch_ttmctc(p, n, ops, d_G_out, p->sc.A, nullptr, stream, fuse));
      // Riemannian gradient at the current point, before U^(n) moves (A rows of
      // empty slices are zero, all I_n rows of U take part)
      if (grad_on) HOQRI_TRY(launch_grad(p, n, p->sc.A, Up[n], d_G_out, ghist + (size_t)t * N + n, stream));
      // rows R_n.. of A are zero (empty slices): orthonormalise the first R_n rows
      // and keep the remaining rows of the factor at zero
      const int64_t Rn = p->md[n].R;
      // f after mode n: the next mode's starting point, or the sweep's end
      double* fdst = n + 1 < N ? (d_f_hist ? d_f_hist + (size_t)t * N + n + 1 : p->sc.f_dev) : fsw + t + 1;
      for (int it = 0; it < inner; ++it) {
        {
          TimerScope to(p, HOQRI_KERNEL_ORTH, stream);
          // rows R_n.. (empty slices) of the new factor are zeroed by the same
          // launch, and the 16-bit forms' copy of rows ..R_n is written with it
          HOQRI_TRY(launch_orth(Rn, p->K[n], p->sc.A, Up[n], nullptr, status, p->sc.orth_ws, p->sc.orth_ws_bytes,
                                stream, true, opts->keep_on_breakdown ? status + 1 : nullptr, p->dims[n],
                                op != OP_FP32 ? p->sc.Uh[n] : nullptr, op, p->sc.status + 2));
        }
        // the 16-bit forms take the core from the stored rows in split bfloat16
        // (the 2 x 2-block BF16 pass stores them in bfloat16)
        if (fuse) HOQRI_TRY(launch_ycore(p, n, d_G_out, fdst, stream, op != OP_FP32, ttm_rows_bf16(p, n, op)));
        // HOOI: next orthogonal-iteration step A = Y_(n) (Y_(n)^T U) from the stored rows
        if (it + 1 < inner) HOQRI_TRY(launch_rows_a(p, n, d_G_out, p->sc.A, stream, ttm_rows_bf16(p, n, op)));
      }
    }
    if (!fuse) HOQRI_TRY(launch_core(p, ops, d_G_out, fsw + t + 1, stream));
    T = t + 1;
    if (T % opts->check_every == 0 || T == opts->max_sweeps) {
      double fv[2];
      double gsum = 0.0;
      int32_t st = 0, pool_fault = 0;
      HOQRI_HIP_TRY(hipMemcpyAsync(fv, fsw + T - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
      HOQRI_HIP_TRY(hipMemcpyAsync(&st, status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
      HOQRI_HIP_TRY(hipMemcpyAsync(&pool_fault, status + 3, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
      if (opts->grad_tol > 0.0) {
        hipLaunchKernelGGL(k_grad_sweep, dim3(1), dim3(64), 0, stream, (const double*)ghist, T - 1, N, p->sc.f_dev + 16);
        HOQRI_HIP_TRY(hipMemcpyAsync(&gsum, p->sc.f_dev + 16, sizeof(double), hipMemcpyDeviceToHost, stream));
      }
      HOQRI_HIP_TRY(hipStreamSynchronize(stream));
      if (pool_fault != 0) return HOQRI_ERR_HIP;  // a slice-pool wait timed out: results are not valid
      if (st != 0) return HOQRI_ERR_BREAKDOWN;
      f_prev = fv[0];
      f_last = fv[1];
      have_prev = true;
      rel = f_last > 0 ? std::fabs(f_last - f_prev) / f_last : 0.0;
      // both rules compare the last two sweeps (f_prev: the sweep before, or the
      // starting factors' f after the first sweep)
      if (opts->tol > 0.0) {
        if (opts->stop_rule == HOQRI_STOP_REL_F && std::fabs(f_last - f_prev) <= opts->tol * f_last) break;
        if (opts->stop_rule == HOQRI_STOP_ERR_CHANGE && std::fabs(rel_err(f_last) - rel_err(f_prev)) < opts->tol)
          break;
      }
      if (opts->grad_tol > 0.0 && std::sqrt(std::fmax(gsum, 0.0)) <= opts->grad_tol * f_last) break;
    }
  }
  // the returned core and f are those of the final factors with float32
  // operands, whatever form the sweeps used
  if (op != OP_FP32) HOQRI_TRY(launch_core(p, plan_operands(p, OP_FP32), d_G_out, fsw + T, stream));
  if (opts->d_grad_hist && T > 0)
    HOQRI_HIP_TRY(hipMemcpyAsync(opts->d_grad_hist, ghist, (size_t)T * N * sizeof(double), hipMemcpyDeviceToDevice,
                                 stream));
  double glast = -1.0;
  if (grad_on && T > 0) {
    hipLaunchKernelGGL(k_grad_sweep, dim3(1), dim3(64), 0, stream, (const double*)ghist, T - 1, N, p->sc.f_dev + 16);
    HOQRI_HIP_TRY(hipMemcpyAsync(&glast, p->sc.f_dev + 16, sizeof(double), hipMemcpyDeviceToHost, stream));
  }
  if (d_f_hist && T > 0) {
    hipLaunchKernelGGL(k_hist_first, dim3(1), dim3(256), 0, stream, fsw, T, N, d_f_hist);
    HOQRI_HIP_TRY(hipGetLastError());
  }
  // factors back to the caller's row order, then final statistics
  if (T > 0) HOQRI_TRY(from_labels(p, d_U_inout, stream));
  double errs[kMaxOrder] = {0, 0, 0, 0};
  for (int n = 0; n < N; ++n)
    HOQRI_TRY(launch_orth_err(p->dims[n], p->K[n], d_U_inout[n], p->sc.f_dev + 8 + n, p->sc.orth_ws,
                              p->sc.orth_ws_bytes, stream));
  double fend = 0.0;
  int32_t st = 0, skips = 0, pool_fault = 0;
  HOQRI_HIP_TRY(hipMemcpyAsync(errs, p->sc.f_dev + 8, N * sizeof(double), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipMemcpyAsync(&fend, fsw + T, sizeof(double), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipMemcpyAsync(&st, status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipMemcpyAsync(&skips, status + 1, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipMemcpyAsync(&pool_fault, status + 3, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HOQRI_HIP_TRY(hipStreamSynchronize(stream));
  if (pool_fault != 0) return HOQRI_ERR_HIP;
  if (st != 0) return HOQRI_ERR_BREAKDOWN;
  (void)have_prev;
  stats->skipped_updates = skips;
  stats->grad_norm2 = glast;
  stats->sweeps = T;
  stats->norm_x2 = p->normx2;
  stats->f = fend;
  stats->fit = 1.0 - std::sqrt(std::fmax(p->normx2 - fend, 0.0)) / std::sqrt(p->normx2);
  stats->rel_change = rel;
  double emax = 0.0;
  for (int n = 0; n < N; ++n) emax = std::fmax(emax, errs[n]);
  stats->orth_err_max = emax;
  return HOQRI_OK;
}

namespace hoqri {
void timing_release(hoqri_plan* p) {
  for (int k = 0; k < kTimingKinds; ++k) {
    if (p->timing.ev[k]) {
      for (int i = 0; i < 2 * kTimingCap; ++i) (void)hipEventDestroy(p->timing.ev[k][i]);
      delete[] p->timing.ev[k];
      p->timing.ev[k] = nullptr;
    }
  }
  p->timing.enabled = false;
}
}  // namespace hoqri

extern "C" hoqri_status hoqri_timing_enable(hoqri_plan* p, int32_t enable) {
  HOQRI_TRY(check_plan(p));
  for (int k = 0; k < kTimingKinds; ++k) p->timing.count[k] = 0;
  if (!enable) {
    p->timing.enabled = false;
    return HOQRI_OK;
  }
  for (int k = 0; k < kTimingKinds; ++k) {
    if (!p->timing.ev[k]) {
      p->timing.ev[k] = new hipEvent_t[2 * kTimingCap];
      for (int i = 0; i < 2 * kTimingCap; ++i)
        if (hipEventCreate(&p->timing.ev[k][i]) != hipSuccess) return HOQRI_ERR_HIP;
    }
  }
  p->timing.enabled = true;
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_timing_read(hoqri_plan* p, int32_t kind, int64_t* launches, double* total_ms) {
  HOQRI_TRY(check_plan(p));
  if (kind < 0 || kind >= kTimingKinds || !launches || !total_ms) return HOQRI_ERR_ARG;
  const int64_t n = p->timing.count[kind];
  double tot = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    HOQRI_HIP_TRY(hipEventSynchronize(p->timing.ev[kind][2 * i + 1]));
    float ms = 0.f;
    HOQRI_HIP_TRY(hipEventElapsedTime(&ms, p->timing.ev[kind][2 * i], p->timing.ev[kind][2 * i + 1]));
    tot += ms;
  }
  *launches = n;
  *total_ms = tot;
  return HOQRI_OK;
}

// ---------------------------------------------------------------------------
// Launch-shape tuning of the TTMcTC passes: per mode, the number of work
// ranges (nonzeros per wave) and the ranges per workgroup. The autotuner times
// one mode update's passes (the TTMcTC pass and, with stored slice rows, the
// core product that follows it) for each candidate on the plan's own
// nonzeros and keeps the fastest; results are cached in a text file, one line
// per shape class (device, order, ranks, operand form, and the powers of two
// of nnz and of every mode's nonempty slices).
// ---------------------------------------------------------------------------
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

namespace hoqri {
namespace {

int ilog2(int64_t v) {
  int e = 0;
  while (v > 1) {
    v >>= 1;
    ++e;
  }
  return e;
}

std::string tune_key(const hoqri_plan* p, hoqri_prec prec) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  std::ostringstream k;
  k << "hoqri-tune-v1 " << arch << " N=" << p->N << " K=";
  for (int n = 0; n < p->N; ++n) k << (n ? "," : "") << p->K[n];
  k << " prec=" << (int)prec << " nnz=2^" << ilog2(p->nnz) << " R=";
  for (int n = 0; n < p->N; ++n) k << (n ? "," : "") << "2^" << ilog2(p->md[n].R);
  return k.str();
}

hoqri_status validate_tuning(const hoqri_plan* p, const hoqri_tuning* t) {
  for (int n = 0; n < p->N; ++n) {
    if (t->ranges[n] < 1 || t->ranges[n] > p->ranges_cap) return HOQRI_ERR_ARG;
    if (t->waves_per_group[n] < 0 || t->waves_per_group[n] > 64) return HOQRI_ERR_ARG;
  }
  return HOQRI_OK;
}

void apply_tuning(hoqri_plan* p, const hoqri_tuning* t) {
  for (int n = 0; n < p->N; ++n) {
    p->md[n].ranges = t->ranges[n];
    p->md[n].rpw = t->waves_per_group[n];
  }
}

void read_tuning(const hoqri_plan* p, hoqri_tuning* t) {
  *t = hoqri_tuning{};
  for (int n = 0; n < p->N; ++n) {
    t->ranges[n] = p->md[n].ranges;
    t->waves_per_group[n] = p->md[n].rpw;
  }
}

// "key | W_0 rpw_0 W_1 rpw_1 ..." lines; the last line with the key wins
bool cache_lookup(const char* path, const std::string& key, int N, hoqri_tuning* t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const size_t bar = line.find(" | ");
    if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
    std::istringstream in(line.substr(bar + 3));
    hoqri_tuning v{};
    bool ok = true;
    for (int n = 0; n < N && ok; ++n) ok = static_cast<bool>(in >> v.ranges[n] >> v.waves_per_group[n]);
    if (ok) {
      *t = v;
      found = true;
    }
  }
  return found;
}

bool cache_store(const char* path, const std::string& key, int N, const hoqri_tuning& t) {
  std::ofstream f(path, std::ios::app);
  if (!f) return false;
  f << key << " |";
  for (int n = 0; n < N; ++n) f << " " << t.ranges[n] << " " << t.waves_per_group[n];
  f << "\n";
  return static_cast<bool>(f);
}

// Deterministic finite operands for timing: every factor entry 1/sqrt(R_m)
// (the stored rows of nonempty slices), the core 1/sqrt(prod K).
hoqri_status tuning_operands(hoqri_plan* p, int op, hipStream_t s) {
  int64_t PK = 1;
  for (int n = 0; n < p->N; ++n) PK *= p->K[n];
  for (int n = 0; n < p->N; ++n) {
    const int64_t cnt = p->dims[n] * p->K[n];
    const float v = 1.0f / std::sqrt((float)std::max<int64_t>(p->md[n].R, 1));
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(cnt)), dim3(256), 0, s, p->sc.Up[n], cnt, v);
    HOQRI_TRY(refresh16(p, op, n, s));
  }
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(PK)), dim3(256), 0, s, p->sc.G, PK, 1.0f / std::sqrt((float)PK));
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

// Median time (ms) of one mode update's passes with the plan's current tuning.
hoqri_status time_mode(hoqri_plan* p, int n, int op, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
  const Operands ops = plan_operands(p, op);
  const bool fuse = p->yfuse != 0;
  auto once = [&]() -> hoqri_status {
    HOQRI_TRY(launch_ttmctc(p, n, ops, p->sc.G, p->sc.A, nullptr, s, fuse));
    if (fuse) HOQRI_TRY(launch_ycore(p, n, p->sc.G, p->sc.f_dev, s, op != OP_FP32, ttm_rows_bf16(p, n, op)));
    return HOQRI_OK;
  };
  HOQRI_TRY(once());  // warm-up (kernel load, caches)
  float t[3];
  for (int r = 0; r < 3; ++r) {
    HOQRI_HIP_TRY(hipEventRecord(e0, s));
    HOQRI_TRY(once());
    HOQRI_HIP_TRY(hipEventRecord(e1, s));
    HOQRI_HIP_TRY(hipEventSynchronize(e1));
    HOQRI_HIP_TRY(hipEventElapsedTime(&t[r], e0, e1));
  }
  std::sort(t, t + 3);
  *ms = t[1];
  return HOQRI_OK;
}

}  // namespace
}  // namespace hoqri

extern "C" hoqri_status hoqri_plan_get_tuning(const hoqri_plan* p, hoqri_tuning* t) {
  if (!p || !t) return HOQRI_ERR_ARG;
  read_tuning(p, t);
  return HOQRI_OK;
}

extern "C" int32_t hoqri_plan_max_ranges(const hoqri_plan* p) { return p ? p->ranges_cap : 0; }

extern "C" hoqri_status hoqri_plan_set_tuning(hoqri_plan* p, const hoqri_tuning* t) {
  if (!p || !t) return HOQRI_ERR_ARG;
  HOQRI_TRY(validate_tuning(p, t));
  apply_tuning(p, t);
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_autotune(hoqri_plan* p, hoqri_prec prec, const char* cache_path, hoqri_tuning* chosen,
                                       int32_t* from_cache, hipStream_t stream) {
  HOQRI_TRY(check_plan(p));
  int op = 0;
  HOQRI_TRY(check_prec(prec, &op));
  if (from_cache) *from_cache = 0;
  const std::string key = tune_key(p, prec);
  hoqri_tuning t{};
  if (cache_path && cache_lookup(cache_path, key, p->N, &t) && validate_tuning(p, &t) == HOQRI_OK) {
    apply_tuning(p, &t);
    if (chosen) *chosen = t;
    if (from_cache) *from_cache = 1;
    return HOQRI_OK;
  }
  if (op == OP_FP16) {
    float as, ys;
    if (!fp16_scales(p, p->N - 1, &as, &ys)) return HOQRI_ERR_UNSUPPORTED;
  }
  HOQRI_TRY(tuning_operands(p, op, stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return HOQRI_ERR_HIP;
  }
  hoqri_status st = HOQRI_OK;
  read_tuning(p, &t);
  for (int n = 0; n < p->N && st == HOQRI_OK; ++n) {
    if (!segpass_supported(p, n)) continue;  // generic kernels: nothing to tune
    const int64_t W0 = p->md[n].ranges0;
    std::vector<int32_t> Ws;
    for (int64_t w : {W0 / 4, W0 / 2, W0, 2 * W0}) {
      const int64_t c = std::min<int64_t>(std::max<int64_t>(w, 1), std::min<int64_t>(p->ranges_cap, p->nnz));
      if (std::find(Ws.begin(), Ws.end(), (int32_t)c) == Ws.end()) Ws.push_back((int32_t)c);
    }
    const int rmax = ttm_max_rpw(p, n, op);
    std::vector<int32_t> Rs = {0};  // the library's rule first
    for (int r : {1, 2, 4, 8, 12})
      if (r <= rmax) Rs.push_back(r);
    float best = 0.f;
    int32_t bw = p->md[n].ranges0, br = 0;
    bool have = false;
    for (int32_t w : Ws) {
      for (int32_t r : Rs) {
        p->md[n].ranges = w;
        p->md[n].rpw = r;
        float ms = 0.f;
        st = time_mode(p, n, op, stream, e0, e1, &ms);
        if (st != HOQRI_OK) break;
        if (!have || ms < best) {
          best = ms;
          bw = w;
          br = r;
          have = true;
        }
      }
      if (st != HOQRI_OK) break;
    }
    p->md[n].ranges = bw;
    p->md[n].rpw = br;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HOQRI_OK) {
    for (int n = 0; n < p->N; ++n) {
      p->md[n].ranges = p->md[n].ranges0;
      p->md[n].rpw = 0;
    }
    return st;
  }
  read_tuning(p, &t);
  if (chosen) *chosen = t;
  if (cache_path) (void)cache_store(cache_path, key, p->N, t);
  return HOQRI_OK;
}
