/*
 * hoqri.h — C ABI of the MI355X (gfx950) HOQRI library.
 *
 * HOQRI (higher-order QR iteration) computes a low multilinear rank (Tucker)
 * approximation X ~ G x {U} of a sparse N-way tensor X by maximising
 * ||X x {U^T}||^2 over factors U^(n) with orthonormal columns (§2.2). Each
 * iteration sweeps n = 1..N (Alg. 2): A^(n) = TTMcTC(X, {U}, n), then U^(n) =
 * an orthonormal basis of A^(n) by QR. TTMcTC is A^(n) = Y_(n) G_(n)^T where
 * Y = X x_{-n} {U^T} and G = X x {U^T} (definition in §4.1); Y is never formed.
 *
 * Conventions used by every entry point:
 *  - Pointers named d_* are device (HBM) memory owned by the caller; this
 *    library never frees them. Host arrays are read during the call only.
 *  - Indices are 0-based int32. A sparse tensor is given as coordinates
 *    d_idx[N][nnz] (structure of arrays: mode m's indices at d_idx + m*nnz) and
 *    values d_vals[nnz] (float32).
 *  - A factor U^(n) is row-major I_n x K_n float32. The core G is a dense
 *    K_1 x ... x K_N float32 array in C order (last mode fastest), so its
 *    mode-n unfolding G_(n) has the other modes ascending, last fastest.
 *  - Every call is asynchronous on `stream` unless documented otherwise and
 *    returns a hoqri_status; argument errors are detected on the host before
 *    any launch and leave outputs untouched. No C++ exception crosses the ABI.
 *  - Calls on one plan must not overlap (they share its scratch memory);
 *    distinct plans may run concurrently on distinct streams.
 *  - Results are deterministic: the same inputs give bitwise-identical outputs
 *    (fixed-order reductions, no floating-point atomics).
 */
#ifndef HOQRI_H
#define HOQRI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOQRI_OK = 0,
  HOQRI_ERR_ARG = -1,         /* invalid argument (null pointer, bad order/size, nnz < 1, ...) */
  HOQRI_ERR_INDEX = -2,       /* a coordinate lies outside [0, I_n) */
  HOQRI_ERR_RANK = -3,        /* K_n outside [1, I_n], or K_n > prod_{m!=n} K_m */
  HOQRI_ERR_BREAKDOWN = -4,   /* A^(n) numerically rank deficient: no orthonormal basis */
  HOQRI_ERR_NOMEM = -5,       /* caller workspace too small */
  HOQRI_ERR_HIP = -6,         /* a HIP runtime call failed (no device, launch failure, ...) */
  HOQRI_ERR_UNSUPPORTED = -7  /* shape not supported by the compiled kernels (see limits below) */
} hoqri_status;

/* Operand precision of the Kronecker x core contraction. Accumulation is always
 * float32; Gram matrices, Cholesky factors and scalars are float64. */
typedef enum {
  HOQRI_FP32 = 1,  /* float32 operands on the float32 matrix cores */
  HOQRI_BF16 = 2,  /* bfloat16 operands (round to nearest even), float32 accumulate */
  HOQRI_FP16 = 3   /* float16 operands, float32 accumulate: factor copies scaled by 2^15 and the
                      value x row-entries operand by a power of two chosen from max|x|, both
                      removed exactly. Factor entries must have magnitude below 1.5 (orthonormal
                      columns give at most 1): hoqri_core, hoqri_ttmctc and hoqri_run check this
                      with one synchronisation before any pass and return HOQRI_ERR_ARG otherwise */
} hoqri_prec;

/* Limits: 2 <= N <= 5; 1 <= K_n <= 32; nnz < 2^30 and 4 N ceil16(nnz) bytes
 * < 2^32 (one mode's block records: nnz below about 268M at N = 4, 358M at
 * N = 3); every I_n < 2^31, I_1 * ... * I_N <= 2^63 (C-order linear keys in
 * 64 bits) and I_n * K_n * 4 bytes < 2^32. Shapes beyond these return
 * HOQRI_ERR_UNSUPPORTED (HOQRI_ERR_ARG for nnz or I_n out of range). Modes
 * with N <= 4 and prod_{m!=n} K_m within 8 blocks of 16 x 16 take the segment
 * passes (every operand form, stored slice rows, HOOI, the server); other
 * modes (N = 5, wider Kronecker rows) take the generic kernels, float32
 * operands only (HOQRI_ERR_UNSUPPORTED otherwise). */
#define HOQRI_MAX_ORDER 5
#define HOQRI_MAX_RANK 32

typedef struct hoqri_plan hoqri_plan; /* opaque; host object pointing into the caller's workspace */

/* Exact device workspace (bytes) that hoqri_plan_create needs for this shape.
 * nnz is the number of stored coordinates before duplicates are merged.
 * Host-side only apart from querying the device's sort temporary size; needs a
 * visible HIP device (HOQRI_ERR_HIP otherwise). Used for admission by footprint. */
hoqri_status hoqri_plan_workspace_size(int32_t order, const int64_t* dims, const int32_t* ranks,
                                       int64_t nnz, size_t* bytes);

/* Builds the plan for tensor X with target ranks K (§2.2): merges duplicate
 * coordinates by summing their values, computes ||X||^2 in float64, and for each
 * mode n keeps a copy of the nonzeros stably sorted by i_n together with the
 * table of nonempty index sets I^(n)_{i_n} (Table 1: the nonzeros whose mode-n
 * index is i_n). d_idx and d_vals are read only during this call and may be
 * freed afterwards. d_ws (ws_bytes >= hoqri_plan_workspace_size) must stay
 * allocated until hoqri_plan_destroy. Synchronises `stream` twice (index check
 * and sizes). Errors: HOQRI_ERR_INDEX for a coordinate out of range,
 * HOQRI_ERR_RANK for invalid ranks, HOQRI_ERR_NOMEM for a short workspace. */
hoqri_status hoqri_plan_create(hoqri_plan** plan, int32_t order, const int64_t* dims,
                               const int32_t* ranks, int64_t nnz, const int32_t* d_idx,
                               const float* d_vals, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Information about a built plan (host values): number of distinct coordinates,
 * ||X||^2 and, if R is not NULL, the number of nonempty mode-n slices R[n]. */
hoqri_status hoqri_plan_info(const hoqri_plan* plan, int64_t* nnz_coalesced, double* norm_x2, int64_t* R);

/* Releases the host object. Frees nothing the caller owns. */
void hoqri_plan_destroy(hoqri_plan* plan);

/* Core G = X x {U^T} (§2.2; the core Alg. 3 forms before its loop): G(k) = sum over nonzeros of
 * x(i) prod_m U^(m)(i_m, k_m). d_U is a HOST array of N device pointers (factor
 * m row-major I_m x K_m). Writes all prod K_m entries of d_G (C order). If
 * d_f is not NULL, writes f = ||G||^2 (float64, device) there. */
hoqri_status hoqri_core(hoqri_plan* plan, const float* const* d_U, float* d_G, double* d_f,
                        hoqri_prec prec, hipStream_t stream);

/* TTMcTC (definition in §4.1; Alg. 3): A^(n) = Y_(n) G_(n)^T with
 * Y = X x_{-n} {U^T}, i.e. A(i_n, k_n) = sum over nonzeros with mode-n index
 * i_n and over k_{-n} of x(i) G(k) prod_{m!=n} U^(m)(i_m, k_m). Y is never
 * formed. d_G is the core (C order) the caller supplies, usually hoqri_core's
 * output for the same factors. d_A (I_n x K_n row-major) is fully overwritten;
 * rows of empty slices are zero. */
hoqri_status hoqri_ttmctc(hoqri_plan* plan, int32_t mode, const float* const* d_U, const float* d_G,
                          float* d_A, hoqri_prec prec, hipStream_t stream);

/* The core G = X x {U^T} (§2.2) by the route of hoqri_run's mode update with
 * stored rows (§4.2): the TTMcTC pass of `mode` (core operand d_G_stage, its
 * output A discarded) keeps the rows Y_(mode) of the nonempty slices, and
 * G_(mode) = U^(mode)T Y_(mode) follows from them. Same arguments as
 * hoqri_core (d_f optional), plus the pass's mode and core operand (C order,
 * the caller's). For checking that route against the definition; hoqri_core
 * computes G directly. HOQRI_ERR_UNSUPPORTED if the plan's passes cannot keep
 * rows. Overwrites the plan's run scratch. */
hoqri_status hoqri_core_rows(hoqri_plan* plan, int32_t mode, const float* const* d_U, const float* d_G_stage,
                             float* d_G, double* d_f, hoqri_prec prec, hipStream_t stream);

/* Device workspace bytes hoqri_orth needs for `rows` x `cols`. Host only. */
size_t hoqri_orth_workspace_size(int64_t rows, int32_t cols);

/* Orthonormal basis of A (the QR step of Alg. 2) by CholeskyQR2 with float64
 * Gram matrices and Cholesky factors: W1 = A^T A, R1 = chol(W1), Q1 = A R1^-1,
 * W2 = Q1^T Q1, R2 = chol(W2), U = A (R2 R1)^-1. This is the thin QR with a
 * positive diagonal of R. d_A: rows x cols float32 row-major, 1 <= cols <= min(rows, 32).
 * d_U: output, may alias d_A. d_R: optional (NULL allowed) cols x cols float64
 * upper-triangular R = R2 R1 (row-major). d_status: device int32 set to 0 on
 * success or HOQRI_ERR_BREAKDOWN when a Cholesky pivot is <= 1e-13 * trace(W)
 * (A numerically rank deficient); then d_U is left unchanged. */
hoqri_status hoqri_orth(int64_t rows, int32_t cols, const float* d_A, float* d_U, double* d_R,
                        int32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* hoqri_orth without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same kernels and results (bitwise those of
 * hoqri_orth), with the scratch taken from a fixed device array of
 * hoqri_orth_noalloc_scratch_bytes() bytes (about 8 MiB) per GPU, set up on
 * the first call on each device and held until the process ends. Allocates
 * nothing. Arguments and errors as hoqri_orth; HOQRI_ERR_UNSUPPORTED if the
 * shape needed more scratch than the array holds (no valid shape does).
 * Calls that overlap on one GPU (several streams or threads) share the array
 * and race: serialise them. */
hoqri_status hoqri_orth_noalloc(int64_t rows, int32_t cols, const float* d_A, float* d_U, double* d_R,
                                int32_t* d_status, hipStream_t stream);
size_t hoqri_orth_noalloc_scratch_bytes(void);

typedef struct {
  int32_t max_sweeps;   /* sweeps over all N modes (one sweep = one HOQRI iteration) */
  double tol;           /* stop rule threshold (0 disables); the rule is chosen by stop_rule */
  hoqri_prec prec;      /* operand precision of the segment passes */
  int32_t check_every;  /* read f back every this many sweeps (>= 1) */
  int32_t orthonormalize_input; /* nonzero: first replace each U^(n) by its orthonormal basis */
  int32_t keep_on_breakdown;  /* nonzero: a rank-deficient A^(n) leaves U^(n) unchanged for that
                                 step (counted in skipped_updates) instead of ending the run */
  double* d_grad_hist;  /* optional (device, max_sweeps * N doubles): squared norm of the
                           Riemannian gradient of f with respect to U^(n) at every mode step
                           (§5.2: grad_n = 2 (A^(n) - U^(n) G_(n) G_(n)^T), evaluated before
                           U^(n) is updated); NULL and grad_tol == 0 turn the monitor off */
  double grad_tol;      /* > 0: also stop when sqrt(sum_n ||grad_n||^2) over a sweep <= grad_tol * f_t */
  int32_t method;       /* HOQRI_METHOD_HOQRI (0, Alg. 2) or HOQRI_METHOD_HOOI (Alg. 1) */
  int32_t inner_iters;  /* HOOI: orthogonal-iteration steps per mode update (>= 1; 0 means 1) */
  int32_t stop_rule;    /* HOQRI_STOP_REL_F (0): stop when |f_t - f_{t-1}| <= tol * f_t;
                           HOQRI_STOP_ERR_CHANGE (1): stop when the relative approximation error
                           eps_t = sqrt(max(||X||^2 - f_t, 0) / ||X||^2) changes by less than tol,
                           |eps_t - eps_{t-1}| < tol (the rule of the experiments in §6.1).
                           Both rules compare the last two sweeps (f_0: the starting factors)
                           at every check (every check_every sweeps) */
} hoqri_run_opts;

#define HOQRI_STOP_REL_F 0
#define HOQRI_STOP_ERR_CHANGE 1

/* Methods of hoqri_run. HOOI (Alg. 1) replaces the single QR step of a mode
 * update by the K_n leading left singular vectors of Y_(n), computed by
 * orthogonal iteration on Y_(n) Y_(n)^T from the current U^(n):
 * U <- orth(Y_(n) Y_(n)^T U), inner_iters times. The first product is the
 * TTMcTC of the mode (Y_(n) G_(n)^T with G_(n) = U^T Y_(n)); the others reuse
 * the slice rows Y_(n) that pass stored. With inner_iters == 1 a mode update
 * is the HOQRI update. */
#define HOQRI_METHOD_HOQRI 0
#define HOQRI_METHOD_HOOI 1

typedef struct {
  int32_t sweeps;       /* sweeps performed */
  double norm_x2;       /* ||X||^2 */
  double f;             /* ||G||^2 for the returned factors */
  double fit;           /* 1 - sqrt(max(||X||^2 - f, 0)) / ||X|| */
  double rel_change;    /* |f_t - f_{t-1}| / f_t at the last sweep */
  double orth_err_max;  /* max_n ||U^(n)T U^(n) - I||_F of the returned factors */
  int32_t skipped_updates; /* mode updates skipped for rank deficiency (keep_on_breakdown) */
  double grad_norm2;    /* sum_n ||grad_n||^2 of the last sweep (-1 when the monitor is off) */
} hoqri_run_stats;

/* HOQRI (Alg. 2): for each sweep, for n = 1..N: G from the current factors,
 * A^(n) = TTMcTC, U^(n) = orthonormal basis of A^(n) (Gauss-Seidel order);
 * or HOOI (opts->method, see above) on the same passes.
 * d_U_inout: host array of N device pointers, read as the start and overwritten
 * with the result (orthonormal columns required unless orthonormalize_input).
 * d_G_out: receives G = X x {U^T} for the returned factors (last line of
 * Alg. 2). d_f_hist (optional, device, max_sweeps * N doubles) receives f
 * before every mode update. stats (host) is filled at the end. Synchronises
 * `stream` every check_every sweeps and at the end. Returns
 * HOQRI_ERR_BREAKDOWN if some A^(n) is rank deficient (unless keep_on_breakdown),
 * or before any sweep if some mode has fewer nonempty slices than K_n. */
hoqri_status hoqri_run(hoqri_plan* plan, float* const* d_U_inout, float* d_G_out, double* d_f_hist,
                       const hoqri_run_opts* opts, hoqri_run_stats* stats, hipStream_t stream);

/* HOSVD-style start for Alg. 2 (which may start from HOSVD), by a randomized
 * range finder of every unfolding: A^(n) = X_(n) (kron over m != n of Omega_m)
 * Gamma_(n)^T, i.e. TTMcTC (definition in §4.1) with the factors replaced by
 * d_Omega and the core by d_Gamma, then U^(n) = the orthonormal basis of A^(n)
 * with positive-diagonal R (as hoqri_orth). Every mode is sketched from X alone.
 * d_Omega: host array of N device pointers, Omega_m row-major I_m x K_m float32
 * (random draws, e.g. N(0,1), supplied by the caller); d_Gamma: K_1 x ... x K_N
 * float32 (C order, random). d_U_out: host array of N device pointers, written
 * I_n x K_n (rows of empty slices zero). HOQRI_ERR_BREAKDOWN if some sketch is
 * rank deficient (fewer than K_n nonempty slices, or degenerate draws). */
hoqri_status hoqri_sketch_start(hoqri_plan* plan, const float* const* d_Omega, const float* d_Gamma,
                                float* const* d_U_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Launch-shape tuning of the TTMcTC passes. Per mode: the number of work
 * ranges the mode-sorted nonzeros are cut into (one wave walks one range) and
 * the ranges per workgroup. Results depend on them only through the summation
 * order (each choice is deterministic); the library's own rule is the default.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t ranges[HOQRI_MAX_ORDER];          /* 1 .. hoqri_plan_max_ranges(plan) */
  int32_t waves_per_group[HOQRI_MAX_ORDER]; /* 0: the library's rule; else capped by what the pass holds */
} hoqri_tuning;
/* Current tuning of a plan (host). */
hoqri_status hoqri_plan_get_tuning(const hoqri_plan* plan, hoqri_tuning* tuning);
/* Sets the tuning (host; takes effect at the next call). HOQRI_ERR_ARG for
 * values out of range. Entries of modes >= N are ignored. */
hoqri_status hoqri_plan_set_tuning(hoqri_plan* plan, const hoqri_tuning* tuning);
/* Most work ranges per mode the plan's workspace holds. */
int32_t hoqri_plan_max_ranges(const hoqri_plan* plan);
/* Autotuner: for every mode whose TTMcTC takes the segment passes, times one
 * mode update (the TTMcTC pass and, when the passes store slice rows, the core
 * product that follows) on the plan's own nonzeros for each candidate (ranges
 * 1/4, 1/2, 1 and 2 times the library's choice; every admissible ranges per
 * workgroup), median of 3 after a warm-up, and applies the fastest. With
 * cache_path (a text file, may be NULL) a previous result for the same shape
 * class (device architecture, order, ranks, operand form, floor(log2) of nnz
 * and of every mode's nonempty slices) is applied without timing
 * (*from_cache = 1), and a new result is appended. Overwrites the plan's run
 * scratch (factors, core) with timing operands; synchronises `stream`. */
hoqri_status hoqri_autotune(hoqri_plan* plan, hoqri_prec prec, const char* cache_path, hoqri_tuning* chosen,
                            int32_t* from_cache, hipStream_t stream);

/* Kernel timing (diagnostics). When enabled on a plan, every launch of the
 * listed kernels made through that plan is bracketed by HIP events recorded on
 * the launch stream, and hoqri_timing_read returns the number of launches and
 * their summed duration (milliseconds) since the last enable, for `kind`:
 *   HOQRI_KERNEL_TTMCTC = the TTMcTC segment-pass kernel,
 *   HOQRI_KERNEL_CORE   = the core segment-pass kernel (without its reduction),
 *   HOQRI_KERNEL_ORTH   = one CholeskyQR2 (all its kernels),
 *   HOQRI_KERNEL_FIXUP  = TTMcTC operand preparation and split-slice fix-up.
 * Enabling resets the counters. At most 4096 launches per kind are recorded.
 * hoqri_timing_read synchronises the recorded events. */
typedef enum { HOQRI_KERNEL_TTMCTC = 0, HOQRI_KERNEL_CORE = 1, HOQRI_KERNEL_ORTH = 2, HOQRI_KERNEL_FIXUP = 3 } hoqri_kernel;
hoqri_status hoqri_timing_enable(hoqri_plan* plan, int32_t enable);
hoqri_status hoqri_timing_read(hoqri_plan* plan, int32_t kind, int64_t* launches, double* total_ms);

/* ------------------------------------------------------------------------
 * Device memory arena (host-side bookkeeping only; no HIP calls).
 * First-fit allocator over [0, bytes) in 256-byte granules with coalescing of
 * neighbouring free blocks. Offsets are relative to whatever device buffer the
 * caller associates with the arena. Used by the request server for admission
 * by footprint; exported for callers that pack several plans in one buffer.
 * ------------------------------------------------------------------------ */
typedef struct hoqri_arena hoqri_arena;
hoqri_status hoqri_arena_create(size_t bytes, hoqri_arena** arena);
/* HOQRI_ERR_NOMEM when no free block is large enough (nothing changes). */
hoqri_status hoqri_arena_alloc(hoqri_arena* arena, size_t bytes, size_t* offset);
/* HOQRI_ERR_ARG for an offset that is not the start of a live block. */
hoqri_status hoqri_arena_free(hoqri_arena* arena, size_t offset);
hoqri_status hoqri_arena_stats(const hoqri_arena* arena, size_t* used, size_t* largest_free, int32_t* live_blocks);
void hoqri_arena_destroy(hoqri_arena* arena);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of many HOQRI runs (Alg. 2) on one GPU.
 *
 * Requests are admitted first-come first-served when a slot is free and the
 * plan's workspace (hoqri_plan_workspace_size) fits in the server's arena;
 * a request that does not fit waits (later requests do not overtake it). Each
 * hoqri_server_step advances every admitted request by one mode update (core,
 * TTMcTC, orthonormalisation), with one launch per kernel kind covering all
 * admitted requests (blocks are split among requests by a table), so requests
 * admitted at different times overlap on the device. A request's launches use
 * the same work split as hoqri_run, so its results are bitwise those of
 * hoqri_run with the same options (float32 operands, check_every = 1).
 * Requests finish when the stop rule of hoqri_run holds or after max_sweeps.
 * ------------------------------------------------------------------------ */
typedef struct {
  void* d_arena;            /* device memory owned by the caller, kept until destroy */
  size_t arena_bytes;       /* plans are admitted while their workspaces fit in here */
  int32_t max_slots;        /* requests in flight at once (1 .. 1024) */
  int32_t max_sweeps;       /* per request (>= 1) */
  double tol;               /* stop rule |f_t - f_{t-1}| <= tol * f_t (0 disables) */
  int32_t max_admit_per_step; /* plan builds per step (0: no limit) */
  int32_t report_orth_err;  /* nonzero: compute ||U^T U - I||_F of finished requests */
  int32_t keep_on_breakdown; /* as in hoqri_run_opts */
  int32_t use_graphs;       /* nonzero: each step's batched launches are captured into a HIP graph and
                               replayed as one launch (the previous step's executable graph is updated
                               in place when its topology is unchanged); results are bitwise the same */
  int32_t time_passes;      /* nonzero (and use_graphs zero): HIP events around each step's batched
                               TTMcTC launches, read by hoqri_server_ttm_stats */
} hoqri_server_opts;

typedef struct {
  int64_t id;               /* caller's tag, returned in the result */
  int32_t order;
  const int64_t* dims;      /* host [order], copied at submit */
  const int32_t* ranks;     /* host [order], copied at submit */
  int64_t nnz;
  const int32_t* d_idx;     /* device [order][nnz]; read when the request is admitted */
  const float* d_vals;      /* device [nnz]; read when the request is admitted */
  float* const* d_U;        /* host array of order device pointers (copied at submit): orthonormal
                               start factors, overwritten with the result when the request finishes */
  float* d_G;               /* device, prod K floats: receives the core of the result */
} hoqri_request;

typedef struct {
  int64_t id;
  hoqri_status status;      /* HOQRI_OK, or the error that ended the request */
  int32_t sweeps;
  double norm_x2, f, fit, rel_change, orth_err_max;
  int64_t admitted_step, finished_step;
  int32_t skipped_updates;
} hoqri_result;

typedef struct hoqri_server hoqri_server;
/* Allocates pinned host memory for the per-step launch tables; takes the first
 * part of the arena for their device copy. Needs a visible device. */
hoqri_status hoqri_server_create(const hoqri_server_opts* opts, hoqri_server** server);
/* Queues a request (host only; no device work). The caller keeps d_idx,
 * d_vals, the factors and d_G allocated until the request's result is returned. */
hoqri_status hoqri_server_submit(hoqri_server* server, const hoqri_request* request);
/* Admits queued requests, advances all admitted requests by one mode update on
 * `stream`, and writes the results of requests that finished during this step
 * (at most `cap`; the rest are returned by later calls) to `results`. Results
 * are complete (factors and core written) when the call returns. Synchronises
 * `stream` once per step, plus once per admitted request (plan build). */
hoqri_status hoqri_server_step(hoqri_server* server, hipStream_t stream, hoqri_result* results, int32_t cap,
                               int32_t* n_results);
/* Requests queued, requests in flight, bytes of the arena in use. */
hoqri_status hoqri_server_info(const hoqri_server* server, int32_t* queued, int32_t* active, size_t* arena_used);
/* With time_passes: the steps whose TTMcTC launches were timed, their total
 * duration (ms, HIP events on the step's stream around the batched stage-two
 * operand, segment pass and split-slice fix-up launches) and the algorithmic
 * HBM bytes and flops of the passes they ran (per request and mode: indices
 * and values streamed once, the slice table, each needed factor row once in
 * float32, A^(n) written once; 2 nnz prod_{m!=n} K_m + 2 R_n prod K flops).
 * Steps whose events have not completed yet are not counted. Host only. */
hoqri_status hoqri_server_ttm_stats(const hoqri_server* server, int64_t* steps, double* ms, double* bytes,
                                    double* flops);
/* Frees the server's host memory; nothing the caller owns. In-flight requests are dropped. */
void hoqri_server_destroy(hoqri_server* server);

/* Human-readable name of a status code (static string). */
const char* hoqri_status_string(hoqri_status status);

#ifdef __cplusplus
}
#endif

#endif /* HOQRI_H */
