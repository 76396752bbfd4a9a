"""ctypes binding of libhoqri.so (include/hoqri.h).

Argument marshalling only: every step of HOQRI runs in the library's HIP
kernels. PyTorch provides device memory (tensors, including the plan
workspace) and the stream (the current torch stream). If the library is not
built, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# HOQRI_LIB may point at another build of the same library (same ABI)
LIB_PATH = os.environ.get("HOQRI_LIB") or os.path.join(_HERE, "libhoqri.so")

HOQRI_OK = 0
STATUS = {
    0: "HOQRI_OK", -1: "HOQRI_ERR_ARG", -2: "HOQRI_ERR_INDEX", -3: "HOQRI_ERR_RANK",
    -4: "HOQRI_ERR_BREAKDOWN", -5: "HOQRI_ERR_NOMEM", -6: "HOQRI_ERR_HIP", -7: "HOQRI_ERR_UNSUPPORTED",
}
PREC = {"fp32": 1, "bf16": 2, "fp16": 3}

# every symbol the header declares
EXPORTS = (
    "hoqri_plan_workspace_size", "hoqri_plan_create", "hoqri_plan_info", "hoqri_plan_destroy",
    "hoqri_core", "hoqri_core_rows", "hoqri_ttmctc", "hoqri_orth_workspace_size", "hoqri_orth", "hoqri_run",
    "hoqri_status_string", "hoqri_timing_enable", "hoqri_timing_read",
    "hoqri_arena_create", "hoqri_arena_alloc", "hoqri_arena_free", "hoqri_arena_stats", "hoqri_arena_destroy",
    "hoqri_server_create", "hoqri_server_submit", "hoqri_server_step", "hoqri_server_info", "hoqri_server_destroy",
    "hoqri_server_ttm_stats", "hoqri_sketch_start", "hoqri_orth_noalloc", "hoqri_orth_noalloc_scratch_bytes",
    "hoqri_plan_get_tuning", "hoqri_plan_set_tuning", "hoqri_plan_max_ranges", "hoqri_autotune",
)
KERNEL = {"ttmctc": 0, "core": 1, "orth": 2, "fixup": 3}


class HoqriError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class RunOpts(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("tol", ctypes.c_double), ("prec", ctypes.c_int),
                ("check_every", ctypes.c_int32), ("orthonormalize_input", ctypes.c_int32),
                ("keep_on_breakdown", ctypes.c_int32), ("d_grad_hist", ctypes.c_void_p),
                ("grad_tol", ctypes.c_double), ("method", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32)]


METHOD = {"hoqri": 0, "hooi": 1}
STOP = {"rel_f": 0, "err": 1}


class Tuning(ctypes.Structure):
    _fields_ = [("ranges", ctypes.c_int32 * 5), ("waves_per_group", ctypes.c_int32 * 5)]


class RunStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("norm_x2", ctypes.c_double), ("f", ctypes.c_double),
                ("fit", ctypes.c_double), ("rel_change", ctypes.c_double), ("orth_err_max", ctypes.c_double),
                ("skipped_updates", ctypes.c_int32), ("grad_norm2", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("d_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("tol", ctypes.c_double), ("max_admit_per_step", ctypes.c_int32),
                ("report_orth_err", ctypes.c_int32), ("keep_on_breakdown", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("time_passes", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("order", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("ranks", ctypes.POINTER(ctypes.c_int32)), ("nnz", ctypes.c_int64), ("d_idx", ctypes.c_void_p),
                ("d_vals", ctypes.c_void_p), ("d_U", ctypes.POINTER(ctypes.c_void_p)), ("d_G", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("sweeps", ctypes.c_int32),
                ("norm_x2", ctypes.c_double), ("f", ctypes.c_double), ("fit", ctypes.c_double),
                ("rel_change", ctypes.c_double), ("orth_err_max", ctypes.c_double),
                ("admitted_step", ctypes.c_int64), ("finished_step", ctypes.c_int64),
                ("skipped_updates", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libhoqri.so and declares the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    P = ctypes.POINTER
    L.hoqri_plan_workspace_size.argtypes = [i32, P(i64), P(i32), i64, P(sz)]
    L.hoqri_plan_create.argtypes = [P(vp), i32, P(i64), P(i32), i64, vp, vp, vp, sz, vp]
    L.hoqri_plan_info.argtypes = [vp, P(i64), P(dbl), P(i64)]
    L.hoqri_plan_destroy.argtypes = [vp]
    L.hoqri_plan_destroy.restype = None
    L.hoqri_core.argtypes = [vp, P(vp), vp, vp, ctypes.c_int, vp]
    L.hoqri_ttmctc.argtypes = [vp, i32, P(vp), vp, vp, ctypes.c_int, vp]
    L.hoqri_core_rows.argtypes = [vp, i32, P(vp), vp, vp, vp, ctypes.c_int, vp]
    L.hoqri_orth_workspace_size.argtypes = [i64, i32]
    L.hoqri_orth_workspace_size.restype = sz
    L.hoqri_orth.argtypes = [i64, i32, vp, vp, vp, vp, vp, sz, vp]
    L.hoqri_orth_noalloc.argtypes = [i64, i32, vp, vp, vp, vp, vp]
    L.hoqri_orth_noalloc_scratch_bytes.argtypes = []
    L.hoqri_orth_noalloc_scratch_bytes.restype = sz
    L.hoqri_run.argtypes = [vp, P(vp), vp, vp, P(RunOpts), P(RunStats), vp]
    L.hoqri_sketch_start.argtypes = [vp, P(vp), vp, P(vp), vp]
    L.hoqri_plan_get_tuning.argtypes = [vp, P(Tuning)]
    L.hoqri_plan_set_tuning.argtypes = [vp, P(Tuning)]
    L.hoqri_plan_max_ranges.argtypes = [vp]
    L.hoqri_plan_max_ranges.restype = i32
    L.hoqri_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, P(Tuning), P(i32), vp]
    L.hoqri_timing_enable.argtypes = [vp, i32]
    L.hoqri_timing_read.argtypes = [vp, i32, P(i64), P(dbl)]
    L.hoqri_status_string.argtypes = [ctypes.c_int]
    L.hoqri_status_string.restype = ctypes.c_char_p
    L.hoqri_arena_create.argtypes = [sz, P(vp)]
    L.hoqri_arena_alloc.argtypes = [vp, sz, P(sz)]
    L.hoqri_arena_free.argtypes = [vp, sz]
    L.hoqri_arena_stats.argtypes = [vp, P(sz), P(sz), P(i32)]
    L.hoqri_arena_destroy.argtypes = [vp]
    L.hoqri_arena_destroy.restype = None
    L.hoqri_server_create.argtypes = [P(ServerOpts), P(vp)]
    L.hoqri_server_submit.argtypes = [vp, P(Request)]
    L.hoqri_server_step.argtypes = [vp, vp, P(Result), i32, P(i32)]
    L.hoqri_server_info.argtypes = [vp, P(i32), P(i32), P(sz)]
    L.hoqri_server_destroy.argtypes = [vp]
    L.hoqri_server_destroy.restype = None
    L.hoqri_server_ttm_stats.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_double), P(ctypes.c_double),
                                         P(ctypes.c_double)]
    for name in ("hoqri_plan_workspace_size", "hoqri_plan_create", "hoqri_plan_info", "hoqri_core", "hoqri_core_rows",
                 "hoqri_ttmctc", "hoqri_orth", "hoqri_orth_noalloc", "hoqri_run", "hoqri_timing_enable", "hoqri_timing_read",
                 "hoqri_arena_create", "hoqri_arena_alloc", "hoqri_arena_free", "hoqri_arena_stats",
                 "hoqri_server_create", "hoqri_server_submit", "hoqri_server_step", "hoqri_server_info",
                 "hoqri_server_ttm_stats", "hoqri_sketch_start", "hoqri_plan_get_tuning", "hoqri_plan_set_tuning", "hoqri_autotune"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, where: str):
    if status != HOQRI_OK:
        raise HoqriError(status, where)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def _need_cuda(t, dtype, name):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


def hoqri_status_string(status: int) -> str:
    return load().hoqri_status_string(int(status)).decode()


def hoqri_plan_workspace_size(order: int, dims: Sequence[int], ranks: Sequence[int], nnz: int) -> int:
    L = load()
    d = (ctypes.c_int64 * order)(*dims)
    r = (ctypes.c_int32 * order)(*ranks)
    out = ctypes.c_size_t(0)
    _check(L.hoqri_plan_workspace_size(order, d, r, int(nnz), ctypes.byref(out)), "hoqri_plan_workspace_size")
    return int(out.value)


def hoqri_orth_workspace_size(rows: int, cols: int) -> int:
    return int(load().hoqri_orth_workspace_size(int(rows), int(cols)))


class Plan:
    """A built plan: owns its device workspace (a torch uint8 tensor)."""

    def __init__(self, handle, workspace, dims, ranks):
        self._h = handle
        self.workspace = workspace
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(k) for k in ranks)
        self.order = len(self.dims)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def destroy(self):
        if self._h is not None:
            load().hoqri_plan_destroy(self._h)
            self._h = None
            self.workspace = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hoqri_plan_create(idx, vals, dims: Sequence[int], ranks: Sequence[int], stream=None,
                      workspace=None) -> Plan:
    """idx: int32 CUDA tensor [N, nnz]; vals: float32 CUDA tensor [nnz]."""
    import torch
    L = load()
    _need_cuda(idx, torch.int32, "idx")
    _need_cuda(vals, torch.float32, "vals")
    N = len(dims)
    if idx.dim() != 2 or idx.shape[0] != N or vals.numel() != idx.shape[1]:
        raise ValueError("idx must be [N, nnz] with nnz = len(vals)")
    nnz = int(vals.numel())
    nbytes = hoqri_plan_workspace_size(N, dims, ranks, nnz)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=vals.device)
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * N)(*dims)
    r = (ctypes.c_int32 * N)(*ranks)
    _check(L.hoqri_plan_create(ctypes.byref(h), N, d, r, nnz, _ptr(idx), _ptr(vals), _ptr(workspace),
                               workspace.numel(), _stream(stream)), "hoqri_plan_create")
    return Plan(h, workspace, dims, ranks)


def hoqri_plan_info(plan: Plan):
    """Returns (nnz after merging duplicates, ||X||^2, [R_n nonempty slices])."""
    L = load()
    n = ctypes.c_int64()
    x2 = ctypes.c_double()
    R = (ctypes.c_int64 * plan.order)()
    _check(L.hoqri_plan_info(plan.handle, ctypes.byref(n), ctypes.byref(x2), R), "hoqri_plan_info")
    return int(n.value), float(x2.value), [int(v) for v in R]


def hoqri_core(plan: Plan, Us, G=None, f=None, prec: str = "fp32", stream=None):
    """G = X x {U^T}; returns G (float32, shape K) and, if f is given, fills f[0] = ||G||^2."""
    import torch
    L = load()
    for U in Us:
        _need_cuda(U, torch.float32, "U")
    if G is None:
        G = torch.empty(plan.ranks, dtype=torch.float32, device=Us[0].device)
    _check(L.hoqri_core(plan.handle, _ptr_array(Us), _ptr(G), _ptr(f) if f is not None else None,
                        PREC[prec], _stream(stream)), "hoqri_core")
    return G


def hoqri_core_rows(plan: Plan, mode: int, Us, G_stage, G=None, f=None, prec: str = "fp32", stream=None):
    """G = X x {U^T} by the stored-row route of a mode update (TTMcTC pass of
    `mode` with core operand G_stage, then U^(mode)T Y_(mode)); returns G."""
    import torch
    L = load()
    for U in Us:
        _need_cuda(U, torch.float32, "U")
    _need_cuda(G_stage, torch.float32, "G_stage")
    if G is None:
        G = torch.empty(plan.ranks, dtype=torch.float32, device=Us[0].device)
    _check(L.hoqri_core_rows(plan.handle, int(mode), _ptr_array(Us), _ptr(G_stage), _ptr(G),
                             _ptr(f) if f is not None else None, PREC[prec], _stream(stream)), "hoqri_core_rows")
    return G


def hoqri_ttmctc(plan: Plan, mode: int, Us, G, A=None, prec: str = "fp32", stream=None):
    """A^(n) = Y_(n) G_(n)^T; returns A (float32, I_n x K_n)."""
    import torch
    L = load()
    for U in Us:
        _need_cuda(U, torch.float32, "U")
    _need_cuda(G, torch.float32, "G")
    if A is None:
        A = torch.empty((plan.dims[mode], plan.ranks[mode]), dtype=torch.float32, device=G.device)
    _check(L.hoqri_ttmctc(plan.handle, int(mode), _ptr_array(Us), _ptr(G), _ptr(A), PREC[prec],
                          _stream(stream)), "hoqri_ttmctc")
    return A


def hoqri_orth(A, U=None, R=None, status=None, workspace=None, stream=None):
    """CholeskyQR2 orthonormal basis of A. Returns (U, status tensor)."""
    import torch
    L = load()
    _need_cuda(A, torch.float32, "A")
    rows, cols = A.shape
    if U is None:
        U = torch.empty_like(A)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
    if workspace is None:
        workspace = torch.empty(hoqri_orth_workspace_size(rows, cols), dtype=torch.uint8, device=A.device)
    _check(L.hoqri_orth(rows, cols, _ptr(A), _ptr(U), _ptr(R) if R is not None else None, _ptr(status),
                        _ptr(workspace), workspace.numel(), _stream(stream)), "hoqri_orth")
    return U, status


def hoqri_orth_noalloc(A, U, R=None, status=None, stream=None):
    """hoqri_orth with the library's fixed per-GPU scratch instead of a
    workspace (allocates nothing; the caller passes U and status). Returns
    (U, status tensor)."""
    import torch
    L = load()
    _need_cuda(A, torch.float32, "A")
    _need_cuda(U, torch.float32, "U")
    rows, cols = A.shape
    _check(L.hoqri_orth_noalloc(rows, cols, _ptr(A), _ptr(U), _ptr(R) if R is not None else None, _ptr(status),
                                _stream(stream)), "hoqri_orth_noalloc")
    return U, status


@dataclass
class Stats:
    sweeps: int
    norm_x2: float
    f: float
    fit: float
    rel_change: float
    orth_err_max: float
    skipped_updates: int = 0
    grad_norm2: float = -1.0


def hoqri_run(plan: Plan, Us, max_sweeps: int, tol: float = 0.0, prec: str = "fp32", check_every: int = 1,
              orthonormalize_input: bool = False, G=None, f_hist=None, stream=None, keep_on_breakdown: bool = False,
              grad_hist=None, grad_tol: float = 0.0, method: str = "hoqri", inner_iters: int = 1,
              stop: str = "rel_f"):
    """Runs HOQRI (or HOOI with `inner_iters` orthogonal-iteration steps per mode
    update) in place on Us. `stop` picks the rule `tol` applies to: "rel_f"
    (|f_t - f_{t-1}| <= tol f_t) or "err" (change of the relative approximation
    error below tol). Returns (G, Stats)."""
    import torch
    L = load()
    for U in Us:
        _need_cuda(U, torch.float32, "U")
    if G is None:
        G = torch.empty(plan.ranks, dtype=torch.float32, device=Us[0].device)
    if grad_hist is not None:
        _need_cuda(grad_hist, torch.float64, "grad_hist")
    opts = RunOpts(int(max_sweeps), float(tol), PREC[prec], int(check_every), int(bool(orthonormalize_input)),
                   int(bool(keep_on_breakdown)), ctypes.c_void_p(grad_hist.data_ptr()) if grad_hist is not None else None,
                   float(grad_tol), METHOD[method], int(inner_iters), STOP[stop])
    st = RunStats()
    _check(L.hoqri_run(plan.handle, _ptr_array(Us), _ptr(G), _ptr(f_hist) if f_hist is not None else None,
                       ctypes.byref(opts), ctypes.byref(st), _stream(stream)), "hoqri_run")
    return G, Stats(st.sweeps, st.norm_x2, st.f, st.fit, st.rel_change, st.orth_err_max, st.skipped_updates,
                    st.grad_norm2)


def hoqri_sketch_start(plan: Plan, Omega, Gamma, U=None, stream=None):
    """HOSVD-style start by a randomized range finder (hoqri_sketch_start): Omega is
    a list of random I_m x K_m float32 tensors, Gamma a random K_1 x ... x K_N core.
    Returns the N orthonormal factors (float32, I_n x K_n)."""
    import torch
    for O_ in Omega:
        _need_cuda(O_, torch.float32, "Omega")
    _need_cuda(Gamma, torch.float32, "Gamma")
    if U is None:
        U = [torch.empty((d, k), dtype=torch.float32, device=Gamma.device) for d, k in zip(plan.dims, plan.ranks)]
    _check(load().hoqri_sketch_start(plan.handle, _ptr_array(Omega), _ptr(Gamma), _ptr_array(U), _stream(stream)),
           "hoqri_sketch_start")
    return U


def _tuning_dict(t: Tuning, N: int):
    return {"ranges": [int(t.ranges[n]) for n in range(N)],
            "waves_per_group": [int(t.waves_per_group[n]) for n in range(N)]}


def hoqri_plan_get_tuning(plan: Plan):
    """The plan's launch shapes per mode: {"ranges": [...], "waves_per_group": [...]}."""
    L = load()
    t = Tuning()
    _check(L.hoqri_plan_get_tuning(plan.handle, ctypes.byref(t)), "hoqri_plan_get_tuning")
    return _tuning_dict(t, len(plan.dims))


def hoqri_plan_set_tuning(plan: Plan, ranges, waves_per_group=None):
    L = load()
    t = Tuning()
    for n, w in enumerate(ranges):
        t.ranges[n] = int(w)
        t.waves_per_group[n] = int(waves_per_group[n]) if waves_per_group is not None else 0
    _check(L.hoqri_plan_set_tuning(plan.handle, ctypes.byref(t)), "hoqri_plan_set_tuning")


def hoqri_plan_max_ranges(plan: Plan) -> int:
    return int(load().hoqri_plan_max_ranges(plan.handle))


def hoqri_autotune(plan: Plan, prec: str = "fp32", cache_path: str | None = None, stream=None):
    """Times the candidate launch shapes on the plan and applies the fastest
    (or a cached result for the same shape class). Returns (tuning dict,
    from_cache)."""
    L = load()
    t = Tuning()
    fc = ctypes.c_int32(0)
    path = cache_path.encode() if cache_path else None
    _check(L.hoqri_autotune(plan.handle, PREC[prec], path, ctypes.byref(t), ctypes.byref(fc), _stream(stream)),
           "hoqri_autotune")
    return _tuning_dict(t, len(plan.dims)), bool(fc.value)


def hoqri_timing_enable(plan: Plan, enable: bool = True):
    """Starts (and resets) or stops per-kernel HIP-event timing on the plan."""
    _check(load().hoqri_timing_enable(plan.handle, int(bool(enable))), "hoqri_timing_enable")


def hoqri_timing_read(plan: Plan, kind: str):
    """Returns (launches, total milliseconds) for kernel kind ttmctc/core/orth/fixup."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().hoqri_timing_read(plan.handle, KERNEL[kind], ctypes.byref(n), ctypes.byref(ms)),
           "hoqri_timing_read")
    return int(n.value), float(ms.value)


class Arena:
    """Host-side first-fit allocator over [0, size) (hoqri_arena_*)."""

    def __init__(self, size: int):
        L = load()
        h = ctypes.c_void_p()
        _check(L.hoqri_arena_create(int(size), ctypes.byref(h)), "hoqri_arena_create")
        self._h = h

    def alloc(self, nbytes: int):
        """Offset of a new block, or None when nothing fits."""
        off = ctypes.c_size_t(0)
        st = load().hoqri_arena_alloc(self._h, int(nbytes), ctypes.byref(off))
        if st == -5:
            return None
        _check(st, "hoqri_arena_alloc")
        return int(off.value)

    def free(self, offset: int):
        _check(load().hoqri_arena_free(self._h, int(offset)), "hoqri_arena_free")

    def stats(self):
        used, largest, live = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_int32(0)
        _check(load().hoqri_arena_stats(self._h, ctypes.byref(used), ctypes.byref(largest), ctypes.byref(live)),
               "hoqri_arena_stats")
        return int(used.value), int(largest.value), int(live.value)

    def close(self):
        if self._h:
            load().hoqri_arena_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class ServeResult:
    id: int
    status: int
    sweeps: int
    norm_x2: float
    f: float
    fit: float
    rel_change: float
    orth_err_max: float
    admitted_step: int
    finished_step: int
    skipped_updates: int


class Server:
    """Request server (hoqri_server_*): continuous batching of HOQRI runs.

    The arena is a torch uint8 tensor of `arena_bytes` on the current device.
    Tensors handed to submit() are kept referenced until their result is
    returned by step().
    """

    def __init__(self, arena_bytes: int, max_slots: int = 64, max_sweeps: int = 30, tol: float = 1e-6,
                 max_admit_per_step: int = 0, report_orth_err: bool = False, keep_on_breakdown: bool = True,
                 device=None, use_graphs: bool = False, time_passes: bool = False):
        import torch
        L = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device or "cuda")
        opts = ServerOpts(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(max_slots), int(max_sweeps),
                          float(tol), int(max_admit_per_step), int(bool(report_orth_err)),
                          int(bool(keep_on_breakdown)), int(bool(use_graphs)), int(bool(time_passes)))
        h = ctypes.c_void_p()
        _check(L.hoqri_server_create(ctypes.byref(opts), ctypes.byref(h)), "hoqri_server_create")
        self._h = h
        self._keep = {}
        self._cap = 1024
        self._res = (Result * self._cap)()

    def submit(self, rid: int, idx, vals, dims, ranks, Us, G):
        """Queues request `rid`: coordinates idx [N, nnz] int32 and values float32 on
        the device, orthonormal start factors Us (overwritten with the result) and
        the core output G."""
        import torch
        _need_cuda(idx, torch.int32, "idx")
        _need_cuda(vals, torch.float32, "vals")
        for U in Us:
            _need_cuda(U, torch.float32, "U")
        _need_cuda(G, torch.float32, "G")
        N = len(dims)
        d = (ctypes.c_int64 * N)(*[int(x) for x in dims])
        r = (ctypes.c_int32 * N)(*[int(x) for x in ranks])
        u = _ptr_array(Us)
        req = Request(int(rid), N, d, r, int(vals.numel()), ctypes.c_void_p(idx.data_ptr()),
                      ctypes.c_void_p(vals.data_ptr()), u, ctypes.c_void_p(G.data_ptr()))
        _check(load().hoqri_server_submit(self._h, ctypes.byref(req)), "hoqri_server_submit")
        self._keep[int(rid)] = (idx, vals, Us, G)

    def step(self, stream=None):
        """One engine step; returns the results of requests that finished."""
        n = ctypes.c_int32(0)
        _check(load().hoqri_server_step(self._h, _stream(stream), self._res, self._cap, ctypes.byref(n)),
               "hoqri_server_step")
        out = []
        for i in range(n.value):
            r = self._res[i]
            out.append(ServeResult(int(r.id), int(r.status), int(r.sweeps), r.norm_x2, r.f, r.fit, r.rel_change,
                                   r.orth_err_max, int(r.admitted_step), int(r.finished_step),
                                   int(r.skipped_updates)))
            self._keep.pop(int(r.id), None)
        return out

    def info(self):
        q, a, used = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_size_t(0)
        _check(load().hoqri_server_info(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(used)),
               "hoqri_server_info")
        return int(q.value), int(a.value), int(used.value)

    def ttm_stats(self):
        """(steps timed, total ms, algorithmic bytes, algorithmic flops) of the
        TTMcTC launches of the steps so far (time_passes=True)."""
        st, ms, by, fl = ctypes.c_int64(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        _check(load().hoqri_server_ttm_stats(self._h, ctypes.byref(st), ctypes.byref(ms), ctypes.byref(by),
                                             ctypes.byref(fl)), "hoqri_server_ttm_stats")
        return int(st.value), ms.value, by.value, fl.value

    def close(self):
        if self._h:
            load().hoqri_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
