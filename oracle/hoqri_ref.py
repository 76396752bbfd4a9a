"""FP64 CPU oracle for HOQRI — test infrastructure only.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may import
this module. The GPU library never calls it, and it shares no code with it.

Everything here is plain numpy in float64, written from the paper
(Sun, Bhat, Wang, Huang: "HOQRI: Higher-order QR Iteration for Low Multilinear
Rank Approximation of Large and Sparse Tensors"):

* the mode-n unfolding, n-mode product and Kronecker form of the
  tensor-times-matrix chain (TTMc) of §2.1;
* the core G = X x {U^T} that is optimal for orthonormal factors (§2.2);
* TTMcTC, A^(n) = Y_(n) G_(n)^T with Y = X x_{-n} {U^T} (definition in §4.1),
  in three independent forms: element by element as in Alg. 3, one column of
  Y_(n) at a time as in Alg. 4, and slice by slice over the index sets
  I^(n)_{i_n} of Table 1 (the same sum, grouped by row; reaches the second
  complexity of §4.2 without storing Y);
* the HOQRI loop of Alg. 2 (Gauss-Seidel over modes, the single-mode update
  rule of §5), with the QR step taken as a Householder QR whose R has a
  positive diagonal;
* the quantities of the convergence analysis (§5): the objective f = ||G||^2,
  the Riemannian gradient norm, the subspace distance d(U, V);
* a HOSVD-style start (Alg. 2 allows one) by a randomized range finder of
  every unfolding, computed as TTMcTC with random factors and a random core;
* HOOI (Alg. 1), the method HOQRI is contrasted with: each mode update takes
  the leading left singular vectors of Y_(n) (an SVD of its nonempty rows).

Readings where the paper is silent (all also listed in the design doc):
* QR basis: the thin QR with diag(R) > 0, unique for full-rank A (the paper
  allows any orthonormal basis, Remark after Theorem 2).
* Iteration: one iteration = one sweep over all N modes (§6.1 counts them so).
* Error and fit: ||X - G x {U}||^2 = ||X||^2 - ||G||^2 for orthonormal U
  (§2.2); fit = 1 - sqrt(max(||X||^2 - ||G||^2, 0)) / ||X||.
* Duplicate coordinates are summed (TTMcTC and the core are linear in X).
* Rank deficiency: a QR pivot with R_kk^2 <= 1e-13 * ||A||_F^2 is a breakdown
  (the paper does not discuss it); it either ends the run or, on request,
  leaves that mode's factor unchanged for that step.
* Unfolding column order: C order (last remaining mode fastest), which matches
  the ascending-mode Kronecker chain of the TTMc formula in §2.1.

Pins: every function here is checked against something other than itself in
tests/test_oracle_*.py (dense brute force, closed forms, the paper's
identities and inequalities, textbook SVD/eigen routines). None is unpinned.
"""
from __future__ import annotations

import itertools
import math
import string
from typing import Sequence

import numpy as np

__all__ = [
    "RankDeficient",
    "validate",
    "coalesce",
    "norm_x2",
    "to_dense",
    "unfold",
    "mode_product",
    "kron_except",
    "core_dense",
    "ttmctc_dense",
    "core_elementwise",
    "ttmctc_elementwise",
    "ttmctc_matrix",
    "slices",
    "ttmctc_segment",
    "core_segment",
    "qr_positive",
    "orthonormal_start",
    "hoqri",
    "fit_from",
    "subspace_dist",
    "grad_norm2_mode",
    "grad_norm2_direct",
    "tucker_dense",
    "sketch_start",
    "leading_left",
    "hooi",
    "core_entry",
    "ttmctc_slice_row",
]

BREAKDOWN_REL = 1e-13


class RankDeficient(ArithmeticError):
    """A^(n) has (numerically) lower rank than K_n, so no orthonormal basis exists."""


# --------------------------------------------------------------------------
# Inputs
# --------------------------------------------------------------------------

def validate(idx: np.ndarray, dims: Sequence[int], ranks: Sequence[int]) -> None:
    """Reject inputs outside the problem statement of §2.2.

    0 <= idx < dims, 1 <= K_n <= I_n, and K_n <= prod_{m != n} K_m (otherwise
    A^(n), whose columns lie in a space of that dimension, cannot have rank K_n).
    """
    idx = np.asarray(idx)
    N = len(dims)
    if idx.ndim != 2 or idx.shape[0] != N:
        raise ValueError("idx must be [N, nnz]")
    if idx.shape[1] < 1:
        raise ValueError("nnz must be >= 1")
    if len(ranks) != N or N < 2:
        raise ValueError("need N >= 2 modes with one rank each")
    for n in range(N):
        if idx[n].min() < 0 or idx[n].max() >= dims[n]:
            raise IndexError(f"mode {n} index out of range")
        if not (1 <= ranks[n] <= dims[n]):
            raise ValueError(f"rank K_{n} must be in [1, I_{n}]")
        other = math.prod(int(ranks[m]) for m in range(N) if m != n)
        if ranks[n] > other:
            raise ValueError(f"rank K_{n} exceeds the product of the other ranks")


def coalesce(idx: np.ndarray, vals: np.ndarray, dims: Sequence[int]):
    """Merge duplicate coordinates by summing their values.

    Returns (idx, vals) sorted by the C-order linear index. TTMcTC and the core
    are linear in X, so summing duplicates changes neither; ||X||^2 needs it.
    """
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = np.ravel_multi_index(tuple(idx), tuple(int(d) for d in dims))
    uk, inv = np.unique(key, return_inverse=True)
    v = np.zeros(uk.size, dtype=np.float64)
    np.add.at(v, inv, vals)
    out = np.stack(np.unravel_index(uk, tuple(int(d) for d in dims))).astype(np.int64)
    return out, v


def norm_x2(vals: np.ndarray) -> float:
    """||X||^2, the sum of squared entries (§2.1), of coalesced values."""
    v = np.asarray(vals, dtype=np.float64)
    return float(np.dot(v, v))


def to_dense(idx, vals, dims) -> np.ndarray:
    """Dense array of a (small) COO tensor; duplicates add."""
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    np.add.at(X, tuple(np.asarray(idx, dtype=np.int64)), np.asarray(vals, dtype=np.float64))
    return X


# --------------------------------------------------------------------------
# Dense definitions (§2.1, §2.2, §4.1): brute force on tiny tensors
# --------------------------------------------------------------------------

def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n): mode n gives the rows, the other modes (ascending,
    last fastest) give the columns (§2.1)."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def mode_product(X: np.ndarray, B: np.ndarray, n: int) -> np.ndarray:
    """n-mode product X x_n B for B of shape K x I_n, element by element (§2.1)."""
    out = np.tensordot(B, X, axes=([1], [n]))  # K x (other modes in order)
    return np.moveaxis(out, 0, n)


def kron_except(Us: Sequence[np.ndarray], n: int) -> np.ndarray:
    """U^(1) (x) ... (x) U^(n-1) (x) U^(n+1) (x) ... (x) U^(N): the Kronecker chain of
    the TTMc formula in §2.1 (ascending modes)."""
    out = np.ones((1, 1))
    for m, U in enumerate(Us):
        if m != n:
            out = np.kron(out, U)
    return out


def core_dense(X: np.ndarray, Us: Sequence[np.ndarray]) -> np.ndarray:
    """G = X x {U^T} (§2.2) by successive n-mode products."""
    G = X
    for n, U in enumerate(Us):
        G = mode_product(G, U.T, n)
    return G


def ttmctc_dense(X: np.ndarray, Us: Sequence[np.ndarray], n: int) -> np.ndarray:
    """A^(n) = Y_(n) G_(n)^T (§4.1) with Y_(n) = X_(n) (Kronecker chain of U) from the
    TTMc formula of §2.1 — the explicit, memory-exploding form."""
    Y = unfold(X, n) @ kron_except(Us, n)
    G = core_dense(X, Us)
    return Y @ unfold(G, n).T


def tucker_dense(G: np.ndarray, Us: Sequence[np.ndarray]) -> np.ndarray:
    """The Tucker model G x {U} (§2.2)."""
    X = G
    for n, U in enumerate(Us):
        X = mode_product(X, U, n)
    return X


# --------------------------------------------------------------------------
# Sparse forms
# --------------------------------------------------------------------------

def _letters(N: int):
    return string.ascii_lowercase[:N]


def core_elementwise(idx, vals, Us: Sequence[np.ndarray], chunk: int = 65536) -> np.ndarray:
    """G(k_1..k_N) = sum over nonzeros x(i) prod_m U^(m)(i_m, k_m): the core of §2.2
    written out over the nonzero set I(X) of Table 1 (the core Alg. 3 forms first)."""
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    N = len(Us)
    ks = _letters(N)
    spec = "z," + ",".join("z" + k for k in ks) + "->" + ks
    G = np.zeros(tuple(U.shape[1] for U in Us))
    for s in range(0, vals.size, chunk):
        e = slice(s, s + chunk)
        G += np.einsum(spec, vals[e], *[Us[m][idx[m, e]] for m in range(N)], optimize=True)
    return G


def ttmctc_elementwise(idx, vals, Us: Sequence[np.ndarray], n: int, G: np.ndarray | None = None,
                       chunk: int = 65536) -> np.ndarray:
    """Alg. 3: A^(n)(i_n, k_n) = sum over i_{-n} in I^(n)_{i_n} and over k_{-n} of
    x(i) G(k) prod_{v != n} U^(v)(i_v, k_v). G is formed first (its first line)
    unless given."""
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    N = len(Us)
    if G is None:
        G = core_elementwise(idx, vals, Us)
    ks = _letters(N)
    others = [m for m in range(N) if m != n]
    spec = "z," + ks + "," + ",".join("z" + ks[m] for m in others) + "->z" + ks[n]
    A = np.zeros((Us[n].shape[0], Us[n].shape[1]))
    for s in range(0, vals.size, chunk):
        e = slice(s, s + chunk)
        contrib = np.einsum(spec, vals[e], G, *[Us[m][idx[m, e]] for m in others], optimize=True)
        np.add.at(A, idx[n, e], contrib)
    return A


def ttmctc_matrix(idx, vals, Us: Sequence[np.ndarray], n: int) -> np.ndarray:
    """Alg. 4: A^(n) = sum over k_{-n} of y y^T U^(n), where y is the column of
    Y_(n) for that k_{-n}: the sparse mode product of X with one column of every
    other factor. Uses no G (G_(n) = U^(n)T Y_(n), §4.2). One column at a time,
    so only for small ranks."""
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    N = len(Us)
    others = [m for m in range(N) if m != n]
    In = Us[n].shape[0]
    A = np.zeros((In, Us[n].shape[1]))
    for kk in itertools.product(*[range(Us[m].shape[1]) for m in others]):
        w = vals.copy()
        for m, k in zip(others, kk):
            w *= Us[m][idx[m], k]
        y = np.zeros(In)
        np.add.at(y, idx[n], w)
        A += np.outer(y, y @ Us[n])
    return A


def slices(idx, n: int):
    """The nonempty index sets I^(n)_{i_n} of Table 1: returns (order, rows, starts)
    where order stably sorts the nonzeros by i_n, rows[s] is the i_n of slice s and
    slice s is order[starts[s]:starts[s+1]]."""
    key = np.asarray(idx[n], dtype=np.int64)
    order = np.argsort(key, kind="stable")
    k = key[order]
    brk = np.flatnonzero(np.diff(k)) + 1
    starts = np.concatenate([[0], brk, [k.size]])
    rows = k[starts[:-1]]
    return order, rows, starts


def _slice_rows(idx, vals, Us, n, chunk=None):
    """y_i = sum over e in I^(n)_i of x_e (Kronecker over m != n, ascending, of
    U^(m)(i_m^e, :)) for every nonempty slice i — row i of Y_(n) (§4.1), computed
    slice by slice without forming X_(n). Returns (rows, Y_rows[R, prod K_{-n}])."""
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    N = len(Us)
    others = [m for m in range(N) if m != n]
    order, rows, starts = slices(idx, n)
    P = math.prod(Us[m].shape[1] for m in others)
    Yr = np.zeros((rows.size, P))
    chunk = chunk or max(4096, (1 << 24) // P)
    seg_of = np.repeat(np.arange(rows.size), np.diff(starts))
    for s in range(0, order.size, chunk):
        e = order[s:s + chunk]
        z = vals[e][:, None]
        for m in others:
            z = (z[:, :, None] * Us[m][idx[m, e]][:, None, :]).reshape(e.size, -1)
        _seg_add(Yr, seg_of[s:s + chunk], z)
    return rows, Yr


def _seg_add(out, seg, z):
    """out[seg[j]] += z[j] for sorted seg (segmented sum via reduceat)."""
    brk = np.flatnonzero(np.diff(seg)) + 1
    st = np.concatenate([[0], brk])
    out[seg[st]] += np.add.reduceat(z, st, axis=0)


def ttmctc_segment(idx, vals, Us: Sequence[np.ndarray], n: int, G: np.ndarray) -> np.ndarray:
    """A^(n)(i, :) = y_i G_(n)^T for each nonempty slice i (zero rows elsewhere):
    the TTMcTC definition of §4.1 evaluated slice by slice."""
    rows, Yr = _slice_rows(idx, vals, Us, n)
    A = np.zeros((Us[n].shape[0], Us[n].shape[1]))
    A[rows] = Yr @ unfold(G, n).T
    return A


def core_entry(idx, vals, Us: Sequence[np.ndarray], ks: Sequence[int]) -> float:
    """One entry G(k_1, ..., k_N) = sum_e x_e prod_m U^(m)(i_m^e, k_m) of the core
    (§2.2), as one sum over all nonzeros (for sampling large tensors)."""
    idx = np.asarray(idx, dtype=np.int64)
    t = np.asarray(vals, dtype=np.float64).copy()
    for m, k in enumerate(ks):
        t *= Us[m][idx[m], k]
    return float(t.sum())


def ttmctc_slice_row(idx, vals, Us: Sequence[np.ndarray], n: int, i: int, G: np.ndarray,
                     chunk: int = 1 << 20) -> np.ndarray:
    """Row i of A^(n) = Y_(n) G_(n)^T (definition in §4.1) from slice i's
    nonzeros only: y_i = sum over the slice of x_e (Kronecker over m != n of
    U^(m)(i_m^e, :)), with the last Kronecker factor contracted by a matrix
    product over the nonzeros (chunks of `chunk`), then y_i G_(n)^T."""
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    sel = np.flatnonzero(idx[n] == i)
    others = [m for m in range(len(Us)) if m != n]
    first, last = others[:-1], others[-1]
    P1 = math.prod(Us[m].shape[1] for m in first)
    y = np.zeros((P1, Us[last].shape[1]))
    for s in range(0, sel.size, chunk):
        e = sel[s:s + chunk]
        W = vals[e][:, None]
        for m in first:
            W = (W[:, :, None] * Us[m][idx[m, e]][:, None, :]).reshape(e.size, -1)
        y += W.T @ Us[last][idx[last, e]]
    return y.reshape(-1) @ unfold(G, n).T


def core_segment(idx, vals, Us: Sequence[np.ndarray], n: int = 0) -> np.ndarray:
    """G_(n) = U^(n)T Y_(n) (§4.2) accumulated slice by slice; returns G as a tensor."""
    rows, Yr = _slice_rows(idx, vals, Us, n)
    Gn = Us[n][rows].T @ Yr
    shape = [U.shape[1] for U in Us]
    moved = [shape[n]] + [shape[m] for m in range(len(Us)) if m != n]
    return np.moveaxis(Gn.reshape(moved), 0, n)


# --------------------------------------------------------------------------
# QR step and the HOQRI loop (Alg. 2)
# --------------------------------------------------------------------------

def qr_positive(A: np.ndarray):
    """Thin QR with a positive diagonal of R: an orthonormal basis of A (Alg. 2's
    QR step). Householder QR from LAPACK, then column signs flipped. Raises
    RankDeficient when some R_kk^2 <= 1e-13 ||A||_F^2."""
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    d = np.diag(R)
    s = np.where(d < 0, -1.0, 1.0)
    fro2 = float(np.sum(np.asarray(A, dtype=np.float64) ** 2))
    if fro2 == 0.0 or np.any(d * d <= BREAKDOWN_REL * fro2):
        raise RankDeficient("A^(n) is rank deficient")
    return Q * s[None, :], R * s[:, None]


def orthonormal_start(raw: Sequence[np.ndarray]):
    """Random initialisation of Alg. 2: the orthonormal basis of each raw matrix."""
    return [qr_positive(np.asarray(R, dtype=np.float64))[0] for R in raw]


def fit_from(normx2: float, f: float) -> float:
    """fit = 1 - ||X - G x {U}|| / ||X||, using ||X - G x {U}||^2 = ||X||^2 - ||G||^2
    for orthonormal U (§2.2)."""
    return 1.0 - math.sqrt(max(normx2 - f, 0.0)) / math.sqrt(normx2)


def hoqri(idx, vals, dims, ranks, U0: Sequence[np.ndarray], sweeps: int, tol: float | None = None,
          stop: str = "rel_f", impl: str = "segment", record_A: bool = False, on_breakdown: str = "raise"):
    """Alg. 2 (HOQRI). Sweeps over n = 1..N in order (Gauss-Seidel: the update of
    mode n sees the already-updated factors of modes < n, as in the single-mode
    update rule of §5). Per mode: G from the current factors (the core
    Alg. 3 forms first), A^(n) = TTMcTC, U^(n) = orthonormal basis of A^(n) by QR.

    U0 must be orthonormal. Stops after `sweeps` sweeps, or earlier when
    stop == "rel_f" and |f_t - f_{t-1}| <= tol * f_t, or stop == "err" and the
    relative approximation error changes by less than tol (§6.1's rule).

    A numerically rank-deficient A^(n) (the QR pivot test of qr_positive) raises
    RankDeficient, or with on_breakdown == "keep" leaves U^(n) as it was for that
    step (the paper does not treat this case; keeping the factor skips one
    single-mode update, so f still does not decrease) and counts it in
    history["skipped"].

    Returns (U, G, history) where history has per-mode-step f (before the update),
    per-sweep f, fit, and optionally every A^(n).
    """
    if on_breakdown not in ("raise", "keep"):
        raise ValueError(on_breakdown)
    validate(idx, dims, ranks)
    idx, vals = coalesce(idx, vals, dims)
    nx2 = norm_x2(vals)
    N = len(dims)
    U = [np.array(u, dtype=np.float64, copy=True) for u in U0]
    core = core_segment if impl == "segment" else (lambda i, v, Us: core_elementwise(i, v, Us))
    tt = ttmctc_segment if impl == "segment" else (lambda i, v, Us, n, G: ttmctc_elementwise(i, v, Us, n, G))
    hist = {"f_step": [], "f_sweep": [], "fit": [], "A": [], "G_step": [], "normx2": nx2, "skipped": 0}
    f_prev = float(np.sum(core(idx, vals, U) ** 2))
    err_prev = math.sqrt(max(nx2 - f_prev, 0.0) / nx2)
    for t in range(sweeps):
        for n in range(N):
            G = core(idx, vals, U)
            hist["f_step"].append(float(np.sum(G * G)))
            A = tt(idx, vals, U, n, G)
            if record_A:
                hist["A"].append(A)
                hist["G_step"].append(G)
            try:
                U[n] = qr_positive(A)[0]
            except RankDeficient:
                if on_breakdown == "raise":
                    raise
                hist["skipped"] += 1
        G = core(idx, vals, U)
        f = float(np.sum(G * G))
        hist["f_sweep"].append(f)
        hist["fit"].append(fit_from(nx2, f))
        if tol is not None:
            if stop == "rel_f" and abs(f - f_prev) <= tol * f:
                break
            if stop == "err":
                err = math.sqrt(max(nx2 - f, 0.0) / nx2)
                if abs(err - err_prev) < tol:
                    break
                err_prev = err
        f_prev = f
    G = core(idx, vals, U)
    return U, G, hist


# --------------------------------------------------------------------------
# HOOI (Alg. 1), the method HOQRI is contrasted with
# --------------------------------------------------------------------------

def leading_left(idx, vals, Us: Sequence[np.ndarray], n: int, K: int):
    """The K leading left singular vectors of Y_(n) = X_(n) (Kronecker over m != n
    of U^(m)), the HOOI update of Alg. 1, from the SVD of its nonempty rows (rows
    of empty slices are zero and add nothing). Returns (U_n with zero rows for
    empty slices, the K leading singular values). Raises RankDeficient when
    fewer than K rows are nonempty."""
    rows, Yr = _slice_rows(idx, vals, Us, n)
    if rows.size < K:
        raise RankDeficient(f"mode {n}: {rows.size} nonempty slices < K = {K}")
    W, s, _ = np.linalg.svd(Yr, full_matrices=False)
    U = np.zeros((Us[n].shape[0], K))
    U[rows] = W[:, :K]
    return U, s[:K]


def hooi(idx, vals, dims, ranks, U0: Sequence[np.ndarray], sweeps: int, tol: float | None = None):
    """Alg. 1 (HOOI): sweeps over n = 1..N in order (Gauss-Seidel, as hoqri);
    per mode U^(n) <- the K_n leading left singular vectors of Y_(n), which
    maximises ||U^T Y_(n)||^2 = f over orthonormal U^(n) with the other factors
    fixed. The basis within the subspace is free (f, the fit and the subspaces do
    not depend on it). Stops after `sweeps` sweeps or when |f_t - f_{t-1}| <=
    tol * f_t. Returns (U, G, history) with history["f_step"] (f after every mode
    update), ["f_sweep"] and ["fit"]."""
    validate(idx, dims, ranks)
    idx, vals = coalesce(idx, vals, dims)
    nx2 = norm_x2(vals)
    N = len(dims)
    U = [np.array(u, dtype=np.float64, copy=True) for u in U0]
    hist = {"f_step": [], "f_sweep": [], "fit": [], "normx2": nx2}
    f_prev = float(np.sum(core_segment(idx, vals, U) ** 2))
    for t in range(sweeps):
        for n in range(N):
            U[n], s = leading_left(idx, vals, U, n, ranks[n])
            hist["f_step"].append(float(np.sum(s * s)))
        f = float(np.sum(core_segment(idx, vals, U) ** 2))
        hist["f_sweep"].append(f)
        hist["fit"].append(fit_from(nx2, f))
        if tol is not None and abs(f - f_prev) <= tol * f:
            break
        f_prev = f
    return U, core_segment(idx, vals, U), hist


# --------------------------------------------------------------------------
# Quantities of the convergence analysis (§5)
# --------------------------------------------------------------------------

def subspace_dist(U: np.ndarray, V: np.ndarray) -> float:
    """d(U, V) = min over orthogonal Q of ||U - V Q||^2 (§5.3). The Procrustes
    minimiser gives 2K - 2 ||U^T V||_* (nuclear norm)."""
    K = U.shape[1]
    return float(2 * K - 2 * np.linalg.svd(U.T @ V, compute_uv=False).sum())


def grad_norm2_mode(A: np.ndarray, G: np.ndarray, n: int) -> float:
    """||grad_{U^(n)} f||^2 = 4 (||A^(n)||^2 - ||G_(n) G_(n)^T||^2) (§5.2, valid when
    U^(n) is orthonormal and A^(n) is the TTMcTC at the same point)."""
    Gn = unfold(G, n)
    GG = Gn @ Gn.T
    return float(4.0 * (np.sum(A * A) - np.sum(GG * GG)))


def grad_norm2_direct(A: np.ndarray, U: np.ndarray, G: np.ndarray, n: int) -> float:
    """||2A - 2 U G_(n) G_(n)^T||^2, the Riemannian gradient of §5.2 before the
    simplification."""
    Gn = unfold(G, n)
    R = 2 * A - 2 * U @ (Gn @ Gn.T)
    return float(np.sum(R * R))


# --------------------------------------------------------------------------
# Start from a randomized range finder (HOSVD-style start of Alg. 2)
# --------------------------------------------------------------------------

def sketch_start(idx, vals, dims, ranks, Omega: Sequence[np.ndarray], Gamma: np.ndarray):
    """Alg. 2 may start from HOSVD. A randomized range finder for the leading
    left singular subspace of every unfolding X_(n): the sketch
    A^(n) = X_(n) (kron over m != n of Omega_m) Gamma_(n)^T, which is exactly
    TTMcTC with the factors replaced by the random Omega_m and the core by the
    random Gamma (definition in §4.1), then U^(n) = the positive-diagonal QR
    basis of A^(n). Every mode is sketched from X alone (not Gauss-Seidel).
    Omega_m (I_m x K_m) and Gamma (K_1 x ... x K_N) are inputs (random draws
    belong to the caller)."""
    idx, vals = coalesce(idx, vals, dims)
    Om = [np.asarray(o, dtype=np.float64) for o in Omega]
    Ga = np.asarray(Gamma, dtype=np.float64)
    return [qr_positive(ttmctc_segment(idx, vals, Om, n, Ga))[0] for n in range(len(dims))]
