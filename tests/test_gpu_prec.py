"""GPU parity of the 16-bit operand forms (BF16, FP16) against the FP64 oracle.

Bound used for the segment passes: every term of y_i is a product of one
value and one factor entry per other mode. In the 16-bit forms the factor
copies are rounded once each and the value-times-row-entries operand once
more, all to nearest, so each term carries a relative error of at most
(N-1+1) u16 plus float32 rounding, with u16 = 2^-8 (bfloat16, 8-bit
significand) or 2^-11 (float16, 11-bit significand). Summing terms and
multiplying by the float32 core cannot raise that relative error above the
same factor times the result of the same computation on absolute values:
    |A_gpu - A| <= (N u16 + eps32) * TTMcTC(|X|, {|U|}, |G|)   elementwise,
and likewise for the core. Where a pass also rounds y_i and the core to
bfloat16 before their product (BF16 with y_i of 2 x 2 blocks: 3-way tensors
with both other ranks in 17..32; BF16 and FP16 on 4-way tensors with all
other ranks at most 16), two more bfloat16 roundings enter every term:
N u16 + 2 * 2^-8; the FP16 form of that 4-way pass rounds its A operand in two
steps (x U_a, then the packed product with U_c): (N + 1) u16 + 2 * 2^-8.
The oracle evaluates the right-hand side (the
operation is multilinear, so its absolute-value instance is the same
definition). Float16 gradual underflow adds an absolute error far below
1e-9 max|A| for these shapes (the operand is scaled so its largest
possible magnitude is below 60000).

Whole runs, at each workload's own sweep count from the same start: a 16-bit
form qualifies when its fit is within 1e-4 relative of the FP64 oracle's. On
the Zipf-structured tensors with the benchmark workloads' shapes every form
qualifies (gaps of 1e-6 to 6e-5). On uniformly random tensors the objective is
almost flat (fit ~0.002) and the 16-bit roundings move the trajectory: the
bfloat16 form of the 200^3 parity workload misses 1e-4 after its 10 sweeps
(1.6e-4), as both 16-bit forms do on the uniform rank-32 tensor; such a form is
recorded as not qualifying together with its time to fit (the sweeps and
milliseconds it needs to reach (1 - 1e-4) times the oracle's fit).
"""
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U16 = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
EPS32 = 2e-5  # float32 roundings and accumulation, generous for slices of a few hundred terms


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def make(name):
    if name == "c1":
        dims, K = (200, 200, 200), (5, 5, 5)
        idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    elif name == "n3k32":
        dims, K = (3000, 2000, 400), (32, 32, 32)
        idx, vals = synth.coo_uniform(dims, 60_000, seed=3)
    elif name == "n3rag":
        # ragged ranks: mode 2's other ranks (20, 24) give y_i of 2 x 2 padded blocks
        dims, K = (2500, 1800, 300), (20, 24, 12)
        idx, vals = synth.coo_zipf(dims, 80_000, alpha=1.2, seed=5)
    elif name == "zipf3":
        dims, K = (30000, 15000, 600), (16, 16, 16)
        idx, vals = synth.coo_zipf(dims, 200_000, alpha=1.2, seed=2)
    elif name == "n4k10":
        dims, K = (4000, 4000, 100, 20), (10, 10, 10, 10)
        idx, vals = synth.coo_zipf(dims, 100_000, alpha=1.1, seed=6, values="uniform")
    elif name == "n4rag":
        # ragged 4-way ranks: c-tile waves with 4, 4 and 1 (or 4 x 4) columns
        dims, K = (3000, 2500, 200, 40), (6, 12, 9, 16)
        idx, vals = synth.coo_zipf(dims, 80_000, alpha=1.1, seed=8, values="uniform")
    elif name == "n4kn2":
        # mode 0 of rank 20 (two 16-column blocks of A) through the c-tile pass
        dims, K = (3000, 200, 150, 100), (20, 4, 4, 4)
        idx, vals = synth.coo_zipf(dims, 60_000, alpha=1.1, seed=23, values="uniform")
    elif name == "tiny3":
        # fewer nonzeros than one 16-nonzero block; y_i of 2 x 2 blocks in mode 2
        dims, K = (30, 40, 50), (20, 24, 12)
        idx, vals = synth.coo_uniform(dims, 7, seed=21)
    elif name == "tiny4":
        dims, K = (12, 11, 10, 9), (6, 7, 8, 9)
        idx, vals = synth.coo_uniform(dims, 5, seed=22)
    elif name == "n2":
        dims, K = (3000, 2000), (8, 8)
        idx, vals = synth.coo_uniform(dims, 40_000, seed=7)
    elif name == "wide":
        # values spread over ~12 orders of magnitude: exercises the FP16 operand scale
        dims, K = (800, 700, 600), (6, 7, 5)
        idx, vals = synth.coo_uniform(dims, 30_000, seed=9)
        rng = np.random.default_rng(9)
        vals = vals * np.exp(rng.normal(0.0, 4.0, vals.size))
    else:
        raise KeyError(name)
    vals32 = vals.astype(np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 100))]
    return dims, K, idx, vals32, U


def ttmctc_tol(prec, K, n):
    """Relative bound of a TTMcTC pass: N u16 + eps32, plus 2 u_bf16 where the
    pass also rounds y_i and the core to bfloat16 for their product (BF16,
    3-way with both other ranks in 17..32; BF16 and FP16, 4-way with all other
    ranks at most 16)."""
    N = len(K)
    others = [K[m] for m in range(N) if m != n]
    ctile = prec in ("bf16", "fp16") and N == 4 and all(k <= 16 for k in others)
    bf16_core = (prec == "bf16" and N == 3 and all(16 < k <= 32 for k in others)) or ctile
    # the FP16 c-tile pass rounds x U_a to float16 before the packed product with U_c
    n_round = N + 1 if (ctile and prec == "fp16") else N
    return n_round * U16[prec] + (2 * U16["bf16"] if bf16_core else 0.0) + EPS32


def bound_check(got, ref, absref, tol_rel, what):
    err = np.abs(np.asarray(got, np.float64) - ref)
    lim = tol_rel * absref + 1e-9 * absref.max()
    bad = err > lim
    assert not bad.any(), f"{what}: {bad.sum()} entries over the bound, worst ratio {np.max(err / lim):.3g}"
    # the bound is not vacuous: the 16-bit error is visible but well inside it
    return float(np.max(err / np.maximum(lim, 1e-300)))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("name", ["c1", "n2", "zipf3", "n3k32", "n3rag", "n4k10", "n4rag", "n4kn2", "tiny3", "tiny4", "wide"])
def test_16bit_passes_within_rounding_bound(name, prec):
    print(f"[prec] case={name} prec={prec}", flush=True)
    dims, K, idx, vals32, U = make(name)
    N = len(dims)
    tol_rel = N * U16[prec] + EPS32
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U64 = [u.astype(np.float64) for u in U]
    Uabs = [np.abs(u) for u in U64]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    G = H.hoqri_core(plan, Ud, prec=prec)
    Gref = O.core_segment(ci, cv, U64)
    Gabs = O.core_segment(ci, np.abs(cv), Uabs)
    torch.cuda.synchronize()
    bound_check(G.cpu().numpy(), Gref, Gabs, tol_rel, "core")
    G32 = Gref.astype(np.float32)
    Gd = dev(G32)
    G64 = G32.astype(np.float64)
    for n in range(N):
        A = H.hoqri_ttmctc(plan, n, Ud, Gd, prec=prec)
        Aref = O.ttmctc_segment(ci, cv, U64, n, G64)
        Aabs = O.ttmctc_segment(ci, np.abs(cv), Uabs, n, np.abs(G64))
        torch.cuda.synchronize()
        Ah = A.cpu().numpy()
        bound_check(Ah, Aref, Aabs, ttmctc_tol(prec, K, n), f"ttmctc mode {n}")
        empty = np.setdiff1d(np.arange(dims[n]), idx[n])
        assert np.all(Ah[empty] == 0.0)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_16bit_forms_are_deterministic(prec):
    dims, K, idx, vals32, U = make("zipf3")
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    G1 = H.hoqri_core(plan, Ud, prec=prec).clone()
    G2 = H.hoqri_core(plan, Ud, prec=prec).clone()
    A1 = H.hoqri_ttmctc(plan, 1, Ud, G1, prec=prec).clone()
    A2 = H.hoqri_ttmctc(plan, 1, Ud, G1, prec=prec).clone()
    torch.cuda.synchronize()
    assert torch.equal(G1, G2) and torch.equal(A1, A2)


def run_fit(name, prec, sweeps):
    dims, K, idx, vals32, U0 = make(name)
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Us = [dev(u) for u in U0]
    G, st = H.hoqri_run(plan, Us, max_sweeps=sweeps, prec=prec)
    torch.cuda.synchronize()
    Uo, Go, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in U0], sweeps=sweeps)
    return dims, K, idx, vals32, [u.cpu().numpy().astype(np.float64) for u in Us], G.cpu().numpy(), st, Uo, h, plan, U0


# (form, tensor, the workload's own sweep count, qualifies). A form qualifies
# when its fit after those sweeps is within 1e-4 relative of the FP64
# oracle's after the same sweeps from the same start. The Zipf tensors have
# the shapes of the benchmark workloads (3-way K = 16 and 32 at 20 sweeps;
# 4-way K = 10 at 15); the 200^3 uniform tensor is the 10-sweep parity
# workload, whose objective is almost flat (fit ~0.002): there the 16-bit
# roundings move the trajectory by more than 1e-4 at 10 sweeps and the forms
# do not qualify; for them the test measures the time to fit, the sweeps (and
# milliseconds) until the form's fit reaches (1 - 1e-4) times the oracle's fit
# after the workload's sweeps.
FIT_GATE = [("bf16", "c1", 10, False), ("fp16", "c1", 10, None), ("bf16", "zipf3", 20, True),
            ("fp16", "zipf3", 20, True), ("bf16", "n3rag", 20, True), ("bf16", "n4k10", 15, True),
            ("fp16", "n4k10", 15, True), ("bf16", "n3k32", 15, False), ("fp16", "n3k32", 15, False)]


@pytest.mark.parametrize("prec,name,sweeps,qualifies", FIT_GATE)
def test_16bit_fit_at_the_workload_sweeps(prec, name, sweeps, qualifies):
    print(f"[prec-run] case={name} prec={prec} sweeps={sweeps}", flush=True)
    dims, K, idx, vals32, U, G, st, Uo, h, plan, U0 = run_fit(name, prec, sweeps)
    assert st.sweeps == sweeps
    fit_o = h["fit"][-1]
    gap = abs(st.fit - fit_o) / abs(fit_o)
    ok = gap <= 1e-4
    assert st.orth_err_max < 1e-5
    # the returned core and f are the float32-operand ones for the returned factors
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    Gchk = O.core_segment(ci, cv, U)
    assert np.linalg.norm(G - Gchk) / np.linalg.norm(Gchk) < 1e-5
    assert st.f == pytest.approx(float(np.sum(Gchk ** 2)), rel=2e-5)
    if qualifies is not None:
        assert ok == qualifies, f"{prec} {name}: fit gap {gap:.3g} after {sweeps} sweeps"
    if ok:
        print(f"[fit-gate] {prec} {name} {sweeps} sweeps: qualifies, gap {gap:.2e}", flush=True)
        return
    # not qualifying: time to fit, i.e. the first sweep count at which the form's
    # fit reaches (1 - 1e-4) fit_o, measured by runs of that many sweeps from the
    # same start (at most 4x the workload's sweeps), against the FP32 form's time
    # for the workload's sweeps
    target = (1.0 - 1e-4) * fit_o

    def timed(p, T):
        Us = [dev(u) for u in U0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s2 = H.hoqri_run(plan, Us, max_sweeps=T, prec=p)
        torch.cuda.synchronize()
        return s2, 1e3 * (time.perf_counter() - t0)

    T = None
    for t in range(sweeps + 1, 4 * sweeps + 1):
        s2, ms = timed(prec, t)
        if s2.fit >= target:
            T = t
            break
    assert T is not None, f"{prec} {name}: fit {s2.fit} still below {target} after {4 * sweeps} sweeps"
    _, ms32 = timed("fp32", sweeps)
    print(f"[fit-gate] {prec} {name} {sweeps} sweeps: does not qualify (gap {gap:.2e}); "
          f"time to fit {T} sweeps, {ms:.2f} ms (FP32 form, {sweeps} sweeps: {ms32:.2f} ms)", flush=True)


def test_fp16_rejects_factors_out_of_range():
    # the float16 copies are u * 2^15: entries of magnitude 1.5 or more (never
    # in a factor with orthonormal columns) would leave the float16 range, so
    # the FP16 form refuses them before any pass, leaving the outputs untouched
    dims, K, idx, vals32, U = make("c1")
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    bad = [u.copy() for u in U]
    bad[1][7, 2] = 3.0
    Ud = [dev(u) for u in bad]
    G = torch.full(K, 5.0, dtype=torch.float32, device=DEV)
    with pytest.raises(H.HoqriError) as e:
        H.hoqri_core(plan, Ud, G=G, prec="fp16")
    assert e.value.status == -1 and torch.all(G == 5.0)
    A = torch.full((dims[0], K[0]), 5.0, dtype=torch.float32, device=DEV)
    with pytest.raises(H.HoqriError) as e:
        H.hoqri_ttmctc(plan, 0, Ud, dev(np.ones(K, np.float32)), A=A, prec="fp16")
    assert e.value.status == -1 and torch.all(A == 5.0)
    # the mode being updated is not cast: its factor may hold anything
    H.hoqri_ttmctc(plan, 1, Ud, dev(np.ones(K, np.float32)), prec="fp16")
    # BF16 copies keep float32's range: no such limit
    H.hoqri_core(plan, Ud, prec="bf16")
    torch.cuda.synchronize()
