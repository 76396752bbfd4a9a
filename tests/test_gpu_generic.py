"""The split-Kronecker pass against the FP64 oracle: the 5-way workload of
Fig. 5 (I = 80, K = 10 per mode, so 10^4 Kronecker entries per nonzero) and
modes whose y_i spans more 16x16 tiles than the segment passes take.

Float32 form: single calls agree with the oracle within 1e-5 relative
(Frobenius) and elementwise within the float32 bound; whole runs in fit within
1e-5 relative after the same sweeps from the same start. BF16 form: elementwise
within its rounding bound.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def fp32_bound_check(got, ref, absref, terms, what):
    """Elementwise float32 bound gamma_T |.|-instance (T roundings along one
    term's path, u32 = 2^-24), valid for any summation order."""
    err = np.abs(np.asarray(got, np.float64) - ref)
    t = np.asarray(terms, np.float64) * 2.0 ** -24
    lim = t / (1.0 - t) * absref
    bad = err > lim
    assert not bad.any(), f"{what}: {bad.sum()} entries over the float32 bound"


@pytest.mark.parametrize("dims,K,nnz", [((30, 25, 20, 15, 12), (3, 4, 2, 5, 3), 3000),
                                        ((60, 50, 40, 30), (12, 12, 4, 4), 6000),
                                        ((40, 30, 20, 10), (20, 20, 12, 8), 4000)])
def test_single_calls_match_oracle(dims, K, nnz):
    print(f"[generic] dims={dims} K={K}", flush=True)
    idx, vals = synth.coo_uniform(dims, nnz, seed=sum(K))
    vals32 = vals.astype(np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 5))]
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U64 = [u.astype(np.float64) for u in U]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    G = H.hoqri_core(plan, Ud)
    Gref = O.core_segment(ci, cv, U64)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy()
    assert rel(Gh, Gref) < 1e-5
    N = len(dims)
    Uabs = [np.abs(u) for u in U64]
    fp32_bound_check(Gh, Gref, O.core_segment(ci, np.abs(cv), Uabs), cv.size + N + 1, "core")
    G32 = Gref.astype(np.float32)
    for n in range(N):
        A = H.hoqri_ttmctc(plan, n, Ud, dev(G32))
        Aref = O.ttmctc_segment(ci, cv, U64, n, G32.astype(np.float64))
        torch.cuda.synchronize()
        Ah = A.cpu().numpy()
        assert rel(Ah, Aref) < 1e-5, n
        Aabs = O.ttmctc_segment(ci, np.abs(cv), Uabs, n, np.abs(G32.astype(np.float64)))
        L = np.bincount(ci[n], minlength=dims[n]).astype(np.float64)
        P = int(np.prod(K)) // K[n]
        fp32_bound_check(Ah, Aref, Aabs, (L + P + N + 1)[:, None], f"ttmctc mode {n}")


@pytest.mark.parametrize("nnz", [800, 8000])
def test_five_way_run_follows_oracle(nnz):
    # Fig. 5's workload: 80^5 tensor, nnz = 10 I or 100 I, rank 10 per mode
    dims, K = (80,) * 5, (10,) * 5
    idx, vals = synth.coo_uniform(dims, nnz, seed=nnz)
    vals32 = vals.astype(np.float32)
    U0 = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 6))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Us = [dev(u) for u in U0]
    G, st = H.hoqri_run(plan, Us, max_sweeps=3, keep_on_breakdown=True)
    torch.cuda.synchronize()
    Uo, Go, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in U0], sweeps=3,
                        on_breakdown="keep")
    assert st.skipped_updates == h["skipped"]
    assert st.fit == pytest.approx(h["fit"][-1], rel=1e-5)
    assert st.orth_err_max < 1e-5


def test_split_kronecker_forms():
    # the split-Kronecker pass takes float32 and bfloat16 operands; float16 is refused
    dims, K = (30, 25, 20, 15, 12), (3, 4, 2, 5, 3)
    idx, vals = synth.coo_uniform(dims, 2000, seed=3)
    plan = H.hoqri_plan_create(dev(idx), dev(vals.astype(np.float32)), dims, K)
    U = [dev(u.astype(np.float32)) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 4))]
    with pytest.raises(H.HoqriError):
        H.hoqri_run(plan, [u.clone() for u in U], max_sweeps=1, prec="fp16")
    H.hoqri_run(plan, [u.clone() for u in U], max_sweeps=1, prec="bf16", keep_on_breakdown=True)


@pytest.mark.parametrize("dims,K,nnz", [((30, 25, 20, 15, 12), (3, 4, 2, 5, 3), 3000),
                                        ((80,) * 5, (10,) * 5, 8000),
                                        ((40, 30, 20, 10), (20, 20, 12, 8), 4000)])
def test_bf16_split_kronecker_within_rounding_bound(dims, K, nnz):
    # BF16 form: every term's two Kronecker halves are rounded once each to
    # bfloat16 (2 u16, u16 = 2^-8), float32 accumulation and a float32 product
    # with the core: |A_gpu - A| <= (2 u16 + 2e-5) TTMcTC(|X|, {|U|}, |G|)
    print(f"[generic-bf16] dims={dims} K={K}", flush=True)
    idx, vals = synth.coo_uniform(dims, nnz, seed=sum(K) + 1)
    vals32 = vals.astype(np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 8))]
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U64 = [u.astype(np.float64) for u in U]
    Uabs = [np.abs(u) for u in U64]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    Gref = O.core_segment(ci, cv, U64)
    Gabs = O.core_segment(ci, np.abs(cv), Uabs)
    N = len(dims)
    if N == 5:  # every mode takes the split-Kronecker pass, the core too
        G = H.hoqri_core(plan, Ud, prec="bf16").cpu().numpy().astype(np.float64)
        lim = (2 * 2.0 ** -8 + 2e-5) * Gabs + 1e-9 * Gabs.max()
        assert np.all(np.abs(G - Gref) <= lim)
    G32 = Gref.astype(np.float32)
    for n in range(N):
        if N == 4 and np.prod([K[m] for m in range(N) if m != n]) <= 2048:
            continue  # segment-pass modes are covered by test_gpu_prec
        A = H.hoqri_ttmctc(plan, n, Ud, dev(G32), prec="bf16").cpu().numpy().astype(np.float64)
        Aref = O.ttmctc_segment(ci, cv, U64, n, G32.astype(np.float64))
        Aabs = O.ttmctc_segment(ci, np.abs(cv), Uabs, n, np.abs(G32.astype(np.float64)))
        lim = (2 * 2.0 ** -8 + 2e-5) * Aabs + 1e-9 * Aabs.max()
        err = np.abs(A - Aref)
        assert np.all(err <= lim), (n, float(np.max(err / lim)))


def test_bf16_five_way_run():
    # a BF16 run on Fig. 5's shape: orthonormal factors, and the returned core
    # and f are those of the returned factors with float32 operands
    dims, K = (80,) * 5, (10,) * 5
    idx, vals = synth.coo_uniform(dims, 8000, seed=8000)
    vals32 = vals.astype(np.float32)
    U0 = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 6))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Us = [dev(u) for u in U0]
    G, st = H.hoqri_run(plan, Us, max_sweeps=3, prec="bf16", keep_on_breakdown=True)
    torch.cuda.synchronize()
    assert st.orth_err_max < 1e-5
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    Gchk = O.core_segment(ci, cv, [u.cpu().numpy().astype(np.float64) for u in Us])
    assert np.linalg.norm(G.cpu().numpy() - Gchk) / np.linalg.norm(Gchk) < 1e-5
    assert st.f == pytest.approx(float(np.sum(Gchk ** 2)), rel=2e-5)
