"""The core of the fused mode update (G_(n) = U^(n)T Y_(n) from the rows the
TTMcTC pass stores, §4.2) against the FP64 oracle's core G = X x {U^T}.

hoqri_core_rows runs exactly the route hoqri_run takes after each mode's QR
step: the TTMcTC pass of that mode keeps its slice rows (bfloat16 in the
2 x 2-block BF16 pass, float32 otherwise), and the core follows from them and
the mode's factor. The shapes have most slices of two modes holding a few
nonzeros (Zipf tails), ranges that split some slices (their partial rows go
through the split-slice path), ranks below 32, and a mode rank of at most 16.

Bound, elementwise against the |.|-instance of the same definition (see
test_gpu_prec): a stored bfloat16 row's term carries the two bfloat16 factor
copies, x U_a and y_i rounded to bfloat16 (4 roundings of 2^-9; the factor of
the mode enters through split bfloat16 products), so
|G - G_ref| <= (3 u16 + 2 u16 + eps32) G_abs with u16 = 2^-8, as for the
2 x 2-block pass's TTMcTC. With nonnegative values and factors G is its own
|.|-instance and the bound is tight (with signed random factors G is far
below it). Float32 form: the float32 bound gamma_T.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U16 = 2.0 ** -8
EPS32 = 2e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = {
    # most slices of modes 0 and 1 hold a few nonzeros (Zipf tails), mode 2 long ones
    "short32": ((40_000, 20_000, 800), (32, 32, 32), 150_000),
    # ranks below 32 (every mode's other ranks even in 17..32) and a mode rank of 20
    "short_rag": ((30_000, 25_000, 600), (20, 24, 18), 120_000),
    # the mode's own rank at most 16 (partials of 16 rows) for mode 0
    "short_k12": ((30_000, 12_000, 500), (12, 24, 20), 100_000),
}


def short_fraction(idx, dims, n):
    cnt = np.bincount(idx[n], minlength=dims[n])
    cnt = cnt[cnt > 0]
    return float(np.mean(cnt <= 8))


@pytest.mark.parametrize("sign", ["signed", "nonnegative"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_core_from_rows_bf16_within_rounding_bound(name, sign):
    # nonnegative values and factors: G is its own |.|-instance, so the bound
    # is tight and a lost or misplaced share of any slice breaks it
    dims, K, nnz = CASES[name]
    print(f"[core-rows] case={name} {sign} dims={dims} K={K}", flush=True)
    idx, vals = synth.coo_zipf(dims, nnz, alpha=1.2, seed=len(name))
    vals32 = vals.astype(np.float32)
    if sign == "nonnegative":
        vals32 = np.abs(vals32)
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    # most slices of modes 0 and 1 hold at most 8 nonzeros
    assert short_fraction(ci, dims, 0) > 0.5 and short_fraction(ci, dims, 1) > 0.3
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 31))]
    if sign == "nonnegative":
        U = [np.abs(u) for u in U]
    U64 = [u.astype(np.float64) for u in U]
    Gref = O.core_segment(ci, cv, U64)
    Gabs = O.core_segment(ci, np.abs(cv), [np.abs(u) for u in U64])
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    Gst = dev(Gref.astype(np.float32))
    tol = 5 * U16 + EPS32
    for n in range(3):
        f = torch.zeros(1, dtype=torch.float64, device=DEV)
        G = H.hoqri_core_rows(plan, n, Ud, Gst, f=f, prec="bf16")
        G2 = H.hoqri_core_rows(plan, n, Ud, Gst, prec="bf16")
        torch.cuda.synchronize()
        Gh = G.cpu().numpy().astype(np.float64)
        err = np.abs(Gh - Gref)
        lim = tol * Gabs + 1e-9 * Gabs.max()
        assert np.all(err <= lim), (n, float(np.max(err / lim)))
        assert torch.equal(G, G2)  # fixed summation order
        assert f.item() == pytest.approx(float(np.sum(G.cpu().numpy().astype(np.float64) ** 2)), rel=1e-6)


@pytest.mark.parametrize("dims,K,nnz", [((40_000, 20_000, 800), (16, 16, 16), 150_000),
                                        ((30_000, 25_000, 600), (20, 24, 18), 120_000)])
def test_core_from_rows_fp32_matches_oracle(dims, K, nnz):
    print(f"[core-rows] fp32 dims={dims} K={K}", flush=True)
    idx, vals = synth.coo_zipf(dims, nnz, alpha=1.2, seed=sum(K))
    vals32 = vals.astype(np.float32)
    ci, cv = O.coalesce(idx, vals32.astype(np.float64), dims)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 32))]
    U64 = [u.astype(np.float64) for u in U]
    Gref = O.core_segment(ci, cv, U64)
    Gabs = O.core_segment(ci, np.abs(cv), [np.abs(u) for u in U64])
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Ud = [dev(u) for u in U]
    Gst = dev(Gref.astype(np.float32))
    for n in range(3):
        G = H.hoqri_core_rows(plan, n, Ud, Gst, prec="fp32").cpu().numpy().astype(np.float64)
        err = np.abs(G - Gref)
        # gamma_T with T bounding the roundings along one term's path: the
        # products, the slice sum (its longest slice), and the float32 sum over
        # one partial's rows (at most an eighth of the rows and split partials,
        # ranges <= 16384), then the float64 reduction
        L = int(np.bincount(ci[n]).max())
        R = int(np.unique(ci[n]).size)
        t = (L + 8 + (R + 2 * 16384) // 8 + 1) * 2.0 ** -24
        lim = t / (1 - t) * Gabs + 1e-12 * Gabs.max()
        assert np.all(err <= lim), (n, float(np.max(err / lim)))
        assert np.linalg.norm(G - Gref) / np.linalg.norm(Gref) < 1e-5


def test_bf16_run_from_warm_start_follows_oracle():
    # a BF16 run on a tensor whose slices are mostly a few nonzeros long: f
    # before every mode update (each from the previous update's core from
    # stored rows) follows the FP64 oracle's trajectory from the same start.
    # The start is warm (3 FP64 oracle sweeps from a random one): at a random
    # start A is tiny against its |.|-instance, and the 16-bit roundings,
    # bounded relative to that instance, can move the first updates by percents.
    dims, K, nnz = (24_000, 12_000, 500), (32, 32, 32), 70_000
    idx, vals = synth.coo_zipf(dims, nnz, alpha=1.2, seed=7)
    v64 = vals.astype(np.float32).astype(np.float64)
    U0 = O.orthonormal_start(synth.gaussian_start(dims, K, 33))
    Uw, _, hw = O.hoqri(idx, v64, dims, K, [u.astype(np.float64) for u in U0], sweeps=3, on_breakdown="keep")
    assert hw["skipped"] == 0
    Uw32 = [u.astype(np.float32) for u in Uw]
    plan = H.hoqri_plan_create(dev(idx), dev(vals.astype(np.float32)), dims, K)
    Us = [dev(u) for u in Uw32]
    fh = torch.zeros(2 * 3, dtype=torch.float64, device=DEV)
    G, st = H.hoqri_run(plan, Us, max_sweeps=2, prec="bf16", f_hist=fh, keep_on_breakdown=True)
    torch.cuda.synchronize()
    Uo, Go, h = O.hoqri(idx, v64, dims, K, [u.astype(np.float64) for u in Uw32], sweeps=2, on_breakdown="keep")
    assert st.sweeps == 2 and st.skipped_updates == 0 and h["skipped"] == 0
    np.testing.assert_allclose(fh.cpu().numpy(), h["f_step"], rtol=5e-3)
    assert abs(st.fit - h["fit"][-1]) / h["fit"][-1] < 1e-3
