"""Parity at the benchmark's full size (the 50M-nonzero 3-way Zipf tensor
1e6 x 5e5 x 2e4, ranks 16^3 in FP32 and 32^3 in BF16), in the launch
configuration bench.py times, on outputs the FP64 oracle can compute one by
one from the same nonzeros:

* core entries G(a, b, c) = sum_e x_e U1(i_e, a) U2(j_e, b) U3(k_e, c) (§2.2),
  each a dot product over all 50M nonzeros;
* TTMcTC rows A^(n)(i, :) of single slices (the heaviest slice of each mode and
  random ones), from the oracle's slice-by-slice definition on that slice's
  nonzeros only;
and on properties that hold at any size: U^T A = G_(n) G_(n)^T (§5.2), a run's
factors orthonormal with f = ||G||^2 of the returned core.

Tolerances: FP32 accumulation over up to 4M terms per slice row: 1e-5
relative (Frobenius over the sampled outputs); BF16 form: the rounding bound of
test_gpu_prec on the sampled values (core: N 2^-8 + 2e-5 times the
|.|-instance; TTMcTC rows at ranks 32^3: (N + 2) 2^-8 + 2e-5, since y_i and the
core are rounded to bfloat16 for their product).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DIMS = (1_000_000, 500_000, 20_000)
NNZ = 50_000_000


@pytest.fixture(scope="module")
def tensor():
    print("[fullsize] generating the 50M-nonzero tensor", flush=True)
    idx, vals = synth.coo_zipf_torch(DIMS, NNZ, 1.2, 12, "lognormal", device=DEV)
    torch.cuda.synchronize()
    return idx, vals, idx.cpu().numpy().astype(np.int64), vals.cpu().numpy().astype(np.float64)


def start(K, seed):
    return [H.hoqri_orth(r)[0] for r in synth.gaussian_start_torch(DIMS, K, seed, device=DEV)]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def sample_slices(ih, n, rng, k=4):
    counts = np.bincount(ih[n], minlength=DIMS[n])
    nonempty = np.flatnonzero(counts)
    return [int(np.argmax(counts))] + [int(x) for x in rng.choice(nonempty, size=k - 1, replace=False)]


@pytest.mark.parametrize("K,prec", [((16, 16, 16), "fp32"), ((32, 32, 32), "bf16")])
def test_fullsize_core_entries_and_slice_rows(tensor, K, prec):
    idx, vals, ih, vh = tensor
    print(f"[fullsize] K={K} prec={prec}", flush=True)
    plan = H.hoqri_plan_create(idx, vals, DIMS, K)
    Ud = start(K, 112 if K[0] == 16 else 113)
    G = H.hoqri_core(plan, Ud, prec=prec)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().astype(np.float64)
    Uh = [u.cpu().numpy().astype(np.float64) for u in Ud]
    rng = np.random.default_rng(1)
    # sampled core entries, each over all nonzeros (float32 operands: 1e-5 on
    # the sample; the 16-bit form within its rounding bound)
    picks = [tuple(int(rng.integers(k)) for k in K) for _ in range(6)]
    got, ref, absref = [], [], []
    Uabs = [np.abs(u) for u in Uh]
    for ks in picks:
        ref.append(O.core_entry(ih, vh, Uh, ks))
        absref.append(O.core_entry(ih, np.abs(vh), Uabs, ks))
        got.append(Gh[ks])
    got, ref, absref = map(np.array, (got, ref, absref))
    if prec == "fp32":
        assert rel(got, ref) < 1e-5
    else:
        assert np.all(np.abs(got - ref) <= (3 * 2.0 ** -8 + 2e-5) * absref)
    # sampled TTMcTC rows with the float32 core the GPU used
    G64 = Gh
    for n in range(3):
        A = H.hoqri_ttmctc(plan, n, Ud, G, prec=prec)
        torch.cuda.synchronize()
        for i in sample_slices(ih, n, rng):
            print(f"[fullsize] mode {n} slice {i}", flush=True)
            row = A[i].cpu().numpy().astype(np.float64)
            want = O.ttmctc_slice_row(ih, vh, Uh, n, i, G64)
            if prec == "fp32":
                assert rel(row, want) < 1e-5, (n, i)
            else:
                wabs = O.ttmctc_slice_row(ih, np.abs(vh), Uabs, n, i, np.abs(G64))
                # y_i and the core are rounded to bfloat16 for their product too
                lim = (5 * 2.0 ** -8 + 2e-5) * wabs + 1e-9 * wabs.max()
                assert np.all(np.abs(row - want) <= lim), (n, i)
    plan.destroy()


def test_fullsize_identities_and_run(tensor):
    idx, vals, ih, vh = tensor
    K = (16, 16, 16)
    plan = H.hoqri_plan_create(idx, vals, DIMS, K)
    Ud = start(K, 112)
    G = H.hoqri_core(plan, Ud)
    for n in range(3):
        A = H.hoqri_ttmctc(plan, n, Ud, G).double()
        Gn = O.unfold(G.cpu().double().numpy(), n)
        lhs = (Ud[n].double().T @ A).cpu().numpy()
        assert rel(lhs, Gn @ Gn.T) < 1e-5, n
    # two sweeps as bench.py runs them: orthonormal factors, f = ||G||^2, and
    # the returned core equals the core of the returned factors (sampled)
    Us = [u.clone() for u in Ud]
    G2, st = H.hoqri_run(plan, Us, max_sweeps=2, keep_on_breakdown=True)
    torch.cuda.synchronize()
    assert st.orth_err_max < 1e-5
    Gh = G2.cpu().numpy().astype(np.float64)
    assert st.f == pytest.approx(float(np.sum(Gh * Gh)), rel=1e-6)
    Uh = [u.cpu().numpy().astype(np.float64) for u in Us]
    rng = np.random.default_rng(2)
    got, ref = [], []
    for _ in range(4):
        ks = tuple(int(rng.integers(16)) for _ in range(3))
        ref.append(O.core_entry(ih, vh, Uh, ks))
        got.append(Gh[ks])
    assert rel(got, ref) < 1e-5
    plan.destroy()


# The 4-way workload at full size: 2e5 x 2e5 x 5e3 x 1e3, 100M Zipf(1.1)
# nonzeros with uniform(0,1) values, ranks 10^4, in the FP16 form bench.py
# times and in the FP32 form (both through the c-tile pass).
DIMS4 = (200_000, 200_000, 5_000, 1_000)
NNZ4 = 100_000_000
K4 = (10, 10, 10, 10)


def test_fullsize_4way_core_entries_and_slice_rows():
    print("[fullsize4] generating the 100M-nonzero 4-way tensor", flush=True)
    idx, vals = synth.coo_zipf_torch(DIMS4, NNZ4, 1.1, 14, "uniform", device=DEV)
    torch.cuda.synchronize()
    ih = idx.cpu().numpy().astype(np.int64)
    vh = vals.cpu().numpy().astype(np.float64)
    plan = H.hoqri_plan_create(idx, vals, DIMS4, K4)
    del idx, vals
    Ud = [H.hoqri_orth(r)[0] for r in synth.gaussian_start_torch(DIMS4, K4, 114, device=DEV)]
    torch.cuda.synchronize()
    Uh = [u.cpu().numpy().astype(np.float64) for u in Ud]
    Uabs = [np.abs(u) for u in Uh]
    vabs = np.abs(vh)
    rng = np.random.default_rng(4)
    picks = [tuple(int(rng.integers(k)) for k in K4) for _ in range(4)]
    ref = np.array([O.core_entry(ih, vh, Uh, ks) for ks in picks])
    absref = np.array([O.core_entry(ih, vabs, Uabs, ks) for ks in picks])
    slices = [sample_slices_dims(ih, n, DIMS4, rng, k=3) for n in range(4)]
    for prec in ("fp16", "fp32"):
        print(f"[fullsize4] prec={prec} core", flush=True)
        G = H.hoqri_core(plan, Ud, prec=prec)
        torch.cuda.synchronize()
        Gh = G.cpu().numpy().astype(np.float64)
        got = np.array([Gh[ks] for ks in picks])
        if prec == "fp32":
            assert rel(got, ref) < 1e-5
        else:
            # core pass of the FP16 form (the c-tile walk rounds its A operand in two
            # steps): (N + 1) u16 of the |.|-instance, float32 accumulation
            assert np.all(np.abs(got - ref) <= (5 * 2.0 ** -11 + 2e-5) * absref)
        for n in range(4):
            A = H.hoqri_ttmctc(plan, n, Ud, G, prec=prec)
            torch.cuda.synchronize()
            for i in slices[n]:
                print(f"[fullsize4] prec={prec} mode {n} slice {i}", flush=True)
                row = A[i].cpu().numpy().astype(np.float64)
                want = O.ttmctc_slice_row(ih, vh, Uh, n, i, Gh)
                if prec == "fp32":
                    assert rel(row, want) < 1e-5, (n, i)
                else:
                    wabs = O.ttmctc_slice_row(ih, vabs, Uabs, n, i, np.abs(Gh))
                    # the FP16 c-tile pass: (N + 1) u16 for the factor copies and the
                    # two-step A operand, plus 2 bfloat16 roundings of y_i and the core
                    lim = (5 * 2.0 ** -11 + 2 * 2.0 ** -8 + 2e-5) * wabs + 1e-9 * wabs.max()
                    assert np.all(np.abs(row - want) <= lim), (n, i)
    plan.destroy()


def sample_slices_dims(ih, n, dims, rng, k=3):
    counts = np.bincount(ih[n], minlength=dims[n])
    nonempty = np.flatnonzero(counts)
    return [int(np.argmax(counts))] + [int(x) for x in rng.choice(nonempty, size=k - 1, replace=False)]
