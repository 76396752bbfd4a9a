"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Both sides get identical inputs: the same coordinates, the float32 values and
float32 factors (the oracle promotes them to float64). Float32 results must be
within 1e-5 relative Frobenius error of the oracle (the bar for the TTMcTC
output); integer work (merged nonzero count, slice counts) must match exactly.
Shapes span several work ranges (slices split across ranges), ragged tails and
empty slices.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2510_16930_amd import _lib as H
from paper_2510_16930_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def rel_fro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


U32 = 2.0 ** -24


def fp32_bound_check(got, ref, absref, terms, what):
    """Elementwise float32 bound: a float32 evaluation of a sum of products, in
    any order, with every product and partial sum rounded to nearest, is within
    gamma_T = T u32 / (1 - T u32) (T roundings along one term's path, u32 =
    2^-24) times the same computation on absolute values; `terms` is T per
    output entry (broadcast against the outputs)."""
    err = np.abs(np.asarray(got, np.float64) - ref)
    t = np.asarray(terms, np.float64) * U32
    lim = t / (1.0 - t) * absref
    bad = err > lim
    assert not bad.any(), f"{what}: {bad.sum()} entries over the float32 bound, worst ratio {np.max(err / np.maximum(lim, 1e-300)):.3g}"


def make_case(name):
    if name == "c1":
        dims, K = (200, 200, 200), (5, 5, 5)
        idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    elif name == "zipf3":
        dims, K = (30000, 15000, 600), (16, 16, 16)
        idx, vals = synth.coo_zipf(dims, 200_000, alpha=1.2, seed=2)
    elif name == "n3k32":
        dims, K = (3000, 2000, 400), (32, 32, 32)
        idx, vals = synth.coo_uniform(dims, 60_000, seed=3)
    elif name == "n3mixed":
        dims, K = (500, 400, 300), (7, 20, 12)
        idx, vals = synth.coo_uniform(dims, 30_000, seed=4)
    elif name == "n4":
        dims, K = (40, 30, 20, 10), (3, 4, 2, 3)
        idx, vals = synth.coo_uniform(dims, 5000, seed=5)
    elif name == "n4k10":
        dims, K = (4000, 4000, 100, 20), (10, 10, 10, 10)
        idx, vals = synth.coo_zipf(dims, 100_000, alpha=1.1, seed=6, values="uniform")
    elif name == "n2":
        dims, K = (3000, 2000), (8, 8)
        idx, vals = synth.coo_uniform(dims, 40_000, seed=7)
    elif name == "k1":
        dims, K = (50, 60, 70), (1, 1, 1)
        idx, vals = synth.coo_uniform(dims, 2000, seed=8)
    else:
        raise KeyError(name)
    vals32 = vals.astype(np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 100))]
    return dims, K, idx, vals32, U


CASES = ["c1", "n4", "n2", "k1", "n3mixed", "zipf3", "n3k32", "n4k10"]


def dev_plan(dims, K, idx, vals32):
    return H.hoqri_plan_create(torch.from_numpy(np.ascontiguousarray(idx)).to(DEV),
                               torch.from_numpy(np.ascontiguousarray(vals32)).to(DEV), dims, K)


def dev_list(Us):
    return [torch.from_numpy(np.ascontiguousarray(u)).to(DEV) for u in Us]


@pytest.mark.parametrize("name", CASES)
def test_core_and_ttmctc_match_oracle(name):
    print(f"[parity] case={name}", flush=True)
    dims, K, idx, vals32, U = make_case(name)
    v64 = vals32.astype(np.float64)
    U64 = [u.astype(np.float64) for u in U]
    plan = dev_plan(dims, K, idx, vals32)
    nnz, nx2, R = H.hoqri_plan_info(plan)
    ci, cv = O.coalesce(idx, v64, dims)
    assert nnz == cv.size
    assert nx2 == pytest.approx(O.norm_x2(cv), rel=1e-12)
    for n in range(len(dims)):
        assert R[n] == np.unique(idx[n]).size
    Ud = dev_list(U)
    f = torch.zeros(1, dtype=torch.float64, device=DEV)
    G = H.hoqri_core(plan, Ud, f=f)
    Gref = O.core_segment(ci, cv, U64)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy()
    assert rel_fro(Gh, Gref) < TOL
    assert f.item() == pytest.approx(float(np.sum(Gref ** 2)), rel=2 * TOL)
    # elementwise: every core entry is a sum over all nonzeros of N-factor products
    N = len(dims)
    U64abs = [np.abs(u) for u in U64]
    Gabs = O.core_segment(ci, np.abs(cv), U64abs)
    fp32_bound_check(Gh, Gref, Gabs, cv.size + N + 1, "core")
    # TTMcTC with the same core on both sides (the float32 core)
    G32 = Gref.astype(np.float32)
    Gd = torch.from_numpy(G32).to(DEV)
    for n in range(len(dims)):
        A = H.hoqri_ttmctc(plan, n, Ud, Gd)
        Aref = O.ttmctc_segment(ci, cv, U64, n, G32.astype(np.float64))
        torch.cuda.synchronize()
        Ah = A.cpu().numpy()
        assert rel_fro(Ah, Aref) < TOL, f"mode {n}"
        # elementwise: row i sums L_i nonzeros' Kronecker rows (N roundings per
        # term) and then P = prod_{m != n} K_m products with the core
        Aabs = O.ttmctc_segment(ci, np.abs(cv), U64abs, n, np.abs(G32.astype(np.float64)))
        L = np.bincount(ci[n], minlength=dims[n]).astype(np.float64)
        P = math.prod(K) // K[n]
        fp32_bound_check(Ah, Aref, Aabs, (L + P + N + 1)[:, None], f"ttmctc mode {n}")
        empty = np.setdiff1d(np.arange(dims[n]), idx[n])
        assert np.all(Ah[empty] == 0.0)


def test_duplicates_are_merged():
    dims, K, idx, vals32, U = make_case("c1")
    rng = np.random.default_rng(0)
    pick = rng.choice(idx.shape[1], 500, replace=False)
    idx2 = np.concatenate([idx, idx[:, pick]], axis=1)
    vals2 = np.concatenate([vals32, rng.standard_normal(500).astype(np.float32)])
    perm = rng.permutation(idx2.shape[1])
    idx2, vals2 = idx2[:, perm], vals2[perm]
    plan = dev_plan(dims, K, idx2, vals2)
    nnz, nx2, R = H.hoqri_plan_info(plan)
    ci, cv = O.coalesce(idx2, vals2.astype(np.float64), dims)
    assert nnz == idx.shape[1]
    assert nx2 == pytest.approx(O.norm_x2(cv.astype(np.float32).astype(np.float64)), rel=1e-12)
    Ud = dev_list(U)
    G = H.hoqri_core(plan, Ud)
    Gref = O.core_segment(ci, cv, [u.astype(np.float64) for u in U])
    assert rel_fro(G.cpu().numpy(), Gref) < TOL


def test_bitwise_deterministic():
    dims, K, idx, vals32, U = make_case("zipf3")
    plan = dev_plan(dims, K, idx, vals32)
    Ud = dev_list(U)
    G1 = H.hoqri_core(plan, Ud).clone()
    G2 = H.hoqri_core(plan, Ud).clone()
    A1 = H.hoqri_ttmctc(plan, 0, Ud, G1).clone()
    A2 = H.hoqri_ttmctc(plan, 0, Ud, G1).clone()
    torch.cuda.synchronize()
    assert torch.equal(G1, G2) and torch.equal(A1, A2)


def test_gpu_outputs_satisfy_AU_identity():
    # U^T A = G_(n) G_(n)^T (§5.2), checked on GPU outputs with no oracle
    dims, K, idx, vals32, U = make_case("zipf3")
    plan = dev_plan(dims, K, idx, vals32)
    Ud = dev_list(U)
    G = H.hoqri_core(plan, Ud)
    for n in range(3):
        A = H.hoqri_ttmctc(plan, n, Ud, G).double()
        Gn = O.unfold(G.cpu().double().numpy(), n)
        lhs = (Ud[n].double().T @ A).cpu().numpy()
        assert rel_fro(lhs, Gn @ Gn.T) < 1e-5


@pytest.mark.parametrize("rows,cols,cond", [(1000, 16, 1e2), (257, 5, 1e4), (100_000, 32, 10.0), (64, 1, 1.0)])
def test_orth_matches_householder(rows, cols, cond):
    rng = np.random.default_rng(rows + cols)
    Q0, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    V0, _ = np.linalg.qr(rng.standard_normal((cols, cols)))
    s = np.geomspace(1.0, 1.0 / cond, cols)
    A = ((Q0 * s) @ V0.T * 3.0).astype(np.float32)
    Qref, Rref = O.qr_positive(A.astype(np.float64))
    Ad = torch.from_numpy(A).to(DEV)
    Rd = torch.zeros((cols, cols), dtype=torch.float64, device=DEV)
    Ud, st = H.hoqri_orth(Ad, R=Rd)
    torch.cuda.synchronize()
    assert st.item() == 0
    Uh = Ud.cpu().numpy().astype(np.float64)
    assert np.abs(Uh.T @ Uh - np.eye(cols)).max() < 2e-6
    # the positive-diagonal QR factor is unique: compare elementwise (scaled by conditioning)
    assert np.abs(Uh - Qref).max() < 1e-6 * cond + 1e-6
    assert rel_fro(Rd.cpu().numpy(), Rref) < 1e-6


@pytest.mark.parametrize("rows,cols,cond", [(1_000_000, 32, 1e3), (1_000_000, 32, 1e5), (200_000, 16, 3e5)])
def test_orth_ill_conditioned_tall(rows, cols, cond):
    # CholeskyQR2 with the second Gram taken from Q1 = A R1^-1 itself: orthonormality
    # at the float32 rounding of U while kappa(A)^2 u64 < 1 (here up to 1e-5), and the
    # positive-diagonal factor equal to Householder's up to that rounding plus the
    # forward error kappa u64. Forming the second Gram from the first (R1^-T W1 R1^-1)
    # loses kappa^2 u64 of orthonormality: 1e-6 at kappa 1e5, 1e-5 at 3e5.
    print(f"[orth] rows={rows} cols={cols} cond={cond:g}", flush=True)
    rng = np.random.default_rng(int(cond) + cols)
    Q0, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    V0, _ = np.linalg.qr(rng.standard_normal((cols, cols)))
    s = np.geomspace(1.0, 1.0 / cond, cols)
    A = ((Q0 * s) @ V0.T * 3.0).astype(np.float32)
    Qref, Rref = O.qr_positive(A.astype(np.float64))
    Ad = torch.from_numpy(A).to(DEV)
    Rd = torch.zeros((cols, cols), dtype=torch.float64, device=DEV)
    Ud, st = H.hoqri_orth(Ad, R=Rd)
    torch.cuda.synchronize()
    assert st.item() == 0
    Uh = Ud.cpu().numpy().astype(np.float64)
    assert np.abs(Uh.T @ Uh - np.eye(cols)).max() < 5e-7
    assert np.abs(Uh - Qref).max() < 2e-7 + 1e-13 * cond
    assert rel_fro(Rd.cpu().numpy(), Rref) < 1e-8


def test_orth_in_place_and_breakdown():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((500, 6)).astype(np.float32)
    A[:, 4] = A[:, 0] - 2 * A[:, 1]
    Ad = torch.from_numpy(A).to(DEV)
    U, st = H.hoqri_orth(Ad, U=Ad)
    torch.cuda.synchronize()
    assert st.item() == -4
    assert torch.equal(Ad.cpu(), torch.from_numpy(A))   # untouched on breakdown
    B = rng.standard_normal((500, 6)).astype(np.float32)
    Bd = torch.from_numpy(B).to(DEV)
    U, st = H.hoqri_orth(Bd, U=Bd)                      # aliasing allowed
    Qref, _ = O.qr_positive(B.astype(np.float64))
    torch.cuda.synchronize()
    assert st.item() == 0 and np.abs(Bd.cpu().numpy() - Qref).max() < 1e-6


def test_index_out_of_range_is_reported():
    dims, K = (10, 10, 10), (2, 2, 2)
    idx = np.array([[0, 1, 10], [0, 1, 2], [3, 4, 5]], dtype=np.int32)
    vals = np.ones(3, dtype=np.float32)
    with pytest.raises(H.HoqriError) as e:
        dev_plan(dims, K, idx, vals)
    assert e.value.status == -2


def test_single_nonzero_and_tiny():
    dims, K = (5, 6, 7), (1, 1, 1)
    idx = np.array([[3], [1], [4]], dtype=np.int32)
    vals = np.array([-1.5], dtype=np.float32)
    U = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 3))]
    plan = dev_plan(dims, K, idx, vals)
    Ud = dev_list(U)
    G = H.hoqri_core(plan, Ud)
    ref = -1.5 * U[0][3, 0] * U[1][1, 0] * U[2][4, 0]
    assert G.item() == pytest.approx(ref, rel=1e-6)
    for n in range(3):
        A = H.hoqri_ttmctc(plan, n, Ud, G).cpu().numpy()
        i = (3, 1, 4)[n]
        s = 1.5 ** 2 * math.prod(float(U[m][(3, 1, 4)[m], 0]) ** 2 for m in range(3) if m != n)
        expect = np.zeros((dims[n], 1))
        expect[i, 0] = s * U[n][i, 0]
        assert np.abs(A - expect).max() <= 1e-6 * abs(expect).max()
