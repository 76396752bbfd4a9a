"""GPU parity of the whole HOQRI loop (hoqri_run) against the FP64 oracle."""
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


def run_both(dims, K, idx, vals32, U0_32, sweeps, tol=0.0):
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Us = [dev(u) for u in U0_32]
    fh = torch.zeros(sweeps * len(dims), dtype=torch.float64, device=DEV)
    G, st = H.hoqri_run(plan, Us, max_sweeps=sweeps, tol=tol, f_hist=fh)
    torch.cuda.synchronize()
    Uo, Go, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in U0_32],
                        sweeps=sweeps, tol=(tol if tol > 0 else None))
    return [u.cpu().numpy().astype(np.float64) for u in Us], G.cpu().numpy(), st, fh.cpu().numpy(), Uo, Go, h


def test_c1_trajectory_matches_oracle():
    # 200^3, 20k uniform nonzeros, N(0,1) values, ranks (5,5,5), 10 sweeps
    print("[run] c1 10 sweeps", flush=True)
    dims, K = (200, 200, 200), (5, 5, 5)
    idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    U0 = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 111))]
    U, G, st, fh, Uo, Go, h = run_both(dims, K, idx, vals.astype(np.float32), U0, 10)
    assert st.sweeps == 10
    # f before every mode update, for all 30 mode steps
    np.testing.assert_allclose(fh, h["f_step"], rtol=1e-5)
    assert st.f == pytest.approx(h["f_sweep"][-1], rel=1e-5)
    assert st.fit == pytest.approx(h["fit"][-1], rel=1e-4)
    for n in range(3):
        # canonical QR (positive diagonal): the factors are comparable elementwise
        assert np.abs(U[n] - Uo[n]).max() < 1e-4
        # d is a squared Frobenius distance: 1000 entries within 1e-4 give at most 1e-5;
        # float32 drift over 30 mode steps is observed at ~1e-7
        assert O.subspace_dist(U[n], Uo[n]) < 1e-6
    assert np.linalg.norm(G - Go) / np.linalg.norm(Go) < 1e-5
    assert st.orth_err_max < 1e-5
    # Theorem 1 on the GPU trajectory (float32 slack)
    assert np.all(np.diff(fh) >= -1e-6 * fh[1:])


def test_planted_tucker_recovered():
    rng = np.random.default_rng(12)
    dims, K, support = (400, 500, 600), (3, 4, 2), (9, 11, 9)
    U0t, rows = [], []
    for d, k, s in zip(dims, K, support):
        r = np.sort(rng.choice(d, size=s, replace=False))
        M = np.zeros((d, k))
        M[r] = rng.standard_normal((s, k))
        U0t.append(np.linalg.qr(M)[0])
        rows.append(r)
    G0 = rng.standard_normal(K)
    block = O.tucker_dense(G0, [u[r] for u, r in zip(U0t, rows)])
    grids = np.meshgrid(*rows, indexing="ij")
    idx = np.stack([g.ravel() for g in grids]).astype(np.int32)
    vals32 = block.ravel().astype(np.float32)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 77))]
    U, G, st, fh, Uo, Go, h = run_both(dims, K, idx, vals32, start, 2)
    # exact in exact arithmetic; with float32 sums the subspace moves by ~kappa(A) u32 per
    # update (kappa(A) <= 67 here). A float32 emulation of the same sums in numpy reaches
    # d = 4.5e-8 .. 1.0e-7, so 1e-7 is the float32 bar.
    for n in range(3):
        assert O.subspace_dist(U[n], U0t[n]) < 1e-7
    # squared relative residual (fit loses half the digits near 1)
    assert (st.norm_x2 - st.f) / st.norm_x2 < 1e-5


def test_matrix_case_top_singular_subspace():
    rng = np.random.default_rng(13)
    I1, I2, K = 300, 200, 4
    Ul = np.linalg.qr(rng.standard_normal((I1, I2)))[0]
    Vr = np.linalg.qr(rng.standard_normal((I2, I2)))[0]
    s = np.concatenate([[10.0, 8.0, 6.0, 5.0], 1.0 / (1 + np.arange(I2 - 4))])
    M = (Ul * s) @ Vr.T
    idx = np.stack(np.unravel_index(np.arange(I1 * I2), (I1, I2))).astype(np.int32)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start((I1, I2), (K, K), 3))]
    U, G, st, fh, Uo, Go, h = run_both((I1, I2), (K, K), idx, M.ravel().astype(np.float32), start, 30)
    M32 = M.astype(np.float32).astype(np.float64)
    sv = np.linalg.svd(M32, compute_uv=False)
    assert st.f == pytest.approx(np.sum(sv[:K] ** 2), rel=1e-5)
    Ls, _, Rs = np.linalg.svd(M32)
    assert O.subspace_dist(U[0], Ls[:, :K]) < 1e-7
    assert O.subspace_dist(U[1], Rs[:K].T) < 1e-7


def test_rank_one_and_stopping_rule():
    # K = (1,1,1) with the stop rule |f_t - f_{t-1}| <= tol f_t. Near the threshold
    # float32 and float64 f may decide differently, so the unique facts are checked:
    # the GPU stops at the first sweep where its own f sequence meets the rule, the
    # oracle's stop is within one sweep, and the GPU state equals the oracle's after
    # the same number of sweeps.
    dims, K = (50, 60, 70), (1, 1, 1)
    idx, vals = synth.coo_uniform(dims, 2000, seed=14)
    tol = 1e-6
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 5))]
    U, G, st, fh, Uo, Go, h = run_both(dims, K, idx, vals.astype(np.float32), start, 200, tol=tol)
    T = st.sweeps
    F = [fh[t * 3] for t in range(T)] + [st.f]          # f before sweep 1, after sweep 1, ..., after T
    for t in range(1, T):
        assert abs(F[t] - F[t - 1]) > tol * F[t]
    assert abs(F[T] - F[T - 1]) <= tol * F[T]
    assert abs(T - len(h["f_sweep"])) <= 1
    Uo2, Go2, h2 = O.hoqri(idx, vals.astype(np.float32).astype(np.float64), dims, K,
                           [u.astype(np.float64) for u in start], sweeps=T)
    assert st.f == pytest.approx(h2["f_sweep"][-1], rel=1e-5)
    for n in range(3):
        assert np.abs(U[n] - Uo2[n]).max() < 1e-4


def test_order4_run():
    dims, K = (60, 50, 40, 30), (3, 4, 2, 3)
    idx, vals = synth.coo_uniform(dims, 20000, seed=15)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 6))]
    U, G, st, fh, Uo, Go, h = run_both(dims, K, idx, vals.astype(np.float32), start, 4)
    np.testing.assert_allclose(fh, h["f_step"], rtol=1e-5)
    for n in range(4):
        assert np.abs(U[n] - Uo[n]).max() < 1e-4


def test_rank_deficient_update_raises():
    # fewer nonempty mode-0 slices than K_0
    dims, K = (50, 40, 30), (4, 3, 3)
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, 2, 400), rng.integers(0, 40, 400), rng.integers(0, 30, 400)]).astype(np.int32)
    vals = rng.standard_normal(400).astype(np.float32)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 1))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals), dims, K)
    with pytest.raises(H.HoqriError) as e:
        H.hoqri_run(plan, [dev(u) for u in start], max_sweeps=2)
    assert e.value.status == -4


def test_orthonormalize_input_from_raw_gaussian():
    dims, K = (200, 200, 200), (5, 5, 5)
    idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    raw = synth.gaussian_start(dims, K, 111)
    plan = H.hoqri_plan_create(dev(idx), dev(vals.astype(np.float32)), dims, K)
    Us = [dev(r.astype(np.float32)) for r in raw]
    G, st = H.hoqri_run(plan, Us, max_sweeps=3, orthonormalize_input=True)
    U0 = O.orthonormal_start([r.astype(np.float32).astype(np.float64) for r in raw])
    Uo, Go, h = O.hoqri(idx, vals.astype(np.float32).astype(np.float64), dims, K, U0, sweeps=3)
    assert st.f == pytest.approx(h["f_sweep"][-1], rel=1e-5)


def test_rank_deficient_mode_kept_like_oracle():
    # sum of two rank-one terms on a 20x25x30 block inside 60x70x80: the mode-0
    # unfolding has rank 2 < K_0 = 3, so every mode-0 update is rank deficient
    rng = np.random.default_rng(22)
    dims, K = (60, 70, 80), (3, 2, 2)
    rows = [np.sort(rng.choice(d, size=s, replace=False)) for d, s in zip(dims, (20, 25, 30))]
    block = sum(np.einsum("i,j,k->ijk", rng.standard_normal(20), rng.standard_normal(25), rng.standard_normal(30))
                for _ in range(2))
    grids = np.meshgrid(*rows, indexing="ij")
    idx = np.stack([g.ravel() for g in grids]).astype(np.int32)
    vals32 = block.ravel().astype(np.float32)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 9))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    with pytest.raises(H.HoqriError) as e:
        H.hoqri_run(plan, [dev(u) for u in start], max_sweeps=2)
    assert e.value.status == -4
    Us = [dev(u) for u in start]
    G, st = H.hoqri_run(plan, Us, max_sweeps=3, keep_on_breakdown=True)
    Uo, Go, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in start], sweeps=3,
                        on_breakdown="keep")
    assert st.skipped_updates == h["skipped"] == 3
    assert torch.equal(Us[0].cpu(), torch.from_numpy(start[0]))
    for n in (1, 2):
        assert np.abs(Us[n].cpu().numpy() - Uo[n]).max() < 1e-4
    assert st.f == pytest.approx(h["f_sweep"][-1], rel=1e-5)


def test_riemannian_gradient_monitor():
    # ||grad_n||^2 = ||2 (A^(n) - U^(n) G_(n) G_(n)^T)||^2 at every mode step (§5.2), before
    # U^(n) moves; the oracle evaluates the equivalent 4 (||A||^2 - ||G_(n) G_(n)^T||^2) in float64
    dims, K = (200, 200, 200), (5, 5, 5)
    idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    U0 = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 111))]
    plan = H.hoqri_plan_create(dev(idx), dev(vals.astype(np.float32)), dims, K)
    Us = [dev(u) for u in U0]
    gh = torch.zeros(6 * 3, dtype=torch.float64, device=DEV)
    G, st = H.hoqri_run(plan, Us, max_sweeps=6, grad_hist=gh)
    Uo, Go, h = O.hoqri(idx, vals.astype(np.float32).astype(np.float64), dims, K, [u.astype(np.float64) for u in U0],
                        sweeps=6, record_A=True)
    ref = np.array([O.grad_norm2_mode(A, Gs, i % 3) for i, (A, Gs) in enumerate(zip(h["A"], h["G_step"]))])
    got = gh.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-4)
    assert st.grad_norm2 == pytest.approx(float(ref[-3:].sum()), rel=1e-4)
    # stop rule on the gradient: the run ends at the first sweep whose gradient is small enough
    r = [float(np.sqrt(ref[3 * t:3 * t + 3].sum()) / h["f_sweep"][t]) for t in range(6)]
    assert r[0] > r[1] > r[2]
    tol = float(np.sqrt(r[1] * r[2]))  # met after sweep 3, not before
    Us = [dev(u) for u in U0]
    G, st2 = H.hoqri_run(plan, Us, max_sweeps=20, grad_tol=tol)
    assert st2.sweeps == 3
    # off by default
    Us = [dev(u) for u in U0]
    G, st3 = H.hoqri_run(plan, Us, max_sweeps=2)
    assert st3.grad_norm2 == -1.0


def test_sketch_start_matches_oracle_and_recovers_planted():
    # c1 shape: GPU range-finder start against the oracle's (same random draws)
    dims, K = (200, 200, 200), (5, 5, 5)
    idx, vals = synth.coo_uniform(dims, 20000, seed=11)
    rng = np.random.default_rng(41)
    Om = [rng.standard_normal((d, k)).astype(np.float32) for d, k in zip(dims, K)]
    Ga = rng.standard_normal(K).astype(np.float32)
    plan = H.hoqri_plan_create(dev(idx), dev(vals.astype(np.float32)), dims, K)
    U = [u.cpu().numpy().astype(np.float64) for u in H.hoqri_sketch_start(plan, [dev(o) for o in Om], dev(Ga))]
    Uo = O.sketch_start(idx, vals.astype(np.float32).astype(np.float64), dims, K,
                        [o.astype(np.float64) for o in Om], Ga.astype(np.float64))
    for n in range(3):
        assert np.abs(U[n] - Uo[n]).max() < 1e-3
        assert O.subspace_dist(U[n], Uo[n]) < 1e-6
        np.testing.assert_allclose(U[n].T @ U[n], np.eye(K[n]), atol=1e-5)
        empty = np.setdiff1d(np.arange(dims[n]), idx[n])
        assert np.all(U[n][empty] == 0.0)
    # planted exact multilinear rank: the start already spans the planted subspaces
    rng = np.random.default_rng(42)
    dims, K, support = (400, 500, 600), (3, 4, 2), (9, 11, 9)
    U0t, rows = [], []
    for d, k, s in zip(dims, K, support):
        r = np.sort(rng.choice(d, size=s, replace=False))
        M = np.zeros((d, k))
        M[r] = rng.standard_normal((s, k))
        U0t.append(np.linalg.qr(M)[0])
        rows.append(r)
    block = O.tucker_dense(rng.standard_normal(K), [u[r] for u, r in zip(U0t, rows)])
    grids = np.meshgrid(*rows, indexing="ij")
    pidx = np.stack([g.ravel() for g in grids]).astype(np.int32)
    plan = H.hoqri_plan_create(dev(pidx), dev(block.ravel().astype(np.float32)), dims, K)
    Om = [dev(rng.standard_normal((d, k)).astype(np.float32)) for d, k in zip(dims, K)]
    U = H.hoqri_sketch_start(plan, Om, dev(rng.standard_normal(K).astype(np.float32)))
    for n in range(3):
        assert O.subspace_dist(U[n].cpu().numpy().astype(np.float64), U0t[n]) < 1e-7


def test_error_change_stop_rule():
    # §6.1's rule: stop when the relative approximation error
    # eps_t = sqrt(max(||X||^2 - f_t, 0) / ||X||^2) changes by less than tol between
    # consecutive sweeps. The GPU must stop at the first sweep where its own f
    # sequence meets the rule, within one sweep of the oracle's stop (float32 and
    # float64 f may decide differently next to the threshold), and its state must
    # equal the oracle's after the same number of sweeps.
    dims, K = (30, 30, 30), (2, 2, 2)
    idx, vals = synth.coo_uniform(dims, 300, seed=15)
    start = [u.astype(np.float32) for u in O.orthonormal_start(synth.gaussian_start(dims, K, 9))]
    vals32 = vals.astype(np.float32)
    tol = 9e-6
    plan = H.hoqri_plan_create(dev(idx), dev(vals32), dims, K)
    Us = [dev(u) for u in start]
    fh = torch.zeros(40 * 3, dtype=torch.float64, device=DEV)
    G, st = H.hoqri_run(plan, Us, max_sweeps=40, tol=tol, f_hist=fh, stop="err")
    torch.cuda.synchronize()
    T = st.sweeps
    fh = fh.cpu().numpy()
    F = np.array([fh[t * 3] for t in range(T)] + [st.f])
    eps = np.sqrt(np.maximum(st.norm_x2 - F, 0.0) / st.norm_x2)
    d = np.abs(np.diff(eps))
    assert 1 < T < 40
    assert np.all(d[:-1] >= tol) and d[-1] < tol
    _, _, h = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in start],
                      sweeps=40, tol=tol, stop="err")
    assert abs(T - len(h["f_sweep"])) <= 1
    Uo, _, h2 = O.hoqri(idx, vals32.astype(np.float64), dims, K, [u.astype(np.float64) for u in start], sweeps=T)
    assert st.f == pytest.approx(h2["f_sweep"][-1], rel=1e-5)
    for n in range(3):
        assert np.abs(Us[n].cpu().numpy() - Uo[n]).max() < 1e-4
    # the relative-change rule with the same threshold stops elsewhere: the rules differ
    Us2 = [dev(u) for u in start]
    _, st2 = H.hoqri_run(plan, Us2, max_sweeps=40, tol=tol, stop="rel_f")
    assert st2.sweeps != T
    with pytest.raises(H.HoqriError):
        _bad_stop(plan, Us2)


def _bad_stop(plan, Us):
    # an unknown stop rule is an argument error, detected before any launch
    import ctypes
    L = H.load()
    opts = H.RunOpts(3, 1e-6, H.PREC["fp32"], 1, 0, 0, None, 0.0, 0, 1, 7)
    st = H.RunStats()
    H._check(L.hoqri_run(plan.handle, H._ptr_array(Us), H._ptr(torch.empty(plan.ranks, device=DEV)), None,
                         ctypes.byref(opts), ctypes.byref(st), H._stream(None)), "hoqri_run")
