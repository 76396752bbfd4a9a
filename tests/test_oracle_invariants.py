"""Pins of the oracle's HOQRI loop against the paper's analysis (§5) and against
special cases with textbook answers (planted Tucker, N=2 SVD, K=1 power method)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2510_16930_amd import synth


def _run_record(dims, K, nnz, seed, sweeps):
    idx, vals = synth.coo_uniform(dims, nnz, seed=seed)
    U0 = O.orthonormal_start(synth.gaussian_start(dims, K, seed + 1000))
    # replay the loop by hand to get every (U before, A, G) triple
    idx, vals = O.coalesce(idx, vals, dims)
    U = [u.copy() for u in U0]
    steps = []
    for t in range(sweeps):
        for n in range(len(dims)):
            G = O.core_segment(idx, vals, U)
            A = O.ttmctc_segment(idx, vals, U, n, G)
            Unew = O.qr_positive(A)[0]
            steps.append((n, [u.copy() for u in U], A, G))
            U[n] = Unew
    return idx, vals, U0, steps


def test_AU_identity_and_trace():
    # eq. in §5.2: A^T U = U^T A = G_(n) G_(n)^T, so tr(A^T U) = ||G||^2
    idx, vals, U0, steps = _run_record((30, 40, 50), (3, 4, 2), 400, seed=3, sweeps=1)
    for n, U, A, G in steps:
        Gn = O.unfold(G, n)
        np.testing.assert_allclose(U[n].T @ A, Gn @ Gn.T, atol=1e-12)
        np.testing.assert_allclose(A.T @ U[n], Gn @ Gn.T, atol=1e-12)
        assert np.trace(U[n].T @ A) == pytest.approx(np.sum(G * G), rel=1e-12)


def test_core_norm_bounded_by_data_norm():
    # G = X x {U^T} is an orthogonal projection of X, so ||G|| <= ||X||
    idx, vals, U0, steps = _run_record((20, 25, 30), (4, 4, 4), 300, seed=4, sweeps=2)
    nx2 = O.norm_x2(vals)
    for _, _, _, G in steps:
        assert np.sum(G * G) <= nx2 * (1 + 1e-14)


def test_theorem1_monotone_and_per_step_bounds():
    # Theorem 1: f non-decreasing per mode step. Proof of Theorem 2:
    # f_{t+1} >= ||A||_* >= f_t, and ||grad||^2 <= 4 f_sup (f_{t+1} - f_t) with f_sup <= ||X||^2.
    idx, vals, U0, steps = _run_record((40, 50, 30), (4, 3, 5), 900, seed=5, sweeps=4)
    nx2 = O.norm_x2(vals)
    fs = [float(np.sum(G * G)) for _, _, _, G in steps]
    for j, (n, U, A, G) in enumerate(steps):
        f_t = fs[j]
        Unext = [u.copy() for u in U]
        Unext[n] = O.qr_positive(A)[0]
        f_next = float(np.sum(O.core_segment(idx, vals, Unext) ** 2))
        nuc = float(np.linalg.svd(A, compute_uv=False).sum())
        assert f_next >= nuc * (1 - 1e-12)
        assert nuc >= f_t * (1 - 1e-12)
        g2 = O.grad_norm2_mode(A, G, n)
        assert g2 == pytest.approx(O.grad_norm2_direct(A, U[n], G, n), rel=1e-9, abs=1e-12 * nx2 ** 2)
        assert g2 <= 4 * nx2 * (f_next - f_t) * (1 + 1e-9) + 1e-12 * nx2 ** 2
        if j + 1 < len(fs):
            assert fs[j + 1] >= f_t * (1 - 1e-13)


def test_lemma1_interlacing():
    # Appendix lemma: sigma_k(A^(n)) >= lambda_k(G_(n) G_(n)^T)
    idx, vals, U0, steps = _run_record((25, 35, 45), (3, 3, 3), 500, seed=6, sweeps=2)
    for n, U, A, G in steps:
        s = np.linalg.svd(A, compute_uv=False)
        Gn = O.unfold(G, n)
        lam = np.sort(np.linalg.eigvalsh(Gn @ Gn.T))[::-1]
        assert np.all(s >= lam * (1 - 1e-11) - 1e-14)


def test_hoqri_driver_matches_hand_replay():
    dims, K = (30, 40, 50), (3, 4, 2)
    idx, vals = synth.coo_uniform(dims, 400, seed=3)
    U0 = O.orthonormal_start(synth.gaussian_start(dims, K, 1003))
    _, _, _, steps = _run_record(dims, K, 400, seed=3, sweeps=2)
    U, G, h = O.hoqri(idx, vals, dims, K, U0, sweeps=2, record_A=True)
    assert len(h["A"]) == len(steps)
    for A, (_, _, Ar, _) in zip(h["A"], steps):
        np.testing.assert_allclose(A, Ar, atol=1e-13)
    # element-wise and slice forms of the loop agree
    U2, G2, h2 = O.hoqri(idx, vals, dims, K, U0, sweeps=2, impl="elementwise")
    np.testing.assert_allclose(h["f_step"], h2["f_step"], rtol=1e-12)
    for a, b in zip(U, U2):
        np.testing.assert_allclose(a, b, atol=1e-11)


def _planted(dims, K, support, seed):
    """Noiseless Tucker tensor G0 x {U0} supported on a dense block of rows."""
    rng = np.random.default_rng(seed)
    U0 = []
    rows = []
    for d, k, s in zip(dims, K, support):
        r = np.sort(rng.choice(d, size=s, replace=False))
        M = np.zeros((d, k))
        M[r] = rng.standard_normal((s, k))
        U0.append(np.linalg.qr(M)[0])
        rows.append(r)
    G0 = rng.standard_normal(K)
    block = O.tucker_dense(G0, [u[r] for u, r in zip(U0, rows)])
    grids = np.meshgrid(*rows, indexing="ij")
    idx = np.stack([g.ravel() for g in grids]).astype(np.int32)
    return idx, block.ravel(), U0, G0


def test_planted_tucker_recovered_in_one_sweep():
    dims, K = (40, 50, 60), (3, 4, 2)
    idx, vals, U0true, G0 = _planted(dims, K, (9, 11, 9), seed=12)
    start = O.orthonormal_start(synth.gaussian_start(dims, K, 77))
    U, G, h = O.hoqri(idx, vals, dims, K, start, sweeps=1)
    for u, ut in zip(U, U0true):
        assert O.subspace_dist(u, ut) < 1e-12
    nx2 = h["normx2"]
    assert (nx2 - h["f_sweep"][0]) / nx2 < 1e-12


def test_matrix_case_converges_to_top_singular_subspaces():
    # N = 2: HOQRI is orthogonal iteration (§4.3) -> top-K singular subspaces,
    # f* = sum of the K largest sigma^2 (Eckart-Young)
    rng = np.random.default_rng(13)
    I1, I2, K = 60, 50, 3
    Ul = np.linalg.qr(rng.standard_normal((I1, I1)))[0]
    Vr = np.linalg.qr(rng.standard_normal((I2, I2)))[0]
    s = np.concatenate([[10.0, 8.0, 6.0], 1.0 / (1 + np.arange(I2 - 3))])
    M = (Ul[:, :I2] * s) @ Vr.T
    idx = np.stack(np.unravel_index(np.arange(I1 * I2), (I1, I2))).astype(np.int32)
    start = O.orthonormal_start(synth.gaussian_start((I1, I2), (K, K), 3))
    U, G, h = O.hoqri(idx, M.ravel(), (I1, I2), (K, K), start, sweeps=40)
    sv = np.linalg.svd(M, compute_uv=False)
    assert h["f_sweep"][-1] == pytest.approx(np.sum(sv[:K] ** 2), rel=1e-12)
    Ls, _, Rs = np.linalg.svd(M)
    assert O.subspace_dist(U[0], Ls[:, :K]) < 1e-10
    assert O.subspace_dist(U[1], Rs[:K].T) < 1e-10


def test_rank_one_case_is_higher_order_power_method():
    # K = (1,..,1): the QR of the single column A = y g gives u = sign(g) y / ||y||
    dims = (8, 9, 10)
    idx, vals = synth.coo_uniform(dims, 200, seed=14)
    start = O.orthonormal_start(synth.gaussian_start(dims, (1, 1, 1), 5))
    U, G, h = O.hoqri(idx, vals, dims, (1, 1, 1), start, sweeps=3)
    X = O.to_dense(idx, vals, dims)
    u = [s[:, 0].copy() for s in start]
    for t in range(3):
        for n in range(3):
            others = [m for m in range(3) if m != n]
            y = X
            for m in sorted(others, reverse=True):
                y = np.tensordot(y, u[m], axes=([m], [0]))
            g = float(y @ u[n])
            u[n] = math.copysign(1.0, g) * y / np.linalg.norm(y)
    for a, b in zip(U, u):
        np.testing.assert_allclose(a[:, 0], b, atol=1e-12)


def test_rank_deficient_update_raises():
    # fewer nonempty mode-0 slices than K_0 -> A^(0) has rank < K_0
    idx = np.array([[0, 0, 1, 1], [0, 1, 2, 3], [0, 1, 0, 1]], dtype=np.int32)
    vals = np.array([1.0, 2.0, 3.0, 4.0])
    dims, K = (5, 4, 2), (3, 2, 2)
    start = O.orthonormal_start(synth.gaussian_start(dims, K, 1))
    with pytest.raises(O.RankDeficient):
        O.hoqri(idx, vals, dims, K, start, sweeps=1)


def test_stopping_rules():
    dims, K = (30, 30, 30), (2, 2, 2)
    idx, vals = synth.coo_uniform(dims, 300, seed=15)
    start = O.orthonormal_start(synth.gaussian_start(dims, K, 9))
    _, _, h = O.hoqri(idx, vals, dims, K, start, sweeps=200, tol=1e-6, stop="rel_f")
    f = h["f_sweep"]
    assert len(f) < 200 and abs(f[-1] - f[-2]) <= 1e-6 * f[-1]


def test_error_change_stop_rule_replayed_by_hand():
    # §6.1 stops when the change of the relative approximation error
    # eps_t = ||X - G x {U}||_F / ||X||_F = sqrt((||X||^2 - f_t) / ||X||^2)
    # between consecutive iterations is below tol. Replay it from an unstopped
    # run: the stopped run must end at the first sweep t with
    # |eps_t - eps_{t-1}| < tol (eps_0 from the starting factors), and the
    # fixture is chosen so that comparing squared errors, or not advancing
    # eps_{t-1}, would stop elsewhere.
    dims, K = (30, 30, 30), (2, 2, 2)
    idx, vals = synth.coo_uniform(dims, 300, seed=15)
    start = O.orthonormal_start(synth.gaussian_start(dims, K, 9))
    _, _, full = O.hoqri(idx, vals, dims, K, start, sweeps=40)
    nx2 = float(np.sum(np.asarray(vals, np.float64) ** 2))
    assert full["normx2"] == pytest.approx(nx2, rel=1e-14)
    fs = [full["f_step"][0]] + full["f_sweep"]          # f before sweep 1, after each sweep
    eps = np.sqrt(np.maximum(nx2 - np.array(fs), 0.0) / nx2)
    tol = 9e-6
    d = np.abs(np.diff(eps))                            # d[t-1] = |eps_t - eps_{t-1}|
    k = int(np.argmax(d < tol)) + 1
    assert d[k - 1] < tol and np.all(d[:k - 1] >= tol) and 1 < k < 40
    k_sq = int(np.argmax(np.abs(np.diff(eps ** 2)) < tol)) + 1
    stale = np.abs(eps[1:] - eps[0]) < tol
    assert k_sq != k and not stale.any()                # the plausible mistakes differ
    _, _, h = O.hoqri(idx, vals, dims, K, start, sweeps=40, tol=tol, stop="err")
    assert len(h["f_sweep"]) == k
    np.testing.assert_allclose(h["f_sweep"], full["f_sweep"][:k], rtol=0, atol=0)
    # a tolerance no change reaches runs every sweep
    _, _, h0 = O.hoqri(idx, vals, dims, K, start, sweeps=12, tol=1e-300, stop="err")
    assert len(h0["f_sweep"]) == 12


def test_rank_deficient_mode_is_kept_on_request():
    # X = sum of two rank-one terms on a 6x7x8 support: every mode-0 unfolding has
    # rank 2 < K_0 = 3, so A^(0) = X_(0) (U_1 kron U_2) G_(0)^T is rank deficient at
    # every step while modes 1 and 2 (K = 2) update normally.
    rng = np.random.default_rng(21)
    dims, K = (6, 7, 8), (3, 2, 2)
    X = sum(np.einsum("i,j,k->ijk", rng.standard_normal(6), rng.standard_normal(7), rng.standard_normal(8))
            for _ in range(2))
    idx = np.stack(np.unravel_index(np.arange(X.size), dims)).astype(np.int32)
    vals = X.ravel()
    U0 = O.orthonormal_start(synth.gaussian_start(dims, K, 4))
    with pytest.raises(O.RankDeficient):
        O.hoqri(idx, vals, dims, K, U0, sweeps=2)
    U, G, h = O.hoqri(idx, vals, dims, K, U0, sweeps=3, on_breakdown="keep")
    assert h["skipped"] == 3                      # mode 0 in each of the 3 sweeps
    np.testing.assert_array_equal(U[0], U0[0])    # kept exactly
    assert not np.array_equal(U[1], U0[1])        # the other modes moved
    f = h["f_step"] + [h["f_sweep"][-1]]
    assert all(b >= a - 1e-12 * abs(b) for a, b in zip(f, f[1:]))  # Theorem 1 still holds


def test_sketch_start_recovers_planted_subspaces_and_hosvd():
    # exact multilinear rank K: the range finder spans the column space of every
    # unfolding, which is span(U0_n) (probability one over the Gaussian draws)
    rng = np.random.default_rng(31)
    dims, K = (30, 25, 20), (3, 4, 2)
    U0 = [np.linalg.qr(rng.standard_normal((d, k)))[0] for d, k in zip(dims, K)]
    X = O.tucker_dense(rng.standard_normal(K), U0)
    idx = np.stack(np.unravel_index(np.arange(X.size), dims)).astype(np.int32)
    Om = [rng.standard_normal((d, k)) for d, k in zip(dims, K)]
    Ga = rng.standard_normal(K)
    U = O.sketch_start(idx, X.ravel(), dims, K, Om, Ga)
    for n in range(3):
        assert O.subspace_dist(U[n], U0[n]) < 1e-12
        np.testing.assert_allclose(U[n].T @ U[n], np.eye(K[n]), atol=1e-12)
    # against the dense definition: the sketch of X_(n) is X_(n) (kron Omega) Gamma_(n)^T
    n = 1
    S = O.unfold(X, n) @ O.kron_except(Om, n) @ O.unfold(Ga, n).T
    np.testing.assert_allclose(U[n], O.qr_positive(S)[0], atol=1e-12)


# --------------------------------------------------------------------------
# HOOI (Alg. 1)
# --------------------------------------------------------------------------

def _dense_Y(idx, vals, dims, Us, n):
    """Y_(n) = unfold(X x_{m != n} U^(m)T, n) from the dense tensor (mode products)."""
    X = O.to_dense(idx, vals, dims)
    for m in range(len(dims)):
        if m != n:
            X = O.mode_product(X, Us[m].T, m)
    return O.unfold(X, n)


def test_hooi_update_is_the_dense_eigen_solution_and_dominates():
    # the update maximises ||U^T Y_(n)||^2: its value equals the sum of the K
    # largest eigenvalues of Y Y^T from the dense tensor, its subspace is their
    # eigenvectors', and no other orthonormal U (HOQRI's step, random ones) does better
    dims, K = (12, 9, 10), (3, 2, 4)
    idx, vals = synth.coo_uniform(dims, 300, seed=41)
    U = O.orthonormal_start(synth.gaussian_start(dims, K, 42))
    ci, cv = O.coalesce(idx, vals, dims)
    rng = np.random.default_rng(43)
    for n in range(3):
        Un, s = O.leading_left(ci, cv, U, n, K[n])
        Y = _dense_Y(ci, cv, dims, U, n)
        w, V = np.linalg.eigh(Y @ Y.T)
        assert np.sum(s ** 2) == pytest.approx(np.sum(w[-K[n]:]), rel=1e-12)
        assert O.subspace_dist(Un, V[:, -K[n]:]) < 1e-10
        assert np.allclose(Un.T @ Un, np.eye(K[n]), atol=1e-12)
        f_hooi = np.sum((Un.T @ Y) ** 2)
        G = O.core_segment(ci, cv, U)
        Uq = O.qr_positive(O.ttmctc_segment(ci, cv, U, n, G))[0]
        assert np.sum((Uq.T @ Y) ** 2) <= f_hooi * (1 + 1e-12)
        for _ in range(5):
            Ur = np.linalg.qr(rng.standard_normal((dims[n], K[n])))[0]
            assert np.sum((Ur.T @ Y) ** 2) <= f_hooi * (1 + 1e-12)


def test_hooi_planted_tucker_recovered_in_one_sweep_and_monotone():
    dims, K = (40, 50, 60), (3, 4, 2)
    idx, vals, U0true, G0 = _planted(dims, K, (9, 11, 9), seed=12)
    start = O.orthonormal_start(synth.gaussian_start(dims, K, 77))
    U, G, h = O.hooi(idx, vals, dims, K, start, sweeps=1)
    for u, ut in zip(U, U0true):
        assert O.subspace_dist(u, ut) < 1e-12
    assert (h["normx2"] - h["f_sweep"][0]) / h["normx2"] < 1e-12
    # f never decreases along the mode updates on a generic tensor
    dims2, K2 = (30, 25, 20), (4, 3, 5)
    idx2, vals2 = synth.coo_uniform(dims2, 2000, seed=44)
    st2 = O.orthonormal_start(synth.gaussian_start(dims2, K2, 45))
    _, _, h2 = O.hooi(idx2, vals2, dims2, K2, st2, sweeps=4)
    f = np.array(h2["f_step"])
    assert np.all(np.diff(f) >= -1e-12 * f[:-1])


def test_hooi_matrix_case_is_the_truncated_svd():
    # N = 2: alternating leading subspaces converge to the top-K singular pair
    # subspaces, f* = sum of the K largest sigma^2 (Eckart-Young)
    rng = np.random.default_rng(13)
    I1, I2, K = 60, 50, 3
    Ul = np.linalg.qr(rng.standard_normal((I1, I1)))[0]
    Vr = np.linalg.qr(rng.standard_normal((I2, I2)))[0]
    s = np.concatenate([[10.0, 8.0, 6.0], 1.0 / (1 + np.arange(I2 - 3))])
    M = (Ul[:, :I2] * s) @ Vr.T
    idx = np.stack(np.unravel_index(np.arange(I1 * I2), (I1, I2))).astype(np.int32)
    start = O.orthonormal_start(synth.gaussian_start((I1, I2), (K, K), 3))
    U, G, h = O.hooi(idx, M.ravel(), (I1, I2), (K, K), start, sweeps=20)
    sv = np.linalg.svd(M, compute_uv=False)
    assert h["f_sweep"][-1] == pytest.approx(np.sum(sv[:K] ** 2), rel=1e-12)
    Ls, _, Rs = np.linalg.svd(M)
    assert O.subspace_dist(U[0], Ls[:, :K]) < 1e-10
    assert O.subspace_dist(U[1], Rs[:K].T) < 1e-10
