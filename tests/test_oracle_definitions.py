"""Pins of the oracle's definitions against independent brute force and closed forms.

Each test checks an oracle function against something other than itself:
explicit loops over the §2.1 definitions, the Kronecker/unfolding form of
TTMc (§2.1), closed forms derived by hand, or library routines.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_2510_16930_amd import synth


def _tiny(dims, K, nnz, seed):
    idx, vals = synth.coo_uniform(dims, nnz, seed=seed)
    U = O.orthonormal_start(synth.gaussian_start(dims, K, seed + 100))
    return idx, vals, U


def test_mode_product_matches_loop_definition():
    # §2.1: [X x_n B](i_1..k..i_N) = sum_{i_n} B(k, i_n) X(i_1..i_N)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 5))
    for n in range(3):
        B = rng.standard_normal((2, X.shape[n]))
        Y = O.mode_product(X, B, n)
        ref = np.zeros(Y.shape)
        for out_idx in itertools.product(*[range(s) for s in Y.shape]):
            k = out_idx[n]
            acc = 0.0
            for i in range(X.shape[n]):
                src = list(out_idx)
                src[n] = i
                acc += B[k, i] * X[tuple(src)]
            ref[out_idx] = acc
        np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-12)


def test_unfolding_turns_mode_product_into_matrix_product():
    # §2.1: [X x_n B]_(n) = B X_(n), which fixes the unfolding to be consistent
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 5, 2))
    for n in range(4):
        B = rng.standard_normal((3, X.shape[n]))
        np.testing.assert_allclose(O.unfold(O.mode_product(X, B, n), n), B @ O.unfold(X, n), atol=1e-12)


def test_kronecker_form_of_ttmc_matches_successive_mode_products():
    # §2.1: [X x_{-n} {B}]_(n) = X_(n) (B^(1) (x) ... skip n ... (x) B^(N))^T
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, 4, 5))
    Bs = [rng.standard_normal((2, s)) for s in X.shape]
    for n in range(3):
        Y = X
        for m in range(3):
            if m != n:
                Y = O.mode_product(Y, Bs[m], m)
        # the chain holds B^(m) of shape K x I; the formula multiplies by its transpose
        kr = O.kron_except([B for B in Bs], n)          # (prod K) x (prod I)
        np.testing.assert_allclose(O.unfold(Y, n), O.unfold(X, n) @ kr.T, atol=1e-12)


def test_kron_except_entry_formula():
    # C-order Kronecker: row index (i_a * I_b + i_b), column (k_a * K_b + k_b)
    rng = np.random.default_rng(3)
    Us = [rng.standard_normal((4, 2)), rng.standard_normal((3, 2)), rng.standard_normal((5, 3))]
    Kr = O.kron_except(Us, 0)
    for ia, ib, ka, kb in itertools.product(range(3), range(5), range(2), range(3)):
        assert Kr[ia * 5 + ib, ka * 3 + kb] == pytest.approx(Us[1][ia, ka] * Us[2][ib, kb])


@pytest.mark.parametrize("dims,K", [((4, 5, 6), (2, 3, 2)), ((3, 4, 5, 6), (2, 2, 3, 2)), ((6, 7), (2, 3)),
                                    ((3, 4, 3, 2, 3), (2, 2, 2, 1, 2))])
def test_three_ttmctc_forms_match_dense_brute_force(dims, K):
    nnz = min(40, math.prod(dims) // 2)
    idx, vals, U = _tiny(dims, K, nnz, seed=7)
    X = O.to_dense(idx, vals, dims)
    Gd = O.core_dense(X, U)
    np.testing.assert_allclose(O.core_elementwise(idx, vals, U), Gd, atol=1e-13)
    for n in range(len(dims)):
        Ad = O.ttmctc_dense(X, U, n)
        np.testing.assert_allclose(O.ttmctc_elementwise(idx, vals, U, n), Ad, atol=1e-13)
        np.testing.assert_allclose(O.ttmctc_matrix(idx, vals, U, n), Ad, atol=1e-13)
        np.testing.assert_allclose(O.ttmctc_segment(idx, vals, U, n, Gd), Ad, atol=1e-13)
        np.testing.assert_allclose(O.core_segment(idx, vals, U, n), Gd, atol=1e-13)


@pytest.mark.parametrize("dims,K", [((5, 4, 6), (2, 3, 2)), ((3, 4, 2, 3), (2, 2, 2, 2))])
def test_sampled_entries_match_dense_brute_force(dims, K):
    # the one-entry core and one-row TTMcTC forms used to sample large outputs
    idx, vals, U = _tiny(dims, K, min(30, math.prod(dims) // 2), seed=17)
    X = O.to_dense(idx, vals, dims)
    Gd = O.core_dense(X, U)
    for ks in itertools.product(*[range(k) for k in K]):
        assert O.core_entry(idx, vals, U, ks) == pytest.approx(Gd[ks], abs=1e-13)
    for n in range(len(dims)):
        Ad = O.ttmctc_dense(X, U, n)
        for i in range(dims[n]):
            for chunk in (1, 1 << 20):
                np.testing.assert_allclose(O.ttmctc_slice_row(idx, vals, U, n, i, Gd, chunk=chunk),
                                           Ad[i], atol=1e-13)


def test_single_nonzero_closed_forms():
    # One nonzero x at i: G = x (x)_m U_m(i_m,:), and
    # A^(n)(i_n,:) = x^2 prod_{m!=n} ||U_m(i_m,:)||^2 U_n(i_n,:); other rows zero.
    dims, K = (5, 6, 7), (2, 3, 2)
    U = O.orthonormal_start(synth.gaussian_start(dims, K, 9))
    i = (3, 1, 4)
    x = -1.7
    idx = np.array(i, dtype=np.int32)[:, None]
    vals = np.array([x])
    G = O.core_elementwise(idx, vals, U)
    ref = x * np.einsum("a,b,c->abc", U[0][i[0]], U[1][i[1]], U[2][i[2]])
    np.testing.assert_allclose(G, ref, atol=1e-15)
    for n in range(3):
        A = O.ttmctc_segment(idx, vals, U, n, G)
        s = x * x * math.prod(float(U[m][i[m]] @ U[m][i[m]]) for m in range(3) if m != n)
        expect = np.zeros_like(A)
        expect[i[n]] = s * U[n][i[n]]
        np.testing.assert_allclose(A, expect, atol=1e-15)


def test_hand_worked_example():
    # 2x2x2 tensor with X(0,0,0)=1 and X(1,1,1)=2, K=(1,1,1),
    # U_m = (1/sqrt2)[1,1]^T for all m. G = (1 + 2)/2^{3/2};
    # A^(1)(0) = 1 * G * (1/2) = 3/8 * sqrt2 ... computed by hand:
    # A^(n)(i) = sum_{e in slice i} x_e G prod_{m!=n} u = x_e * G * 1/2
    idx = np.array([[0, 1], [0, 1], [0, 1]], dtype=np.int32)
    vals = np.array([1.0, 2.0])
    u = np.full((2, 1), 1 / math.sqrt(2))
    U = [u, u, u]
    G = O.core_elementwise(idx, vals, U)
    g = 3.0 / (2.0 * math.sqrt(2.0))
    assert G.shape == (1, 1, 1) and G[0, 0, 0] == pytest.approx(g, abs=1e-15)
    A = O.ttmctc_elementwise(idx, vals, U, 0, G)
    np.testing.assert_allclose(A[:, 0], [1.0 * g * 0.5, 2.0 * g * 0.5], atol=1e-15)
    # one HOQRI mode step: A has two positive entries, so U^(1) = A/||A|| = [1,2]/sqrt5
    Q, R = O.qr_positive(A)
    np.testing.assert_allclose(Q[:, 0], [1 / math.sqrt(5), 2 / math.sqrt(5)], atol=1e-15)


def test_linearity_and_duplicates():
    dims, K = (5, 6, 7), (2, 2, 3)
    idx, vals, U = _tiny(dims, K, 30, seed=21)
    # doubling every nonzero by listing it twice equals doubling the values
    idx2 = np.concatenate([idx, idx], axis=1)
    vals2 = np.concatenate([vals, vals])
    for n in range(3):
        G2 = O.core_elementwise(idx2, vals2, U)
        np.testing.assert_allclose(G2, O.core_elementwise(idx, 2 * vals, U), atol=1e-13)
        np.testing.assert_allclose(O.ttmctc_elementwise(idx2, vals2, U, n, G2),
                                   O.ttmctc_elementwise(idx, 2 * vals, U, n, G2), atol=1e-13)
    ci, cv = O.coalesce(idx2, vals2, dims)
    assert ci.shape[1] == idx.shape[1]
    assert O.norm_x2(cv) == pytest.approx(4 * float(vals @ vals), rel=1e-14)
    np.testing.assert_allclose(O.to_dense(ci, cv, dims), O.to_dense(idx2, vals2, dims), atol=0)


def test_equivariance_under_rotations():
    # A^(n)(U Q) = A^(n)(U) Q_n for orthogonal Q_m (derived from the TTMcTC definition)
    dims, K = (6, 7, 8), (2, 3, 2)
    idx, vals, U = _tiny(dims, K, 50, seed=31)
    rng = np.random.default_rng(5)
    Qs = [np.linalg.qr(rng.standard_normal((k, k)))[0] for k in K]
    UQ = [u @ q for u, q in zip(U, Qs)]
    for n in range(3):
        A = O.ttmctc_elementwise(idx, vals, U, n)
        AQ = O.ttmctc_elementwise(idx, vals, UQ, n)
        np.testing.assert_allclose(AQ, A @ Qs[n], atol=1e-13)


def test_fit_matches_dense_residual():
    dims, K = (6, 7, 8), (2, 3, 2)
    idx, vals, U = _tiny(dims, K, 60, seed=41)
    X = O.to_dense(idx, vals, dims)
    G = O.core_dense(X, U)
    res = np.sum((X - O.tucker_dense(G, U)) ** 2)
    nx2 = O.norm_x2(vals)
    assert res == pytest.approx(nx2 - np.sum(G * G), rel=1e-12)
    assert O.fit_from(nx2, float(np.sum(G * G))) == pytest.approx(1 - math.sqrt(res) / math.sqrt(nx2), rel=1e-12)


def test_qr_positive_against_cholesky_route_and_breakdown():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((50, 6))
    Q, R = O.qr_positive(A)
    np.testing.assert_allclose(Q @ R, A, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-14)
    assert np.all(np.diag(R) > 0)
    # the same factor from the normal equations: R = chol(A^T A)^T (textbook identity)
    Rc = np.linalg.cholesky(A.T @ A).T
    np.testing.assert_allclose(R, Rc, rtol=1e-10, atol=1e-12)
    B = A.copy()
    B[:, 3] = B[:, 0] + B[:, 1]
    with pytest.raises(O.RankDeficient):
        O.qr_positive(B)
    with pytest.raises(O.RankDeficient):
        O.qr_positive(np.zeros((5, 2)))


def test_subspace_distance_against_procrustes():
    from scipy.linalg import orthogonal_procrustes
    rng = np.random.default_rng(8)
    U = np.linalg.qr(rng.standard_normal((20, 4)))[0]
    V = np.linalg.qr(rng.standard_normal((20, 4)))[0]
    Q, _ = orthogonal_procrustes(V, U)   # argmin ||V Q - U||
    assert O.subspace_dist(U, V) == pytest.approx(np.sum((U - V @ Q) ** 2), rel=1e-10)
    W = np.linalg.qr(rng.standard_normal((4, 4)))[0]
    assert abs(O.subspace_dist(U, U @ W)) < 1e-12


def test_validate_rejects_bad_inputs():
    idx = np.array([[0, 1], [0, 2], [1, 1]])
    O.validate(idx, (2, 3, 2), (1, 1, 1))
    with pytest.raises(IndexError):
        O.validate(idx, (2, 2, 2), (1, 1, 1))
    with pytest.raises(ValueError):
        O.validate(idx, (2, 3, 2), (3, 1, 1))          # K > I
    with pytest.raises(ValueError):
        O.validate(idx, (2, 3, 2), (2, 1, 1))          # K_0 > K_1 K_2
    with pytest.raises(ValueError):
        O.validate(np.zeros((3, 0), dtype=int), (2, 3, 2), (1, 1, 1))
