"""Pins of the oracle's rank-K column-pivoted QR and interpolation matrix
(Algorithm 1; Fact 1; the CPQR remark in Section 1.2.1)."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


def _separated(l, n, seed):
    g = np.random.default_rng(seed)
    Y = g.standard_normal((l, n))
    Y *= g.uniform(0.5, 4.0, n)[None, :]
    return Y


@pytest.mark.parametrize("l,n,k", [(12, 30, 5), (30, 200, 20), (64, 64, 40), (40, 15, 15)])
def test_pivots_match_lapack_geqp3(l, n, k):
    # special case: greedy CPQR pivots equal LAPACK's dgeqp3 pivots when no
    # near-ties occur (well separated random columns)
    Y = _separated(l, n, l * n + k)
    J, P, keff, R, nu = oracle.cpqr_id(Y, k, trace=True)
    assert keff == k
    _, Rl, piv = sla.qr(Y, pivoting=True, mode="economic")
    assert np.array_equal(J, piv[:k])
    np.testing.assert_allclose(np.abs(R[np.arange(k), J]), np.abs(np.diag(Rl)[:k]), rtol=1e-12)


def test_pivot_certificate_and_decreasing_diagonal():
    Y = np.random.default_rng(3).standard_normal((25, 300))
    k = 20
    J, P, keff, R, nu = oracle.cpqr_id(Y, k, trace=True)
    d = np.abs(R[np.arange(k), J])
    for t in range(k):
        # |r_tt|^2 is the largest trailing squared column norm at step t
        assert d[t] ** 2 == pytest.approx(nu[t].max(), rel=1e-12)
        assert nu[t, J[t]] == nu[t].max()
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))


def test_identity_on_skeleton_exact():
    # Fact 1(i): P[:, J] = I_K exactly
    Y = np.random.default_rng(4).standard_normal((30, 100))
    J, P, keff, R, _ = oracle.cpqr_id(Y, 17)
    assert np.array_equal(P[:, J], np.eye(17))


def test_R11_times_T_equals_R12():
    Y = np.random.default_rng(5).standard_normal((40, 120))
    k = 25
    J, P, keff, R, _ = oracle.cpqr_id(Y, k)
    rest = np.setdiff1d(np.arange(120), J)
    R11 = R[:, J]
    assert np.allclose(np.tril(R11, -1), 0.0)
    T = sla.solve_triangular(R11, R[:, rest], lower=False)
    np.testing.assert_allclose(P[:, rest], T, rtol=1e-11, atol=1e-11)


def test_residual_equals_trailing_norm():
    # Y Pi = Q [R11 R12; 0 R22]  =>  ||Y - Y_J P||_F^2 = ||R22||_F^2, which is the
    # sum of the trailing squared norms at step K.
    Y = np.random.default_rng(6).standard_normal((30, 90))
    k = 12
    J, P, _, _, _ = oracle.cpqr_id(Y, k)
    _, _, _, _, nu = oracle.cpqr_id(Y, k + 1, trace=True)
    res2 = np.sum((Y - Y[:, J] @ P) ** 2)
    tail = np.sum(nu[k][nu[k] >= 0])
    assert res2 == pytest.approx(tail, rel=1e-10)


def test_K_equals_rows_is_exact():
    # Fact 1(v): K = I (number of rows) reproduces the matrix
    Y = np.random.default_rng(7).standard_normal((16, 70))
    J, P, keff, _, _ = oracle.cpqr_id(Y, 16)
    assert keff == 16
    np.testing.assert_allclose(Y[:, J] @ P, Y, atol=1e-12 * np.abs(Y).max())


def test_exact_rank_k_matrix_id():
    A = synth.config0(seed=3, exact=True, m=400, n=200, k=10)
    G = synth.gaussian(20, 64, 3)
    r = oracle.matrix_id(A, k=10, l1=64, seed=3, G=G)
    assert r["k_eff"] == 10
    assert oracle.residual_fro(A, r["J"], r["P"]) < 1e-13


def test_rank_deficient_stops_early():
    g = np.random.default_rng(8)
    Y = g.standard_normal((20, 4)) @ g.standard_normal((4, 50))
    Y[:, 10:] = 0.0
    Y = Y[:, :10]                           # rank 4, 10 columns
    Yr = np.zeros((20, 30))
    Yr[:, ::3] = Y                          # + exact zero columns
    J, P, keff, _, _ = oracle.cpqr_id(Yr, 8)
    # floating rank is 4; exact zeros beyond it are not guaranteed, so accept
    # either an early stop or tiny trailing pivots
    assert keff <= 8
    Z = np.zeros((10, 6))
    J2, P2, keff2, _, _ = oracle.cpqr_id(Z, 3)
    assert keff2 == 0 and np.all(J2 == -1) and np.all(P2 == 0)
    Y3 = np.zeros((10, 6))
    Y3[:, 2] = 1.0
    J3, P3, keff3, _, _ = oracle.cpqr_id(Y3, 3)
    assert keff3 == 1 and J3[0] == 2 and np.all(J3[1:] == -1)


def test_ties_go_to_lowest_index():
    Y = np.zeros((4, 6))
    Y[0, 1] = 1.0
    Y[1, 3] = 1.0
    Y[2, 5] = -1.0
    J, _, keff, _, _ = oracle.cpqr_id(Y, 3)
    assert list(J) == [1, 3, 5]


def _best_subset(A, k):
    best, bestJ = np.inf, None
    for J in itertools.combinations(range(A.shape[1]), k):
        C = A[:, J]
        X, *_ = np.linalg.lstsq(C, A, rcond=None)
        r = np.linalg.norm(A - C @ X)
        if r < best:
            best, bestJ = r, J
    return best, bestJ


def test_bruteforce_best_subset_lower_bound():
    # CPQR-ID can never beat the best k-subset projection
    for seed in range(6):
        A = np.random.default_rng(seed).standard_normal((8, 7))
        best, _ = _best_subset(A, 3)
        J, P, _, _, _ = oracle.cpqr_id(A, 3)
        r = np.linalg.norm(A - A[:, J] @ P)
        assert r >= best * (1 - 1e-12)
        # the interpolation coefficients are the least-squares ones only up to
        # the sketch; here Y = A so P is the projection coefficient on A_J
        X, *_ = np.linalg.lstsq(A[:, J], A, rcond=None)
        assert r <= np.linalg.norm(A - A[:, J] @ X) * 10


def test_bruteforce_planted_skeleton():
    # k dominant columns plus small combinations of them: the unique best subset
    # is the planted one, and the ID finds it
    for seed in range(5):
        g = np.random.default_rng(100 + seed)
        k, n, l = 3, 8, 9
        planted = np.sort(g.choice(n, k, replace=False))
        B = g.standard_normal((l, k)) * 10
        A = 0.05 * g.standard_normal((l, n)) + 1e-3 * g.standard_normal((l, n))
        A[:, planted] = B
        A += 0  # others are small
        _, bestJ = _best_subset(A, k)
        J, P, _, _, _ = oracle.cpqr_id(A, k)
        assert tuple(sorted(J)) == tuple(bestJ) == tuple(planted)


def test_fact1_residual_bound_holds_for_sketched_id():
    # Proposition 1 / Fact 1(vi) style check: ||A_J P - A|| <= sigma_{K+1} sqrt(4K(R-K)+1)
    # comfortably for a well-sketched problem (CPQR in place of SRRQR, so only
    # a loose statistical pin).
    m, n, k = 600, 120, 8
    sig = np.concatenate([np.ones(k), 1e-6 * np.ones(n - k)])
    A = synth.dense_lowrank(m, n, sig, 0.0, 2)
    G = synth.gaussian(k + 10, 64, 2)
    r = oracle.matrix_id(A, k=k, l1=64, seed=2, G=G)
    err = np.linalg.norm(A - A[:, r["J"]] @ r["P"], 2)
    assert err <= 1e-6 * np.sqrt(4 * k * (n - k) + 1)


def test_adaptive_rank_clear_gap_and_consistency():
    # sigma = 1 for i <= 10, 1e-6 after: at tol = 1e-3 the fixed-accuracy stop
    # is rank 10; the adaptive ID is the fixed-rank ID of that rank
    g = np.random.default_rng(31)
    m, n = 300, 120
    U, _ = np.linalg.qr(g.standard_normal((m, n)))
    V, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = np.where(np.arange(n) < 10, 1.0, 1e-6)
    A = (U * s) @ V.T
    G = g.standard_normal((40, 128))
    o = oracle.matrix_id_adaptive(A, kmax=30, tol=1e-3, l1=128, seed=1, G=G)
    assert o["rank"] == 10 and o["k_eff"] == 10
    f = oracle.matrix_id(A, k=10, l1=128, seed=1, G=G)
    assert np.array_equal(o["J"], f["J"]) and np.array_equal(o["P"], f["P"])
    assert np.array_equal(o["J"], o["J_kmax"][:10])
    # |r_tt| of column-pivoted QR never increases, so the first step below the
    # threshold is also the count of diagonal entries above it
    d = np.abs(o["R_kmax"][np.arange(30), o["J_kmax"]])
    assert np.all(d[1:] <= d[:-1] * (1 + 1e-12))
    assert int(np.sum(d > 1e-3 * d[0])) == 10


def test_adaptive_rank_tol_zero_is_fixed_rank():
    g = np.random.default_rng(32)
    A = g.standard_normal((200, 80))
    o = oracle.matrix_id_adaptive(A, kmax=25, tol=0.0, l1=64, seed=2, G=g.standard_normal((30, 64)))
    assert o["rank"] == 25
