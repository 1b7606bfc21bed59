"""Pins of the oracle's CountSketch (Section 1.3) and of its plain product."""
import numpy as np
import pytest

import oracle
import synth


def explicit_S(bucket, sign, L):
    """The CountSketch matrix S = Phi D written out (Section 1.3)."""
    m = bucket.shape[0]
    S = np.zeros((L, m))
    S[bucket, np.arange(m)] = sign
    return S


@pytest.mark.parametrize("m,n,L", [(50, 7, 6), (300, 33, 40), (129, 65, 128)])
def test_countsketch_equals_explicit_S_times_A_exactly(m, n, L):
    g = np.random.default_rng(m)
    A = g.integers(-1000, 1000, size=(m, n)).astype(np.float64)
    b, s = oracle.hash_maps(1, 0, m, L)
    Y = oracle.countsketch_dense(A, b, s, L)
    assert np.array_equal(Y, explicit_S(b, s, L) @ A)  # integer sums: exact


def test_countsketch_gaussian_matches_explicit():
    g = np.random.default_rng(0)
    A = g.standard_normal((500, 40))
    b, s = oracle.hash_maps(2, 0, 500, 32)
    Y = oracle.countsketch_dense(A, b, s, 32)
    np.testing.assert_allclose(Y, explicit_S(b, s, 32) @ A, rtol=0, atol=1e-13)


def test_frobenius_norm_of_S_is_sqrt_m():
    # Lemma 4: ||S||_F^2 = I (each column of S has one +-1)
    b, s = oracle.hash_maps(3, 0, 777, 50)
    # S^T applied to the identity: sketch of I_m
    Y = oracle.countsketch_dense(np.eye(777), b, s, 50)
    assert float(np.sum(Y * Y)) == 777.0


def test_csr_equals_dense():
    import scipy.sparse as sp
    g = np.random.default_rng(4)
    A = sp.random(400, 90, density=0.05, random_state=5, format="csr")
    A.data = np.round(A.data * 1000)
    b, s = oracle.hash_maps(9, 0, 400, 24)
    Yc = oracle.countsketch_csr(A.indptr, A.indices, A.data, 90, b, s, 24)
    Yd = oracle.countsketch_dense(A.toarray(), b, s, 24)
    assert np.array_equal(Yc, Yd)


def test_csr_duplicates_are_summed():
    rowptr = np.array([0, 3, 4], dtype=np.int64)
    colind = np.array([1, 1, 2, 0], dtype=np.int32)
    val = np.array([2.0, 3.0, 7.0, 5.0])
    b = np.array([1, 0], dtype=np.int32)
    s = np.array([-1, 1], dtype=np.int8)
    Y = oracle.countsketch_csr(rowptr, colind, val, 3, b, s, 2)
    assert np.array_equal(Y, np.array([[5.0, 0, 0], [0, -5.0, -7.0]]))


def test_fullrank_square_sketch_is_signed_permutation():
    # With h~ and L = I, S is a signed permutation, so Y^T Y = A^T A exactly.
    m, n = 64, 10
    pi, x = synth.fullrank_perm(m, m, 0)
    b = oracle.fullrank_buckets(pi, x, m)
    _, s = oracle.hash_maps(0, 0, m, m)
    A = np.random.default_rng(1).integers(-50, 50, size=(m, n)).astype(np.float64)
    Y = oracle.countsketch_dense(A, b, s, m)
    assert np.array_equal(Y.T @ Y, A.T @ A)


def test_subspace_embedding_lemma2_monte_carlo():
    # Lemma 2: E ||(S U)^T (S U) - I||^2 <= (K^2 + K) / L for U with orthonormal
    # columns.  Check the Monte-Carlo mean over seeds stays below the bound.
    m, K, L = 2000, 4, 200
    U = synth.orthonormal(m, K, np.random.default_rng(0))
    vals = []
    for seed in range(300):
        b, s = oracle.hash_maps(seed, 0, m, L)
        SU = oracle.countsketch_dense(U, b, s, L)
        E = SU.T @ SU - np.eye(K)
        vals.append(np.linalg.norm(E, 2) ** 2)
    assert np.mean(vals) <= (K * K + K) / L


def test_gemm_matches_numpy():
    g = np.random.default_rng(2)
    G = g.standard_normal((17, 40))
    B = g.standard_normal((40, 29))
    np.testing.assert_allclose(oracle.gemm(G, B), G @ B, rtol=1e-13, atol=1e-13)
    Gi = g.integers(-9, 9, size=(8, 30)).astype(np.float64)
    Bi = g.integers(-9, 9, size=(30, 11)).astype(np.float64)
    assert np.array_equal(oracle.gemm(Gi, Bi), Gi @ Bi)


def test_gaussian_stream_draw():
    # the oracle's G generator (Box-Muller on the stream's uniforms): N(0, 1)
    # by moments and a Kolmogorov-Smirnov test, a new stream per (seed, tag),
    # and entry e built from outputs 2e, 2e+1 of the stream (seed, tag | 2^63)
    from scipy import stats
    g = oracle.gaussian(11, 5, 400, 500).ravel()
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1) < 5 * np.sqrt(2 / g.size)
    assert abs(np.mean(g ** 4) - 3) < 0.1
    assert stats.kstest(g, "norm").pvalue > 1e-3
    assert not np.array_equal(oracle.gaussian(11, 6, 4, 5), oracle.gaussian(11, 5, 4, 5))
    z = oracle.stream(11, 5 | (1 << 63), 2 * 20)
    u1 = ((z[0::2] >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (z[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    ref = np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    np.testing.assert_allclose(oracle.gaussian(11, 5, 4, 5).ravel(), ref, rtol=1e-14, atol=1e-15)


def test_cp_sparse_csc_form_holds_the_same_entries():
    import scipy.sparse as sp
    dense, lam = synth.cp_sparse(N=3, I=50, R=7, K=3, density=0.1, seed=4)
    csc, lam2 = synth.cp_sparse(N=3, I=50, R=7, K=3, density=0.1, seed=4, fmt="csc")
    assert np.array_equal(lam, lam2)
    for F, (cp, ri, va) in zip(dense, csc):
        assert np.all(np.diff(ri.reshape(7, -1), axis=1) > 0)
        assert np.array_equal(sp.csc_matrix((va, ri, cp), shape=F.shape).toarray(), F)
