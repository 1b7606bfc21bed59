"""Pins of the oracle's TensorSketch (Section 1.3), s-value update
(Section 4, Algorithm 3) and tensor error evaluator (Gram identity)."""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _khatri_rao(factors):
    """Row (i_1, ..., i_N) of the Khatri-Rao product, in itertools order."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    rows = []
    idx = []
    for tup in itertools.product(*[range(d) for d in dims]):
        v = np.ones(R)
        for n, i in enumerate(tup):
            v = v * factors[n][i, :]
        rows.append(v)
        idx.append(tup)
    return np.array(rows), idx


def _explicit_T(maps, idx, Jlen):
    """TensorSketch matrix: column for tuple i has S(i) in row H(i)."""
    T = np.zeros((Jlen, len(idx)))
    for c, tup in enumerate(idx):
        H = sum(int(maps[n][0][i]) for n, i in enumerate(tup)) % Jlen
        S = np.prod([int(maps[n][1][i]) for n, i in enumerate(tup)])
        T[H, c] = S
    return T


@pytest.mark.parametrize("dims,R,Jlen", [((4, 5, 3), 6, 8), ((3, 4), 5, 7), ((2, 3, 2, 3), 4, 16)])
def test_tensorsketch_equals_explicit_T_times_M(dims, R, Jlen):
    g = np.random.default_rng(sum(dims))
    factors = [g.standard_normal((d, R)) for d in dims]
    lam = g.uniform(0.5, 2.0, R)
    maps = oracle.tensor_maps(4, dims, Jlen)
    KR, idx = _khatri_rao(factors)
    M = KR * lam[None, :]
    TM = _explicit_T(maps, idx, Jlen) @ M
    Y = oracle.tensorsketch(factors, lam, maps, Jlen)
    np.testing.assert_allclose(Y, TM, rtol=1e-13, atol=1e-13)


def test_tensorsketch_integer_exact():
    g = np.random.default_rng(1)
    dims, R, Jlen = (5, 4, 6), 3, 9
    factors = [g.integers(-5, 5, size=(d, R)).astype(np.float64) for d in dims]
    lam = np.array([1.0, -2.0, 3.0])
    maps = oracle.tensor_maps(9, dims, Jlen)
    KR, idx = _khatri_rao(factors)
    TM = _explicit_T(maps, idx, Jlen) @ (KR * lam[None, :])
    assert np.array_equal(oracle.tensorsketch(factors, lam, maps, Jlen), TM)


def test_tensorsketch_matches_fft_formula():
    # eq. for T A: FFT^{-1}( prod_n FFT(S^(n) A^(n)) ) -- numpy FFT as the
    # special-case library routine
    g = np.random.default_rng(2)
    dims, R, Jlen = (60, 50, 40), 7, 64
    factors = [g.standard_normal((d, R)) for d in dims]
    lam = g.uniform(0.1, 10, R)
    maps = oracle.tensor_maps(5, dims, Jlen)
    Y = oracle.tensorsketch(factors, lam, maps, Jlen)
    spec = np.ones((Jlen, R), dtype=complex)
    for f, (b, s) in zip(factors, maps):
        C = oracle.countsketch_dense(f, b, s, Jlen)
        spec *= np.fft.fft(C, axis=0)
    Yf = np.real(np.fft.ifft(spec, axis=0)) * lam[None, :]
    np.testing.assert_allclose(Y, Yf, rtol=0, atol=1e-12 * np.abs(Yf).max())


def test_tensorsketch_column_subset():
    g = np.random.default_rng(3)
    dims, R, Jlen = (30, 20, 10), 9, 32
    factors = [g.standard_normal((d, R)) for d in dims]
    lam = np.ones(R)
    maps = oracle.tensor_maps(6, dims, Jlen)
    Y = oracle.tensorsketch(factors, lam, maps, Jlen)
    cols = [8, 0, 3]
    assert np.array_equal(oracle.tensorsketch(factors, lam, maps, Jlen, cols=cols), Y[:, cols])


def test_tensorsketch_inner_product_unbiased():
    # Fact 6(i): E <T x, T y> = <x, y> for Kronecker-structured x, y
    g = np.random.default_rng(4)
    dims, Jlen = (6, 5, 4), 16
    factors = [g.standard_normal((d, 2)) for d in dims]
    KR, _ = _khatri_rao(factors)
    exact = float(KR[:, 0] @ KR[:, 1])
    vals = []
    for seed in range(3000):
        maps = oracle.tensor_maps(seed, dims, Jlen)
        Y = oracle.tensorsketch(factors, np.ones(2), maps, Jlen)
        vals.append(Y[:, 0] @ Y[:, 1])
    vals = np.array(vals)
    assert abs(vals.mean() - exact) < 5 * vals.std() / np.sqrt(len(vals))


def test_lambda_hat_duplicated_terms_closed_form():
    # Terms that are exact copies of base terms: the ID keeps one term per
    # group and lambda_hat equals the group's lambda sum; the error vanishes.
    factors, lam, base_of = synth.cp_tensor(dims=(30, 25, 20), R=24, nbase=4, pert=0.0,
                                            lam_range=(0.5, 2.0), seed=1)
    r = oracle.tensor_id(factors, lam, k=4, Jlen=64, seed=1)
    assert r["k_eff"] == 4
    groups = base_of[r["J"]]
    assert sorted(groups) == [0, 1, 2, 3]
    for t, gidx in enumerate(groups):
        np.testing.assert_allclose(r["lambda_hat"][t], lam[base_of == gidx].sum(), rtol=1e-10)
    assert oracle.tensor_error(factors, lam, r["J"], r["lambda_hat"]) < 1e-7


def test_tensor_error_gram_matches_dense():
    g = np.random.default_rng(5)
    dims, R = (5, 4, 3), 6
    factors = [g.standard_normal((d, R)) for d in dims]
    lam = g.uniform(0.5, 2, R)
    J = np.array([1, 4])
    lh = np.array([0.7, -1.3])
    KR, _ = _khatri_rao(factors)
    X = KR @ lam
    Xh = KR[:, J] @ lh
    expect = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    assert oracle.tensor_error(factors, lam, J, lh) == pytest.approx(expect, rel=1e-12)


def test_lambda_hat_definition():
    P = np.array([[1.0, 0.5, 0.0], [0.0, 2.0, 1.0]])
    J = np.array([0, 2])
    lam = np.array([3.0, 5.0, -7.0])
    np.testing.assert_array_equal(oracle.lambda_hat(P, J, lam), [3.0 * 1.5, -7.0 * 3.0])
