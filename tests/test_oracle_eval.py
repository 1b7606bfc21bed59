"""Pins of the oracle's error evaluators and of its hash stream for nonzero
(seed, tag), against things other than the evaluators themselves:

  * residual_fro: a direct library evaluation (numpy's Frobenius norm of the
    whole difference, no chunking), the QR identity ||Y - Y_J P||_F^2 =
    ||R22||_F^2 (the sum of the trailing squared column norms after K steps,
    Algorithm 1), and its handling of unused skeleton slots (J = -1).
  * residual_fro_csr: the dense evaluation of the same matrix, duplicates
    summed (CSR definition), on matrices small enough to densify.
  * spectral_est: the exact 2-norm from an SVD (the randomized spectral-norm
    estimate of the matrix experiments, Section 6.1, is a lower bound that
    power iteration drives to the exact value when the top singular value is
    separated).
  * hash stream: an independent arbitrary-precision Python SplitMix64
    (Steele, Lea & Flood 2014), written here from the publication, for several
    nonzero seeds and tags (the CountSketch maps h, D of Section 1.3).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

M64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# residual_fro
# --------------------------------------------------------------------------
def _lowrank(m, n, r, noise, seed):
    sig = np.where(np.arange(1, min(m, n) + 1) <= r, 1.0, 0.0)[: min(m, n)]
    return synth.dense_lowrank(m, n, sig[:min(m, n)], noise, seed=seed)


def test_residual_fro_chunked_equals_direct_norm():
    # 70000 rows: the default chunk (65536) splits the rows in two, chunk=1000
    # in 70 with a ragged last piece; both must equal one direct evaluation.
    m, n, k = 70000, 30, 8
    A = _lowrank(m, n, k, 1e-3, seed=11)
    r = oracle.matrix_id(A, k=k, l1=64, seed=11)
    J, P = r["J"], r["P"]
    direct = np.linalg.norm(A - A[:, J] @ P) / np.linalg.norm(A)
    assert direct > 0
    assert oracle.residual_fro(A, J, P) == pytest.approx(direct, rel=1e-12)
    assert oracle.residual_fro(A, J, P, chunk=1000) == pytest.approx(direct, rel=1e-12)
    assert oracle.residual_fro(A, J, P, chunk=1 << 30) == pytest.approx(direct, rel=1e-12)


def test_residual_fro_equals_trailing_norms_after_k_steps():
    # Y Pi = Q [R11 R12; 0 R22] with Q orthogonal, and Y_J P = Q [R11 R12; 0 0] Pi^T,
    # so ||Y - Y_J P||_F^2 = ||R22||_F^2: the sum over unchosen columns of the
    # trailing squared norms the pivoted QR holds before step K + 1.
    g = np.random.default_rng(21)
    for (l, n, k) in ((40, 120, 10), (25, 300, 24), (70000 // 1000, 500, 30)):
        Y = g.standard_normal((l, n)) * np.logspace(0, -6, n)[None, :]
        J, P, keff, _, _ = oracle.cpqr_id(Y, k)
        _, _, _, _, nu = oracle.cpqr_id(Y, k + 1, trace=True)
        tail = float(np.sum(nu[k][nu[k] >= 0]))
        res = oracle.residual_fro(Y, J, P)
        assert res ** 2 * float(np.sum(Y * Y)) == pytest.approx(tail, rel=1e-9)


def test_residual_fro_ignores_unused_slots():
    # rows of P whose J entry is -1 (rank deficiency) take no part
    A = _lowrank(300, 40, 5, 1e-4, seed=12)
    r = oracle.matrix_id(A, k=5, l1=32, seed=12)
    J2 = np.concatenate([r["J"], [-1, -1]])
    P2 = np.vstack([r["P"], np.full((2, 40), 123.0)])
    assert oracle.residual_fro(A, J2, P2) == oracle.residual_fro(A, r["J"], r["P"])


def test_residual_fro_zero_for_exact_identity_and_full_rank():
    # Fact 1(v): K = R (all columns) reproduces A exactly
    A = np.random.default_rng(13).standard_normal((50, 7))
    J = np.arange(7)
    assert oracle.residual_fro(A, J, np.eye(7)) == 0.0


# --------------------------------------------------------------------------
# residual_fro_csr
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k,seed", [(400, 60, 6, 1), (1500, 200, 20, 2)])
def test_residual_fro_csr_equals_dense(m, n, k, seed):
    g = np.random.default_rng(seed)
    # sparse plus a planted low-rank part, with duplicate (row, col) entries
    counts = g.integers(0, 9, size=m)
    rows = np.repeat(np.arange(m), counts)
    cols = g.integers(0, n, size=rows.shape[0]).astype(np.int32)
    vals = g.standard_normal(rows.shape[0])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dense = np.zeros((m, n))
    np.add.at(dense, (rows, cols), vals)          # duplicates summed
    assert sp.csr_matrix((vals, cols, rowptr), shape=(m, n)).nnz >= 0
    J = np.sort(g.choice(n, size=k, replace=False)).astype(np.int64)
    P = g.standard_normal((k, n))
    P[:, J] = np.eye(k)
    direct = np.linalg.norm(dense - dense[:, J] @ P) / np.linalg.norm(dense)
    got = oracle.residual_fro_csr(rowptr, cols, vals, n, J, P)
    assert got == pytest.approx(direct, rel=1e-10)
    assert got == pytest.approx(oracle.residual_fro(dense, J, P), rel=1e-10)


# --------------------------------------------------------------------------
# spectral_est
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [3, 4])
def test_spectral_est_matches_svd(seed):
    # residual with a separated top singular value: power iteration converges
    m, n, k = 300, 80, 10
    sig = np.concatenate([np.logspace(0, -3, k), [1e-4, 3e-5], np.full(n - k - 2, 1e-6)])
    A = synth.dense_lowrank(m, n, sig, 0.0, seed=seed)
    r = oracle.matrix_id(A, k=k, l1=48, seed=seed)
    E = A - A[:, r["J"]] @ r["P"]
    exact = np.linalg.norm(E, 2) / np.linalg.norm(A, 2)
    est = oracle.spectral_est(A, r["J"], r["P"], iters=50)
    assert est <= exact * (1 + 1e-10)            # a Rayleigh-quotient lower bound
    assert est >= 0.97 * exact
    # and the spectral norm of E sits between ||E||_F / sqrt(rank) and ||E||_F
    fro = oracle.residual_fro(A, r["J"], r["P"]) * np.linalg.norm(A) / np.linalg.norm(A, 2)
    assert est <= fro * (1 + 1e-10)
    assert est >= fro / np.sqrt(n) * 0.97


def test_spectral_est_exact_rank_is_tiny():
    A = synth.config0(seed=3, exact=True, m=400, n=200, k=10)
    r = oracle.matrix_id(A, k=10, l1=64, seed=3, G=synth.gaussian(20, 64, 3))
    assert oracle.spectral_est(A, r["J"], r["P"]) < 1e-13


# --------------------------------------------------------------------------
# hash stream for nonzero (seed, tag): independent big-int SplitMix64
# --------------------------------------------------------------------------
def _mix(z: int) -> int:
    # the SplitMix64 output function, evaluated with Python integers mod 2^64
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _py_maps(seed: int, tag: int, m: int, L: int):
    key = _mix(seed ^ _mix(tag))
    gamma = 0x9E3779B97F4A7C15
    b = np.empty(m, dtype=np.int64)
    s = np.empty(m, dtype=np.int64)
    for i in range(m):
        z = _mix(key + (i + 1) * gamma)
        b[i] = ((z >> 32) * L) >> 32
        s[i] = -1 if (z & 1) else 1
    return key, b, s


@pytest.mark.parametrize("seed,tag", [(1, 0), (0, 1), (7, 3), (0xDEADBEEF, 15),
                                      (2**63 + 5, 2**40 + 3), (M64, M64)])
@pytest.mark.parametrize("L", [1, 3, 480, 4096, 32768])
def test_hash_matches_independent_bigint_splitmix(seed, tag, L):
    m = 700
    key, b, s = _py_maps(seed, tag, m, L)
    assert oracle.lib().orc_stream_key(seed, tag) == key
    ob, os_ = oracle.hash_maps(seed, tag, m, L)
    assert np.array_equal(ob.astype(np.int64), b)
    assert np.array_equal(os_.astype(np.int64), s)


def test_tensor_mode_streams_are_tags_one_up():
    # mode n of the TensorSketch draws h_n, s_n from tag n + 1
    dims = (37, 50, 21)
    maps = oracle.tensor_maps(9, dims, 64)
    for n, d in enumerate(dims):
        _, b, s = _py_maps(9, n + 1, d, 64)
        assert np.array_equal(maps[n][0].astype(np.int64), b)
        assert np.array_equal(maps[n][1].astype(np.int64), s)


def test_pool_drivers_match_serial_oracle():
    # the process-pool drivers only split independent work: a batch's oracle
    # IDs and a TensorSketch's columns equal the serial oracle's bit for bit
    import tempfile

    from oracle import pool
    m, n, flat = synth.batched_inputs(12, seed=3)
    G = synth.bf16_bits(synth.gaussian(20, 64, seed=3))
    d = tempfile.mkdtemp()
    a_path = os.path.join(d, "A.npy")
    np.save(a_path, flat)
    jo, po, keff, _, _ = pool.batched_oracle(a_path, G, m, n, 15, 64, 3, d, workers=2)
    Jo = np.load(jo)
    Po = np.load(po)
    a_off = np.concatenate([[0], np.cumsum(m * n)])
    p_off = np.concatenate([[0], np.cumsum(15 * n)])
    for p in (0, 7, 11):
        A = synth.bf16_to_f64(flat[a_off[p]:a_off[p + 1]]).reshape(m[p], n[p])
        l1 = min(int(m[p]), 64)
        o = oracle.matrix_id(A, k=15, l1=l1, seed=3, tag=p, G=synth.bf16_to_f64(G)[:, :l1])
        assert np.array_equal(Jo[p], o["J"])
        assert np.array_equal(Po[p_off[p]:p_off[p + 1]].reshape(15, n[p]), o["P"])
    res = pool.batched_ratios(a_path, m, n, 15, Jo, Po, jo, po, d, workers=2)
    assert np.all(res[:, 0] == res[:, 1])
    f, lam, _ = synth.cp_tensor(dims=(40, 30, 20), R=60, nbase=6, pert=1e-6, seed=6)
    maps = oracle.tensor_maps(0, [40, 30, 20], 64)
    assert np.array_equal(pool.tensorsketch(f, lam, maps, 64, workers=3), oracle.tensorsketch(f, lam, maps, 64))


def test_tensor_error_sampled_all_entries_is_exact():
    # every entry of a small CP tensor: the sampled evaluator is the plain
    # Frobenius-norm ratio of the explicit tensors (def-X-tensor)
    f, lam, _ = synth.cp_tensor(dims=(6, 5, 4), R=9, nbase=3, pert=1e-3, seed=2)
    J = np.array([0, 4, -1])
    lhat = np.array([1.7, -0.3, 0.0])
    X = np.einsum("r,ir,jr,kr->ijk", lam, *f)
    Xh = lhat[0] * np.einsum("i,j,k->ijk", f[0][:, 0], f[1][:, 0], f[2][:, 0]) + \
        lhat[1] * np.einsum("i,j,k->ijk", f[0][:, 4], f[1][:, 4], f[2][:, 4])
    exact = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    ent = np.array(np.meshgrid(np.arange(6), np.arange(5), np.arange(4), indexing="ij")).reshape(3, -1).T
    assert abs(oracle.tensor_error_sampled(f, lam, J, lhat, entries=ent) - exact) <= 1e-13 * exact
    # and the Gram-identity evaluator agrees on the same case
    assert abs(oracle.tensor_error(f, lam, J, lhat) - exact) <= 1e-12 * exact


def test_tensor_error_sparse_matches_dense_evaluators():
    # sparse factor columns (the synthetic sparse 5-way generator, scaled down):
    # the sparse Gram path equals the dense long-double Gram identity, and both
    # equal the explicit tensor difference on a tensor small enough to form
    f, lam = synth.cp_sparse(N=3, I=7, R=10, K=4, density=0.3, seed=1)
    J = np.array([1, 3, 6, -1])
    lhat = np.array([0.9, -0.2, 0.05, 0.0])
    X = np.einsum("r,ir,jr,kr->ijk", lam, *f)
    Xh = sum(lhat[t] * np.einsum("i,j,k->ijk", f[0][:, j], f[1][:, j], f[2][:, j]) for t, j in enumerate(J) if j >= 0)
    exact = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    assert abs(oracle.tensor_error_sparse(f, lam, J, lhat) - exact) <= 1e-12 * exact
    f5, lam5 = synth.cp_sparse(N=5, I=300, R=80, K=20, density=0.05, seed=2)
    J5 = np.arange(0, 80, 4)
    lh5 = lam5[J5] * 1.01
    a = oracle.tensor_error_sparse(f5, lam5, J5, lh5)
    b = oracle.tensor_error(f5, lam5, J5, lh5)
    assert abs(a - b) <= 1e-10 * b
