"""Seeded synthetic inputs for the interpolative-decomposition workloads.

This module only draws random inputs (numpy PCG64 streams keyed by seed and a
purpose tag) and lays them out; it holds none of the decomposition's
arithmetic.  Both the GPU library's tests/benchmark and the CPU oracle take
their inputs from here, so the two sides always see the same bytes.

The paper's datasets (SuiteSparse matrices, the Enron tensor) are not
available; these generators stand in for them with the shapes, value
distributions and structure of the five workloads:

  dense_lowrank ..... U diag(sigma) V^T (+ noise), U, V Gaussian-orthonormal
  csr_zipf .......... 1e6 x 2e4 CSR, Zipf(1.5) row counts + planted rank-50 part
  cp_tensor ......... CP tensor whose terms are perturbed copies of base terms
  batched_problems .. thousands of small low-rank problems stored in BF16
  gaussian .......... the N(0,1) matrix of the second sketch stage
"""
from __future__ import annotations

import numpy as np

# purpose tags for independent generator streams
_T_U, _T_V, _T_NOISE, _T_G, _T_CSR, _T_CP, _T_BATCH, _T_PERM, _T_SPARSE = range(1, 10)


def rng(seed: int, tag: int, *more: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag), *[int(x) for x in more]])


def orthonormal(m: int, r: int, g: np.random.Generator, dtype=np.float64) -> np.ndarray:
    """m x r with orthonormal columns: Q factor of an m x r Gaussian."""
    q, rr = np.linalg.qr(g.standard_normal((m, r)))
    # fix signs so the result is a deterministic function of the Gaussian
    q *= np.sign(np.diag(rr))[None, :]
    return q.astype(dtype, copy=False)


def dense_lowrank(m: int, n: int, sigma: np.ndarray, noise: float = 0.0, seed: int = 0,
                  dtype=np.float64) -> np.ndarray:
    """A = U diag(sigma) V^T + noise * N(0,1), row-major m x n.

    len(sigma) = r <= min(m, n); U (m x r), V (n x r) Gaussian-orthonormal.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    U = orthonormal(m, r, rng(seed, _T_U))
    V = orthonormal(n, r, rng(seed, _T_V))
    A = (U * sigma[None, :]) @ V.T
    del U
    if noise:
        A += noise * rng(seed, _T_NOISE).standard_normal((m, n))
    return np.ascontiguousarray(A.astype(dtype, copy=False))


def gaussian(l: int, q: int, seed: int = 0, tag: int = 0) -> np.ndarray:
    """l x q matrix of iid N(0,1) (the second-stage Gaussian sketch)."""
    return rng(seed, _T_G, tag).standard_normal((l, q))


def default_l1(m: int, k: int, p: int) -> int:
    """Intermediate CountSketch height: min(m, 4(k+p) rounded up to 16)."""
    t = 4 * (k + p)
    t = (t + 15) // 16 * 16
    return min(m, t)


# --------------------------------------------------------------------------
# workload 0: 2000 x 1000 dense, sigma = 1 (i <= 20), 1e-10 after, + 1e-12 noise
# --------------------------------------------------------------------------
def config0(seed: int = 0, exact: bool = False, m: int = 2000, n: int = 1000, k: int = 20):
    r = min(m, n)
    sigma = np.where(np.arange(1, r + 1) <= k, 1.0, 0.0 if exact else 1e-10)
    if exact:
        sigma = sigma[:k]
    A = dense_lowrank(m, n, sigma, 0.0 if exact else 1e-12, seed)
    return A


# --------------------------------------------------------------------------
# workload 1: 200000 x 2000, sigma_i = i^-2, stored FP32
# --------------------------------------------------------------------------
def config1(seed: int = 0, m: int = 200000, n: int = 2000) -> np.ndarray:
    r = min(m, n)
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -2.0
    return dense_lowrank(m, n, sigma, 0.0, seed, dtype=np.float32)


# --------------------------------------------------------------------------
# workload 2: CSR, Zipf(1.5) row counts truncated to 1..681 (mean ~20),
# uniform distinct columns, N(0,1) values, plus a planted part
# Gp (nplant random rows x 50, Gaussian) times C (50 x ncols random columns,
# 3 random +-1 entries per column).  Overlapping entries are summed.
# --------------------------------------------------------------------------
def zipf_counts(m: int, g: np.random.Generator, a: float = 1.5, kmax: int = 681) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** -a
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    return (np.searchsorted(cdf, g.random(m), side="right") + 1).astype(np.int64)


def csr_zipf(m: int = 1_000_000, n: int = 20_000, seed: int = 0, kmax: int = 681,
             rank: int = 50, nplant_rows: int = 10_000, nplant_cols: int = 1_000):
    """Returns (rowptr int64[m+1], colind int32[nnz] sorted per row, val f64[nnz])."""
    import scipy.sparse as sp
    g = rng(seed, _T_CSR)
    kmax = min(kmax, n)
    cnt = zipf_counts(m, g, kmax=kmax)
    nnz = int(cnt.sum())
    rows = np.repeat(np.arange(m, dtype=np.int64), cnt)
    cols = g.integers(0, n, size=nnz, dtype=np.int64)
    vals = g.standard_normal(nnz)
    # planted dense-by-sparse rank-`rank` block
    if rank > 0 and nplant_rows > 0 and nplant_cols > 0:
        prow = g.choice(m, size=min(nplant_rows, m), replace=False)
        pcol = g.choice(n, size=min(nplant_cols, n), replace=False)
        Gp = g.standard_normal((prow.shape[0], rank))
        C = np.zeros((rank, pcol.shape[0]))
        for j in range(pcol.shape[0]):
            sel = g.choice(rank, size=min(3, rank), replace=False)
            C[sel, j] = g.choice([-1.0, 1.0], size=sel.shape[0])
        B = Gp @ C
        rows = np.concatenate([rows, np.repeat(prow.astype(np.int64), pcol.shape[0])])
        cols = np.concatenate([cols, np.tile(pcol.astype(np.int64), prow.shape[0])])
        vals = np.concatenate([vals, B.ravel()])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


# --------------------------------------------------------------------------
# workload 3: CP tensor, order N, R terms as perturbed copies of `nbase`
# unit-norm Gaussian base terms; every factor vector perturbed by
# `pert` relative Gaussian noise and renormalised; lambda log-uniform.
# Factors are returned column-major (column r contiguous) as I_n x R arrays.
# --------------------------------------------------------------------------
def cp_tensor(dims=(2000, 2000, 2000), R: int = 2000, nbase: int = 50, pert: float = 1e-8,
              lam_range=(1e-2, 1e2), seed: int = 0):
    g = rng(seed, _T_CP)
    base_of = np.arange(R) % nbase
    base_of = base_of[g.permutation(R)]
    factors = []
    for In in dims:
        B = g.standard_normal((In, nbase))
        B /= np.linalg.norm(B, axis=0, keepdims=True)
        F = B[:, base_of] + pert * g.standard_normal((In, R)) / np.sqrt(In)
        F /= np.linalg.norm(F, axis=0, keepdims=True)
        factors.append(np.asfortranarray(F))
    lo, hi = np.log10(lam_range[0]), np.log10(lam_range[1])
    lam = 10.0 ** g.uniform(lo, hi, size=R)
    return factors, lam, base_of


def cp_sparse(N: int = 5, I: int = 10000, R: int = 2000, K: int = 200, density: float = 0.01, seed: int = 0,
              fmt: str = "dense"):
    """Sparse N-way CP tensor of the paper's synthetic tensor experiment (Section
    on tensor ID experiments, experiment 1): every factor column is a random
    sparse vector with the given density (nonzero positions uniform without
    replacement, N(0, 1) values), scaled to unit 2-norm as the CP form requires;
    lambda_r = 10^(-8 (r - 1) / R) for r <= K and 10^-8 beyond (the schedule
    as printed, with the paper's R = 10000 and K = 1000 scaled down to R, K).
    Factors are returned dense, I x R, column-major, or with fmt="csc" as
    (colptr int64[R+1], rowind int32 ascending within a column, val) triples
    holding the same entries (the same draws)."""
    g = rng(seed, _T_SPARSE)
    nnz = max(1, int(round(density * I)))
    factors = []
    for _ in range(N):
        if fmt == "csc":
            ri = np.empty(R * nnz, dtype=np.int32)
            va = np.empty(R * nnz, dtype=np.float64)
            for r in range(R):
                rows = g.choice(I, size=nnz, replace=False)
                v = g.standard_normal(nnz)
                o = np.argsort(rows)
                ri[r * nnz:(r + 1) * nnz] = rows[o]
                va[r * nnz:(r + 1) * nnz] = (v / np.linalg.norm(v))[o]
            factors.append((np.arange(0, (R + 1) * nnz, nnz, dtype=np.int64), ri, va))
            continue
        F = np.zeros((I, R), dtype=np.float64, order="F")
        for r in range(R):
            rows = g.choice(I, size=nnz, replace=False)
            v = g.standard_normal(nnz)
            F[rows, r] = v / np.linalg.norm(v)
        factors.append(F)
    r = np.arange(1, R + 1)
    lam = np.where(r <= K, 10.0 ** (-8.0 * (r - 1) / R), 1e-8)
    return factors, lam


# --------------------------------------------------------------------------
# workload 4: batched problems, m ~ logU[256, 4096], n ~ logU[128, 1024],
# sigma_i = exp(-i/8) (truncated at rank 128, where sigma_i < 1.2e-7 sigma_1,
# far below the BF16 rounding of the stored entries), stored BF16
# (float64 -> float32 RNE -> bfloat16 RNE).
# --------------------------------------------------------------------------
def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float64/float32 -> bfloat16 bit pattern (uint16), round-to-nearest-even
    via float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    return u.astype(np.uint16)


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def batched_shapes(nprob: int = 4096, seed: int = 0, mrange=(256, 4096), nrange=(128, 1024)):
    g = rng(seed, _T_BATCH)
    m = np.rint(np.exp(g.uniform(np.log(mrange[0]), np.log(mrange[1]), size=nprob))).astype(np.int64)
    n = np.rint(np.exp(g.uniform(np.log(nrange[0]), np.log(nrange[1]), size=nprob))).astype(np.int64)
    return m, n


def batched_problem(m: int, n: int, seed: int, p: int, rmax: int = 128) -> np.ndarray:
    r = min(m, n, rmax)
    sigma = np.exp(-np.arange(1, r + 1, dtype=np.float64) / 8.0)
    g = rng(seed, _T_BATCH, p + 1)
    U, _ = np.linalg.qr(g.standard_normal((m, r)))
    V, _ = np.linalg.qr(g.standard_normal((n, r)))
    return bf16_bits((U * sigma[None, :]) @ V.T)


def fullrank_perm(m: int, L: int, seed: int = 0, tag: int = 0):
    """Random inputs of the modified hash: a uniform permutation pi of [m] and
    iid uniform x_q in [L] (entries q < L are unused by the map)."""
    g = rng(seed, _T_PERM, tag)
    return g.permutation(m).astype(np.int64), g.integers(0, L, size=m, dtype=np.int32)


def _batched_worker(args):
    m, n, seed, p = args
    return batched_problem(m, n, seed, p)


def batched_inputs(nprob: int = 4096, seed: int = 0, workers: int = 0, mrange=(256, 4096), nrange=(128, 1024)):
    """All problems of a batch: (m, n, flat bf16 bits of A_0, A_1, ... back to
    back).  Problems are drawn independently (stream per problem), so the
    result does not depend on `workers` (a process pool; 0 = serial)."""
    m, n = batched_shapes(nprob, seed, mrange, nrange)
    jobs = [(int(m[p]), int(n[p]), seed, p) for p in range(nprob)]
    if workers and workers > 1:
        import multiprocessing as mp
        import os
        # fresh interpreters (a forked BLAS thread pool can deadlock), one
        # BLAS thread each
        old = {v: os.environ.get(v) for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
        for v in old:
            os.environ[v] = "1"
        try:
            with mp.get_context("spawn").Pool(workers) as pool:
                parts = pool.map(_batched_worker, jobs, chunksize=16)
        finally:
            for v, val in old.items():
                if val is None:
                    os.environ.pop(v, None)
                else:
                    os.environ[v] = val
    else:
        parts = [_batched_worker(j) for j in jobs]
    flat = np.concatenate([q.ravel() for q in parts])
    return m, n, flat
