"""FP64 CPU oracle for CountSketch / TensorSketch interpolative decomposition.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against (Malik & Becker, "Fast randomized matrix and
tensor interpolative decomposition using CountSketch").  It shares no code with
the GPU library and never imports it; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

The arithmetic lives in ``oracle.c`` (plain double-precision loops, increasing
summation order).  This module loads it with ctypes, marshals numpy arrays, and
holds the error evaluators (numpy, float64 / long double).

Paper map:
  * CountSketch S = Phi D and Y = S A ......... Section 1.3, Algorithm 2
  * Gaussian sketch of the sketch ............. Section 1.2.1 (Gaussian ID)
  * rank-K CPQR, R11^{-1} R12, P ............... Algorithm 1 (+ CPQR remark)
  * TensorSketch T, eq. for T A via (*) ........ Section 1.3, Algorithm 3
  * lambda_hat_k = lambda_{j_k} sum_r p_kr ...... Section 4, Algorithm 3
  * modified hash h~ = f o pi .................. Remark 2, Proposition 4
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None

c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_i32 = ctypes.c_int32
c_vp = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, no BLAS, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_mix64.restype = c_u64
        L.orc_mix64.argtypes = [c_u64]
        L.orc_stream_key.restype = c_u64
        L.orc_stream_key.argtypes = [c_u64, c_u64]
        L.orc_stream.argtypes = [c_u64, c_u64, c_i64, c_vp]
        L.orc_hash.argtypes = [c_u64, c_u64, c_i64, c_i64, c_vp, c_vp]
        L.orc_fullrank_hash.argtypes = [c_i64, c_i64, c_vp, c_vp, c_vp]
        L.orc_countsketch_dense.argtypes = [c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp]
        L.orc_countsketch_csr.argtypes = [c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]
        L.orc_gemm.argtypes = [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp]
        L.orc_cpqr_id.restype = c_i64
        L.orc_cpqr_id.argtypes = [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp]
        L.orc_tensorsketch.argtypes = [c_i32, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp]
        L.orc_lambda_hat.argtypes = [c_i64, c_i64, c_vp, c_vp, c_vp, c_vp]
        L.orc_gaussian.argtypes = [c_u64, c_u64, c_i64, c_vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(c_vp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# random maps
# --------------------------------------------------------------------------
def mix64(z: int) -> int:
    return int(lib().orc_mix64(c_u64(z & (2**64 - 1))))


def stream(seed: int, tag: int, m: int) -> np.ndarray:
    z = np.empty(m, dtype=np.uint64)
    lib().orc_stream(c_u64(seed), c_u64(tag), c_i64(m), _p(z))
    return z


def hash_maps(seed: int, tag: int, m: int, L: int):
    """CountSketch maps (h, D) of Section 1.3 from the seeded stream."""
    b = np.empty(m, dtype=np.int32)
    s = np.empty(m, dtype=np.int8)
    lib().orc_hash(c_u64(seed), c_u64(tag), c_i64(m), c_i64(L), _p(b), _p(s))
    return b, s


def fullrank_buckets(pi: np.ndarray, x: np.ndarray, L: int) -> np.ndarray:
    """Modified map h~(i) = f(pi(i)) of Remark 2 / Proposition 4."""
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.empty(pi.shape[0], dtype=np.int32)
    lib().orc_fullrank_hash(c_i64(pi.shape[0]), c_i64(L), _p(pi), _p(x), _p(out))
    return out


def gaussian(seed: int, tag: int, l: int, q: int) -> np.ndarray:
    """l x q N(0, 1) matrix from the stream (seed, tag | 2^63) by the
    Box-Muller transform of its uniforms (the generator a NULL G asks the
    library to run on the device)."""
    g = np.empty(l * q, dtype=np.float64)
    lib().orc_gaussian(c_u64(seed), c_u64(tag), c_i64(l * q), _p(g))
    return g.reshape(l, q)


# --------------------------------------------------------------------------
# sketches
# --------------------------------------------------------------------------
def countsketch_dense(A, bucket, sign, L: int) -> np.ndarray:
    A = _f64(A)
    m, n = A.shape
    b = np.ascontiguousarray(bucket, dtype=np.int32)
    s = np.ascontiguousarray(sign, dtype=np.int8)
    Y = np.empty((L, n), dtype=np.float64)
    lib().orc_countsketch_dense(c_i64(m), c_i64(n), _p(A), c_i64(n), _p(b), _p(s), c_i64(L), _p(Y))
    return Y


def countsketch_csr(rowptr, colind, val, n: int, bucket, sign, L: int) -> np.ndarray:
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = _f64(val)
    b = np.ascontiguousarray(bucket, dtype=np.int32)
    s = np.ascontiguousarray(sign, dtype=np.int8)
    m = rp.shape[0] - 1
    Y = np.empty((L, n), dtype=np.float64)
    lib().orc_countsketch_csr(c_i64(m), c_i64(n), _p(rp), _p(ci), _p(v), _p(b), _p(s), c_i64(L), _p(Y))
    return Y


def gemm(G, B) -> np.ndarray:
    G = _f64(G)
    B = _f64(B)
    l, q = G.shape
    q2, n = B.shape
    assert q == q2
    C = np.empty((l, n), dtype=np.float64)
    lib().orc_gemm(c_i64(l), c_i64(q), c_i64(n), _p(G), _p(B), _p(C))
    return C


def gaussian_id(A, k: int, Omega, blas: bool = False, trace: bool = False):
    """The Gaussian-sketch ID the paper compares with (Section 1.2.1): Y = Omega A,
    then Algorithm 1.  blas=True forms Y with numpy's FP64 matmul (a library
    primitive) for inputs too large for the plain triple loop."""
    if blas:
        Y = np.asarray(Omega, dtype=np.float64) @ np.asarray(A, dtype=np.float64)
    else:
        Y = gemm(Omega, A)
    J, P, keff, R, nu = cpqr_id(Y, k, trace=trace)
    return dict(Y=Y, J=J, P=P, k_eff=keff, nu=nu)


def cpqr_id(Y, k: int, trace: bool = False):
    """Algorithm 1 with column-pivoted QR.  Returns (J, P, k_eff, Rtop, nu)."""
    Y = _f64(Y)
    l, n = Y.shape
    J = np.full(k, -1, dtype=np.int64)
    P = np.zeros((k, n), dtype=np.float64)
    R = np.zeros((k, n), dtype=np.float64)
    nu = np.zeros((k, n), dtype=np.float64) if trace else None
    keff = lib().orc_cpqr_id(c_i64(l), c_i64(n), c_i64(k), _p(Y), _p(J), _p(P), _p(R),
                             _p(nu) if trace else None)
    return J, P, int(keff), R, nu


def tensorsketch(factors, lam, maps, Jlen: int, cols=None) -> np.ndarray:
    """T M of Algorithm 3 by direct circular convolution.

    factors: list of I_n x R arrays (any layout; converted to column-major).
    maps: list of (bucket, sign) per mode.  Returns Jlen x len(cols).
    """
    N = len(factors)
    R = factors[0].shape[1]
    fc = [np.asfortranarray(_f64(f)) for f in factors]  # column r contiguous
    dims = np.array([f.shape[0] for f in fc], dtype=np.int64)
    ld = dims.copy()
    fptr = (c_vp * N)(*[f.ctypes.data for f in fc])
    bs = [np.ascontiguousarray(m[0], dtype=np.int32) for m in maps]
    ss = [np.ascontiguousarray(m[1], dtype=np.int8) for m in maps]
    bptr = (c_vp * N)(*[b.ctypes.data for b in bs])
    sptr = (c_vp * N)(*[s.ctypes.data for s in ss])
    lam = _f64(lam)
    if cols is None:
        ncols = R
        cptr = None
        carr = None
    else:
        carr = np.ascontiguousarray(cols, dtype=np.int64)
        ncols = carr.shape[0]
        cptr = _p(carr)
    Yc = np.empty((ncols, Jlen), dtype=np.float64)
    lib().orc_tensorsketch(c_i32(N), _p(dims), _p(ld), c_i64(R), ctypes.cast(fptr, c_vp),
                           _p(lam), ctypes.cast(bptr, c_vp), ctypes.cast(sptr, c_vp),
                           c_i64(Jlen), cptr, c_i64(ncols), _p(Yc))
    return np.ascontiguousarray(Yc.T)


def lambda_hat(P, J, lam) -> np.ndarray:
    P = _f64(P)
    k, n = P.shape
    J = np.ascontiguousarray(J, dtype=np.int64)
    lam = _f64(lam)
    out = np.empty(k, dtype=np.float64)
    lib().orc_lambda_hat(c_i64(k), c_i64(n), _p(P), _p(J), _p(lam), _p(out))
    return out


# --------------------------------------------------------------------------
# pipelines (Algorithm 2 with an optional Gaussian second stage; Algorithm 3)
# --------------------------------------------------------------------------
def matrix_sketch(A=None, *, csr=None, n=None, l1: int, seed: int, tag: int = 0,
                  G=None, bucket=None, sign=None):
    """Y1 = S A (CountSketch to l1 rows) then Y = G Y1 when G is given."""
    m = A.shape[0] if A is not None else csr[0].shape[0] - 1
    if bucket is None:
        bucket, sign = hash_maps(seed, tag, m, l1)
    elif sign is None:
        _, sign = hash_maps(seed, tag, m, l1)
    if A is not None:
        Y1 = countsketch_dense(A, bucket, sign, l1)
    else:
        Y1 = countsketch_csr(csr[0], csr[1], csr[2], n, bucket, sign, l1)
    Y = gemm(G, Y1) if G is not None else Y1
    return Y1, Y


def matrix_id(A=None, *, csr=None, n=None, k: int, l1: int, seed: int, tag: int = 0,
              G=None, bucket=None, sign=None, trace: bool = False):
    Y1, Y = matrix_sketch(A, csr=csr, n=n, l1=l1, seed=seed, tag=tag, G=G,
                          bucket=bucket, sign=sign)
    J, P, keff, R, nu = cpqr_id(Y, k, trace=trace)
    return dict(Y1=Y1, Y=Y, J=J, P=P, k_eff=keff, R=R, nu=nu)


def adaptive_rank(R, J, keff: int, tol: float) -> int:
    """Fixed-accuracy stop of Algorithm 1's pivoted QR: the first step t >= 1
    with |r_tt| <= tol |r_11| (r_tt = R[t, J[t]]); keff when no step meets it."""
    d = np.abs(R[np.arange(keff), np.asarray(J[:keff])])
    for t in range(1, keff):
        if d[t] <= tol * d[0]:
            return t
    return keff


def matrix_id_adaptive(A, *, kmax: int, tol: float, l1: int, seed: int, tag: int = 0, G=None):
    """Fixed-accuracy ID: the rank-kmax factorisation decides the rank t by
    adaptive_rank, then the ID of rank t (the first t pivots are the same)."""
    Y1, Y = matrix_sketch(A, l1=l1, seed=seed, tag=tag, G=G)
    J, P, keff, R, nu = cpqr_id(Y, kmax)
    t = adaptive_rank(R, J, keff, tol)
    J2, P2, keff2, R2, _ = cpqr_id(Y, t)
    return dict(Y=Y, J=J2, P=P2, k_eff=keff2, rank=t, J_kmax=J, R_kmax=R)


def tensor_maps(seed: int, dims, Jlen: int):
    """Independent per-mode maps h_n, s_n: stream tag n+1 for mode n."""
    return [hash_maps(seed, n + 1, int(d), Jlen) for n, d in enumerate(dims)]


def tensor_id(factors, lam, *, k: int, Jlen: int, seed: int, G=None, trace: bool = False):
    """Algorithm 3; with G (l x Jlen) the Gaussian second stage G (T M) is
    factored instead of T M (Section 1.2.1's Gaussian sketch on the sketch)."""
    maps = tensor_maps(seed, [f.shape[0] for f in factors], Jlen)
    Y = tensorsketch(factors, lam, maps, Jlen)
    Yf = Y if G is None else gemm(G, Y)
    J, P, keff, R, nu = cpqr_id(Yf, k, trace=trace)
    lh = lambda_hat(P[:keff], J[:keff], lam)
    return dict(Y=Y, J=J, P=P, k_eff=keff, lambda_hat=lh, nu=nu, R=R)


# --------------------------------------------------------------------------
# evaluators (applied to any (J, P); float64 / long double)
# --------------------------------------------------------------------------
def residual_fro(A, J, P, chunk: int = 65536) -> float:
    """||A - A[:, J] P||_F / ||A||_F, A dense (rows processed in chunks)."""
    J = np.asarray(J)
    keep = J >= 0
    J = J[keep]
    P = _f64(P)[keep]
    num = 0.0
    den = 0.0
    for r0 in range(0, A.shape[0], chunk):
        a = np.asarray(A[r0:r0 + chunk], dtype=np.float64)
        e = a - a[:, J] @ P
        num += float(np.sum(e * e))
        den += float(np.sum(a * a))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def residual_fro_csr(rowptr, colind, val, n, J, P) -> float:
    """||A - A[:, J] P||_F / ||A||_F for A in CSR form, without forming the
    m x n difference."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(colind), np.asarray(rowptr)),
                      shape=(len(rowptr) - 1, n))
    # a CSR matrix with repeated (row, col) entries stands for their sum (the
    # definition CountSketch is applied to); ||A||_F needs the summed entries
    A.sum_duplicates()
    J = np.asarray(J)
    keep = J >= 0
    AJ = A[:, J[keep]]
    # ||A - AJ P||^2 = ||A||^2 - 2 <A, AJ P> + ||AJ P||^2, evaluated without
    # forming the m x n difference: <A, AJ P> = trace(P^T AJ^T A).
    Pk = _f64(P)[keep]
    nA2 = float(np.sum(A.data.astype(np.float64) ** 2))
    AJtA = (AJ.T @ A).toarray()                 # k x n
    cross = float(np.sum(AJtA * Pk))
    Gj = (AJ.T @ AJ).toarray()                   # k x k
    quad = float(np.sum((Gj @ Pk) * Pk))
    num = max(nA2 - 2.0 * cross + quad, 0.0)
    return float(np.sqrt(num / nA2))


def spectral_est(A, J, P, iters: int = 50, seed: int = 1) -> float:
    """Power-iteration estimate of ||A - A_J P||_2 / ||A||_2 (lower bound)."""
    rng = np.random.default_rng(seed)
    J = np.asarray(J)
    keep = J >= 0
    J = J[keep]
    P = _f64(P)[keep]
    A = np.asarray(A, dtype=np.float64)
    AJ = A[:, J]

    def op(x):
        return A @ x - AJ @ (P @ x)

    def opT(y):
        return A.T @ y - P.T @ (AJ.T @ y)

    def power(f, fT, n):
        x = rng.standard_normal(n)
        x /= np.linalg.norm(x)
        s = 0.0
        for _ in range(iters):
            y = f(x)
            z = fT(y)
            nz = np.linalg.norm(z)
            if nz == 0:
                return 0.0
            s = np.sqrt(nz)
            x = z / nz
        return float(s)

    e = power(op, opT, A.shape[1])
    a = power(lambda x: A @ x, lambda y: A.T @ y, A.shape[1])
    return e / a if a > 0 else e


def tensor_error(factors, lam, J, lhat) -> float:
    """||X - X_hat||_F / ||X||_F via the Gram identity (eq. for M^T M) in long
    double: X - X_hat = sum_r d_r X^(r) with d_r = lambda_r - [r = j_k] lambda_hat_k,
    so ||X - X_hat||^2 = d^T (G_1 * ... * G_N) d with G_n = A^(n)T A^(n)."""
    R = factors[0].shape[1]
    H = np.ones((R, R), dtype=np.longdouble)
    for f in factors:
        fl = np.asarray(f, dtype=np.longdouble)
        H *= fl.T @ fl
    lam_l = np.asarray(lam, dtype=np.longdouble)
    d = lam_l.copy()
    for t, j in enumerate(np.asarray(J)):
        if j >= 0:
            d[j] -= np.longdouble(lhat[t])
    num = d @ (H @ d)
    den = lam_l @ (H @ lam_l)
    return float(np.sqrt(max(num, 0) / den))


def tensor_error_sampled(factors, lam, J, lhat, nsamp: int = 200000, seed: int = 7, entries=None) -> float:
    """||X - X_hat||_F / ||X||_F estimated from uniformly sampled entries
    (i_1, ..., i_N) of the CP tensors (def-X-tensor): each sampled entry of
    X - X_hat is sum_r d_r prod_n A^(n)[i_n, r] with d_r = lambda_r -
    [r = j_k] lambda_hat_k, evaluated directly (no Gram cancellation), and the
    ratio of the two sums of squares estimates the ratio of the norms.  With
    `entries` (an nsamp x N index array) those entries are used instead; all
    entries of a small tensor give the exact value."""
    N = len(factors)
    R = factors[0].shape[1]
    lam = np.asarray(lam, dtype=np.float64)
    d = lam.copy()
    for t, j in enumerate(np.asarray(J)):
        if j >= 0:
            d[j] -= float(lhat[t])
    if entries is None:
        g = np.random.default_rng(seed)
        entries = np.stack([g.integers(0, f.shape[0], size=nsamp) for f in factors], axis=1)
    num = 0.0
    den = 0.0
    for c0 in range(0, entries.shape[0], 8192):
        idx = entries[c0:c0 + 8192]
        prod = np.ones((idx.shape[0], R), dtype=np.float64)
        for n_, f in enumerate(factors):
            prod *= np.asarray(f)[idx[:, n_], :]
        e = prod @ d
        x = prod @ lam
        num += float(e @ e)
        den += float(x @ x)
    return float(np.sqrt(num / den))


def _gram_sparse_ld(F) -> np.ndarray:
    """A^T A of a sparse-column factor in long double, summing v_ir v_is over
    the rows i where both columns are nonzero (row by row, pairs within a row)."""
    F = np.asarray(F, dtype=np.float64)
    R = F.shape[1]
    G = np.zeros((R, R), dtype=np.longdouble)
    rows, cols = np.nonzero(F)
    order = np.argsort(rows, kind="stable")
    rows, cols = rows[order], cols[order]
    vals = F[rows, cols].astype(np.longdouble)
    starts = np.flatnonzero(np.r_[True, rows[1:] != rows[:-1]])
    ends = np.r_[starts[1:], rows.shape[0]]
    # group rows by their nonzero count, so each group is one vectorised outer product
    cnt = ends - starts
    for c in np.unique(cnt):
        sel = starts[cnt == c]
        idx = sel[:, None] + np.arange(c)[None, :]
        cc = cols[idx]
        vv = vals[idx]
        np.add.at(G, (np.repeat(cc, c, axis=1).ravel(), np.tile(cc, (1, c)).ravel()),
                  (vv[:, :, None] * vv[:, None, :]).reshape(-1))
    return G


def tensor_error_sparse(factors, lam, J, lhat) -> float:
    """tensor_error (the Gram identity in long double) for factors whose
    columns are sparse: each G_n = A^(n)T A^(n) is summed over the nonzeros of
    the factor only, so the cost follows the number of nonzero pairs per row
    instead of I_n R^2."""
    R = factors[0].shape[1]
    H = np.ones((R, R), dtype=np.longdouble)
    for f in factors:
        H *= _gram_sparse_ld(f)
    lam_l = np.asarray(lam, dtype=np.longdouble)
    d = lam_l.copy()
    for t, j in enumerate(np.asarray(J)):
        if j >= 0:
            d[j] -= np.longdouble(lhat[t])
    num = d @ (H @ d)
    den = lam_l @ (H @ lam_l)
    return float(np.sqrt(max(num, 0) / den))
