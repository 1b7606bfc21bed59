"""Process-pool drivers of the FP64 oracle.

TEST INFRASTRUCTURE ONLY (used by the tests and the benchmark's CPU-baseline
leg).  Nothing here changes the oracle's arithmetic: each worker calls the
same plain functions of this package on a share of independent work (columns
of a TensorSketch, problems of a batch).  Workers are fresh interpreters
(spawn: no inherited GPU context or BLAS thread pool) with one BLAS thread
each; large inputs reach them through memory-mapped .npy files.
"""
from __future__ import annotations

import os
import time

import numpy as np

_BLAS_VARS = ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")


def default_workers() -> int:
    """Host cores to use: the scheduler affinity, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pool_map(fn, jobs, workers: int, chunksize: int = 1):
    import multiprocessing as mp
    old = {v: os.environ.get(v) for v in _BLAS_VARS}
    for v in old:
        os.environ[v] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(fn, jobs, chunksize=chunksize)
    finally:
        for v, val in old.items():
            if val is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = val


# --------------------------------------------------------------------------
# TensorSketch T M by direct circular convolution, columns split over workers
# --------------------------------------------------------------------------
def _ts_worker(job):
    import oracle
    fcols, lam, maps, Jlen = job
    return oracle.tensorsketch(fcols, lam, maps, Jlen)


def tensorsketch(factors, lam, maps, Jlen: int, workers: int = 0) -> np.ndarray:
    """oracle.tensorsketch over all R columns (Jlen x R); column r of T M
    depends only on column r of every factor, so column blocks are
    independent."""
    R = factors[0].shape[1]
    workers = workers or default_workers()
    bounds = np.linspace(0, R, min(R, 4 * workers) + 1).astype(int)
    jobs = [([np.asfortranarray(f[:, a:b]) for f in factors], np.asarray(lam)[a:b], maps, Jlen)
            for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    parts = _pool_map(_ts_worker, jobs, workers)
    return np.concatenate(parts, axis=1)


# --------------------------------------------------------------------------
# batched matrix IDs: every problem through oracle.matrix_id
# --------------------------------------------------------------------------
def _bf16_to_f64(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def _batch_id_worker(job):
    """Oracle IDs of problems [p0, p1): inputs from memory-mapped files, the
    oracle's J and P written into memory-mapped outputs."""
    import oracle
    d, p0, p1 = job
    m, n, a_off, p_off = d["m"], d["n"], d["a_off"], d["p_off"]
    A = np.load(d["A"], mmap_mode="r")
    G = _bf16_to_f64(np.load(d["G"]))
    Jo = np.load(d["Jo"], mmap_mode="r+")
    Po = np.load(d["Po"], mmap_mode="r+")
    keff = []
    for p in range(p0, p1):
        Ap = _bf16_to_f64(A[a_off[p]:a_off[p + 1]]).reshape(m[p], n[p])
        l1 = min(int(m[p]), d["l1max"])
        o = oracle.matrix_id(Ap, k=d["k"], l1=l1, seed=d["seed"], tag=p, G=G[:, :l1])
        Jo[p] = o["J"]
        Po[p_off[p]:p_off[p + 1]] = o["P"].reshape(-1)
        keff.append(o["k_eff"])
    Jo.flush()
    Po.flush()
    return keff


def _batch_res_worker(job):
    """Residual ratios ||A - A_J P||_F (the library's J, P) over the oracle's,
    for problems [p0, p1)."""
    import oracle
    d, p0, p1 = job
    m, n, a_off, p_off, k = d["m"], d["n"], d["a_off"], d["p_off"], d["k"]
    A = np.load(d["A"], mmap_mode="r")
    Jg = np.load(d["Jg"], mmap_mode="r")
    Pg = np.load(d["Pg"], mmap_mode="r")
    Jo = np.load(d["Jo"], mmap_mode="r")
    Po = np.load(d["Po"], mmap_mode="r")
    out = []
    for p in range(p0, p1):
        Ap = _bf16_to_f64(A[a_off[p]:a_off[p + 1]]).reshape(m[p], n[p])
        kg = int(np.sum(Jg[p] >= 0))
        ko = int(np.sum(Jo[p] >= 0))
        rg = oracle.residual_fro(Ap, Jg[p, :kg], np.asarray(Pg[p_off[p]:p_off[p + 1]]).reshape(k, n[p])[:kg])
        ro = oracle.residual_fro(Ap, Jo[p, :ko], np.asarray(Po[p_off[p]:p_off[p + 1]]).reshape(k, n[p])[:ko])
        out.append((rg, ro))
    return out


def batched_oracle(A_path: str, G_bits, m, n, k: int, l1max: int, seed: int, workdir: str, workers: int = 0):
    """Oracle IDs of every problem of a batch (A_p: BF16 bits back to back in
    the .npy at A_path; G: l x l1max BF16 bits).  Returns (Jo path, Po path,
    keff, wall seconds, workers): the oracle's outputs in memory-mapped files
    under workdir; the wall time covers the pool's IDs only."""
    workers = workers or default_workers()
    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    nprob = m.shape[0]
    a_off = np.concatenate([[0], np.cumsum(m * n)])
    p_off = np.concatenate([[0], np.cumsum(k * n)])
    os.makedirs(workdir, exist_ok=True)
    g_path = os.path.join(workdir, "G_bits.npy")
    np.save(g_path, np.asarray(G_bits))
    jo_path = os.path.join(workdir, "oracle_J.npy")
    po_path = os.path.join(workdir, "oracle_P.npy")
    np.lib.format.open_memmap(jo_path, mode="w+", dtype=np.int64, shape=(nprob, k))[:] = -1
    np.lib.format.open_memmap(po_path, mode="w+", dtype=np.float64, shape=(int(p_off[-1]),))
    d = dict(m=m, n=n, a_off=a_off, p_off=p_off, k=k, l1max=l1max, seed=seed, A=A_path, G=g_path,
             Jo=jo_path, Po=po_path)
    # small chunks, largest problems spread over the chunks by the shuffle of
    # the generator's draws; 8 chunks per worker for balance
    bounds = np.linspace(0, nprob, min(nprob, 8 * workers) + 1).astype(int)
    jobs = [(d, a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    t0 = time.perf_counter()
    parts = _pool_map(_batch_id_worker, jobs, workers)
    wall = time.perf_counter() - t0
    keff = np.concatenate([np.asarray(x, dtype=np.int64) for x in parts])
    return jo_path, po_path, keff, wall, workers


def batched_ratios(A_path: str, m, n, k: int, Jg, Pg, jo_path: str, po_path: str, workdir: str,
                   workers: int = 0):
    """Per-problem (library residual, oracle residual) for a batch whose
    library results are J (nprob x k) and P (flat, P_p k x n_p at k sum n_q)."""
    workers = workers or default_workers()
    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    nprob = m.shape[0]
    a_off = np.concatenate([[0], np.cumsum(m * n)])
    p_off = np.concatenate([[0], np.cumsum(k * n)])
    jg_path = os.path.join(workdir, "lib_J.npy")
    pg_path = os.path.join(workdir, "lib_P.npy")
    np.save(jg_path, np.asarray(Jg, dtype=np.int64))
    np.save(pg_path, np.asarray(Pg, dtype=np.float64))
    d = dict(m=m, n=n, a_off=a_off, p_off=p_off, k=k, A=A_path, Jg=jg_path, Pg=pg_path, Jo=jo_path, Po=po_path)
    bounds = np.linspace(0, nprob, min(nprob, 8 * workers) + 1).astype(int)
    jobs = [(d, a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    parts = _pool_map(_batch_res_worker, jobs, workers)
    return np.array([x for part in parts for x in part], dtype=np.float64)
