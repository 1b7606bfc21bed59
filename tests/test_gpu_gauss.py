"""The Gaussian G drawn on the device when the caller passes none, against the
oracle's generator (the same stream and Box-Muller transform, host libm):
through the projection of the matrix path (FP64 and FP32), the tensor path's
second stage, and the batched path (BF16 G)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ids = pytest.importorskip("paper_1901_10559_amd")

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_drawn_g_projection_f64():
    # integer-valued A and l1 = m with the identity-like hash is not needed:
    # Y = G Y1, Y1 from the oracle, so G's effect is checked entrywise
    m, n, l1, l, seed, tag = 3000, 257, 160, 40, 9, 3
    A = np.random.default_rng(1).standard_normal((m, n))
    Y = ids.id_sketch(dev(A), l1, l, seed=seed, tag=tag).cpu().numpy()
    b, s = oracle.hash_maps(seed, tag, m, l1)
    Y1 = oracle.countsketch_dense(A, b, s, l1)
    Go = oracle.gaussian(seed, tag, l, l1)
    Yo = oracle.gemm(Go, Y1)
    # host and device libm differ by a few ulps in log / cos
    assert np.max(np.abs(Y - Yo)) <= 1e-12 * np.max(np.abs(Yo))


def test_drawn_g_matrix_id_parity():
    sig = np.where(np.arange(1, 301) <= 12, 1.0, 1e-9)
    A = synth.dense_lowrank(600, 300, sig, 1e-12, seed=5)
    r = ids.matrix_id(dev(A), 12, 96, 22, seed=5, tag=1, check=True)
    o = oracle.matrix_id(A, k=12, l1=96, seed=5, tag=1, G=oracle.gaussian(5, 1, 22, 96))
    assert np.array_equal(r["J"].cpu().numpy(), o["J"])
    assert np.linalg.norm(r["P"].cpu().numpy() - o["P"]) <= 1e-10 * np.linalg.norm(o["P"])


def test_drawn_g_f32_projection():
    m, n, l1, l = 5000, 300, 480, 120
    A = np.random.default_rng(2).standard_normal((m, n)).astype(np.float32)
    Y = ids.id_sketch(dev(A), l1, l, seed=0, acc=ids.F32).cpu().numpy()
    b, s = oracle.hash_maps(0, 0, m, l1)
    Yo = oracle.gemm(oracle.gaussian(0, 0, l, l1).astype(np.float32).astype(np.float64),
                     oracle.countsketch_dense(A, b, s, l1))
    # FP32 sketch (a bucket of ~10 rows) and FP32 MFMA projection over 480 terms
    assert np.max(np.abs(Y - Yo)) <= 1e-4 * np.max(np.abs(Yo))


def test_drawn_g_tensor_projected():
    factors, lam, _ = synth.cp_tensor(dims=(40, 30, 20), R=60, nbase=6, pert=1e-6, seed=6)
    ft = [dev(np.asarray(f).T).t() for f in factors]
    r = ids.tensor_id(ft, dev(lam), 6, 64, seed=6, l=12, check=True)
    o = oracle.tensor_id(factors, lam, k=6, Jlen=64, seed=6, G=oracle.gaussian(6, 0, 12, 64))
    assert np.array_equal(r["J"].cpu().numpy(), o["J"])
    lh = r["lambda_hat"].cpu().numpy()
    assert np.max(np.abs(lh - o["lambda_hat"]) / np.abs(o["lambda_hat"])) <= 1e-10


def test_drawn_g_batched_matches_host_g():
    # the batch with G drawn on the device equals the batch given the host
    # generator's G rounded the same way (FP64 -> FP32 -> BF16)
    nprob, k, l, l1max = 40, 30, 40, 128
    m, n, flat = synth.batched_inputs(nprob, seed=3, mrange=(64, 900), nrange=(40, 700))
    At = dev(flat.view(np.int16)).view(torch.bfloat16)
    Gh = synth.bf16_bits(oracle.gaussian(3, 0, l, l1max))
    plan = ids.batched_plan(m, n, k, l, l1max)
    a = ids.id_batched(plan, At, None, seed=3)
    b = ids.id_batched(plan, At, dev(Gh.view(np.int16)).view(torch.bfloat16), seed=3)
    torch.cuda.synchronize()
    assert np.array_equal(a["J"].cpu().numpy(), b["J"].cpu().numpy())
    assert np.array_equal(a["P"].cpu().numpy(), b["P"].cpu().numpy())
