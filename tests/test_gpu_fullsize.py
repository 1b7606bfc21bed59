"""Full-size GPU checks, in the launch configurations the benchmark times:
dense 200000 x 2000 (FP32), CSR 1e6 x 2e4 with ~3e7 stored entries (FP64),
the 2000^3 CP tensor with 2000 terms and J = 4096 (FP64), and batches of the
mixed-precision problems.  Each compares against the FP64 oracle on outputs it
can compute (whole sketches, sampled columns) or on properties that hold at any
size; the tensor ID and the whole 4096-problem batch are compared with the
oracle's complete result (its work spread over a process pool)."""
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


def tie_aware_J(Jg, Jo, nu, rel=1e-12):
    if np.array_equal(Jg, Jo):
        return True
    t = int(np.argmax(Jg != Jo))
    row = np.sort(nu[t][nu[t] >= 0])[::-1]
    return len(row) > 1 and (row[0] - row[1]) <= rel * row[0]


def test_dense_countsketch_200000x2000_f32():
    m, n, l1 = 200_000, 2000, 480
    A = np.random.default_rng(11).standard_normal((m, n), dtype=np.float32)
    Y = ids.id_sketch(dev(A), l1, seed=0, acc=ids.F32).cpu().numpy()
    b, s = oracle.hash_maps(0, 0, m, l1)
    Yo = oracle.countsketch_dense(A, b, s, l1)
    cnt = np.bincount(b, minlength=l1)
    # FP32 accumulation of cnt[b] terms: |err| <= cnt * 2^-24 * sum |terms|
    absY = oracle.countsketch_dense(np.abs(A), b, np.ones_like(s), l1)
    bound = (cnt[:, None] * 2.0 ** -24) * absY
    assert np.all(np.abs(Y - Yo) <= bound)


def test_dense_matrix_id_200000x2000_f32_residual():
    A = synth.config1()                      # U diag(i^-2) V^T, FP32
    l1 = synth.default_l1(A.shape[0], 100, 20)
    G = synth.gaussian(120, l1, seed=0)
    r = ids.matrix_id(dev(A), 100, l1, 120, seed=0, G=dev(G.astype(np.float32)), acc=ids.F32)
    Jg = r["J"].cpu().numpy()
    Pg = r["P"].cpu().numpy()
    assert int(r["k_eff"].item()) == 100 and len(set(Jg.tolist())) == 100
    assert np.array_equal(Pg[:, Jg], np.eye(100))
    A64 = A.astype(np.float64)
    o = oracle.matrix_id(A64, k=100, l1=l1, seed=0, G=G.astype(np.float32).astype(np.float64))
    rg = oracle.residual_fro(A64, Jg, Pg)
    ro = oracle.residual_fro(A64, o["J"], o["P"])
    # FP32 sketch and projection against the FP64 oracle on the same FP32 input
    assert rg <= 1.05 * ro


def test_csr_matrix_id_1e6x2e4_fp64_parity():
    rp, ci, v = synth.csr_zipf()             # ~3e7 stored entries
    n, k, l1, l = 20_000, 50, 240, 60
    G = synth.gaussian(l, l1, seed=0)
    Ad = (dev(rp), dev(ci), dev(v), n)
    Y1 = ids.id_sketch(Ad, l1, seed=0).cpu().numpy()
    b, s = oracle.hash_maps(0, 0, rp.shape[0] - 1, l1)
    Y1o = oracle.countsketch_csr(rp, ci, v, n, b, s, l1)
    absY = oracle.countsketch_csr(rp, ci, np.abs(v), n, b, np.ones_like(s), l1)
    assert np.all(np.abs(Y1 - Y1o) <= 4096 * 2.0 ** -52 * absY)
    r = ids.matrix_id(Ad, k, l1, l, seed=0, G=dev(G))
    o = oracle.matrix_id(csr=(rp, ci, v), n=n, k=k, l1=l1, seed=0, G=G, trace=True)
    Jg = r["J"].cpu().numpy()
    Pg = r["P"].cpu().numpy()
    assert tie_aware_J(Jg, o["J"], o["nu"])
    if np.array_equal(Jg, o["J"]):
        assert np.linalg.norm(Pg - o["P"]) <= 1e-10 * np.linalg.norm(o["P"])
    assert np.array_equal(Pg[:, Jg], np.eye(k))


def test_csr_ordered_sketch_1e6x2e4_bit_exact():
    # IDS_DETERMINISTIC at the CSR workload's full size (240 buckets x 20
    # column ranges x 17 row chunks = 81600 counters, ten tiles of the counter
    # scan): the sketch equals the oracle's row-order sums bit for bit
    rp, ci, v = synth.csr_zipf()
    A = (dev(rp), dev(ci), dev(v), 20000)
    print("ordered CSR sketch 1e6 x 2e4, l1 = 240", flush=True)
    Y = ids.id_sketch(A, 240, seed=0, deterministic=True).cpu().numpy()
    b, s = oracle.hash_maps(0, 0, rp.size - 1, 240)
    assert np.array_equal(Y, oracle.countsketch_csr(rp, ci, v, 20000, b, s, 240))


def test_tensor_id_2000cubed_R2000_J4096():
    # Algorithm 3 at full size against the oracle's Algorithm 3: the whole
    # 4096 x 2000 sketch (direct circular convolutions, columns over a process
    # pool), its pivoted QR, J (tie-aware), P and lambda_hat
    from oracle import pool
    factors, lam, base_of = synth.cp_tensor()   # 3 x (2000 x 2000), 50 bases, 1e-8 perturbation
    Jlen, k = 4096, 50
    ft = [dev(np.asarray(f).T).t() for f in factors]
    r = ids.tensor_id(ft, dev(lam), k, Jlen, seed=0, return_Y=True)
    torch.cuda.synchronize()
    assert ids.check_status(r["status"]) == {ids.OK}
    J = r["J"].cpu().numpy()
    P = r["P"].cpu().numpy()
    lh = r["lambda_hat"].cpu().numpy()
    Yg = r["Y"].cpu().numpy()
    assert int(r["k_eff"].item()) == k
    maps = oracle.tensor_maps(0, [2000, 2000, 2000], Jlen)
    print("oracle TensorSketch 4096 x 2000 (process pool)", flush=True)
    Yo = pool.tensorsketch(factors, lam, maps, Jlen)
    # FFT against direct convolution: rounding level per column
    scale = np.linalg.norm(Yo, axis=0, keepdims=True)
    assert np.max(np.abs(Yg - Yo) / scale) <= 1e-13
    print("oracle CPQR of the 4096 x 2000 sketch", flush=True)
    Jo, Po, ko, _, nu = oracle.cpqr_id(Yo, k, trace=True)
    assert ko == k
    assert tie_aware_J(J, Jo, nu)
    if np.array_equal(J, Jo):
        assert np.linalg.norm(P - Po) <= 1e-10 * np.linalg.norm(Po)
        lo = oracle.lambda_hat(Po, Jo, lam)
        assert np.max(np.abs(lh - lo) / np.abs(lo)) <= 1e-10
    # properties at full size: one kept term per base cluster, P[:, J] = I,
    # lambda_hat = the cluster's lambda sum up to the 1e-8 perturbation
    assert np.array_equal(P[:, J], np.eye(k))
    assert len(set(base_of[J].tolist())) == k
    for t in range(k):
        grp = lam[base_of == base_of[J[t]]].sum()
        assert abs(lh[t] - grp) <= 1e-6 * abs(grp)


def test_tensor_id_2000cubed_projected_l60():
    factors, lam, base_of = synth.cp_tensor()
    Jlen, k, l = 4096, 50, 60
    G = synth.gaussian(l, Jlen, seed=0)
    ft = [dev(np.asarray(f).T).t() for f in factors]
    r = ids.tensor_id(ft, dev(lam), k, Jlen, seed=0, l=l, G=dev(G))
    J = r["J"].cpu().numpy()
    P = r["P"].cpu().numpy()
    lh = r["lambda_hat"].cpu().numpy()
    assert int(r["k_eff"].item()) == k
    assert np.array_equal(P[:, J], np.eye(k))
    assert len(set(base_of[J].tolist())) == k
    for t in range(k):
        grp = lam[base_of == base_of[J[t]]].sum()
        assert abs(lh[t] - grp) <= 1e-6 * abs(grp)


def test_sparse5way_I10000_R2000_projected():
    # the sparse 5-way workload in the launch configuration the benchmark
    # times: sampled sketch columns against the direct convolution, and the
    # properties of the ID at full size
    factors, lam = synth.cp_sparse(N=5, I=10000, R=2000, K=200, density=0.01, seed=0)
    Jlen, k, l = 2048, 200, 210
    G = synth.gaussian(l, Jlen, seed=0)
    ft = [dev(np.asarray(f).T).t() for f in factors]
    r = ids.tensor_id(ft, dev(lam), k, Jlen, seed=0, l=l, G=dev(G), return_Y=True)
    torch.cuda.synchronize()
    cols = np.linspace(0, 1999, 10).astype(np.int64)
    Yo = oracle.tensorsketch(factors, lam, oracle.tensor_maps(0, [10000] * 5, Jlen), Jlen, cols=cols)
    Yg = r["Y"][:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    scale = np.linalg.norm(Yo, axis=0, keepdims=True)
    assert np.max(np.abs(Yg - Yo) / scale) <= 1e-13
    J = r["J"].cpu().numpy()
    P = r["P"].cpu().numpy()
    assert int(r["k_eff"].item()) == k
    assert np.array_equal(P[:, J], np.eye(k))


def test_batched_full_batch_4096(tmp_path):
    # the whole benchmark batch (4096 problems, seed 0) in its launch
    # configuration; every problem's residual against the FP64 oracle's on the
    # same BF16 inputs and BF16 G (oracle IDs over a process pool)
    from oracle import pool
    nprob, k, l, l1max = 4096, 111, 121, 496
    print("generating the 4096-problem batch", flush=True)
    m, n, flat = synth.batched_inputs(nprob, seed=0, workers=pool.default_workers())
    Gb = synth.bf16_bits(synth.gaussian(l, l1max, seed=0))
    plan = ids.batched_plan(m, n, k, l, l1max)
    At = dev(flat.view(np.int16)).view(torch.bfloat16)
    Gt = dev(Gb.view(np.int16)).view(torch.bfloat16)
    out = ids.id_batched(plan, At, Gt, seed=0)
    torch.cuda.synchronize()
    del At
    J = out["J"].cpu().numpy()
    P = out["P"].cpu().numpy()
    keff = out["k_eff"].cpu().numpy()
    assert np.all(keff == k)
    assert set(out["status"].cpu().numpy().tolist()) == {ids.OK}
    for p in range(nprob):
        Pp = P[plan.p_off[p]:plan.p_off[p + 1]].reshape(k, n[p])
        assert np.array_equal(Pp[:, J[p]], np.eye(k))
    a_path = str(tmp_path / "A_bits.npy")
    np.save(a_path, flat)
    del flat
    print("oracle IDs of 4096 problems (process pool)", flush=True)
    jo, po, ko, wall, workers = pool.batched_oracle(a_path, Gb, m, n, k, l1max, 0, str(tmp_path))
    assert np.all(ko == k)
    res = pool.batched_ratios(a_path, m, n, k, J, P, jo, po, str(tmp_path))
    ratio = res[:, 0] / res[:, 1]
    print(f"residual ratio over {nprob}: median {np.median(ratio):.6f} max {ratio.max():.6f} "
          f"(oracle {wall:.1f} s on {workers} processes)", flush=True)
    assert ratio.max() <= 2.0


def test_sparse5way_paper_scale_I10000_R10000_K1000():
    # the paper's synthetic tensor experiment at its own size (R = 10000 terms,
    # target rank 1000; Section on tensor ID experiments, experiment 1) with
    # CSC factors and J = 1024: sampled sketch columns against the direct
    # convolution, then the oracle's Algorithm 1 on the library's sketch
    # against the library's pivots, P and lambda_hat (this shape takes the
    # column-steps QR and the blocked solve)
    N, I, R, K, Jlen = 5, 10000, 10000, 1000, 1024
    fac, lam = synth.cp_sparse(N=N, I=I, R=R, K=K, density=0.01, seed=0, fmt="csc")
    d = [(dev(cp), dev(ri), dev(va), I) for cp, ri, va in fac]
    print("paper-scale sparse 5-way tensor_id_csc R=10000 k=1000 J=1024", flush=True)
    r = ids.tensor_id_csc(d, dev(lam), K, Jlen, seed=0, return_Y=True, check=True)
    Yg = r["Y"].cpu().numpy()
    cols = np.linspace(0, R - 1, 8).astype(np.int64)
    dense = []
    for cp, ri, va in fac:
        F = np.zeros((I, cols.size))
        for q, c in enumerate(cols):
            F[ri[cp[c]:cp[c + 1]], q] = va[cp[c]:cp[c + 1]]
        dense.append(F)
    Yo = oracle.tensorsketch(dense, lam[cols], oracle.tensor_maps(0, [I] * N, Jlen), Jlen)
    scale = np.linalg.norm(Yo, axis=0, keepdims=True)
    assert np.max(np.abs(Yg[:, cols] - Yo) / scale) <= 1e-13
    print("paper-scale: oracle Algorithm 1 on the 1024 x 10000 sketch", flush=True)
    Jo, Po, ko, _, nu = oracle.cpqr_id(Yg, K, trace=True)
    assert int(r["k_eff"].item()) == ko == K
    Jg = r["J"].cpu().numpy()
    if np.array_equal(Jg, Jo):
        Pg = r["P"].cpu().numpy()
        assert np.linalg.norm(Pg - Po) <= 1e-10 * np.linalg.norm(Po)
        assert np.array_equal(Pg[:, Jg], np.eye(K))
        lo = oracle.lambda_hat(Po, Jo, lam)
        assert np.max(np.abs(r["lambda_hat"].cpu().numpy() - lo) / np.abs(lo)) <= 1e-10
    else:
        t = int(np.argmax(Jg != Jo))
        row = np.sort(nu[t][nu[t] >= 0])[::-1]
        assert len(row) > 1 and row[0] - row[1] <= 1e-12 * row[0], (t, row[:2])
