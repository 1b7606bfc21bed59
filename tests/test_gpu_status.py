"""Device status words (IDS_OK, IDS_ERANKDEF, IDS_ENONFINITE, IDS_ETIMEOUT)
and the introspection of the select plan.  The timeout path is forced from
the host (ids_set_wait_limit(0) raises the give-up flag before the
factorisation starts); every kernel still runs its bounded loops to the end."""
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


def lowrank(m=600, n=300, k=12, seed=5):
    sig = np.where(np.arange(1, n + 1) <= k, 1.0, 1e-9)
    return synth.dense_lowrank(m, n, sig, 1e-12, seed=seed)


def test_status_ok_and_rankdef():
    A = lowrank()
    r = ids.matrix_id(dev(A), 12, 96, 22, seed=5, G=dev(synth.gaussian(22, 96, seed=5)), check=True)
    assert int(r["status"].item()) == ids.OK
    J, P, keff = ids.id_select(dev(np.zeros((30, 100))), 20, status=(st := torch.full((1,), -1, dtype=torch.int32,
                                                                                      device=DEV)))
    assert ids.check_status(st) == {ids.ERANKDEF}
    assert int(keff.item()) == 0


@pytest.mark.parametrize("l,n,k", [(120, 2000, 100), (700, 400, 30)])
def test_forced_timeout_is_reported(l, n, k):
    g = np.random.default_rng(3)
    Y = dev(g.standard_normal((l, n)))
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    print(f"forced timeout: l={l} n={n} k={k} {ids.select_plan_info(l, n, k)}", flush=True)
    ids.set_wait_limit(0)
    try:
        J, P, keff = ids.id_select(Y, k, status=st)
        torch.cuda.synchronize()
    finally:
        ids.set_wait_limit(None)
    assert int(st.item()) == ids.ETIMEOUT
    assert int(keff.item()) == -1
    with pytest.raises(ids.IdsError, match="IDS_ETIMEOUT"):
        ids.check_status(st)
    # the default limit is back: the same call completes and matches the oracle
    J, P, keff = ids.id_select(Y, k, status=st)
    assert ids.check_status(st) == {ids.OK}
    Jo, Po, ko, _, _ = oracle.cpqr_id(Y.cpu().numpy(), k)
    assert int(keff.item()) == ko == k
    assert np.array_equal(J.cpu().numpy(), Jo)


def test_nonfinite_reported_by_sketch_check_and_select():
    A = lowrank()
    A[17, 4] = np.nan
    chk = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    Y = ids.id_sketch(dev(A), 96, 22, seed=5, G=dev(synth.gaussian(22, 96, seed=5)), check_finite=chk)
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ids.id_select(Y, 12, status=st)
    torch.cuda.synchronize()
    assert int(chk.item()) == ids.ENONFINITE
    assert int(st.item()) == ids.ENONFINITE
    with pytest.raises(ids.IdsError, match="IDS_ENONFINITE"):
        ids.check_status(st)
    # the same flag on clean data reports IDS_OK
    Y = ids.id_sketch(dev(lowrank()), 96, 22, seed=5, G=dev(synth.gaussian(22, 96, seed=5)), check_finite=chk)
    torch.cuda.synchronize()
    assert int(chk.item()) == ids.OK


def test_row_band_nonfinite():
    g = np.random.default_rng(4)
    Y = g.standard_normal((700, 400))
    Y[5, 123] = np.inf
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ids.id_select(dev(Y), 30, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == ids.ENONFINITE


def test_batched_status_per_problem():
    m = np.array([300, 400, 500])
    n = np.array([200, 150, 300])
    g = np.random.default_rng(8)
    blocks = [g.standard_normal((mi, ni)) for mi, ni in zip(m, n)]
    blocks[1][3, 7] = np.nan
    bits = np.concatenate([synth.bf16_bits(b).reshape(-1) for b in blocks])
    At = dev(bits.view(np.int16)).view(torch.bfloat16)
    Gt = dev(synth.bf16_bits(synth.gaussian(40, 64, seed=1)).view(np.int16)).view(torch.bfloat16)
    plan = ids.batched_plan(m, n, 30, 40, 64)
    out = ids.id_batched(plan, At, Gt, seed=0)
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [ids.OK, ids.ENONFINITE, ids.OK]


# ---------------------------------------------------------------------------
# the owner-published candidate exchange (more than 256 publishers per step).
# On MI355X only the 512-row band kernel (257 <= l <= 512) has more than 256
# co-resident workgroups (two per CU); the grouped-lane kernels (l <= 256)
# and the longer bands fit one per CU, so they always take the speculative
# exchange (their owner-mode instances serve devices with more residency).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("l,n,k", [(300, 5000, 40), (500, 8000, 30), (257, 8190, 64)])
def test_select_owner_exchange(l, n, k):
    info = ids.select_plan_info(l, n, k)
    print(f"owner exchange: l={l} n={n} k={k} {info}", flush=True)
    assert info["exchange"] == "owner" and info["publishers"] > 256
    g = np.random.default_rng(l + n + k)
    Y = g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    J, P, keff = ids.id_select(dev(Y), k, status=st)
    Jo, Po, ko, _, nu = oracle.cpqr_id(Y, k, trace=True)
    assert ids.check_status(st) == {ids.OK}
    assert int(keff.item()) == ko == k
    Jg = J.cpu().numpy()
    assert np.array_equal(Jg, Jo)
    assert np.linalg.norm(P.cpu().numpy() - Po) <= 1e-10 * np.linalg.norm(Po)


# ---------------------------------------------------------------------------
# dense CountSketch beyond the one-workgroup plan (m > 16384): the fused plan
# (L <= 1024) and the plan with a separate offsets pass (L > 1024) keep rows
# of a bucket in increasing order, so FP64 sums are bitwise the oracle's
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,L", [(40000, 64, 480), (40000, 64, 2048), (70001, 9, 1025)])
def test_countsketch_f64_bit_exact_large_plans(m, n, L):
    g = np.random.default_rng(m + L)
    A = g.standard_normal((m, n))
    Y = ids.id_sketch(dev(A), L, seed=7).cpu().numpy()
    b, s = oracle.hash_maps(7, 0, m, L)
    assert np.array_equal(Y, oracle.countsketch_dense(A, b, s, L))


def test_stream_read_checksum():
    # the measurement utility reads every word: XOR of all 32-bit words
    g = np.random.default_rng(9)
    words = g.integers(0, 2**32, size=(1 << 20) + 12, dtype=np.uint64).astype(np.uint32)
    buf = dev(words.view(np.int32))
    chk = torch.zeros(1, dtype=torch.int32, device=DEV)
    ids.stream_read(buf, chk)
    torch.cuda.synchronize()
    assert int(chk.item()) & 0xFFFFFFFF == int(np.bitwise_xor.reduce(words))


# ---------------------------------------------------------------------------
# every value of the tuned knobs gives the oracle's results
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("l,n,k", [(30, 1000, 20), (60, 20000, 50), (120, 2000, 100), (120, 9000, 60),
                                   (250, 800, 201), (250, 4500, 100)])
def test_select_four_wave_variant(l, n, k):
    lb = "l32" if l <= 32 else "l64" if l <= 64 else "l128" if l <= 128 else "l256"
    nb = "n1k" if n <= 1024 else "n4k" if n <= 4096 else "n16k" if n <= 16384 else "ninf"
    key = f"select.gl.{lb}.{nb}"
    g = np.random.default_rng(l + n + k + 1)
    Y = g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]
    ids.tune_set(key, 1)
    try:
        info = ids.select_plan_info(l, n, k)
        print(f"4-wave variant: l={l} n={n} k={k} {info}", flush=True)
        st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        J, P, keff = ids.id_select(dev(Y), k, status=st)
        torch.cuda.synchronize()
    finally:
        ids.tune_set(key, None)
    Jo, Po, ko, _, nu = oracle.cpqr_id(Y, k, trace=True)
    assert ids.check_status(st) == {ids.OK}
    assert int(keff.item()) == ko == k
    assert np.array_equal(J.cpu().numpy(), Jo)
    assert np.linalg.norm(P.cpu().numpy() - Po) <= 1e-10 * np.linalg.norm(Po)


@pytest.mark.parametrize("key,value,l,n,k", [("trsm.k32", 1, 30, 700, 20), ("trsm.k32", 2, 30, 700, 20),
                                             ("trsm.k32", 4, 30, 700, 20), ("trsm.k64", 2, 60, 900, 50),
                                             ("trsm.k64", 4, 60, 900, 50), ("trsm.k128", 4, 120, 1500, 100),
                                             ("trsm.k128", 8, 120, 1500, 100)])
def test_solve_variants(key, value, l, n, k):
    # the lane-per-column solves (trsm.mfma = 0), each lane count
    g = np.random.default_rng(k + value)
    Y = g.standard_normal((l, n))
    ids.tune_set("trsm.mfma", 0)
    ids.tune_set(key, value)
    try:
        J, P, keff = ids.id_select(dev(Y), k)
        torch.cuda.synchronize()
    finally:
        ids.tune_set(key, None)
        ids.tune_set("trsm.mfma", None)
    Jo, Po, ko, _, _ = oracle.cpqr_id(Y, k)
    assert np.array_equal(J.cpu().numpy(), Jo)
    assert np.linalg.norm(P.cpu().numpy() - Po) <= 1e-10 * np.linalg.norm(Po)
    assert np.array_equal(P.cpu().numpy()[:, Jo], np.eye(k))


@pytest.mark.parametrize("rl512,rl256", [(0, 0), (36, 0), (0, 36)])
def test_batched_row_placement_variants(rl512, rl256):
    # rows in LDS or in registers: the same reflections; the FP32 partial sums
    # of the trailing norms are grouped differently (LDS rows in one run,
    # register rows in chunks of 8), so P agrees to the FP32 data's rounding
    m = np.array([300, 900, 500, 2000, 700])
    n = np.array([200, 400, 100, 700, 300])
    g = np.random.default_rng(4)
    bits = np.concatenate([synth.bf16_bits(g.standard_normal((mi, ni))).reshape(-1) for mi, ni in zip(m, n)])
    At = dev(bits.view(np.int16)).view(torch.bfloat16)
    Gt = dev(synth.bf16_bits(synth.gaussian(60, 128, seed=2)).view(np.int16)).view(torch.bfloat16)
    plan = ids.batched_plan(m, n, 50, 60, 128)
    ref = ids.id_batched(plan, At, Gt, seed=3)
    torch.cuda.synchronize()
    Jr, Pr = ref["J"].cpu().numpy(), ref["P"].cpu().numpy()
    ids.tune_set("batched.rl512", rl512)
    ids.tune_set("batched.rl256", rl256)
    try:
        out = ids.id_batched(plan, At, Gt, seed=3)
        torch.cuda.synchronize()
    finally:
        ids.tune_set("batched.rl512", None)
        ids.tune_set("batched.rl256", None)
    assert np.array_equal(out["J"].cpu().numpy(), Jr)
    assert np.linalg.norm(out["P"].cpu().numpy() - Pr) <= 1e-5 * np.linalg.norm(Pr)


def test_select_wide_shape_falls_back_to_four_waves():
    # 60 x 40000: 8-wave workgroups cannot all be co-resident; the plan takes
    # the 4-wave variant whatever the knob says, and the result is the oracle's
    l, n, k = 60, 40000, 40
    g = np.random.default_rng(40)
    Y = g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]
    ids.tune_set("select.gl.l64.ninf", 0)
    try:
        info = ids.select_plan_info(l, n, k)
        J, P, keff = ids.id_select(dev(Y), k)
        torch.cuda.synchronize()
    finally:
        ids.tune_set("select.gl.l64.ninf", None)
    assert info["workgroups"] == (n + 63) // 64   # 64 columns per 4-wave workgroup
    Jo, Po, ko, _, _ = oracle.cpqr_id(Y, k)
    assert np.array_equal(J.cpu().numpy(), Jo)
    assert np.linalg.norm(P.cpu().numpy() - Po) <= 1e-10 * np.linalg.norm(Po)


# the one-kernel block solve on the FP64 matrix cores (trsm.mfma = 1): k from
# 1 to 128, partial blocks, n below one 16-column tile and off a tile
# boundary, and a rank-deficient sketch (k_eff < k: rows past k_eff zero)
@pytest.mark.parametrize("l,n,k,rank", [(30, 700, 20, None), (60, 900, 50, None), (120, 1500, 100, None),
                                        (130, 2001, 128, None), (20, 300, 1, None), (40, 517, 17, None),
                                        (12, 13, 5, None), (40, 600, 30, 12)])
def test_solve_matrix_core_variant(l, n, k, rank):
    g = np.random.default_rng(l + n + k)
    Y = g.standard_normal((l, n))
    if rank is not None:
        # `rank` nonzero columns: the trailing norms are exactly zero after
        # `rank` steps
        Y = np.zeros((l, n))
        Y[:, g.choice(n, rank, replace=False)] = g.standard_normal((l, rank))
    print(f"matrix-core solve l={l} n={n} k={k} rank={rank}", flush=True)
    ids.tune_set("trsm.mfma", 1)
    try:
        st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        J, P, keff = ids.id_select(dev(Y), k, status=st)
        torch.cuda.synchronize()
    finally:
        ids.tune_set("trsm.mfma", None)
    Jo, Po, ko, _, nu = oracle.cpqr_id(Y, k, trace=True)
    kg = int(keff.item())
    assert kg == ko
    Jg = J.cpu().numpy()
    Pg = P.cpu().numpy()
    if rank is None:
        assert np.array_equal(Jg, Jo)
        assert np.linalg.norm(Pg - Po) <= 1e-10 * np.linalg.norm(Po)
        assert np.array_equal(Pg[:, Jo], np.eye(k))
    else:
        # k_eff = rank pivots, then rows k_eff.. of P are zero
        assert kg == rank
        assert np.array_equal(Jg[:kg], Jo[:ko]) and np.all(Jg[kg:] == -1)
        assert np.linalg.norm(Pg[:kg] - Po[:ko]) <= 1e-10 * np.linalg.norm(Po[:ko])
        assert np.all(Pg[kg:] == 0.0)
        assert np.array_equal(Pg[:kg][:, Jg[:kg]], np.eye(kg))
