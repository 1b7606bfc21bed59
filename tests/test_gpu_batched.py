"""GPU checks of the batched mixed-precision ID (BF16 inputs, FP32 sketch and
projection, FP32 CPQR with FP64 norms, FP64 interpolation matrix) against the
FP64 oracle run on the same BF16-rounded inputs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ids = pytest.importorskip("paper_1901_10559_amd")

DEV = "cuda:0"


def make_batch(ms, ns, seed):
    As = [synth.batched_problem(int(m), int(n), seed, p) for p, (m, n) in enumerate(zip(ms, ns))]
    flat = np.concatenate([a.ravel() for a in As])
    return As, torch.from_numpy(flat.view(np.int16)).to(DEV).view(torch.bfloat16)


def run_batch(ms, ns, k, l, l1max, seed=0):
    As, At = make_batch(ms, ns, seed)
    Gb = synth.bf16_bits(synth.gaussian(l, l1max, seed))
    G64 = synth.bf16_to_f64(Gb)
    Gt = torch.from_numpy(Gb.view(np.int16)).to(DEV).view(torch.bfloat16)
    plan = ids.batched_plan(ms, ns, k, l, l1max)
    out = ids.id_batched(plan, At, Gt, seed=seed, return_Y=True)
    torch.cuda.synchronize()
    return As, G64, plan, out


@pytest.mark.parametrize("ms,ns,k,l,l1max", [
    ([300, 700, 121, 4096, 1500, 497], [130, 1024, 640, 200, 333, 257], 111, 121, 496),
    ([64, 200, 90, 1000], [50, 77, 300, 1000], 20, 40, 128),
    ([150, 333, 2000], [90, 700, 129], 50, 60, 130),   # G rows not 16-byte aligned
    # smallest shapes: n < 8, partial 64-bucket groups, a single bucket group
    ([4, 5, 7, 9, 64, 65, 4096], [3, 5, 8, 9, 127, 129, 1024], 2, 4, 8),
    ([12, 20, 33, 63, 700], [4, 10, 100, 17, 1000], 3, 12, 496),
])
def test_batched_sketch_matches_oracle(ms, ns, k, l, l1max):
    As, G64, plan, out = run_batch(ms, ns, k, l, l1max)
    Y = out["Y"].cpu().numpy()
    for p, (A, m, n) in enumerate(zip(As, ms, ns)):
        A64 = synth.bf16_to_f64(A).reshape(m, n)
        l1 = min(m, l1max)
        b, s = oracle.hash_maps(0, p, m, l1)
        Y1 = oracle.countsketch_dense(A64, b, s, l1)
        Yo = oracle.gemm(G64[:, :l1], Y1)
        Yg = Y[plan.y_off[p]:plan.y_off[p + 1]].reshape(n, l).T
        # hi + lo BF16 split (relative 2^-16) and FP32 accumulation over l1 terms
        absY1 = oracle.countsketch_dense(np.abs(A64), b, np.ones_like(s), l1)
        bound = 4 * (2.0 ** -16 + l1 * 2.0 ** -24) * (np.abs(G64[:, :l1]) @ absY1)
        assert np.all(np.abs(Yg - Yo) <= bound + 1e-30), p


@pytest.mark.parametrize("ms,ns,k,l,l1max", [
    ([300, 700, 121, 4096, 1500, 497], [130, 1024, 640, 200, 333, 257], 111, 121, 496),
    ([64, 200, 90, 1000], [50, 77, 300, 1000], 20, 40, 128),
    ([150, 333, 2000], [90, 700, 129], 50, 60, 130),
    ([4, 5, 7, 9, 64, 65, 4096], [3, 5, 8, 9, 127, 129, 1024], 2, 4, 8),
    ([12, 20, 33, 63, 700], [4, 10, 100, 17, 1000], 3, 12, 496),
])
def test_batched_id_residual_within_2x_of_oracle(ms, ns, k, l, l1max):
    As, G64, plan, out = run_batch(ms, ns, k, l, l1max)
    J = out["J"].cpu().numpy()
    P = out["P"].cpu().numpy()
    keff = out["k_eff"].cpu().numpy()
    for p, (A, m, n) in enumerate(zip(As, ms, ns)):
        A64 = synth.bf16_to_f64(A).reshape(m, n)
        l1 = min(m, l1max)
        o = oracle.matrix_id(A64, k=k, l1=l1, seed=0, tag=p, G=G64[:, :l1])
        assert keff[p] == o["k_eff"] == k
        Pp = P[plan.p_off[p]:plan.p_off[p + 1]].reshape(k, n)
        assert np.array_equal(Pp[:, J[p]], np.eye(k))
        rg = oracle.residual_fro(A64, J[p], Pp)
        ro = oracle.residual_fro(A64, o["J"], o["P"])
        assert rg <= 2.0 * ro, (p, rg, ro)


def test_batched_sketch_unaligned_A_base():
    # A starting 2 bytes past a 16-byte boundary: every chunk takes the element
    # loads; odd n also exercises rows that straddle 16-byte blocks
    ms, ns, k, l, l1max = [300, 129, 77], [77, 200, 33], 20, 40, 128
    As, At = make_batch(ms, ns, 0)
    buf = torch.zeros(At.numel() + 8, dtype=torch.bfloat16, device=DEV)
    buf[1:1 + At.numel()] = At
    Au = buf[1:1 + At.numel()]
    assert Au.data_ptr() % 16 == 2
    Gb = synth.bf16_bits(synth.gaussian(l, l1max, 0))
    G64 = synth.bf16_to_f64(Gb)
    Gt = torch.from_numpy(Gb.view(np.int16)).to(DEV).view(torch.bfloat16)
    plan = ids.batched_plan(ms, ns, k, l, l1max)
    out = ids.id_batched(plan, Au, Gt, seed=0, return_Y=True)
    ref = ids.id_batched(plan, At, Gt, seed=0, return_Y=True)
    torch.cuda.synchronize()
    Y = out["Y"].cpu().numpy()
    # same sums in the same order whatever the load path: bit-identical
    assert np.array_equal(Y, ref["Y"].cpu().numpy())
    for p, (A, m, n) in enumerate(zip(As, ms, ns)):
        A64 = synth.bf16_to_f64(A).reshape(m, n)
        l1 = min(m, l1max)
        b, s = oracle.hash_maps(0, p, m, l1)
        Yo = oracle.gemm(G64[:, :l1], oracle.countsketch_dense(A64, b, s, l1))
        Yg = Y[plan.y_off[p]:plan.y_off[p + 1]].reshape(n, l).T
        absY1 = oracle.countsketch_dense(np.abs(A64), b, np.ones_like(s), l1)
        bound = 4 * (2.0 ** -16 + l1 * 2.0 ** -24) * (np.abs(G64[:, :l1]) @ absY1)
        assert np.all(np.abs(Yg - Yo) <= bound + 1e-30), p


def test_batched_rejects_out_of_range():
    with pytest.raises(ids.IdsError):
        ids.batched_plan([5000], [300], 111, 121, 496)        # m > 4096
    with pytest.raises(ids.IdsError):
        ids.batched_plan([500], [2000], 111, 121, 496)        # n > 1024
    with pytest.raises(ids.IdsError):
        ids.batched_plan([500], [300], 111, 121, 600)         # l1max > 512


def test_batched_fixed_accuracy_rank_and_residual():
    # fixed-accuracy batched ID: problem p stops at |r_tt| <= tol |r_11|; the
    # rank matches the oracle's fixed-accuracy stop on the same BF16 input up
    # to one step (the two sides' norms differ at rounding level near the
    # threshold), and the ID of that rank is as accurate as the oracle's
    nprob, k, l, l1max, tol = 48, 111, 121, 496, 1e-2
    m, n, flat = synth.batched_inputs(nprob, seed=7)
    Gb = synth.bf16_bits(synth.gaussian(l, l1max, seed=7))
    plan = ids.batched_plan(m, n, k, l, l1max)
    At = torch.from_numpy(flat.view(np.int16)).to(DEV).view(torch.bfloat16)
    Gt = torch.from_numpy(Gb.view(np.int16)).to(DEV).view(torch.bfloat16)
    out = ids.id_batched(plan, At, Gt, seed=7, tol=tol)
    keff = out["k_eff"].cpu().numpy()
    J = out["J"].cpu().numpy()
    P = out["P"].cpu().numpy()
    assert np.all((keff >= 1) & (keff < k))
    G64 = synth.bf16_to_f64(Gb)
    for p in range(0, nprob, 6):
        A64 = synth.bf16_to_f64(flat[plan.a_off[p]:plan.a_off[p + 1]]).reshape(m[p], n[p])
        l1 = min(int(m[p]), l1max)
        o = oracle.matrix_id_adaptive(A64, kmax=k, tol=tol, l1=l1, seed=7, tag=p, G=G64[:, :l1])
        r = int(keff[p])
        assert abs(r - o["rank"]) <= 1, (p, r, o["rank"])
        Pp = P[plan.p_off[p]:plan.p_off[p + 1]].reshape(k, n[p])
        assert np.all(J[p, r:] == -1) and np.all(Pp[r:] == 0.0)
        assert np.array_equal(Pp[:r][:, J[p, :r]], np.eye(r))
        of = oracle.matrix_id(A64, k=r, l1=l1, seed=7, tag=p, G=G64[:, :l1])
        assert oracle.residual_fro(A64, J[p, :r], Pp[:r]) <= 2.0 * oracle.residual_fro(A64, of["J"], of["P"])


def test_batched_graph_replays_match_eager():
    # the whole batch recorded into a HIP graph: every replay (with eager work
    # and synchronisations in between) gives the eager call's bits
    nprob, k, l, l1max = 96, 30, 40, 128
    m, n, flat = synth.batched_inputs(nprob, seed=7, mrange=(64, 900), nrange=(40, 1024))
    Gb = synth.bf16_bits(synth.gaussian(l, l1max, seed=7))
    plan = ids.batched_plan(m, n, k, l, l1max)
    At = torch.from_numpy(flat.view(np.int16)).to(DEV).view(torch.bfloat16)
    Gt = torch.from_numpy(Gb.view(np.int16)).to(DEV).view(torch.bfloat16)
    for tol in (0.0, 1e-2):
        eager = ids.id_batched(plan, At, Gt, seed=7, tol=tol)
        torch.cuda.synchronize()
        Je, Pe, ke = eager["J"].cpu().numpy(), eager["P"].cpu().numpy(), eager["k_eff"].cpu().numpy()
        g = ids.batched_graph(plan, At, Gt, seed=7, tol=tol)
        for rep in range(4):
            g.P.fill_(float("nan"))
            g.J.fill_(-7)
            out = g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(out["J"].cpu().numpy(), Je), rep
            assert np.array_equal(out["k_eff"].cpu().numpy(), ke), rep
            assert np.array_equal(out["P"].cpu().numpy(), Pe), rep
            assert set(out["status"].cpu().numpy().tolist()) == {ids.OK}
            # eager work between replays
            ids.id_batched(plan, At, Gt, seed=8, tol=tol)
            torch.cuda.synchronize()
        g.close()
