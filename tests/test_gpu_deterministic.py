"""IDS_DETERMINISTIC: the CSR CountSketch summed in the definition's order
(Section 1.3: row i of A is added, with sign D_ii, to row h(i) of Y1; rows in
increasing order, a row's stored entries in storage order, duplicates summed
where they stand).  The oracle adds in exactly that order, so the FP64 sketch
must equal it bit for bit, and repeated runs must agree bit for bit."""
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


@pytest.fixture(params=[1, 0], ids=["binned", "unbinned"])
def path(request):
    # cs.csr.bin selects the binned ordered kernels (1) or the unbinned one
    # (0, the form wide matrices take); both must give the same bits
    ids.tune_set("cs.csr.bin", request.param)
    yield request.param
    ids.tune_set("cs.csr.bin", -1)


def sketch(rp, ci, v, n, L, seed, **kw):
    print(f"ordered csr sketch m={rp.size - 1} n={n} nnz={ci.size} L={L} seed={seed} "
          f"binned={ids.tune_get('cs.csr.bin')}", flush=True)
    return ids.id_sketch((dev(rp), dev(ci), dev(v), n), L, seed=seed, deterministic=True, **kw).cpu().numpy()


# n > 8192 puts several column ranges on a bucket (and several workgroups);
# L = 1 makes one bucket hold every row
# (200000, 20000, 64): 64 x 20 x 13 = 16640 counters, two tiles of the counter scan
@pytest.mark.parametrize("m,n,L", [(2000, 300, 40), (20000, 1500, 240), (777, 21000, 16), (3000, 40000, 7),
                                   (5000, 64, 1), (1, 1, 1), (200000, 20000, 64)])
def test_ordered_csr_bit_exact(m, n, L, path):
    rp, ci, v = synth.csr_zipf(m=m, n=n, seed=2, kmax=min(681, n), rank=min(5, n), nplant_rows=min(200, m),
                               nplant_cols=min(100, n))
    Y = sketch(rp, ci, v, n, L, seed=4)
    b, s = oracle.hash_maps(4, 0, m, L)
    assert np.array_equal(Y, oracle.countsketch_csr(rp, ci, v, n, b, s, L))


def test_ordered_csr_duplicates_unsorted_empty_and_long_rows(path):
    # unsorted column indices, repeated columns inside a row (several in one
    # 64-entry chunk, so the lane-order rounds run), empty rows and rows much
    # longer than a chunk
    g = np.random.default_rng(21)
    m, n, L = 3000, 2500, 11
    cnt = np.where(g.random(m) < 0.3, 0, g.integers(1, 6, m))
    cnt[5] = 3000
    cnt[400:420] = 500
    cnt[2999] = 1
    rp = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    ci = np.empty(rp[-1], dtype=np.int32)
    for i in range(m):
        a, b_ = rp[i], rp[i + 1]
        # a narrow pool of columns forces repeats inside a row
        pool = g.integers(0, n, size=max(1, (b_ - a) // 4))
        ci[a:b_] = g.choice(pool, size=b_ - a)
    v = g.standard_normal(rp[-1])
    Y = sketch(rp, ci, v, n, L, seed=13)
    b, s = oracle.hash_maps(13, 0, m, L)
    Yo = oracle.countsketch_csr(rp, ci, v, n, b, s, L)
    assert np.array_equal(Y, Yo)
    # the same matrix through the default (atomic) kernel agrees to rounding
    Ya = ids.id_sketch((dev(rp), dev(ci), dev(v), n), L, seed=13).cpu().numpy()
    absum = oracle.countsketch_csr(rp, ci, np.abs(v), n, b, np.ones_like(s), L)
    assert np.all(np.abs(Ya - Yo) <= 64 * 2.0 ** -52 * absum + 1e-300)


def test_ordered_csr_single_entry(path):
    m, n, L = 1000, 50, 9
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[318:] = 1
    ci = np.array([47], dtype=np.int32)
    v = np.array([-2.5])
    Y = sketch(rp, ci, v, n, L, seed=1)
    b, s = oracle.hash_maps(1, 0, m, L)
    Yo = np.zeros((L, n))
    Yo[b[317], 47] = s[317] * -2.5
    assert np.array_equal(Y, Yo)


def test_ordered_matrix_id_repeats_bitwise_and_matches_oracle(path):
    rp, ci, v = synth.csr_zipf(m=20000, n=2000, seed=3, rank=20, nplant_rows=2000, nplant_cols=300)
    A = (dev(rp), dev(ci), dev(v), 2000)
    k, l1 = 20, 120
    G = synth.gaussian(k + 10, l1, seed=3)
    print("ordered matrix_id 20000x2000 k=20 l1=120", flush=True)
    runs = [ids.matrix_id(A, k, l1, k + 10, seed=3, G=dev(G), deterministic=True, check=True) for _ in range(3)]
    for r in runs[1:]:
        for key in ("Y", "J", "P"):
            assert torch.equal(r[key], runs[0][key]), key
    o = oracle.matrix_id(csr=(rp, ci, v), n=2000, k=k, l1=l1, seed=3, G=G, trace=True)
    # the sketch before the projection is the oracle's bit for bit; the
    # projection's sums run in another order, so a pivot may differ only at a
    # numerical tie of the oracle's trailing norms
    Jg = runs[0]["J"].cpu().numpy()
    if not np.array_equal(Jg, o["J"]):
        t = int(np.argmax(Jg != o["J"]))
        row = np.sort(o["nu"][t][o["nu"][t] >= 0])[::-1]
        assert len(row) > 1 and row[0] - row[1] <= 1e-12 * row[0]
    else:
        assert np.linalg.norm(runs[0]["P"].cpu().numpy() - o["P"]) <= 1e-10 * np.linalg.norm(o["P"])


def test_ordered_flag_on_dense_is_a_no_op():
    g = np.random.default_rng(5)
    A = g.standard_normal((3000, 200))
    Y0 = ids.id_sketch(dev(A), 64, seed=2).cpu().numpy()
    Y1 = ids.id_sketch(dev(A), 64, seed=2, deterministic=True).cpu().numpy()
    assert np.array_equal(Y0, Y1)
