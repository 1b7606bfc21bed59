"""The allocation-free select (id_select_noalloc): the same kernels as
id_select with the library's static scratch buffer instead of a caller
workspace.  Called through the C-ABI and compared with id_select on the same
sketch, to the same bar as the select parity tests (the outputs are bitwise
identical: same kernels, same inputs); two calls in a row, the second on a
smaller shape, so the second reuses scratch the first left behind."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ids = pytest.importorskip("paper_1901_10559_amd")

DEV = "cuda:0"


def run_noalloc(Y, k):
    l, n = Y.shape
    J = torch.empty(k, dtype=torch.int64, device=DEV)
    P = torch.empty((k, n), dtype=torch.float64, device=DEV)
    keff = torch.empty(1, dtype=torch.int64, device=DEV)
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ids.id_select_noalloc(Y, k, J, P, keff, status=st)
    return J, P, keff, st


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_matches_select_two_calls(dtype):
    g = np.random.default_rng(11)
    # first call: the c1 sketch shape (grouped lanes, speculative exchange);
    # second: smaller, with fewer workgroups and a shorter sketch
    for (l, n, k) in [(120, 2000, 100), (30, 500, 20)]:
        Yh = (g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]).astype(dtype)
        Y = torch.from_numpy(Yh).to(DEV)
        print(f"noalloc: l={l} n={n} k={k} {dtype.__name__}", flush=True)
        J0, P0, k0 = ids.id_select(Y, k)
        J1, P1, k1, st = run_noalloc(Y, k)
        torch.cuda.synchronize()
        assert int(k1.item()) == int(k0.item()) == k
        assert int(st.item()) == ids.OK
        assert np.array_equal(J1.cpu().numpy(), J0.cpu().numpy())
        assert np.array_equal(P1.cpu().numpy(), P0.cpu().numpy())


def test_noalloc_row_band_then_small():
    g = np.random.default_rng(12)
    for (l, n, k) in [(700, 400, 30), (60, 300, 12)]:
        Y = torch.from_numpy(g.standard_normal((l, n))).to(DEV)
        print(f"noalloc: l={l} n={n} k={k}", flush=True)
        J0, P0, k0 = ids.id_select(Y, k)
        J1, P1, k1, st = run_noalloc(Y, k)
        torch.cuda.synchronize()
        assert int(k1.item()) == int(k0.item()) == k and int(st.item()) == ids.OK
        assert np.array_equal(J1.cpu().numpy(), J0.cpu().numpy())
        assert np.array_equal(P1.cpu().numpy(), P0.cpu().numpy())


def test_noalloc_column_steps_then_small():
    # the column-steps factorisation (forced by the select.steps knob) with its
    # working copy, partials and counters in the static buffer; the second
    # call smaller
    g = np.random.default_rng(13)
    ids.tune_set("select.steps", 1)
    try:
        for (l, n, k) in [(120, 2000, 100), (40, 700, 25)]:
            Y = torch.from_numpy(g.standard_normal((l, n))).to(DEV)
            print(f"noalloc column steps: l={l} n={n} k={k}", flush=True)
            J0, P0, k0 = ids.id_select(Y, k)
            J1, P1, k1, st = run_noalloc(Y, k)
            torch.cuda.synchronize()
            assert int(k1.item()) == int(k0.item()) == k and int(st.item()) == ids.OK
            assert np.array_equal(J1.cpu().numpy(), J0.cpu().numpy())
            assert np.array_equal(P1.cpu().numpy(), P0.cpu().numpy())
    finally:
        ids.tune_set("select.steps", None)


def test_noalloc_rejects_shape_beyond_scratch():
    # 4096 x 2000 with k = 1000 needs more than the static buffer holds:
    # rejected on the host before any launch
    Y = torch.zeros((1, 1), dtype=torch.float64, device=DEV)
    L = ids.lib()
    rc = L.id_select_noalloc(ids.c_vp(Y.data_ptr()), ids.F64, 4096, 2000, 1, 4096, 1000, ids.c_vp(Y.data_ptr()),
                             ids.c_vp(Y.data_ptr()), ids.c_vp(Y.data_ptr()), None, None)
    assert rc == ids.EWORKSPACE
    assert b"static buffer" in L.ids_last_error()
