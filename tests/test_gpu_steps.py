"""The column-steps pivoted QR (columns in HBM, one kernel per pivot step):
taken automatically by shapes too wide for the register-resident
factorisation, and forced on ordinary shapes with the select.steps knob.
Parity with the FP64 oracle's Algorithm 1 as for the other kernels."""
import numpy as np
import pytest

import oracle

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


def check_select(Y, k, Yd=None):
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    J, P, keff = ids.id_select(dev(Y) if Yd is None else Yd, k, status=st)
    torch.cuda.synchronize()
    Jo, Po, ko, _, nu = oracle.cpqr_id(np.asarray(Y, dtype=np.float64), k, trace=True)
    assert int(keff.item()) == ko
    Jg = J.cpu().numpy()
    assert tie_aware_J(Jg, Jo, nu)
    if np.array_equal(Jg, Jo):
        Pg = P.cpu().numpy()
        assert np.linalg.norm(Pg - Po) <= 1e-10 * max(np.linalg.norm(Po), 1e-300)
        assert np.array_equal(Pg[:ko][:, Jg[:ko]], np.eye(ko))
    return int(st.item())


@pytest.mark.parametrize("l,n,k", [(30, 1000, 20), (120, 2000, 100), (300, 900, 64), (1030, 700, 300),
                                   (4096, 300, 30), (65, 129, 64), (12, 40, 5)])
def test_steps_forced(l, n, k):
    g = np.random.default_rng(l + n + k + 3)
    Y = g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]
    ids.tune_set("select.steps", 1)
    try:
        assert ids.select_plan_info(l, n, k)["family"] == "column_steps"
        print(f"steps: l={l} n={n} k={k}", flush=True)
        assert check_select(Y, k) == ids.OK
    finally:
        ids.tune_set("select.steps", None)


def test_steps_rank_deficient_and_nonfinite():
    g = np.random.default_rng(6)
    Y = np.zeros((40, 300))
    Y[:, [3, 17, 29]] = g.standard_normal((40, 3))
    ids.tune_set("select.steps", 1)
    try:
        assert check_select(Y, 6) == ids.ERANKDEF
        Y2 = g.standard_normal((40, 300))
        Y2[7, 11] = np.nan
        st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        ids.id_select(dev(Y2), 6, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == ids.ENONFINITE
    finally:
        ids.tune_set("select.steps", None)


def test_steps_f32_column_major_input():
    g = np.random.default_rng(5)
    Y = g.standard_normal((50, 300)).astype(np.float32)
    Yc = dev(np.asfortranarray(Y).T.copy()).t()
    ids.tune_set("select.steps", 1)
    try:
        assert check_select(Y, 20, Yd=Yc) == ids.OK
    finally:
        ids.tune_set("select.steps", None)


@pytest.mark.parametrize("l,n,k", [(300, 12000, 80), (60, 70000, 30)])
def test_steps_taken_beyond_the_register_resident_limit(l, n, k):
    info = ids.select_plan_info(l, n, k)
    print(f"wide: l={l} n={n} k={k} {info}", flush=True)
    assert info["family"] == "column_steps"
    g = np.random.default_rng(n)
    Y = g.standard_normal((l, n)) * g.uniform(0.1, 10, n)[None, :]
    assert check_select(Y, k) == ids.OK
