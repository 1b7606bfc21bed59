"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/idsketch.h, and rejects bad arguments before touching the
GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_1901_10559_amd as ids

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "idsketch.h")


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_parses():
    names = declared_functions()
    assert "id_sketch" in names and "id_select" in names and "tensor_id" in names
    assert set(names) == set(ids.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = ids.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_constants_match_the_header():
    # the binding restates the header's enums and flag bits by hand
    text = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    consts = {m: int(v) for m, v in re.findall(r"\b(IDS_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    consts.update({m: int(v) for m, v in re.findall(r"#define\s+(IDS_[A-Z0-9_]+)\s+(\d+)u", text)})
    want = {"IDS_OK": ids.OK, "IDS_EINVAL": ids.EINVAL, "IDS_EDTYPE": ids.EDTYPE,
            "IDS_EWORKSPACE": ids.EWORKSPACE, "IDS_EHIP": ids.EHIP, "IDS_ETIMEOUT": ids.ETIMEOUT,
            "IDS_ERANKDEF": ids.ERANKDEF, "IDS_ENONFINITE": ids.ENONFINITE,
            "IDS_F64": ids.F64, "IDS_F32": ids.F32, "IDS_BF16": ids.BF16, "IDS_DENSE": ids.DENSE,
            "IDS_CSR": ids.CSR, "IDS_HASH_FULLRANK": ids.HASH_FULLRANK, "IDS_CHECK_FINITE": ids.CHECK_FINITE,
            "IDS_DETERMINISTIC": ids.DETERMINISTIC}
    for name, val in want.items():
        assert consts.get(name) == val, name


def test_status_strings():
    L = ids.lib()
    assert L.ids_status_string(0) == b"IDS_OK"
    assert L.ids_status_string(1) == b"IDS_EINVAL"
    assert L.ids_status_string(3) == b"IDS_EWORKSPACE"
    assert L.ids_status_string(99) == b"IDS_UNKNOWN"


def test_select_rejects_bad_sizes_without_gpu():
    L = ids.lib()
    nb = ctypes.c_size_t(0)
    assert L.ids_select_workspace_size(10, 5, 5, ctypes.byref(nb)) == 1      # k >= n
    assert b"k must" in L.ids_last_error()
    assert L.ids_select_workspace_size(3, 50, 4, ctypes.byref(nb)) == 1      # k > l
    assert L.ids_select_workspace_size(5000, 50, 4, ctypes.byref(nb)) == 1   # l > 4096
    assert L.id_select(None, 0, 10, 50, 1, 10, 4, None, None, None, None, None, 0, None) == 1
    assert L.id_select_noalloc(None, 0, 10, 50, 1, 10, 4, None, None, None, None, None) == 1


def test_sketch_rejects_bad_arguments_without_gpu():
    L = ids.lib()
    nb = ctypes.c_size_t(0)
    A = ids.IdsMatrix(ids.DENSE, ids.F64, 100, 20, 20, 0, ctypes.c_void_p(16), None, None)
    cfg = ids.IdsSketchCfg(30, 40, 0, 0, 0, ids.F64, ids.F64, None, None, None, None)   # l > l1
    assert L.ids_sketch_workspace_size(ctypes.byref(A), ctypes.byref(cfg), ctypes.byref(nb)) == 1
    cfg = ids.IdsSketchCfg(30, 10, 0, 0, 0, ids.F64, ids.F64, None, None, None, None)   # l < l1, G drawn
    assert L.ids_sketch_workspace_size(ctypes.byref(A), ctypes.byref(cfg), ctypes.byref(nb)) == 0
    without_g = nb.value
    cfg = ids.IdsSketchCfg(30, 10, 0, 0, 0, ids.F64, ids.F64, ctypes.c_void_p(256), None, None, None)
    assert L.ids_sketch_workspace_size(ctypes.byref(A), ctypes.byref(cfg), ctypes.byref(nb)) == 0
    assert without_g - nb.value == 8 * 10 * 30 + (-(8 * 10 * 30)) % 256   # room for the drawn l x l1 G
    cfg = ids.IdsSketchCfg(30, 30, 0, 0, 0, ids.F32, ids.F32, None, None, None, None)   # FP64 in, FP32 acc
    assert L.ids_sketch_workspace_size(ctypes.byref(A), ctypes.byref(cfg), ctypes.byref(nb)) == 2
    A2 = ids.IdsMatrix(ids.DENSE, ids.F64, 100, 20, 10, 0, ctypes.c_void_p(16), None, None)  # ld < n
    cfg = ids.IdsSketchCfg(30, 30, 0, 0, 0, ids.F64, ids.F64, None, None, None, None)
    assert L.ids_sketch_workspace_size(ctypes.byref(A2), ctypes.byref(cfg), ctypes.byref(nb)) == 1
    cfg = ids.IdsSketchCfg(30, 30, 0, 0, ids.HASH_FULLRANK, ids.F64, ids.F64, None, None, None, None)
    assert L.ids_sketch_workspace_size(ctypes.byref(A), ctypes.byref(cfg), ctypes.byref(nb)) == 1
    A3 = ids.IdsMatrix(ids.CSR, ids.F32, 100, 20, 0, 10, ctypes.c_void_p(16), ctypes.c_void_p(16),
                       ctypes.c_void_p(16))
    assert L.ids_sketch_workspace_size(ctypes.byref(A3), ctypes.byref(cfg), ctypes.byref(nb)) == 2


def test_tensor_rejects_bad_arguments_without_gpu():
    L = ids.lib()
    nb = ctypes.c_size_t(0)
    dims = (ctypes.c_int64 * 3)(10, 10, 10)
    p = ctypes.cast(dims, ctypes.c_void_p)
    assert L.ids_tensor_workspace_size(3, p, 20, 5, 100, 0, ctypes.byref(nb)) == 1   # Jlen not power of 2
    assert L.ids_tensor_workspace_size(3, p, 20, 20, 64, 0, ctypes.byref(nb)) == 1   # k >= R
    assert L.ids_tensor_workspace_size(9, p, 20, 5, 64, 0, ctypes.byref(nb)) == 1    # N > 8
    assert L.ids_tensor_workspace_size(3, p, 20, 5, 8192, 0, ctypes.byref(nb)) == 1  # Jlen > 4096
    assert L.ids_tensor_workspace_size(3, p, 20, 5, 64, 4, ctypes.byref(nb)) == 1    # projection l < k
    assert L.ids_tensor_workspace_size(3, p, 20, 5, 64, 65, ctypes.byref(nb)) == 1   # projection l > Jlen


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(ids.IdsError):
        ids.id_select(torch.zeros(4, 8, dtype=torch.float64), 2)


def test_profile_stage_selection_without_gpu():
    L = ids.lib()
    assert L.ids_profile_stages(b"countsketch,cpqr") == 0
    assert L.ids_profile_stages(b"countsketch,nosuch") == 1
    assert b"unknown stage nosuch" in L.ids_last_error()
    assert L.ids_profile_stages(None) == 0
    assert L.ids_profile_stages(b"") == 0


def test_tune_knobs_without_gpu():
    import ctypes as ct
    L = ids.lib()
    v = ct.c_int64(0)
    assert L.ids_tune_get(b"trsm.k64", ct.byref(v)) == 0 and v.value in (2, 4)
    assert L.ids_tune_set(b"trsm.k64", 4) == 0
    assert L.ids_tune_get(b"trsm.k64", ct.byref(v)) == 0 and v.value == 4
    assert L.ids_tune_set(b"trsm.k64", 3) == 1            # not accepted by the knob
    assert b"not accepted" in L.ids_last_error()
    assert L.ids_tune_set(b"no.such.knob", 1) == 1
    assert L.ids_tune_set(b"trsm.k64", -1) == 0           # back to the table's value
    import paper_1901_10559_amd.tune as tune
    assert set(tune.HAND_DEFAULTS) == set(tune.CANDIDATES)
    for key, val in tune.HAND_DEFAULTS.items():
        assert L.ids_tune_get(key.encode(), ct.byref(v)) == 0, key
        assert val in tune.CANDIDATES[key]
    # the compiled table holds exactly the tuner's knobs, each at a value the
    # knob accepts
    import os
    import re
    inc = open(os.path.join(os.path.dirname(tune.__file__), "csrc", "tuned_table.inc")).read()
    table = {k: int(x) for k, x in re.findall(r'\{"([^"]+)", (-?\d+)\}', inc)}
    assert set(table) == set(tune.HAND_DEFAULTS)
    for key, val in table.items():
        assert L.ids_tune_set(key.encode(), val) == 0, key
        assert L.ids_tune_get(key.encode(), ct.byref(v)) == 0 and v.value == val
        assert L.ids_tune_set(key.encode(), -1) == 0
