"""C-ABI checks that need no GPU: the built library loads, exports every
function include/nuasm.h declares, and validates arguments before any device
call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nuasm.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nuasm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    if not os.path.exists(P.lib_path()):
        pytest.skip("libnuasm.so not built")
    P.load()
    return P


def test_header_declares_the_operator_calls():
    names = _declared_functions()
    for need in ("nuasm_plan_create", "nuasm_set_points", "nuasm_execute", "nuasm_execute_adjoint",
                 "nuasm_plan_destroy", "nuasm_status_string", "nuasm_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(P):
    lib = ctypes.CDLL(P.lib_path())
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(P):
    missing = [n for n in _declared_functions() if n not in P._SIGS]
    assert not missing, missing


def test_params_struct_layout_matches_header(P):
    # 4 x int32, int64, 6 doubles, 2 x double[2], double, 2 x uint32
    assert ctypes.sizeof(P.Params) == 4 * 4 + 8 + 6 * 8 + 4 * 8 + 8 + 2 * 4


def _params(P, **kw):
    p = P.Params()
    assert P.load().nuasm_params_default(ctypes.byref(p)) == 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _create(P, p):
    h = ctypes.c_void_p(123)
    st = P.load().nuasm_plan_create(ctypes.byref(p), None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("field,value,expect", [
    ("N", 100, "NUASM_ERR_UNSUPPORTED"),
    ("N", 8, "NUASM_ERR_UNSUPPORTED"),
    ("N", 8192, "NUASM_ERR_UNSUPPORTED"),
    ("type", 4, "NUASM_ERR_INVALID_ARG"),
    ("type", 0, "NUASM_ERR_INVALID_ARG"),
    ("tf", 7, "NUASM_ERR_INVALID_ARG"),
    ("band", 9, "NUASM_ERR_INVALID_ARG"),
    ("lam", 0.0, "NUASM_ERR_INVALID_ARG"),
    ("lam", float("nan"), "NUASM_ERR_INVALID_ARG"),
    ("d2", -1.0, "NUASM_ERR_INVALID_ARG"),
    ("tol", 0.5, "NUASM_ERR_INVALID_ARG"),
    ("flags", 0x80, "NUASM_ERR_INVALID_ARG"),
    ("flags", 0x10, "NUASM_ERR_INVALID_ARG"),
    ("reserved", 1, "NUASM_ERR_INVALID_ARG"),
    ("phase_fp64", 2, "NUASM_ERR_INVALID_ARG"),
])
def test_invalid_params_rejected_before_device_use(P, field, value, expect):
    p = _params(P, **{field: value})
    st, h = _create(P, p)
    lib = P.load()
    assert lib.nuasm_status_string(st).decode() == expect
    assert h.value is None
    assert lib.nuasm_last_error().decode()


def test_type3_rejects_the_crop_flag(P):
    p = _params(P, type=3, flags=0x1)
    st, h = _create(P, p)
    assert P.load().nuasm_status_string(st).decode() == "NUASM_ERR_INVALID_ARG"
    assert h.value is None


def test_plan_info_struct_layout_matches_header(P):
    # 4 x int64, 8 x int32/float, 3 x int64, size_t, int64, 4 x int32
    assert ctypes.sizeof(P.PlanInfo) == 4 * 8 + 8 * 4 + 3 * 8 + 8 + 8 + 4 * 4
    assert [f for f, _ in P.PlanInfo._fields_][-4:] == ["spread_chunk", "interp_chunk", "bin_range_points",
                                                         "Npf"]
    assert ctypes.sizeof(P.Tuning) == 20


def test_tuning_rejects_bad_values_without_a_device(P):
    lib = P.load()
    t = P.Tuning(0, 100, 0, 0, 0)
    assert lib.nuasm_status_string(lib.nuasm_plan_set_tuning(None, ctypes.byref(t))).decode() == \
        "NUASM_ERR_INVALID_ARG"
    assert lib.nuasm_batch_set_branches(None, 2) != 0


def test_stage_names_match_header_count(P):
    src = open(HEADER).read()
    n = int(re.search(r"#define NUASM_NUM_STAGES (\d+)", src).group(1))
    assert len(P.STAGES) == n
    for name, idx in re.findall(r"#define NUASM_STAGE_([A-Z0-9_]+) (\d+)", src):
        assert P.STAGES[int(idx)] == name.lower()


def test_fresnel_needs_nonzero_z(P):
    p = _params(P, tf=1, z=0.0)
    st, h = _create(P, p)
    assert P.load().nuasm_status_string(st).decode() == "NUASM_ERR_INVALID_ARG"


def test_deterministic_flag_passes_validation(P):
    """NUASM_DETERMINISTIC is a known flag: without a device the plan gets as
    far as the device check."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is visible")
    st, h = _create(P, _params(P, flags=0x8 | 0x2))
    assert P.load().nuasm_status_string(st).decode() == "NUASM_ERR_NO_DEVICE"


def test_null_arguments(P):
    lib = P.load()
    h = ctypes.c_void_p()
    assert lib.nuasm_status_string(lib.nuasm_plan_create(None, None, ctypes.byref(h))).decode() == \
        "NUASM_ERR_INVALID_ARG"
    p = _params(P)
    assert lib.nuasm_plan_create(ctypes.byref(p), None, None) != 0
    assert lib.nuasm_plan_destroy(None) == 0
    assert lib.nuasm_execute(None, None, None) != 0
    assert lib.nuasm_set_points(None, 0, None, None) != 0
    assert lib.nuasm_set_dest_points(None, 0, None, None) != 0
    assert lib.nuasm_plan_set_timing(None, 1) != 0
    n = ctypes.c_int64()
    assert lib.nuasm_debug_records(None, 0, None, 0, None, ctypes.byref(n)) != 0


def test_no_device_is_reported(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is visible")
    st, h = _create(P, _params(P))
    assert P.load().nuasm_status_string(st).decode() == "NUASM_ERR_NO_DEVICE"


def test_status_strings(P):
    lib = P.load()
    names = [lib.nuasm_status_string(i).decode() for i in range(8)]
    assert names[0] == "NUASM_OK" and len(set(names)) == 8
    assert lib.nuasm_version() >= 100


def test_boundary_calls_reject_null_handles(P):
    lib = P.load()
    b = ctypes.c_size_t()
    name = lambda st: lib.nuasm_status_string(st).decode()  # noqa: E731
    assert name(lib.nuasm_plan_workspace_bytes(None, 100, ctypes.byref(b))) == "NUASM_ERR_INVALID_ARG"
    assert name(lib.nuasm_plan_set_workspace(None, None, 0)) == "NUASM_ERR_INVALID_ARG"
    M = (ctypes.c_int64 * 1)(10)
    vp = (ctypes.c_void_p * 1)(None)
    assert name(lib.nuasm_set_points_many(None, M, vp, vp)) == "NUASM_ERR_INVALID_ARG"
    assert name(lib.nuasm_execute_many(None, vp, vp)) == "NUASM_ERR_INVALID_ARG"
    h = ctypes.c_void_p(123)
    p = P.Params()
    assert lib.nuasm_params_default(ctypes.byref(p)) == 0
    assert name(lib.nuasm_plan_many_create(0, ctypes.byref(p), None, ctypes.byref(h))) == "NUASM_ERR_INVALID_ARG"
    assert h.value is None
    t = P.Tuning(0, 0, 0, 3, 0)
    assert name(lib.nuasm_plan_set_tuning(None, ctypes.byref(t))) == "NUASM_ERR_INVALID_ARG"
