"""C ABI checks that need no GPU: the library loads, exports every declared
entry point, and rejects invalid problems on the host before any device call."""

import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1602_03395_amd import _lib as L
    return L


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fx_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L.lib, n), n


def test_header_struct_layout_matches_binding():
    L = _lib()
    # int32 ndim, 3 int64, 3x3 doubles, 3 int32, 2 doubles, 2 int32 (with C padding)
    assert ctypes.sizeof(L.fx_problem) == 8 + 24 + 72 + 12 + 4 + 16 + 8


def _create(prob):
    L = _lib()
    h = ctypes.c_void_p()
    st = L.lib.fx_plan_create(ctypes.byref(prob), ctypes.byref(h))
    return st, L.lib.fx_last_error().decode()


@pytest.mark.parametrize("field,value", [
    ("ndim", 0), ("ndim", 4), ("shape0", 0), ("dx0", 0.0), ("dx0", -1.0), ("dx0", math.nan),
    ("lambda0", 0), ("lambda0", -3), ("m_over_hbar", 0.0), ("m_over_hbar", math.inf), ("t_flight", math.nan),
    ("t_flight", math.inf), ("precision", 7), ("schedule", 9), ("a0", math.inf),
])
def test_invalid_problems_are_rejected_on_host(field, value):
    L = _lib()
    p = L.make_problem((16,), 1.0, 3, 1.0, 2.0)
    if field.endswith("0"):
        name = field[:-1]
        arr = getattr(p, "lambda_" if name == "lambda" else name)
        arr[0] = value
    else:
        setattr(p, field, value)
    st, msg = _create(p)
    assert st == L.FX_EINVAL, (st, msg)
    assert msg


def test_unsupported_sizes():
    L = _lib()
    p = L.make_problem((8192,), 1.0, 2, 1.0, 1.0)
    st, msg = _create(p)
    assert st == L.FX_EUNSUPPORTED and "4096" in msg
    p = L.make_problem((4096,), 1.0, 40000, 1.0, 1.0)
    st, _ = _create(p)
    assert st == L.FX_EUNSUPPORTED


def test_null_pointers():
    L = _lib()
    p = L.make_problem((16,), 1.0, 3, 1.0, 2.0)
    assert L.lib.fx_plan_create(ctypes.byref(p), None) == L.FX_EINVAL
    assert L.lib.fx_plan_create(None, ctypes.byref(ctypes.c_void_p())) == L.FX_EINVAL
    assert L.lib.fx_expand(None, None, None, None, None) == L.FX_EINVAL
    assert L.lib.fx_plan_destroy(None) == L.FX_OK
    assert L.lib.fx_problem_init(None) == L.FX_EINVAL


def test_fault_injection_hook_fails_plan_creation(monkeypatch):
    L = _lib()
    monkeypatch.setenv("FX_FAULT_INJECT_PLAN", "1")
    st, msg = _create(L.make_problem((16,), 1.0, 3, 1.0, 2.0))
    assert st == L.FX_ENOMEM and "FAULT_INJECT" in msg


def test_status_strings():
    L = _lib()
    for s in (0, -1, -2, -3, -4):
        assert L.lib.fx_status_string(s).startswith(b"FX_")


def test_problem_init_defaults():
    L = _lib()
    p = L.fx_problem()
    assert L.lib.fx_problem_init(ctypes.byref(p)) == L.FX_OK
    assert p.ndim == 1 and p.lambda_[0] == 1 and math.isnan(p.a[0]) and p.dx[0] == 1.0


def test_python_wrappers_reject_host_tensors():
    torch = pytest.importorskip("torch")
    import paper_1602_03395_amd as fx
    with pytest.raises(ValueError):
        fx.expand(torch.zeros(8, dtype=torch.complex128), 1.0, 1.0, 1.0, 2)
    with pytest.raises(ValueError):
        fx.expand(torch.zeros(8, dtype=torch.float64), 1.0, 1.0, 1.0, 2)


def test_spectrum_plan_rejects_bad_tables_on_host():
    L = _lib()
    import numpy as np
    DP = ctypes.POINTER(ctypes.c_double)
    p = L.make_problem((16,), 1.0, 3, 1.0, 2.0)
    h = ctypes.c_void_p()
    assert L.lib.fx_plan_create_spectrum(ctypes.byref(p), None, ctypes.byref(h)) == L.FX_EINVAL
    bad = np.zeros(48)
    bad[17] = math.nan
    arr = (DP * 3)()
    arr[0] = bad.ctypes.data_as(DP)
    st = L.lib.fx_plan_create_spectrum(ctypes.byref(p), arr, ctypes.byref(h))
    assert st == L.FX_EINVAL and b"non-finite" in L.lib.fx_last_error()
    # an invalid problem is rejected before the table is read
    p.lambda_[0] = 0
    assert L.lib.fx_plan_create_spectrum(ctypes.byref(p), arr, ctypes.byref(h)) == L.FX_EINVAL
    assert not h.value


def test_spectrum_wrapper_checks_table_length():
    torch = pytest.importorskip("torch")
    import numpy as np
    import paper_1602_03395_amd as fx
    with pytest.raises(ValueError):
        fx.Plan((16,), 1.0, 1.0, 2.0, 3, spectrum=[np.zeros(47)])
    with pytest.raises(ValueError):
        fx.Plan((16, 4), 1.0, 1.0, 2.0, 3, spectrum=[np.zeros(48)])
    k = fx.fine_wavenumbers(16, 3, 0.5)
    assert k.shape == (48,) and k[0] < 0 and abs(k[24]) == 0.0


def test_pair_entry_rejects_null_arguments():
    L = _lib()
    assert L.lib.fx_expand_pair(None, None, None, None, None, None, None) == L.FX_EINVAL
    assert L.lib.fx_plan_pair_workspace_size(None, None) == L.FX_EINVAL


def test_far_field_entry_rejects_null_arguments():
    L = _lib()
    assert L.lib.fx_far_field(None, None, None, None, None) == L.FX_EINVAL


def test_brute_force_entry_rejects_null_arguments():
    L = _lib()
    assert L.lib.fx_brute_force(None, None, None, None, None) == L.FX_EINVAL


def test_density_adjoint_entry_rejects_null_arguments():
    L = _lib()
    assert L.lib.fx_density_adjoint(None, None, None, None, None) == L.FX_EINVAL
