"""ctypes binding of ``libfx.so`` (the C ABI declared in ``include/fx.h``).

Argument marshalling only: every step of the expansion runs in the HIP
kernels of the library. Importing this module loads the in-tree library and
raises if it is missing; there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfx.so")

FX_OK = 0
FX_EINVAL = -1
FX_ENOMEM = -2
FX_EDEVICE = -3
FX_EUNSUPPORTED = -4

FX_PREC_C128 = 0
FX_PREC_C64_PHASE64 = 1

FX_SCHED_PAPER = 0
FX_SCHED_AXIS_FACTORISED = 1

FX_MAX_DIM = 3


class fx_problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("shape", ctypes.c_int64 * FX_MAX_DIM),
        ("dx", ctypes.c_double * FX_MAX_DIM),
        ("a", ctypes.c_double * FX_MAX_DIM),
        ("abar", ctypes.c_double * FX_MAX_DIM),
        ("lambda_", ctypes.c_int32 * FX_MAX_DIM),
        ("m_over_hbar", ctypes.c_double),
        ("t_flight", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
    ]


class FxError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _raise(status: int, where: str):
    msg = _lib.fx_last_error().decode(errors="replace")
    if status == FX_EINVAL:
        raise ValueError(f"{where}: {msg}")
    if status == FX_ENOMEM:
        raise MemoryError(f"{where}: {msg}")
    raise FxError(status, where, msg)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1602_03395_amd/build.py` "
            "(or __graft_entry__.build()); there is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P = ctypes.POINTER
    sigs = {
        "fx_problem_init": (ctypes.c_int, [P(fx_problem)]),
        "fx_plan_create": (ctypes.c_int, [P(fx_problem), P(vp)]),
        "fx_plan_create_spectrum": (ctypes.c_int, [P(fx_problem), P(P(ctypes.c_double)), P(vp)]),
        "fx_plan_destroy": (ctypes.c_int, [vp]),
        "fx_plan_num_terms": (ctypes.c_int, [vp, P(ctypes.c_int64)]),
        "fx_plan_workspace_size": (ctypes.c_int, [vp, P(ctypes.c_size_t)]),
        "fx_plan_set_workspace": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "fx_expand": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fx_expand_range": (ctypes.c_int, [vp, vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, vp]),
        "fx_density": (ctypes.c_int, [vp, vp, vp, vp]),
        "fx_column_density": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, vp]),
        "fx_expand_adjoint": (ctypes.c_int, [vp, vp, vp, vp]),
        "fx_density_adjoint": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fx_expand_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fx_expand_many": (ctypes.c_int, [vp, ctypes.c_int64, vp, vp, vp, vp]),
        "fx_density_adjoint_many": (ctypes.c_int, [vp, ctypes.c_int64, vp, vp, vp, vp]),
        "fx_expand_pair": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "fx_plan_pair_workspace_size": (ctypes.c_int, [vp, P(ctypes.c_size_t)]),
        "fx_far_field": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fx_brute_force": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fx_batch_create": (ctypes.c_int, [P(fx_problem), ctypes.c_int32, P(vp)]),
        "fx_batch_destroy": (ctypes.c_int, [vp]),
        "fx_batch_run": (ctypes.c_int, [vp, P(vp), P(vp), P(vp), vp]),
        "fx_batch_num_classes": (ctypes.c_int, [vp, P(ctypes.c_int32)]),
        "fx_batch_class": (ctypes.c_int, [vp, ctypes.c_int32, P(vp), P(ctypes.c_int32), P(ctypes.c_int64),
                                          P(ctypes.c_int32)]),
        "fx_batch_class_members": (ctypes.c_int, [vp, ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32]),
        "fx_batch_set_lanes": (ctypes.c_int, [vp, ctypes.c_int32]),
        "fx_plan_describe": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "fx_plan_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "fx_plan_pass_times": (ctypes.c_int, [vp, P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_double),
                                              ctypes.c_int32]),
        "fx_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "fx_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
lib = _lib


def check(status: int, where: str):
    if status != FX_OK:
        _raise(status, where)


def make_problem(shape, dx, lam, m_over_hbar, t, a=None, abar=None, precision=FX_PREC_C128,
                 schedule=FX_SCHED_PAPER) -> fx_problem:
    d = len(shape)
    if not 1 <= d <= 3:
        raise ValueError("ndim must be 1, 2 or 3")
    p = fx_problem()
    _lib.fx_problem_init(ctypes.byref(p))
    p.ndim = d

    def bc(v, cast):
        if v is None:
            return None
        if isinstance(v, (int, float)):
            return [cast(v)] * d
        v = list(v)
        if len(v) != d:
            raise ValueError("per-axis parameter has the wrong length")
        return [cast(x) for x in v]

    dxs = bc(dx, float)
    lams = bc(lam, int)
    av = bc(a, float)
    abv = bc(abar, float)
    for j in range(d):
        p.shape[j] = int(shape[j])
        p.dx[j] = dxs[j]
        p.lambda_[j] = lams[j]
        p.a[j] = math.nan if av is None else av[j]
        p.abar[j] = math.nan if abv is None else abv[j]
    p.m_over_hbar = float(m_over_hbar)
    p.t_flight = float(t)
    p.precision = int(precision)
    p.schedule = int(schedule)
    return p


def exported_symbols():
    return [n for n in dir(_lib) if n.startswith("fx_")]
