"""PyTorch-facing calls with the names of the C ABI.

PyTorch supplies device memory and the current HIP stream; the expansion
itself (every table product, transform, fold, gather and sum) runs in the
kernels of ``libfx.so``. Precision follows the dtype of the input:
complex128 -> plain FP64 method, complex64 -> FP32 data with FP64-built
phase tables.
"""

from __future__ import annotations

import collections
import ctypes
import threading
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

_PLAN_CACHE: "collections.OrderedDict" = collections.OrderedDict()
_PLAN_LOCK = threading.Lock()
_PLAN_CACHE_MAX = 32


def _stream_ptr() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_field(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {x.device})")
    if x.dtype not in (torch.complex64, torch.complex128):
        raise ValueError(f"{name} must be complex64 or complex128 (got {x.dtype})")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def precision_of(dtype: torch.dtype) -> int:
    return L.FX_PREC_C128 if dtype == torch.complex128 else L.FX_PREC_C64_PHASE64


def real_dtype(dtype: torch.dtype) -> torch.dtype:
    return torch.float64 if dtype == torch.complex128 else torch.float32


class Plan:
    """Owns one ``fx_plan`` (tables on the device, tiling, schedule)."""

    def __init__(self, shape, dx, m_over_hbar, t, lam, a=None, abar=None, dtype=torch.complex128,
                 schedule: str = "paper", spectrum=None):
        """``spectrum``: optional per-axis list of t * omega_j in radians on the fine wave
        numbers (``fine_wavenumbers``), None entries keeping the free-particle phase."""
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        sched = {"paper": L.FX_SCHED_PAPER, "axis_factorised": L.FX_SCHED_AXIS_FACTORISED}[schedule]
        prob = L.make_problem(self.shape, dx, lam, m_over_hbar, t, a, abar, precision_of(dtype), sched)
        self.problem = prob
        h = ctypes.c_void_p()
        if spectrum is None:
            L.check(L.lib.fx_plan_create(ctypes.byref(prob), ctypes.byref(h)), "fx_plan_create")
        else:
            d = len(self.shape)
            if len(spectrum) != d:
                raise ValueError(f"spectrum needs one entry per axis ({d})")
            DP = ctypes.POINTER(ctypes.c_double)
            keep = []
            arr = (DP * 3)()
            for j, ph in enumerate(spectrum):
                if ph is None:
                    continue
                ph = np.ascontiguousarray(np.asarray(ph, dtype=np.float64))
                n = int(prob.lambda_[j]) * self.shape[j]
                if ph.shape != (n,):
                    raise ValueError(f"spectrum[{j}] must hold lam*M = {n} values")
                keep.append(ph)
                arr[j] = ph.ctypes.data_as(DP)
            L.check(L.lib.fx_plan_create_spectrum(ctypes.byref(prob), arr, ctypes.byref(h)),
                    "fx_plan_create_spectrum")
        self._h = h
        self._ws = None

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            L.lib.fx_plan_destroy(h)
            self._h = None

    def num_terms(self) -> int:
        q = ctypes.c_int64()
        L.check(L.lib.fx_plan_num_terms(self._h, ctypes.byref(q)), "fx_plan_num_terms")
        return q.value

    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        L.check(L.lib.fx_plan_workspace_size(self._h, ctypes.byref(b)), "fx_plan_workspace_size")
        return b.value

    def use_torch_workspace(self, device=None):
        """Let PyTorch own the scratch memory (one uint8 tensor kept alive by the plan)."""
        n = self.workspace_size()
        ws = torch.empty(n + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-ws.data_ptr()) % 256
        L.check(L.lib.fx_plan_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr() + off), n),
                "fx_plan_set_workspace")
        self._ws = ws

    def set_timing(self, enable: bool = True):
        L.check(L.lib.fx_plan_set_timing(self._h, 1 if enable else 0), "fx_plan_set_timing")

    def pass_times(self):
        """[(launches, total_ms)] per pass of the schedule since the last call (waits for the events)."""
        n = ctypes.c_int32()
        cap = 64
        la = (ctypes.c_int64 * cap)()
        ms = (ctypes.c_double * cap)()
        L.check(L.lib.fx_plan_pass_times(self._h, ctypes.byref(n), la, ms, cap), "fx_plan_pass_times")
        return [(la[i], ms[i]) for i in range(min(n.value, cap))]

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        L.check(L.lib.fx_plan_describe(self._h, buf, len(buf)), "fx_plan_describe")
        return buf.value.decode()

    # -- calls ---------------------------------------------------------------------------
    def expand(self, psi0: torch.Tensor, want_psi: bool = True, want_rho: bool = True,
               psi_out: Optional[torch.Tensor] = None, rho_out: Optional[torch.Tensor] = None):
        _check_field(psi0, "psi0")
        self._check_shape(psi0)
        if want_psi and psi_out is None:
            psi_out = torch.empty_like(psi0)
        if want_rho and rho_out is None:
            rho_out = torch.empty(psi0.shape, dtype=real_dtype(psi0.dtype), device=psi0.device)
        L.check(L.lib.fx_expand(self._h, _ptr(psi0), _ptr(psi_out) if want_psi else None,
                                _ptr(rho_out) if want_rho else None, _stream_ptr()), "fx_expand")
        return (psi_out if want_psi else None), (rho_out if want_rho else None)

    def expand_many(self, psi0: torch.Tensor, want_psi: bool = True, want_rho: bool = True,
                    psi_out: Optional[torch.Tensor] = None, rho_out: Optional[torch.Tensor] = None):
        """A stack [count, *shape] of independent fields: returns (psi or None, rho or None), see
        ``fx_expand_many``."""
        _check_field(psi0, "psi0")
        count = self._check_stack(psi0)
        if want_psi and psi_out is None:
            psi_out = torch.empty_like(psi0)
        if want_rho and rho_out is None:
            rho_out = torch.empty(psi0.shape, dtype=real_dtype(psi0.dtype), device=psi0.device)
        L.check(L.lib.fx_expand_many(self._h, count, _ptr(psi0), _ptr(psi_out) if want_psi else None,
                                     _ptr(rho_out) if want_rho else None, _stream_ptr()), "fx_expand_many")
        return (psi_out if want_psi else None), (rho_out if want_rho else None)

    def density_adjoint_many(self, psibar: torch.Tensor, grad_rho: torch.Tensor,
                             grad_in: Optional[torch.Tensor] = None):
        """Stacked form of ``density_adjoint`` ([count, *shape]), see ``fx_density_adjoint_many``."""
        _check_field(psibar, "psibar")
        count = self._check_stack(psibar)
        if grad_rho.dtype != real_dtype(self.dtype) or grad_rho.device.type != "cuda":
            raise ValueError("grad_rho must be a device tensor of the plan's real dtype")
        grad_rho = grad_rho.contiguous()
        if tuple(grad_rho.shape) != tuple(psibar.shape):
            raise ValueError("grad_rho has the wrong shape")
        if grad_in is None:
            grad_in = torch.empty_like(psibar)
        L.check(L.lib.fx_density_adjoint_many(self._h, count, _ptr(psibar), _ptr(grad_rho), _ptr(grad_in),
                                              _stream_ptr()), "fx_density_adjoint_many")
        return grad_in

    def _check_stack(self, x: torch.Tensor) -> int:
        if x.dim() != len(self.shape) + 1 or tuple(x.shape[1:]) != self.shape:
            raise ValueError(f"a stack of fields must have shape [count, *{self.shape}] (got {tuple(x.shape)})")
        if x.dtype != self.dtype:
            raise ValueError(f"tensor dtype {x.dtype} does not match the plan's {self.dtype}")
        if x.shape[0] < 1:
            raise ValueError("a stack needs at least one field")
        return int(x.shape[0])

    def expand_range(self, psi0: torch.Tensor, psi_acc: torch.Tensor, q_begin: int, q_end: int,
                     accumulate: bool = False):
        _check_field(psi0, "psi0")
        _check_field(psi_acc, "psi_acc")
        self._check_shape(psi0)
        self._check_shape(psi_acc)
        L.check(L.lib.fx_expand_range(self._h, _ptr(psi0), _ptr(psi_acc), int(q_begin), int(q_end),
                                      1 if accumulate else 0, _stream_ptr()), "fx_expand_range")
        return psi_acc

    def density(self, psi: torch.Tensor, rho: Optional[torch.Tensor] = None):
        _check_field(psi, "psi")
        self._check_shape(psi)
        if rho is None:
            rho = torch.empty(psi.shape, dtype=real_dtype(psi.dtype), device=psi.device)
        L.check(L.lib.fx_density(self._h, _ptr(psi), _ptr(rho), _stream_ptr()), "fx_density")
        return rho

    def column_density(self, rho: torch.Tensor, axis: int):
        if rho.dtype != real_dtype(self.dtype) or rho.device.type != "cuda" or not rho.is_contiguous():
            raise ValueError("rho must be a contiguous device tensor of the plan's real dtype")
        if tuple(rho.shape) != self.shape:
            raise ValueError("rho has the wrong shape")
        d = len(self.shape)
        if not 0 <= axis < d:
            raise ValueError("axis out of range")
        img_shape = tuple(s for i, s in enumerate(self.shape) if i != axis)
        img = torch.empty(img_shape, dtype=rho.dtype, device=rho.device)
        L.check(L.lib.fx_column_density(self._h, _ptr(rho), int(axis), _ptr(img), _stream_ptr()),
                "fx_column_density")
        return img

    def expand_adjoint(self, grad_out: torch.Tensor, grad_in: Optional[torch.Tensor] = None):
        _check_field(grad_out, "grad_psi_out")
        self._check_shape(grad_out)
        if grad_in is None:
            grad_in = torch.empty_like(grad_out)
        L.check(L.lib.fx_expand_adjoint(self._h, _ptr(grad_out), _ptr(grad_in), _stream_ptr()),
                "fx_expand_adjoint")
        return grad_in

    def density_adjoint(self, psibar: torch.Tensor, grad_rho: torch.Tensor,
                        grad_in: Optional[torch.Tensor] = None):
        """grad_psi0 = U^H (2 grad_rho psibar), see ``fx_density_adjoint``."""
        _check_field(psibar, "psibar")
        self._check_shape(psibar)
        if grad_rho.dtype != real_dtype(self.dtype) or grad_rho.device.type != "cuda":
            raise ValueError("grad_rho must be a device tensor of the plan's real dtype")
        grad_rho = grad_rho.contiguous()
        if tuple(grad_rho.shape) != self.shape:
            raise ValueError("grad_rho has the wrong shape")
        if grad_in is None:
            grad_in = torch.empty_like(psibar)
        L.check(L.lib.fx_density_adjoint(self._h, _ptr(psibar), _ptr(grad_rho), _ptr(grad_in), _stream_ptr()),
                "fx_density_adjoint")
        return grad_in

    def pair_workspace_size(self) -> int:
        b = ctypes.c_size_t()
        L.check(L.lib.fx_plan_pair_workspace_size(self._h, ctypes.byref(b)), "fx_plan_pair_workspace_size")
        return b.value

    def expand_pair(self, psi: torch.Tensor, psi_plus: torch.Tensor):
        """Positive-P pair: returns (Psibar, Psibar^+, n = Psibar^+ * Psibar), see ``fx_expand_pair``."""
        _check_field(psi, "psi")
        _check_field(psi_plus, "psi_plus")
        self._check_shape(psi)
        self._check_shape(psi_plus)
        out = torch.empty_like(psi)
        out_plus = torch.empty_like(psi)
        n = torch.empty_like(psi)
        L.check(L.lib.fx_expand_pair(self._h, _ptr(psi), _ptr(psi_plus), _ptr(out), _ptr(out_plus), _ptr(n),
                                     _stream_ptr()), "fx_expand_pair")
        return out, out_plus, n

    def far_field(self, psi0: torch.Tensor, want_amp: bool = True):
        """Far-field estimate on the magnified lattice: returns (amp or None, rho_ff), see ``fx_far_field``."""
        _check_field(psi0, "psi0")
        self._check_shape(psi0)
        amp = torch.empty_like(psi0) if want_amp else None
        rho = torch.empty(psi0.shape, dtype=real_dtype(psi0.dtype), device=psi0.device)
        L.check(L.lib.fx_far_field(self._h, _ptr(psi0), _ptr(amp), _ptr(rho), _stream_ptr()), "fx_far_field")
        return amp, rho

    def brute_force(self, psi0: torch.Tensor, want_psi: bool = True):
        """Padded-lattice propagation (comparator): returns (psi or None, rho), see ``fx_brute_force``."""
        _check_field(psi0, "psi0")
        self._check_shape(psi0)
        out = torch.empty_like(psi0) if want_psi else None
        rho = torch.empty(psi0.shape, dtype=real_dtype(psi0.dtype), device=psi0.device)
        L.check(L.lib.fx_brute_force(self._h, _ptr(psi0), _ptr(out), _ptr(rho), _stream_ptr()), "fx_brute_force")
        return out, rho

    def _check_shape(self, x: torch.Tensor):
        if tuple(x.shape) != self.shape:
            raise ValueError(f"tensor shape {tuple(x.shape)} does not match the plan's {self.shape}")
        if x.dtype != self.dtype:
            raise ValueError(f"tensor dtype {x.dtype} does not match the plan's {self.dtype}")


def _key(shape, dx, m_over_hbar, t, lam, a, abar, dtype, schedule):
    def tup(v):
        if v is None:
            return None
        if isinstance(v, (int, float)):
            return (float(v),)
        return tuple(float(x) for x in v)
    return (tuple(shape), tup(dx), float(m_over_hbar), float(t), tup(lam), tup(a), tup(abar), str(dtype),
            schedule, torch.cuda.current_device())


def get_plan(shape, dx, m_over_hbar, t, lam, a=None, abar=None, dtype=torch.complex128,
             schedule: str = "paper") -> Plan:
    k = _key(shape, dx, m_over_hbar, t, lam, a, abar, dtype, schedule)
    with _PLAN_LOCK:
        if k in _PLAN_CACHE:
            _PLAN_CACHE.move_to_end(k)
            return _PLAN_CACHE[k]
    plan = Plan(shape, dx, m_over_hbar, t, lam, a, abar, dtype, schedule)
    with _PLAN_LOCK:
        _PLAN_CACHE[k] = plan
        while len(_PLAN_CACHE) > _PLAN_CACHE_MAX:
            _PLAN_CACHE.popitem(last=False)
    return plan


def fine_wavenumbers(M: int, lam: int, dx: float) -> np.ndarray:
    """The lam*M fine wave numbers 2 pi l / (lam M dx), ascending from l = -floor(lam M / 2):
    the points at which a ``spectrum`` table samples t * omega."""
    N = int(lam) * int(M)
    return 2.0 * np.pi * np.arange(-(N // 2), -(N // 2) + N, dtype=np.float64) / (N * float(dx))


def _plan_for(x, dx, m_over_hbar, t, lam, a, abar, schedule, spectrum):
    if spectrum is None:
        return get_plan(x.shape, dx, m_over_hbar, t, lam, a, abar, x.dtype, schedule)
    return Plan(x.shape, dx, m_over_hbar, t, lam, a, abar, x.dtype, schedule, spectrum=spectrum)


def expand(psi0: torch.Tensor, dx, m_over_hbar: float, t: float, lam, a=None, abar=None,
           want_psi: bool = True, schedule: str = "paper",
           spectrum=None) -> Tuple[Optional[torch.Tensor], torch.Tensor]:
    """Free flight of ``psi0`` for time t onto the lattice magnified by ``lam``: returns (psi, rho).

    ``spectrum`` (optional) replaces the free-particle phase per axis, see ``Plan``."""
    _check_field(psi0, "psi0")
    plan = _plan_for(psi0, dx, m_over_hbar, t, lam, a, abar, schedule, spectrum)
    return plan.expand(psi0, want_psi=want_psi, want_rho=True)


def expand_adjoint(grad_out: torch.Tensor, dx, m_over_hbar: float, t: float, lam, a=None, abar=None,
                   schedule: str = "paper", spectrum=None) -> torch.Tensor:
    _check_field(grad_out, "grad_psi_out")
    plan = _plan_for(grad_out, dx, m_over_hbar, t, lam, a, abar, schedule, spectrum)
    return plan.expand_adjoint(grad_out)


def column_density(rho: torch.Tensor, axis: int, dx, m_over_hbar: float, t: float, lam, a=None, abar=None,
                   dtype=None) -> torch.Tensor:
    dtype = dtype or (torch.complex128 if rho.dtype == torch.float64 else torch.complex64)
    plan = get_plan(rho.shape, dx, m_over_hbar, t, lam, a, abar, dtype)
    return plan.column_density(rho, axis)


class Batch:
    """Owns one ``fx_batch``: a ragged list of problems run as one captured graph per call.

    ``problems`` is a list of dicts with keys shape, dx, m_over_hbar, t, lam and
    optionally a, abar; all realizations share ``dtype``.
    """

    def __init__(self, problems, dtype=torch.complex64, schedule: str = "paper"):
        sched = {"paper": L.FX_SCHED_PAPER, "axis_factorised": L.FX_SCHED_AXIS_FACTORISED}[schedule]
        self.dtype = dtype
        self.shapes = [tuple(int(x) for x in pr["shape"]) for pr in problems]
        arr = (L.fx_problem * len(problems))()
        for i, pr in enumerate(problems):
            arr[i] = L.make_problem(pr["shape"], pr["dx"], pr["lam"], pr.get("m_over_hbar", 1.0), pr["t"],
                                    pr.get("a"), pr.get("abar"), precision_of(dtype), sched)
        self._arr = arr
        h = ctypes.c_void_p()
        L.check(L.lib.fx_batch_create(arr, len(problems), ctypes.byref(h)), "fx_batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            L.lib.fx_batch_destroy(h)
            self._h = None

    def __len__(self):
        return len(self.shapes)

    def classes(self):
        """Shape classes in issue order: dicts with the class plan (owned by the batch), the
        batch indices of its realizations, the realizations per work item and the lane."""
        n = ctypes.c_int32()
        L.check(L.lib.fx_batch_num_classes(self._h, ctypes.byref(n)), "fx_batch_num_classes")
        out = []
        for i in range(n.value):
            h = ctypes.c_void_p()
            mem = ctypes.c_int32()
            grp = ctypes.c_int64()
            lane = ctypes.c_int32()
            L.check(L.lib.fx_batch_class(self._h, i, ctypes.byref(h), ctypes.byref(mem), ctypes.byref(grp),
                                         ctypes.byref(lane)), "fx_batch_class")
            idx = (ctypes.c_int32 * max(1, mem.value))()
            L.check(L.lib.fx_batch_class_members(self._h, i, idx, mem.value), "fx_batch_class_members")
            members = [int(idx[k]) for k in range(mem.value)]
            plan = _BatchClassPlan(h, self.shapes[members[0]], self.dtype, self)
            out.append({"plan": plan, "members": members, "group": int(grp.value), "lane": int(lane.value)})
        return out

    def set_lanes(self, lanes: int):
        """Lane streams the classes run on (1: one kernel at a time on the caller's stream, for
        per-pass timing of each kernel alone; 0: the tuned value), see ``fx_batch_set_lanes``."""
        L.check(L.lib.fx_batch_set_lanes(self._h, int(lanes)), "fx_batch_set_lanes")

    def run(self, psis, psi_outs=None, rho_outs=None, want_psi=True, want_rho=True):
        n = len(self.shapes)
        if len(psis) != n:
            raise ValueError("wrong number of input fields")
        for x, shp in zip(psis, self.shapes):
            _check_field(x, "psi0")
            if tuple(x.shape) != shp or x.dtype != self.dtype:
                raise ValueError("input field does not match its problem")
        if want_psi and psi_outs is None:
            psi_outs = [torch.empty_like(x) for x in psis]
        if want_rho and rho_outs is None:
            rho_outs = [torch.empty(x.shape, dtype=real_dtype(x.dtype), device=x.device) for x in psis]
        VP = ctypes.c_void_p * n
        pin = VP(*[x.data_ptr() for x in psis])
        pout = VP(*[x.data_ptr() for x in psi_outs]) if want_psi else None
        prho = VP(*[x.data_ptr() for x in rho_outs]) if want_rho else None
        L.check(L.lib.fx_batch_run(self._h, pin, pout, prho, _stream_ptr()), "fx_batch_run")
        return (psi_outs if want_psi else None), (rho_outs if want_rho else None)


class _BatchClassPlan(Plan):
    """A class plan owned by a ``Batch`` (describe, per-pass timing); never destroyed here."""

    def __init__(self, handle, shape, dtype, owner):
        self.shape = tuple(int(x) for x in shape)
        self.dtype = dtype
        self._h = handle
        self._ws = None
        self._owner = owner  # keeps the batch, and so the plan, alive

    def __del__(self):
        pass


def expand_batch(psis, specs, schedule: str = "paper"):
    """Expands a ragged list of fields; ``specs`` is one dict (shared) or one per field."""
    if isinstance(specs, dict):
        specs = [specs] * len(psis)
    probs = [dict(s, shape=tuple(x.shape)) for s, x in zip(specs, psis)]
    b = Batch(probs, dtype=psis[0].dtype, schedule=schedule)
    return b.run(psis)


def _problem_ndim(x: torch.Tensor, lam) -> int:
    """Number of lattice axes: len(lam) when lam is a sequence, else every axis of x."""
    if isinstance(lam, (int, float, np.integer, np.floating)):
        return x.dim()
    return len(lam)


class ExpandDensity(torch.autograd.Function):
    """rho = |U psi0|^2 with the hand-written adjoint U^H for the backward pass.

    For a real loss L(rho), PyTorch's complex gradient convention
    (dL/dRe + i dL/dIm) gives grad_psi0 = U^H (2 * grad_rho * Psibar).

    psi0 holds one field of d = len(lam) axes, or a stack [count, *shape] of independent
    fields (one more leading axis than lam has entries), which forward and backward each
    process in one library call. A scalar lam means one field over every axis of psi0.
    """

    @staticmethod
    def forward(ctx, psi0, dx, m_over_hbar, t, lam, a=None, abar=None, schedule="paper"):
        psi0 = psi0.contiguous()
        d = _problem_ndim(psi0, lam)
        if psi0.dim() == d:
            plan = get_plan(psi0.shape, dx, m_over_hbar, t, lam, a, abar, psi0.dtype, schedule)
            psi, rho = plan.expand(psi0, want_psi=True, want_rho=True)
            ctx.stacked = False
        elif psi0.dim() == d + 1:
            plan = get_plan(psi0.shape[1:], dx, m_over_hbar, t, lam, a, abar, psi0.dtype, schedule)
            psi, rho = plan.expand_many(psi0, want_psi=True, want_rho=True)
            ctx.stacked = True
        else:
            raise ValueError(f"psi0 must have {d} axes (one field) or {d + 1} (a stack of fields), "
                             f"got {psi0.dim()}")
        ctx.plan = plan
        ctx.save_for_backward(psi)
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        (psi,) = ctx.saved_tensors
        g = grad_rho.to(psi.real.dtype)
        if ctx.stacked:
            grad = ctx.plan.density_adjoint_many(psi, g)
        else:
            grad = ctx.plan.density_adjoint(psi, g)
        return grad, None, None, None, None, None, None, None


def expand_density(psi0, dx, m_over_hbar, t, lam, a=None, abar=None, schedule="paper"):
    return ExpandDensity.apply(psi0, dx, m_over_hbar, t, lam, a, abar, schedule)
