"""Parity of the one-wave-per-tile structured EA kernel (k_EAW: g = 8, pruned lengths P = 2, 3, 4, 6,
8) with the oracle, through the C ABI: contiguous lines (1-D, and partial term ranges, so the
kernel starts at q_b != 0 and accumulates), strided lines (2-D and 3-D), both precisions. Each case
checks that the plan really runs k_EAW on the axis."""

import json
import os

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    # shape, lam, dx, t
    ((16,), (8,), (0.5,), 3.0),            # P = 2
    ((24,), (8,), (0.7,), 4.0),            # P = 3
    ((32,), (8,), (1.0,), 9.0),            # P = 4
    ((48,), (40,), (1.0,), 40.0),          # P = 6
    ((64,), (40,), (1.0,), 60.0),          # P = 8
    ((64, 24), (40, 3), (1.0, 0.8), 30.0),   # strided lines, P = 8
    ((48, 20), (8, 5), (0.9, 1.0), 12.0),    # strided lines, P = 6
    ((24, 16, 12), (16, 8, 3), (1.0, 1.0, 1.2), 10.0),  # 3-D, EA along axis 0 with P = 3
    ((32, 16, 24), (40, 8, 2), (1.0, 0.7, 1.0), 25.0),  # 3-D, P = 4
    # table rows too large to stage in LDS (qn M beyond 64 KiB; FP64 only for the second case): the
    # kernel reads them from memory and keeps the first-step flip instead of the rotated reduction
    ((64,), (136,), (1.0,), 60.0),           # P = 8
    ((64, 4), (72, 2), (1.0, 0.9), 40.0),    # P = 8, strided
]


def _plan(fx, shape, lam, dx, t, dtype, monkeypatch):
    monkeypatch.setenv("FX_NO_SPLIT", "1")  # small cases would otherwise split EA into E + A
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    passes = json.loads(plan.describe())["passes"]
    assert any(p["kind"] == "EA" and p["kernel"] == "k_EAW" for p in passes), passes
    return plan


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_eaw_expansion_matches_oracle(fx, case, dtype, tol, monkeypatch):
    shape, lam, dx, t = CASES[case]
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 900 + case).astype(npdt)
    plan = _plan(fx, shape, lam, dx, t, dtype, monkeypatch)
    out, rho = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(rho.cpu().numpy().astype(np.float64), oracle.density(ref)) <= tol
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_eaw_blocked_and_partial_term_ranges(fx, dtype, tol, monkeypatch):
    # 1-D: term ranges run the kernel on partial blocks of the magnification index (q_b = 0, 13, 29,
    # block lengths not multiples of 8) and accumulate into the output
    shape, lam, dx, t = (64,), (40,), (1.0,), 60.0
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 77).astype(npdt)
    x = torch.from_numpy(f).cuda()
    plan = _plan(fx, shape, lam, dx, t, dtype, monkeypatch)
    acc = torch.zeros_like(x)
    plan.expand_range(x, acc, 0, 13)
    plan.expand_range(x, acc, 13, 29, accumulate=True)
    plan.expand_range(x, acc, 29, 40, accumulate=True)
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(acc.cpu().numpy().astype(np.complex128), ref) <= (tol if dtype == torch.complex128 else 1e-5)


E6_CASES = [
    # E along a 48-point axis with g = 8 (P = 6) in the register kernel k_ER: contiguous and strided lines
    ((5, 48), (3, 40), (1.0, 0.9), 20.0),
    ((3, 48, 4), (2, 40, 3), (1.0, 1.0, 0.7), 15.0),
    ((2, 7, 48), (3, 2, 8), (0.8, 1.0, 1.1), 6.0),
]


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", range(len(E6_CASES)))
def test_register_e_six_matches_oracle(fx, case, dtype, tol):
    shape, lam, dx, t = E6_CASES[case]
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 950 + case).astype(npdt)
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    passes = json.loads(plan.describe())["passes"]
    assert any(p["kind"] == "E" and p["kernel"] == "k_ER" and p["P"] == 6 for p in passes), passes
    out, rho = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(rho.cpu().numpy().astype(np.float64), oracle.density(ref)) <= tol
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= tol
