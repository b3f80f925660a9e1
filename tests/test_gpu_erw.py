"""Parity of the register E kernel with a line per 8 P / V lanes (k_ERW: g = 8, pruned lengths P = 16,
32, 48, 64, contiguous lines) with the oracle, through the C ABI: 1-D (the fused pass split into E + A),
2-D and 3-D problems whose last axis runs through it, blocked and partial term ranges (the kernel
starting at q_b != 0), both precisions. Each case checks that the plan really runs k_ERW."""

import json

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
    ((512,), (40,), (1.0,), 60.0),               # P = 64
    ((256,), (8,), (0.7,), 9.0),                 # P = 32
    ((128,), (24,), (0.9,), 5.0),                # P = 16
    ((6, 512), (5, 40), (1.0, 0.8), 30.0),       # E along the contiguous axis of a 2-D problem
    ((3, 5, 256), (2, 3, 24), (1.1, 1.0, 0.6), 12.0),  # 3-D
    ((9, 384 // 3), (4, 40), (1.0, 1.0), 20.0),  # P = 16 with 9 lines per slice (a ragged tile)
    ((384,), (40,), (1.0,), 45.0),               # P = 48 (six values per lane)
    ((5, 384), (3, 8), (0.9, 1.0), 18.0),        # P = 48, 2-D
    ((2, 3, 384), (2, 5, 40), (1.0, 1.2, 0.8), 22.0),  # P = 48, 3-D
]


def _plan(fx, shape, lam, dx, t, dtype, monkeypatch):
    monkeypatch.setenv("FX_ERW", "2")  # also P = 16
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    passes = json.loads(plan.describe())["passes"]
    assert any(p["kind"] == "E" and p["kernel"] == "k_ERW" for p in passes), passes
    return plan


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_erw_expansion_matches_oracle(fx, case, dtype, tol, monkeypatch):
    shape, lam, dx, t = CASES[case]
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 700 + case).astype(npdt)
    plan = _plan(fx, shape, lam, dx, t, dtype, monkeypatch)
    out, rho = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(rho.cpu().numpy().astype(np.float64), oracle.density(ref)) <= tol
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_erw_partial_term_ranges(fx, dtype, tol, monkeypatch):
    # 2-D, outer index along the contiguous axis: ranges start the kernel at q_b = 0, 7, 131 with
    # block lengths that are not multiples of the workgroup's term chunk
    shape, lam, dx, t = (6, 512), (5, 40), (1.0, 0.8), 30.0
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 71).astype(npdt)
    x = torch.from_numpy(f).cuda()
    plan = _plan(fx, shape, lam, dx, t, dtype, monkeypatch)
    acc = torch.zeros_like(x)
    plan.expand_range(x, acc, 0, 7)
    plan.expand_range(x, acc, 7, 131, accumulate=True)
    plan.expand_range(x, acc, 131, 200, accumulate=True)
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(acc.cpu().numpy().astype(np.complex128), ref) <= tol


def test_erw_blocked_outer_index(fx, monkeypatch):
    # a workspace cap forces blocks of the outer magnification index through the same passes
    shape, lam, dx, t = (4, 8, 512), (3, 2, 40), (1.0, 1.0, 1.0), 25.0
    f = workloads.random_field(shape, 5).astype(np.complex64)
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    plan = _plan(fx, shape, lam, dx, t, torch.complex64, monkeypatch)
    assert json.loads(plan.describe())["outer_block"] < 40
    _, rho = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.density(oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam))
    assert rel(rho.cpu().numpy().astype(np.float64), ref) <= 1e-5
