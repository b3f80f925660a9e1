"""Parity of the register E / EA kernel with a line over g P / 8 lanes (k_ERG: g = 2, 4, 8; pruned
lengths P = 16, 32, 64; contiguous and strided lines) with the oracle, through the C ABI: the fused
EA form (structured accumulate over q mod g) and the E form, partial term ranges (q_b != 0), both
precisions. Each case checks that the plan runs k_ERG for the pass kind it is meant to test."""

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
    # shape, lam, dx, t, kind of the k_ERG pass, keep EA fused
    ((64,), (50,), (1.0,), 40.0, "EA", True),                 # g = 2, P = 32, contiguous
    ((64,), (50,), (1.0,), 40.0, "E", False),                 # split into E + A
    ((256,), (20,), (1.0,), 60.0, "EA", True),                # g = 4, P = 64
    ((256,), (20,), (0.8,), 25.0, "E", False),
    ((64, 12), (50, 3), (1.0, 0.9), 30.0, "EA", True),        # strided EA (S = 4)
    ((6, 256), (3, 20), (1.1, 1.0), 50.0, "E", True),         # contiguous E (g = 4) in 2-D
    ((5, 64, 12), (2, 50, 3), (1.0, 0.7, 1.2), 20.0, "E", True),  # strided E (g = 2)
    ((128, 10), (24, 5), (0.9, 1.0), 15.0, "EA", True),       # g = 8, P = 16, strided
    ((512, 6), (40, 1), (1.0, 1.0), 45.0, "EA", True),        # g = 8, P = 64, strided
    ((32, 3), (6, 2), (1.0, 1.0), 8.0, "EA", True),           # g = 2, P = 16
]


def _plan(fx, case, dtype, monkeypatch):
    shape, lam, dx, t, kind, fused = case
    monkeypatch.setenv("FX_ERW", "2")  # also P = 16
    if fused:
        monkeypatch.setenv("FX_NO_SPLIT", "1")
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    passes = json.loads(plan.describe())["passes"]
    assert any(p["kind"] == kind and p["kernel"] == "k_ERG" for p in passes), passes
    return plan


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_erg_expansion_matches_oracle(fx, case, dtype, tol, monkeypatch):
    shape, lam, dx, t, _, _ = CASES[case]
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 1300 + case).astype(npdt)
    plan = _plan(fx, CASES[case], dtype, monkeypatch)
    out, rho = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(rho.cpu().numpy().astype(np.float64), oracle.density(ref)) <= tol
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", [0, 4])
def test_erg_partial_term_ranges(fx, case, dtype, tol, monkeypatch):
    # ranges of the term index start the fused pass at q_b != 0 (odd and even) and accumulate
    shape, lam, dx, t, _, _ = CASES[case]
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    f = workloads.random_field(shape, 77 + case).astype(npdt)
    x = torch.from_numpy(f).cuda()
    plan = _plan(fx, CASES[case], dtype, monkeypatch)
    nq = int(np.prod(lam))
    cuts = [0, 7, nq // 2 + 3, nq]
    acc = torch.zeros_like(x)
    for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
        plan.expand_range(x, acc, a, b, accumulate=i > 0)
    torch.cuda.synchronize()
    ref = oracle.expand(f.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(acc.cpu().numpy().astype(np.complex128), ref) <= tol


ADJ_CASES = [
    # shape, lam, dx, t (the adjoint schedule runs EH through k_EHG on the listed axes)
    ((64,), (50,), (1.0,), 40.0),                   # g = 2, P = 32, contiguous
    ((256,), (20,), (0.9,), 30.0),                  # g = 4, P = 64
    ((64, 12), (50, 3), (1.0, 0.9), 30.0),          # strided (g = 2)
    ((6, 256), (3, 20), (1.1, 1.0), 50.0),          # contiguous, after another axis
    ((256, 64), (20, 50), (1.0, 1.0), 25.0),        # both axes (g = 4 strided, g = 2 contiguous)
    ((128, 10), (24, 5), (0.9, 1.0), 15.0),         # g = 8, P = 16, strided
]


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("case", range(len(ADJ_CASES)))
def test_ehg_adjoint_matches_oracle(fx, case, dtype, tol, monkeypatch):
    shape, lam, dx, t = ADJ_CASES[case]
    monkeypatch.setenv("FX_ERW", "2")
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    adj = json.loads(plan.describe())["adjoint_passes"]
    assert any(p["kind"] == "EH" and p["kernel"] == "k_EHG" for p in adj), adj
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    y = workloads.random_field(shape, 1500 + case).astype(npdt)
    g = plan.expand_adjoint(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand_adjoint(y.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(g.cpu().numpy().astype(np.complex128), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_ehg_adjoint_blocked(fx, dtype, tol, monkeypatch):
    # a tiny workspace splits the outer magnification index into blocks: the adjoint E pass then
    # starts at a term index qb > 0 and accumulates into its output
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    shape, lam, dx, t = (256, 256), (20, 20), (1.0, 1.0), 23.0
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    d = json.loads(plan.describe())
    assert d["outer_block"] < 20 and any(p["kernel"] == "k_EHG" for p in d["adjoint_passes"]), d
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    y = workloads.random_field(shape, 1999).astype(npdt)
    g = plan.expand_adjoint(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand_adjoint(y.astype(np.complex128), dx, 1.0, t, lam)
    assert rel(g.cpu().numpy().astype(np.complex128), ref) <= tol
