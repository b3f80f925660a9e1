"""Seeded random sweep over the lanes-per-line register kernels (k_ERW, k_ERG, k_EHG): problems whose
axes have g = gcd(lam, M) in {2, 4, 8} and pruned lengths P = M / g in {16, 32, 48, 64}, placed
first, last or between other axes (contiguous and strided lines), with odd and even magnification
cofactors, non-integer output offsets and forward and backward flights. Forward expansion and adjoint
against the oracle in plain FP64 (1e-12), the forward density in the FP32 form (1e-5)."""

import json

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_CASES = 24


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def make_case(i):
    rng = np.random.default_rng(np.random.SeedSequence([2024, i]))
    g = int(rng.choice([2, 4, 8]))
    P = int(rng.choice([16, 32, 48, 64] if g == 8 else [16, 32, 64]))
    M = g * P
    # lam = g k with k coprime to P (then gcd(lam, M) = g)
    ks = [k for k in range(1, 8) if np.gcd(k, P) == 1]
    lam_main = g * int(rng.choice(ks))
    ndim = int(rng.integers(1, 4))
    pos = int(rng.integers(0, ndim))
    shape, lam = [], []
    for j in range(ndim):
        if j == pos:
            shape.append(M)
            lam.append(lam_main)
        else:
            shape.append(int(rng.integers(2, 9)))
            lam.append(int(rng.integers(1, 4)))
    dx = tuple(float(v) for v in rng.uniform(0.6, 1.3, size=ndim))
    t = float(rng.choice([-1.0, 1.0]) * rng.uniform(2.0, 40.0))
    abar = [None] * ndim
    # a non-integer output offset on the main axis
    L = M * dx[pos]
    abar[pos] = -L / 2 + (1 - lam_main) * L / 2 + float(rng.uniform(-0.5, 0.5)) * dx[pos]
    return tuple(shape), tuple(lam), dx, t, abar


def _abar(fx, abar, shape, dx, lam):
    # the binding takes None for the default offset of an axis
    return [a if a is not None else -(s * d) / 2 + (1 - l) * s * d / 2 for a, s, d, l in zip(abar, shape, dx, lam)]


@pytest.mark.parametrize("i", range(N_CASES))
def test_lane_kernels_random_problem(fx, i, monkeypatch):
    monkeypatch.setenv("FX_ERW", "2")
    shape, lam, dx, t, abar = make_case(i)
    ab = _abar(fx, abar, shape, dx, lam)
    a = [-(s * d) / 2 for s, d in zip(shape, dx)]
    plan = fx.Plan(shape, dx, 1.0, t, lam, a=a, abar=ab, dtype=torch.complex128)
    desc = json.loads(plan.describe())
    kernels = {p["kernel"] for p in desc["passes"]} | {p["kernel"] for p in desc["adjoint_passes"]}
    f = workloads.random_field(shape, 3000 + i)
    out, rho = plan.expand(torch.from_numpy(f).cuda())
    y = workloads.random_field(shape, 4000 + i)
    gy = plan.expand_adjoint(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f, dx, 1.0, t, lam, a, ab)
    assert rel(out.cpu().numpy(), ref) <= 1e-12, (shape, lam, kernels)
    assert rel(gy.cpu().numpy(), oracle.expand_adjoint(y, dx, 1.0, t, lam, a, ab)) <= 1e-12, (shape, lam, kernels)
    plan32 = fx.Plan(shape, dx, 1.0, t, lam, a=a, abar=ab, dtype=torch.complex64)
    _, rho32 = plan32.expand(torch.from_numpy(f.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    ref32 = oracle.density(oracle.expand(f.astype(np.complex64).astype(np.complex128), dx, 1.0, t, lam, a, ab))
    assert rel(rho32.cpu().numpy().astype(np.float64), ref32) <= 1e-5, (shape, lam, kernels)


def test_sweep_reaches_every_lane_kernel(fx, monkeypatch):
    # the sweep's plans, taken together, run each of the three kernels
    monkeypatch.setenv("FX_ERW", "2")
    seen = set()
    for i in range(N_CASES):
        shape, lam, dx, t, abar = make_case(i)
        plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=torch.complex128)
        desc = json.loads(plan.describe())
        seen |= {p["kernel"] for p in desc["passes"]} | {p["kernel"] for p in desc["adjoint_passes"]}
    assert {"k_ERW", "k_ERG", "k_EHG"} <= seen, seen
