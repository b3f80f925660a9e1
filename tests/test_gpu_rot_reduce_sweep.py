"""Seeded random sweep over the register kernels whose sum over the lanes of a line is the select-free
rotated reduction (power-of-two P = M / g <= 8 with g >= P: k_ER for E passes, k_EAR and k_EAW for EA
passes): g from 2 to 64, the axis placed first, last or between other axes (contiguous and strided
lines), odd magnification cofactors, non-integer output offsets, forward and backward flights.
Expansion against the oracle in plain FP64 (1e-12) and the density in the FP32 form (1e-5), once with
the default kernel choice and once with the EA pass forced to k_EAR."""

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
    rng = np.random.default_rng(np.random.SeedSequence([1602, i]))
    # every P with the axis both as an E pass (not the slowest active axis: k_ER) and as the EA pass
    P = (2, 4, 8)[i % 3]
    e_pass = (i // 3) % 2 == 1
    g = int(rng.choice([v for v in (2, 4, 8, 16, 32, 64) if v >= P]))
    M = g * P
    # lam = g k with k odd (then gcd(lam, M) = g for power-of-two P)
    lam_main = g * int(rng.choice([1, 3, 5]))
    ndim = int(rng.integers(2, 4)) if e_pass else int(rng.integers(1, 4))
    pos = int(rng.integers(1, ndim)) if e_pass else 0
    shape, lam = [], []
    for j in range(ndim):
        if j == pos:
            shape.append(M)
            lam.append(lam_main)
        else:
            shape.append(int(rng.integers(2, 7)))
            lam.append(int(rng.integers(2, 4)))
    dx = tuple(float(v) for v in rng.uniform(0.6, 1.3, size=ndim))
    t = float(rng.choice([-1.0, 1.0]) * rng.uniform(2.0, 30.0))
    abar = [-(s * d) / 2 + (1 - l) * s * d / 2 for s, d, l in zip(shape, dx, lam)]
    abar[pos] += float(rng.uniform(-0.5, 0.5)) * dx[pos]
    a = [-(s * d) / 2 for s, d in zip(shape, dx)]
    return tuple(shape), tuple(lam), dx, t, a, abar, P


FORCE_EAR = {"FX_NO_EAW": "1", "FX_NO_EAS": "1", "FX_NO_SPLIT": "1"}


@pytest.mark.parametrize("force_ear", [False, True])
@pytest.mark.parametrize("i", range(N_CASES))
def test_rotated_reduction_random_problem(fx, i, force_ear, monkeypatch):
    if force_ear:
        for k, v in FORCE_EAR.items():
            monkeypatch.setenv(k, v)
    shape, lam, dx, t, a, abar, P = make_case(i)
    print("rotated reduction", i, shape, lam, force_ear, flush=True)
    f = workloads.random_field(shape, 5000 + i)
    plan = fx.Plan(shape, dx, 1.0, t, lam, a=a, abar=abar, dtype=torch.complex128)
    kernels = {(p["kernel"], p.get("P")) for p in json.loads(plan.describe())["passes"]}
    out, _ = plan.expand(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = oracle.expand(f, dx, 1.0, t, lam, a, abar)
    assert rel(out.cpu().numpy(), ref) <= 1e-12, (shape, lam, kernels)
    plan32 = fx.Plan(shape, dx, 1.0, t, lam, a=a, abar=abar, dtype=torch.complex64)
    f32 = f.astype(np.complex64)
    _, rho32 = plan32.expand(torch.from_numpy(f32).cuda())
    torch.cuda.synchronize()
    ref32 = oracle.density(oracle.expand(f32.astype(np.complex128), dx, 1.0, t, lam, a, abar))
    assert rel(rho32.cpu().numpy().astype(np.float64), ref32) <= 1e-5, (shape, lam, kernels)


def test_sweep_reaches_the_rotated_kernels(fx, monkeypatch):
    # taken together, the sweep's plans run k_ER and k_EAR with P = 2, 4 and 8
    seen = set()
    for force_ear in (False, True):
        for k in FORCE_EAR:
            monkeypatch.delenv(k, raising=False)
        if force_ear:
            for k, v in FORCE_EAR.items():
                monkeypatch.setenv(k, v)
        for i in range(N_CASES):
            shape, lam, dx, t, a, abar, P = make_case(i)
            plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=torch.complex128)
            seen |= {(p["kernel"], p.get("P")) for p in json.loads(plan.describe())["passes"]}
    for kern in ("k_ER", "k_EAR"):
        assert {(kern, P) for P in (2, 4, 8)} <= seen, sorted(seen)
