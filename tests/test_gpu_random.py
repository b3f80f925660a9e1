"""Seeded sweep of small random problems through every kernel family (register and transform forms,
structured and direct accumulates, odd and power-of-two lengths, 1-D to 3-D), each compared with
the FP64 oracle: Psi-bar to 1e-12 in FP64, the density to 1e-5 in the FP32 form, and the adjoint
to 1e-12 in FP64."""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


def draw_case(seed: int):
    """Shape, magnification, spacing, time and output offset shift of case `seed`: lengths are
    drawn so that g = gcd(lam, M) takes the values the register kernels specialise on."""
    rng = np.random.default_rng(seed)
    ndim = int(rng.integers(1, 4))
    shape, lam, dx = [], [], []
    for _ in range(ndim):
        lj = int(rng.choice([1, 2, 3, 4, 5, 6, 8, 12, 16, 32]))
        pj = int(rng.choice([1, 2, 3, 4, 5, 6, 8, 12, 16]))
        mj = int(np.gcd(lj, 64)) * pj if rng.random() < 0.7 else int(rng.integers(1, 40))
        shape.append(max(1, min(mj, 128 if ndim == 1 else 32)))
        lam.append(lj)
        dx.append(float(rng.uniform(0.5, 1.5)))
    t = float(rng.uniform(1.0, 30.0)) * (1 if rng.random() < 0.8 else -1)
    shift = float(rng.uniform(-0.5, 0.5))
    return tuple(shape), tuple(lam), tuple(dx), t, shift


SEEDS = list(range(100, 160))


@pytest.mark.parametrize("seed", SEEDS)
def test_random_problem_matches_oracle(fx, seed):
    shape, lam, dx, t, shift = draw_case(seed)
    print("random case", seed, shape, lam, flush=True)
    psi_np = workloads.random_field(shape, seed)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    ref = oracle.expand(psi_np, dx, 1.0, t, lam, a, abar)
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        plan = fx.Plan(shape, dx, 1.0, t, lam, list(a), list(abar), dtype)
        out, rho = plan.expand(torch.from_numpy(psi_np).to(dtype).cuda())
        if dtype == torch.complex128:
            assert rel(out.cpu().numpy(), ref) <= tol
        assert rel(rho.cpu().numpy(), oracle.density(ref)) <= tol


@pytest.mark.parametrize("seed", SEEDS[::3])
def test_random_adjoint_matches_oracle(fx, seed):
    shape, lam, dx, t, shift = draw_case(seed)
    print("random adjoint", seed, shape, lam, flush=True)
    y_np = workloads.random_field(shape, seed + 1000)
    plan = fx.Plan(shape, dx, 1.0, t, lam)
    g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, t, lam)) <= 1e-12
