"""Parity of the positive-P pair call (``fx_expand_pair``) with the oracle: psibar,
psibar^+ and the estimator n = psibar^+ psibar. Bars: FP64 relative L2 <= 1e-12 for
all three; FP32 form <= 1e-5 in n (the analogue of rho)."""

import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


CASES = [
    # shape, lam, dx, t, m_over_hbar
    ((96,), (6,), (1.0,), 30.0, 1.0),
    ((48, 40), (3, 4), (1.0, 0.8), 30.0, 1.0),
    ((64, 64), (8, 16), (1.0, 1.0), 200.0, 1.0),
    ((12, 24, 48), (2, 3, 4), (1.0, 1.0, 1.0), 7.0, 1.3),
    ((256, 256), (20, 20), (1.0, 1.0), 600.0, 1.0),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("schedule", ["paper", "axis_factorised"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_pair_parity(fx, case, schedule, dtype):
    shape, lam, dx, t, moh = CASES[case]
    say("pair case", shape, lam, schedule, dtype)
    cdt = np.complex128 if dtype == "c128" else np.complex64
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi_np = workloads.random_field(shape, 500 + case).astype(cdt)
    psip_np = workloads.random_field(shape, 600 + case).astype(cdt)
    pb, pbp, n = oracle.expand_pair(psi_np, psip_np, dx, moh, t, lam)
    plan = fx.Plan(shape, dx, moh, t, lam, dtype=tdt, schedule=schedule)
    psi = torch.from_numpy(psi_np).cuda()
    psip = torch.from_numpy(psip_np).cuda()
    # a single-field call before and after the pair must be unaffected by the pair's workspace mode
    o1, _ = plan.expand(psi)
    g, gp, gn = plan.expand_pair(psi, psip)
    o2, _ = plan.expand(psi)
    torch.cuda.synchronize()
    e = (rel(g.cpu().numpy(), pb), rel(gp.cpu().numpy(), pbp), rel(gn.cpu().numpy(), n))
    say("  rel L2 psibar %.2e psibar+ %.2e n %.2e" % e)
    assert torch.equal(o1, o2)
    if dtype == "c128":
        assert max(e) <= TOL64
        assert rel(o1.cpu().numpy(), pb) <= TOL64
    else:
        assert e[2] <= TOL32


def test_pair_with_spectrum_uses_conjugate_kernel(fx):
    shape, lam, dx, t = (48, 40), (3, 4), (1.0, 0.8), 20.0
    phases = [t * 3.0 * (1 - np.cos(0.9 * oracle.fine_wavenumbers(shape[0], lam[0], dx[0]))),
              t * (0.7 * oracle.fine_wavenumbers(shape[1], lam[1], dx[1]) +
                   0.5 * oracle.fine_wavenumbers(shape[1], lam[1], dx[1]) ** 2)]
    psi_np = workloads.random_field(shape, 1)
    psip_np = workloads.random_field(shape, 2)
    pb = oracle.expand_dispersion(psi_np, dx, lam, phases)
    pbp = oracle.expand_dispersion(psip_np.conj(), dx, lam, phases).conj()
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=torch.complex128, spectrum=phases)
    g, gp, gn = plan.expand_pair(torch.from_numpy(psi_np).cuda(), torch.from_numpy(psip_np).cuda())
    assert rel(g.cpu().numpy(), pb) <= TOL64
    assert rel(gp.cpu().numpy(), pbp) <= TOL64
    assert rel(gn.cpu().numpy(), pbp * pb) <= TOL64


def test_pair_with_too_small_caller_workspace_is_rejected(fx):
    shape, lam = (64, 64), (8, 16)
    plan = fx.Plan(shape, (1.0, 1.0), 1.0, 50.0, lam, dtype=torch.complex64)
    assert plan.pair_workspace_size() > plan.workspace_size()
    plan.use_torch_workspace()
    psi = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(MemoryError):
        plan.expand_pair(psi, psi)
    # the single-field call still works on the caller workspace
    _, rho = plan.expand(psi)
    torch.cuda.synchronize()
    assert float(rho.abs().max()) == 0.0
