"""Parity of the HIP path with the oracle for other spectra (section 7.4): the
free-particle phase replaced per axis by a caller table of t * omega_j on the fine
wave numbers (``fx_plan_create_spectrum``). Same bars as the free-flight cases:
FP64 relative L2 <= 1e-12 in Psibar and rho, FP32 form <= 1e-5 in rho."""

import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_RHO = 1e-5


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


# t * omega(k) in radians
SPECTRA = {
    "bogoliubov": lambda k, t: t * np.sqrt(0.25 * k ** 2 * (0.25 * k ** 2 + 2.0 * 0.8)),
    "lattice": lambda k, t: t * 2.0 * 1.5 * (1.0 - np.cos(0.9 * k)),
    "drift_cubic": lambda k, t: t * (0.7 * k + 0.05 * k ** 3 + 0.5 * k ** 2),
    "free": None,
}

CASES = [
    # shape, lam, dx, t, abar shift (dx units), spectrum per axis
    ((96,), (6,), (1.0,), 30.0, 0.0, ("bogoliubov",)),
    ((45,), (4,), (1.0,), 12.0, 0.3, ("drift_cubic",)),
    ((48, 40), (3, 4), (1.0, 0.8), 20.0, 0.37, ("lattice", "drift_cubic")),
    ((64, 64), (8, 16), (1.0, 1.0), 200.0, 0.0, ("bogoliubov", "bogoliubov")),
    ((12, 24, 48), (2, 3, 4), (1.0, 1.0, 1.0), 7.0, 0.1, ("lattice", "free", "bogoliubov")),
    ((16, 384), (2, 3), (1.0, 1.0), 50.0, 0.0, ("free", "lattice")),
]


def _phases(shape, lam, dx, t, names):
    out = []
    for j, n in enumerate(names):
        f = SPECTRA[n]
        out.append(None if f is None else f(oracle.fine_wavenumbers(shape[j], lam[j], dx[j]), t))
    return out


def _setup(case):
    shape, lam, dx, t, shift, names = CASES[case]
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    return shape, lam, dx, t, a, abar, _phases(shape, lam, dx, t, names)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("schedule", ["paper", "axis_factorised"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_spectrum_parity(fx, case, schedule, dtype):
    shape, lam, dx, t, a, abar, phases = _setup(case)
    say("spectrum case", shape, lam, CASES[case][5], schedule, dtype)
    psi_np = workloads.random_field(shape, 300 + case)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi_np = psi_np.astype(np.complex128 if dtype == "c128" else np.complex64)
    # free axes use m/hbar = 1 and the same t
    ref = oracle.expand_dispersion(psi_np, dx, lam, phases, m_over_hbar=1.0, t=t, a=a, abar=abar)
    plan = fx.Plan(shape, dx, 1.0, t, lam, list(a), list(abar), tdt, schedule, spectrum=phases)
    assert '"table"' in plan.describe()
    out, rho = plan.expand(torch.from_numpy(psi_np).cuda())
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    rho = rho.cpu().numpy()
    e_psi = rel(out, ref)
    e_rho = rel(rho, oracle.density(ref))
    say(f"  rel L2 psi {e_psi:.2e}  rho {e_rho:.2e}")
    if dtype == "c128":
        assert e_psi <= TOL64 and e_rho <= TOL64
    else:
        assert e_rho <= TOL32_RHO


@pytest.mark.parametrize("case", [2, 4])
def test_spectrum_adjoint_fp64(fx, case):
    shape, lam, dx, t, a, abar, phases = _setup(case)
    say("spectrum adjoint", shape, lam)
    y_np = workloads.random_field(shape, 400 + case)
    ref = oracle.expand_dispersion_adjoint(y_np, dx, lam, phases, m_over_hbar=1.0, t=t, a=a, abar=abar)
    plan = fx.Plan(shape, dx, 1.0, t, lam, list(a), list(abar), torch.complex128, spectrum=phases)
    got = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    e = rel(got, ref)
    say(f"  rel L2 {e:.2e}")
    assert e <= TOL64


def test_linear_spectrum_translates_exactly(fx):
    # omega = v k with v t = s0 dx: the padded periodic field moves by s0 cells (closed form).
    M, lam, dx, s0 = 256, 4, 0.5, 37
    psi_np = workloads.random_field((M,), 7)
    a = -0.5 * M * dx
    abar = a
    phase = s0 * dx * oracle.fine_wavenumbers(M, lam, dx)
    plan = fx.Plan((M,), (dx,), 1.0, 0.0, (lam,), [a], [abar], torch.complex128, spectrum=[phase])
    out, _ = plan.expand(torch.from_numpy(psi_np).cuda())
    out = out.cpu().numpy()
    pad = np.zeros(lam * M, dtype=np.complex128)
    pad[:M] = psi_np
    expect = pad[(lam * np.arange(M) - s0) % (lam * M)]
    assert np.max(np.abs(out - expect)) <= 1e-12 * np.max(np.abs(psi_np))
