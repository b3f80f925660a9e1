"""Parity of the brute-force comparator (``fx_brute_force``: padded-lattice propagation,
eq. (Psin) on the vacuum-padded lattice) with the oracle. It computes the same operator as
the method, so the bars are those of the expansion: FP64 relative L2 <= 1e-12 in Psibar and
rho, FP32 <= 1e-5 in rho. Cases cover one-pass lines and two-pass lines (padded length above
one workgroup's LDS), 1-D to 3-D, non-integer output offsets."""

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


CASES = [
    # shape, lam, dx, t, m_over_hbar, abar shift (dx units)
    ((64,), (5,), (0.5,), 3.0, 1.0, 0.0),
    ((100,), (7,), (1.0,), 40.0, 1.0, 0.3),
    ((512,), (32,), (1.0,), 2000.0, 1.0, 0.0),       # two passes (N = 16384)
    ((48, 40), (3, 4), (1.0, 0.8), 30.0, 1.0, 0.37),
    ((64, 96), (100, 2), (1.0, 1.0), 500.0, 1.0, 0.0),  # two passes in FP64 (N = 6400)
    ((12, 20, 33), (2, 3, 4), (1.0, 0.5, 1.0), 9.0, 1.3, 0.2),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_brute_force_parity(fx, case, dtype):
    shape, lam, dx, t, moh, shift = CASES[case]
    print("brute force", shape, lam, dtype, flush=True)
    cdt = np.complex128 if dtype == "c128" else np.complex64
    psi = workloads.random_field(shape, 800 + case).astype(cdt)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    ref = oracle.expand(psi, dx, moh, t, lam, a, abar)
    plan = fx.Plan(shape, dx, moh, t, lam, list(a), list(abar),
                   dtype=torch.complex128 if dtype == "c128" else torch.complex64)
    out, rho = plan.brute_force(torch.from_numpy(psi).cuda())
    out2, _ = plan.expand(torch.from_numpy(psi).cuda())
    torch.cuda.synchronize()
    e_psi, e_rho = rel(out.cpu().numpy(), ref), rel(rho.cpu().numpy(), oracle.density(ref))
    e_ff = rel(out.cpu().numpy(), out2.cpu().numpy())
    print(f"  rel L2 psi {e_psi:.2e} rho {e_rho:.2e}  vs expansion {e_ff:.2e}", flush=True)
    if dtype == "c128":
        assert e_psi <= 1e-12 and e_rho <= 1e-12
    else:
        assert e_rho <= 1e-5
