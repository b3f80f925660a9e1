"""Pins of the oracle's far-field estimate (eq. (farfieldk)), CPU only.

* closed form: for a Gaussian wave packet resolved by the lattice and contained in the box,
  the lattice sum of eq. (Psiwtm) at off-grid kappa equals the continuum transform of
  eq. (FT) to rounding (aliasing and truncation are below 1e-15), so rho_ff must match
  (m / hbar t) (sigma / sqrt(pi)) exp(-sigma^2 (m r / hbar t - k0)^2) per axis (1-D and a 2-D product);
* it is the long-time limit of the finite-time expansion (pinned separately by brute force):
  the relative difference must fall at least like 1/t;
* planted mistakes (conjugated kernel, dropped prefactor) fail the closed form.
"""

import numpy as np
import pytest

import oracle


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def gauss(x, x0, sigma, k0):
    return (np.pi * sigma ** 2) ** -0.25 * np.exp(-(x - x0) ** 2 / (2 * sigma ** 2) + 1j * k0 * x)


def rho_ff_exact(r, t, moh, sigma, k0):
    kap = moh * r / t
    return (moh / abs(t)) * sigma / np.sqrt(np.pi) * np.exp(-sigma ** 2 * (kap - k0) ** 2)


@pytest.mark.parametrize("t,moh,k0,x0", [(200.0, 1.0, 0.4, 3.0), (-150.0, 1.7, -0.25, -2.0), (900.0, 0.8, 0.0, 0.0)])
def test_gaussian_closed_form_1d(t, moh, k0, x0):
    M, dx, lam, sigma = 160, 0.5, 8, 4.0
    a, abar = oracle.default_offsets((M,), (dx,), (lam,))
    x = a[0] + np.arange(M) * dx
    psi = gauss(x, x0, sigma, k0)
    amp, rho = oracle.far_field(psi, (dx,), moh, t, (lam,))
    r = abar[0] + np.arange(M) * lam * dx
    ref = rho_ff_exact(r, t, moh, sigma, k0)
    assert np.max(np.abs(rho - ref)) <= 1e-10 * np.max(ref)
    assert np.allclose(np.abs(amp) ** 2, rho, rtol=0, atol=1e-15 * np.max(rho))


def test_gaussian_closed_form_2d_product():
    shape, dx, lam, t = (128, 160), (0.5, 0.4), (6, 5), 300.0
    sig, k0, x0 = (3.0, 2.5), (0.3, -0.2), (1.0, -2.0)
    a, abar = oracle.default_offsets(shape, dx, lam)
    xs = [a[j] + np.arange(shape[j]) * dx[j] for j in range(2)]
    psi = np.outer(gauss(xs[0], x0[0], sig[0], k0[0]), gauss(xs[1], x0[1], sig[1], k0[1]))
    _, rho = oracle.far_field(psi, dx, 1.0, t, lam)
    rs = [abar[j] + np.arange(shape[j]) * lam[j] * dx[j] for j in range(2)]
    ref = np.outer(rho_ff_exact(rs[0], t, 1.0, sig[0], k0[0]), rho_ff_exact(rs[1], t, 1.0, sig[1], k0[1]))
    assert np.max(np.abs(rho - ref)) <= 1e-10 * np.max(ref)


def test_far_field_is_the_long_time_limit_of_the_expansion():
    M, dx, moh = 32, 1.0, 1.0
    x = -M / 2 * dx + np.arange(M) * dx
    psi = np.exp(-x ** 2 / (2 * 3.0 ** 2)) * (1 + 0.5j * np.tanh(x / 2)) * np.exp(0.3j * x)
    errs = []
    for t, lam in [(100.0, 16), (400.0, 64), (1600.0, 256)]:
        rho = oracle.density(oracle.expand(psi, (dx,), moh, t, (lam,)))
        _, rho_ff = oracle.far_field(psi, (dx,), moh, t, (lam,))
        errs.append(rel(rho, rho_ff))
    slopes = np.diff(np.log(errs)) / np.log(4.0)
    assert errs[-1] < 1e-4 and np.all(slopes <= -0.9), (errs, slopes)


@pytest.mark.parametrize("mutation", ["conjugate", "no_prefactor"])
def test_planted_mistakes_fail_the_closed_form(mutation):
    M, dx, lam, sigma, k0, t = 128, 0.5, 8, 4.0, 0.4, 200.0
    a, abar = oracle.default_offsets((M,), (dx,), (lam,))
    x = a[0] + np.arange(M) * dx
    psi = gauss(x, 3.0, sigma, k0)
    r = abar[0] + np.arange(M) * lam * dx
    kap = r / t
    sign = 1.0 if mutation == "conjugate" else -1.0
    s = np.exp(sign * 1j * np.outer(kap, x)) @ psi
    pref = 1.0 if mutation == "no_prefactor" else (1.0 / t) * dx ** 2 / (2 * np.pi)
    rho_bad = pref * np.abs(s) ** 2
    ref = rho_ff_exact(r, t, 1.0, sigma, k0)
    assert np.max(np.abs(rho_bad - ref)) > 1e-3 * np.max(ref)
