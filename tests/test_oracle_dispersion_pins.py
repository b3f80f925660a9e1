"""Pins of the oracle's general-spectrum expansion (CPU only).

Section 7.4 notes that the method carries over to any spectrum omega_k in place
of the free-particle one, with only the chirp (presB) and the final twiddle
(presf) changed; the vacuum assumption (eq. (vacuum)) is what matters. For a
spectrum that is a sum over axes the expanded field is again a product of
per-axis kernels, tabulated by ``oracle.gtable_phase`` from t * omega_j on the
fine wave numbers. These tests pin that oracle to:

* a brute-force propagation on the vacuum-padded lattice with numpy FFTs, with
  omega evaluated directly on numpy's own frequency grid (not on the oracle's
  ascending table), for even and odd spectra, non-integer offsets, odd lengths;
* the closed form of a linear spectrum omega = v k: a translation by v t, which
  on the padded periodic lattice is an exact index shift;
* unitarity over the lam shifted output grids for any real spectrum;
* the free-particle spectrum, which must reproduce the separately pinned
  free-flight oracle;
* the adjoint identity;
* planted mistakes (conjugated spectrum, reversed table, q-independent chirp),
  each of which the brute-force pin must reject.
"""

import numpy as np
import pytest

import oracle


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# t * omega(k) for a few spectra (radians); each takes k as a numpy array.
SPECTRA = {
    # Bogoliubov-like phonon/particle spectrum, even in k
    "bogoliubov": lambda k: 30.0 * np.sqrt(0.25 * k ** 2 * (0.25 * k ** 2 + 2.0 * 0.8)),
    # tight-binding band 2J(1 - cos(k b)), even, periodic in k
    "lattice": lambda k: 40.0 * (1.0 - np.cos(0.7 * k)),
    # odd part present: drift plus cubic term, catches sign/orientation mistakes
    "drift_cubic": lambda k: 3.1 * k + 0.9 * k ** 3 + 5.0 * k ** 2,
}


def brute_force_spectrum(psi, dx, lam, a, abar, spectra):
    """Pad to lam*M, FFT, multiply by exp(i k (abar - a) - i t omega(k)), inverse FFT, take every lam-th point."""
    d = psi.ndim
    sh = psi.shape
    npad = [lam[j] * sh[j] for j in range(d)]
    pad = np.zeros(npad, dtype=np.complex128)
    pad[tuple(slice(0, m) for m in sh)] = psi
    spec = np.fft.fftn(pad)
    ph = np.zeros(npad)
    for j in range(d):
        k = 2.0 * np.pi * np.fft.fftfreq(npad[j], d=dx[j])
        s = [1] * d
        s[j] = npad[j]
        ph = ph + (k * (abar[j] - a[j]) - spectra[j](k)).reshape(s)
    out = np.fft.ifftn(spec * np.exp(1j * ph))
    return out[tuple(slice(0, None, lam[j]) for j in range(d))]


def tables(shape, dx, lam, spectra):
    return [spectra[j](oracle.fine_wavenumbers(shape[j], lam[j], dx[j])) for j in range(len(shape))]


CASES = [
    # shape, lam, dx, abar shift (units of dx), spectrum names per axis
    ((16,), (3,), (0.5,), 0.37, ("bogoliubov",)),
    ((9,), (4,), (1.0,), 0.0, ("drift_cubic",)),      # odd M, even lam
    ((7,), (3,), (0.3,), -1.25, ("lattice",)),        # odd lam*M
    ((12,), (1,), (1.0,), 0.5, ("drift_cubic",)),     # lam = 1
    ((6, 5), (3, 2), (1.0, 0.5), 0.2, ("bogoliubov", "drift_cubic")),
    ((4, 3, 5), (2, 3, 2), (0.7, 1.0, 0.4), -0.4, ("lattice", "bogoliubov", "drift_cubic")),
]


@pytest.mark.parametrize("shape,lam,dx,shift,names", CASES)
def test_brute_force_padded_lattice_general_spectrum(shape, lam, dx, shift, names):
    psi = rand_field(shape, 11)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    spectra = [SPECTRA[n] for n in names]
    got = oracle.expand_dispersion(psi, dx, lam, tables(shape, dx, lam, spectra), a=a, abar=abar)
    ref = brute_force_spectrum(psi, dx, lam, a, abar, spectra)
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("M,lam,s0,delta", [(10, 3, 7, 0), (9, 4, -5, 3), (8, 2, 0, -2), (11, 5, 23, 1)])
def test_linear_spectrum_is_an_exact_translation(M, lam, s0, delta):
    # omega = v k with v t = s0 dx moves the padded periodic field by s0 fine cells.
    dx = 0.5
    psi = rand_field((M,), 3)
    a = -0.5 * M * dx
    abar = a + delta * dx
    phase = s0 * dx * oracle.fine_wavenumbers(M, lam, dx)
    got = oracle.expand_dispersion(psi, (dx,), (lam,), [phase], a=[a], abar=[abar])
    N = lam * M
    pad = np.zeros(N, dtype=np.complex128)
    pad[:M] = psi
    expect = pad[(lam * np.arange(M) + delta - s0) % N]
    assert np.max(np.abs(got - expect)) <= 1e-13 * np.max(np.abs(psi))


def test_unitarity_over_shifted_grids_any_real_spectrum():
    shape, lam, dx = (6, 5), (3, 2), (1.0, 0.5)
    psi = rand_field(shape, 9)
    rng = np.random.default_rng(4)
    phases = [rng.uniform(-50, 50, lam[j] * shape[j]) for j in range(2)]
    a, abar0 = oracle.default_offsets(shape, dx, lam)
    total = 0.0
    for s0 in range(lam[0]):
        for s1 in range(lam[1]):
            abar = abar0 + np.array([s0 * dx[0], s1 * dx[1]])
            total += np.sum(np.abs(oracle.expand_dispersion(psi, dx, lam, phases, a=a, abar=abar)) ** 2)
    norm = np.sum(np.abs(psi) ** 2)
    assert abs(total - norm) <= 1e-13 * norm


def test_free_particle_spectrum_reproduces_free_flight_oracle():
    shape, lam, dx, t, moh = (8, 6), (4, 3), (0.5, 1.0), 37.0, 1.3
    psi = rand_field(shape, 2)
    phases = [t / moh * 0.5 * oracle.fine_wavenumbers(shape[j], lam[j], dx[j]) ** 2 for j in range(2)]
    got = oracle.expand_dispersion(psi, dx, lam, phases)
    ref = oracle.expand(psi, dx, moh, t, lam)
    assert rel(got, ref) <= 1e-13
    # None on an axis keeps the free-particle phase of (t, m/hbar)
    got2 = oracle.expand_dispersion(psi, dx, lam, [None, phases[1]], m_over_hbar=moh, t=t)
    assert rel(got2, ref) <= 1e-13


def test_adjoint_dot_product_general_spectrum():
    shape, lam, dx = (5, 7), (3, 2), (1.0, 0.6)
    phases = tables(shape, dx, lam, [SPECTRA["drift_cubic"], SPECTRA["lattice"]])
    x = rand_field(shape, 5)
    y = rand_field(shape, 6)
    lhs = np.vdot(y, oracle.expand_dispersion(x, dx, lam, phases))
    rhs = np.vdot(oracle.expand_dispersion_adjoint(y, dx, lam, phases), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# ---- planted mistakes -----------------------------------------------------------------

def _mutant_gtable(M, lam, delta, phase, s_min, count, mutation):
    N = lam * M
    l = np.arange(-(N // 2), -(N // 2) + N)
    if mutation == "conjugated":
        ph = -phase
    elif mutation == "reversed":
        ph = phase[::-1]
    elif mutation == "q_independent":
        # the chirp taken at the coarse wave number lam*l~ instead of the fine one
        ph = phase[(lam * np.floor_divide(l, lam)) + N // 2]
    else:
        raise ValueError(mutation)
    s = s_min + np.arange(count)
    E = np.exp(2j * np.pi * np.outer(s + delta, l) / N - 1j * ph[None, :])
    return E.sum(axis=1) / N


@pytest.mark.parametrize("mutation", ["conjugated", "reversed", "q_independent"])
def test_planted_mistakes_are_caught(mutation):
    M, lam, dx = 9, 4, 1.0
    psi = rand_field((M,), 8)
    a, abar = oracle.default_offsets((M,), (dx,), (lam,))
    abar = abar + 0.3 * dx
    spec = SPECTRA["drift_cubic"]
    phase = spec(oracle.fine_wavenumbers(M, lam, dx))
    delta = (abar[0] - a[0]) / dx
    s_min = -(M - 1)
    tab = _mutant_gtable(M, lam, delta, phase, s_min, (lam + 1) * (M - 1) + 1, mutation)
    G = tab[lam * np.arange(M)[:, None] - np.arange(M)[None, :] - s_min]
    mutant = G @ psi
    ref = brute_force_spectrum(psi, (dx,), (lam,), a, abar, [spec])
    assert rel(mutant, ref) > 1e-3
    # and the unmutated direct sum passes the same check
    good = oracle.expand_dispersion(psi, (dx,), (lam,), [phase], a=a, abar=abar)
    assert rel(good, ref) <= 1e-13
