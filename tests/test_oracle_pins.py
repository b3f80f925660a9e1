"""Pins of the CPU oracle against things other than itself (CPU only).

Each pin checks the oracle against a fact the paper or the mathematics fixes:
a brute-force padded-lattice FFT propagation (eq. (Psin) on the large lattice,
section 3 and section 6), the full d-dimensional sum without factorisation,
the vacuum subsampling at t = 0 (eq. (vacuum)), the plain split-step at
lam = 1 (eqs. (Psiwtm), (Psin)), unitarity on the padded lattice, the
continuum Gaussian and the two-Gaussian formula of section 6, the far-field
limit (eq. (farfieldk)), the failure of the naive prescription (eq. (Psinaive),
figure 3) and the adjoint/gradient identities. The last group plants typical
mistakes into copies of the oracle's arithmetic and checks that the pins catch
them.
"""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import propagator as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def brute_force(psi, dx, m_over_hbar, t, lam, a, abar):
    """Eq. (Psin) on the vacuum-padded lam*M lattice with numpy FFTs, sampled at xbar.

    The padded lattice starts at a with the input's spacing; the field is
    propagated with exp(-i hbar t k^2 / 2m) and returned on the lattice offset
    abar (factor exp(i k (abar - a)), eqs. (Psiwtm), (Psin)); the magnified
    grid is every lam-th point of it.
    """
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
        ph = ph + (k * (abar[j] - a[j]) - (t / m_over_hbar) * k ** 2 / 2.0).reshape(s)
    out = np.fft.ifftn(spec * np.exp(1j * ph))
    return out[tuple(slice(0, None, lam[j]) for j in range(d))]


BRUTE_CASES = [
    # shape, lam, dx, t, m_over_hbar, abar shift in units of dx
    ((16,), (3,), (0.5,), 3.3, 1.7, 0.37),
    ((9,), (4,), (1.0,), 5.0, 1.0, 0.0),      # odd M, even lam (half-integer delta)
    ((7,), (3,), (0.3,), 0.8, 2.0, -1.25),    # odd lam*M
    ((12,), (1,), (1.0,), 4.0, 1.0, 0.5),     # lam = 1
    ((1,), (5,), (1.0,), 2.0, 1.0, 0.0),      # single-point axis
    ((10,), (8,), (0.25,), -2.0, 1.0, 0.0),   # backward flight
    ((6, 5), (2, 3), (1.0, 0.7), 3.3, 1.7, 0.37),
    ((8, 4), (4, 1), (1.0, 1.0), 6.0, 1.0, 0.0),
    ((4, 5, 3), (2, 2, 3), (1.0, 1.0, 1.0), 2.0, 1.0, 0.2),
]


@pytest.mark.parametrize("shape,lam,dx,t,moh,shift", BRUTE_CASES)
def test_p1_brute_force_padded_lattice(shape, lam, dx, t, moh, shift):
    psi = rand_field(shape, 11)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    got = oracle.expand(psi, dx, moh, t, lam, a, abar)
    ref = brute_force(psi, dx, moh, t, lam, a, abar)
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("shape,lam", [((3, 4), (2, 3)), ((5, 2), (1, 4)), ((2, 3, 2), (2, 2, 3))])
def test_p2_full_nd_sum_equals_per_axis(shape, lam):
    psi = rand_field(shape, 5)
    dx = tuple(0.9 + 0.1 * j for j in range(len(shape)))
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + 0.3 * np.asarray(dx)
    full = oracle.direct_nd(psi, dx, 1.3, 2.5, lam, a, abar)
    fact = oracle.expand(psi, dx, 1.3, 2.5, lam, a, abar)
    assert rel(fact, full) <= 1e-14


@pytest.mark.parametrize("M,lam,shift", [(10, 3, -4), (9, 2, 3), (12, 4, 0), (7, 5, -11)])
def test_p3_t0_is_vacuum_subsampling(M, lam, shift):
    psi = rand_field((M,), 3)
    dx = (0.5,)
    a = np.array([-0.25 * M])
    abar = a + shift * dx[0]
    got = oracle.expand(psi, dx, 1.0, 0.0, (lam,), a, abar)
    ref = np.zeros(M, dtype=np.complex128)
    for nb in range(M):
        k = (shift + lam * nb) % (lam * M)
        if k < M:
            ref[nb] = psi[k]
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.max(np.abs(psi)) * 10


def test_p4_lambda_one_is_split_step_with_paper_prefactors():
    # eq. (Psiwtm): Psi~ = dV/(2pi)^{d/2} e^{-i a.k} DFT[Psi]; eq. (free0); then the return to x-space
    # of eq. (Psin) on the lattice offset abar. The return prefactor is taken as (2pi)^{d/2}/dV, as in
    # eq. (iDFTbar) with lam = 1: with the printed (2pi)^{d/2}/V and the 1/M-normalised inverse DFT of
    # eq. (iDFT), t = 0 would return Psi/M.
    shape = (12, 10)
    dx = (0.5, 0.8)
    psi = rand_field(shape, 7)
    a = np.array([-3.0, -4.0])
    abar = a + np.array([0.2, -0.3])
    t, moh = 2.5, 1.0
    d = 2
    dV = dx[0] * dx[1]
    k = [2 * np.pi * np.fft.fftfreq(shape[j], d=dx[j]) for j in range(d)]  # eq. (kj) ordering
    K0, K1 = np.meshgrid(k[0], k[1], indexing="ij")
    psit = dV / (2 * np.pi) ** (d / 2) * np.exp(-1j * (a[0] * K0 + a[1] * K1)) * np.fft.fft2(psi)
    psit = psit * np.exp(-1j * t / moh * (K0 ** 2 + K1 ** 2) / 2)
    ref = (2 * np.pi) ** (d / 2) / dV * np.fft.ifft2(psit * np.exp(1j * (abar[0] * K0 + abar[1] * K1)))
    got = oracle.expand(psi, dx, moh, t, (1, 1), a, abar)
    assert rel(got, ref) <= 1e-14


def test_p5_unitarity_over_shifted_grids():
    shape, lam, dx = (6, 5), (3, 2), (1.0, 0.5)
    psi = rand_field(shape, 9)
    a, abar0 = oracle.default_offsets(shape, dx, lam)
    total = 0.0
    for s0 in range(lam[0]):
        for s1 in range(lam[1]):
            abar = abar0 + np.array([s0 * dx[0], s1 * dx[1]])
            total += np.sum(np.abs(oracle.expand(psi, dx, 1.0, 7.0, lam, a, abar)) ** 2)
    assert abs(total - np.sum(np.abs(psi) ** 2)) <= 1e-14 * np.sum(np.abs(psi) ** 2) * 10


def test_p5_single_grid_norm_for_smooth_density():
    # Poisson summation: for a density smooth on the coarse grid, lam * sum|Psibar|^2 ~ sum|Psi|^2.
    M, dx, lam = 256, 0.25, 8
    x = (-M / 2 + np.arange(M)) * dx
    psi = np.exp(-x ** 2 / (2 * 4.0 ** 2)) * np.exp(0.3j * x)
    pb = oracle.expand(psi, (dx,), 1.0, 60.0, (lam,))
    assert abs(lam * np.sum(np.abs(pb) ** 2) / np.sum(np.abs(psi) ** 2) - 1) < 1e-6


def gaussian_packet(x, x0, sigma, k0, t, nu):
    """Continuum free Gaussian packet, hbar/m = nu (textbook closed form)."""
    w = sigma ** 2 + 1j * nu * t
    return ((np.pi * sigma ** 2) ** -0.25 * np.sqrt(sigma ** 2 / w)
            * np.exp(-(x - x0 - nu * k0 * t) ** 2 / (2 * w) + 1j * k0 * (x - x0) - 0.5j * nu * k0 ** 2 * t))


def test_p6_continuum_gaussian_1d():
    M, dx, lam, t, moh = 64, 0.5, 8, 20.0, 1.0
    a = -M * dx / 2
    x = a + np.arange(M) * dx
    psi = gaussian_packet(x, 0.5, 2.0, 0.7, 0.0, 1 / moh)
    _, abar = oracle.default_offsets((M,), (dx,), (lam,))
    xbar = abar[0] + np.arange(M) * lam * dx
    got = oracle.expand(psi, (dx,), moh, t, (lam,))
    ref = gaussian_packet(xbar, 0.5, 2.0, 0.7, t, 1 / moh)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_p6_continuum_gaussian_2d_product():
    shape, dx, lam, t, moh = (40, 48), (0.5, 0.4), (4, 6), 6.0, 2.0
    a, abar = oracle.default_offsets(shape, dx, lam)
    y = a[0] + np.arange(shape[0]) * dx[0]
    x = a[1] + np.arange(shape[1]) * dx[1]
    gy = lambda yy, tt: gaussian_packet(yy, -0.3, 1.5, -0.4, tt, 1 / moh)
    gx = lambda xx, tt: gaussian_packet(xx, 0.2, 1.2, 0.9, tt, 1 / moh)
    psi = gy(y, 0)[:, None] * gx(x, 0)[None, :]
    yb = abar[0] + np.arange(shape[0]) * lam[0] * dx[0]
    xb = abar[1] + np.arange(shape[1]) * lam[1] * dx[1]
    ref = gy(yb, t)[:, None] * gx(xb, t)[None, :]
    got = oracle.expand(psi, dx, moh, t, lam)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_p6_two_gaussian_formula_of_section6():
    cfg = json.load(open(os.path.join(GOLDEN, "section6_double_gaussian.json")))
    # Units: transverse oscillator length and 1/omega_perp; hbar = m = omega_perp = 1.
    ratio = cfg["omega_perp_hz"] / cfg["omega_hz"]
    D = cfg["D_over_a_ho"] * np.sqrt(ratio)          # a_ho / a_perp = sqrt(omega_perp/omega)
    t = cfg["t_final_times_omega"] * ratio           # omega_perp * t
    M, dx, lam = 96, 0.25, 160
    a = -M * dx / 2
    y = a + np.arange(M) * dx
    Ap, Am = 0.8 * np.exp(0.4j), 1.1 * np.exp(-1.3j)

    def two_gauss(yy, tt):
        # closed form printed before eq. (dphase2), hbar = m = omega_perp = 1
        return (1 / np.sqrt(1 + 1j * tt)) * sum(
            A * np.pi ** -0.25 * np.exp(-(2 * yy - sgn * D) ** 2 / (8 * (1 + 1j * tt)))
            for A, sgn in ((Ap, +1), (Am, -1)))

    psi = two_gauss(y, 0.0)
    _, abar = oracle.default_offsets((M,), (dx,), (lam,))
    yb = abar[0] + np.arange(M) * lam * dx
    got = oracle.expand(psi, (dx,), 1.0, t, (lam,))
    ref = two_gauss(yb, t)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_p7_far_field_limit():
    M, dx, moh = 32, 1.0, 1.0
    a = -M / 2 * dx
    x = a + np.arange(M) * dx
    psi = np.exp(-x ** 2 / (2 * 3.0 ** 2)) * (1 + 0.5j * np.tanh(x / 2)) * np.exp(0.3j * x)
    errs = []
    for t, lam in [(100.0, 16), (400.0, 64), (1600.0, 256)]:
        pb = oracle.expand(psi, (dx,), moh, t, (lam,))
        _, abar = oracle.default_offsets((M,), (dx,), (lam,))
        xbar = abar[0] + np.arange(M) * lam * dx
        kap = moh * xbar / t
        psit = dx / np.sqrt(2 * np.pi) * np.exp(-1j * np.outer(kap, x)) @ psi  # eq. (Psiwtm) at off-grid kappa
        rho_ff = (moh / t) * np.abs(psit) ** 2                               # eq. (farfieldk), d = 1
        errs.append(rel(np.abs(pb) ** 2, rho_ff))
    slopes = np.diff(np.log(errs)) / np.log(4.0)
    assert errs[-1] < 1e-4
    assert np.all(slopes <= -0.9), (errs, slopes)


def test_p8_naive_prescription_fails_where_the_oracle_matches_brute_force():
    cfg = json.load(open(os.path.join(GOLDEN, "fig3_naive_input.json")))
    M = cfg["M"]
    x0, x1 = cfg["x_range"]
    dx = (x1 - x0) / M
    x = x0 + np.arange(M) * dx
    psi = np.exp(-x ** 2 / 2) * np.cos(cfg["k0"] * x)
    lam = int(round((cfg["truth_range"][1] - cfg["truth_range"][0]) / (x1 - x0)))
    assert lam == 2
    a = np.array([x0])
    abar = np.array([cfg["truth_range"][0]])
    k = 2 * np.pi * np.fft.fftfreq(M, d=dx)
    for t, must_fail in [(0.2, False), (1.0, True)]:
        got = oracle.expand(psi, (dx,), 1.0, t, (lam,), a, abar)
        ref = brute_force(psi, (dx,), 1.0, t, (lam,), a, abar)
        assert rel(got, ref) <= 1e-13
        # eq. (Psinaive): one DFT on the small lattice, read at n'' = lam*nbar mod M, times Lambda.
        spec = np.fft.fft(psi) * np.exp(-1j * k * a[0]) * np.exp(-0.5j * t * k ** 2) * np.exp(1j * k * abar[0])
        naive = lam * np.fft.ifft(spec)[(lam * np.arange(M)) % M]
        err = rel(np.abs(naive) ** 2 / lam ** 2, np.abs(ref) ** 2)
        if must_fail:
            assert err > 0.3
    # and the naive form is fine before the cloud reaches the box edge only up to its tiling


def test_p9_adjoint_dot_product_and_fd_gradient():
    shape, dx, lam, t = (6, 7), (1.0, 0.8), (3, 2), 4.0
    u = rand_field(shape, 1)
    v = rand_field(shape, 2)
    lhs = np.vdot(oracle.expand(u, dx, 1.0, t, lam), v)
    rhs = np.vdot(u, oracle.expand_adjoint(v, dx, 1.0, t, lam))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    psi = rand_field(shape, 3)
    tau = np.abs(rand_field(shape, 4)) ** 2 * 0.1
    loss, grad = oracle.loss_and_grad(psi, tau, dx, 1.0, t, lam)
    h = 1e-3
    rng = np.random.default_rng(0)
    for _ in range(6):
        i = tuple(rng.integers(0, s) for s in shape)
        for unit, comp in ((1.0, grad[i].real), (1j, grad[i].imag)):
            pp = psi.copy(); pp[i] += h * unit
            pm = psi.copy(); pm[i] -= h * unit
            fd = (oracle.loss_and_grad(pp, tau, dx, 1.0, t, lam)[0]
                  - oracle.loss_and_grad(pm, tau, dx, 1.0, t, lam)[0]) / (2 * h)
            assert abs(fd - comp) <= 1e-6 * max(1.0, abs(comp))


def test_gtable_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    M, lam, dx, t, moh = 24, 5, 0.7, 13.0, 1.3
    delta = -46.37
    N = lam * M
    s_vals = [-23, -5, 0, 17, 60, 115]
    tab = oracle.gtable(M, lam, delta, t, moh, dx, -(M - 1), (lam + 1) * (M - 1) + 1)
    beta = mp.pi * (mp.mpf(t) / mp.mpf(moh)) / (N * mp.mpf(dx)) ** 2
    for s in s_vals:
        acc = mp.mpc(0)
        for l in range(-(N // 2), -(N // 2) + N):
            acc += mp.expjpi(2 * (l * (s + mp.mpf(delta)) / N - beta * l * l))
        ref = complex(acc / N)
        assert abs(tab[s + M - 1] - ref) <= 1e-15


def test_gtable_c_matches_long_double_numpy():
    if not oracle.have_c_kernel():
        pytest.skip("oracle C kernel not built")
    args = (20, 7, 3.25, 9.0, 1.0, 0.5, -19, 7 * 19 + 20)
    assert np.max(np.abs(oracle.gtable(*args) - oracle.gtable_longdouble(*args))) <= 1e-15


def test_linearity():
    shape, dx, lam = (5, 6), (1.0, 1.0), (2, 3)
    u, v = rand_field(shape, 1), rand_field(shape, 2)
    c = 0.3 - 1.7j
    lhs = oracle.expand(u + c * v, dx, 1.0, 3.0, lam)
    rhs = oracle.expand(u, dx, 1.0, 3.0, lam) + c * oracle.expand(v, dx, 1.0, 3.0, lam)
    assert rel(lhs, rhs) <= 1e-14


# ---------------------------------------------------------------------------------------
# Planted mistakes: copies of the oracle arithmetic with one error each must fail a pin.
# ---------------------------------------------------------------------------------------

def _mutant_expand(psi, dx, moh, t, lam, a, abar, mutation):
    d = psi.ndim
    mats = []
    for j in range(d):
        M = psi.shape[j]
        delta = (abar[j] - a[j]) / dx[j]
        tt = t
        if mutation == "drop_delta":
            delta = round(delta)
        if mutation == "chirp_sign":
            tt = -t
        tab = oracle.gtable(M, lam[j], delta, tt, moh, dx[j], -(M - 1), (lam[j] + 1) * (M - 1) + 1)
        nb = np.arange(M)[:, None]
        n = np.arange(M)[None, :]
        s = lam[j] * nb - n
        if mutation == "index_sign":
            s = n - lam[j] * nb + (lam[j] - 1) * (M - 1)  # wrong sign of s, shifted into table range
        G = tab[s + M - 1]
        if mutation == "transpose":
            G = G.T
        if mutation == "norm":
            G = G * np.sqrt(lam[j])
        mats.append(G)
    return P._apply(mats, psi.astype(np.complex128))


@pytest.mark.parametrize("mutation", ["drop_delta", "chirp_sign", "index_sign", "transpose", "norm"])
def test_planted_mistakes_are_caught_by_brute_force_pin(mutation):
    shape, lam, dx, t, moh = (6, 5), (2, 3), (1.0, 0.7), 3.3, 1.7
    psi = rand_field(shape, 21)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + 0.37 * np.asarray(dx)
    ref = brute_force(psi, dx, moh, t, lam, a, abar)
    good = _mutant_expand(psi, dx, moh, t, lam, a, abar, None)
    assert rel(good, ref) <= 1e-13
    bad = _mutant_expand(psi, dx, moh, t, lam, a, abar, mutation)
    assert rel(bad, ref) > 1e-3
