"""Pins of the oracle's point evaluation (``expand_points``) and of its column
density image (``column_density``), CPU only.

``expand_points`` is the checker of the large-configuration GPU tests, which
compare sampled output points; it is pinned here against the brute-force
propagation on the vacuum-padded lattice (eq. (Psin) on the large lattice,
eq. (vacuum)), against the continuum Gaussian packet, and against the oracle's
own full-field evaluation. ``column_density`` is the density image integrated
along one axis (section 6, rho(x, y) = integral dz |Psi|^2): for a product of
Gaussian packets the integral over the summed axis is the norm of that axis'
packet, which free flight conserves, so the image is the closed-form density of
the remaining axes; at t = 0 the image is the weighted sum of the subsampled
input density. Planted mistakes in copies of both functions fail these pins.
"""

import numpy as np
import pytest

import oracle

from test_oracle_pins import brute_force, gaussian_packet, rand_field, rel

POINT_CASES = [
    # shape, lam, dx, t, m_over_hbar, abar shift (units of dx)
    ((16,), (3,), (0.5,), 3.3, 1.7, 0.37),
    ((9,), (4,), (1.0,), 5.0, 1.0, 0.0),        # odd M
    ((10,), (8,), (0.25,), -2.0, 1.0, 0.41),    # backward flight, non-integer delta
    ((6, 5), (2, 3), (1.0, 0.7), 3.3, 1.7, 0.37),
    ((7, 4), (3, 2), (0.6, 1.1), -1.5, 0.8, -0.23),
    ((4, 5, 3), (2, 2, 3), (1.0, 1.0, 1.0), 2.0, 1.0, 0.2),
    ((5, 3, 6), (3, 1, 2), (0.9, 1.2, 0.5), -0.7, 1.3, 0.61),
]


def _random_points(shape, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, m, size=n) for m in shape], axis=1)


@pytest.mark.parametrize("shape,lam,dx,t,moh,shift", POINT_CASES)
def test_points_match_brute_force_padded_lattice(shape, lam, dx, t, moh, shift):
    psi = rand_field(shape, 17)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    pts = _random_points(shape, 25, 3)
    got = oracle.expand_points(psi, pts, dx, moh, t, lam, a, abar)
    ref = brute_force(psi, dx, moh, t, lam, a, abar)[tuple(pts.T)]
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("shape,lam,dx,t,moh,shift", POINT_CASES)
def test_points_equal_full_field(shape, lam, dx, t, moh, shift):
    psi = rand_field(shape, 23)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    pts = _random_points(shape, 40, 5)
    got = oracle.expand_points(psi, pts, dx, moh, t, lam, a, abar)
    full = oracle.expand(psi, dx, moh, t, lam, a, abar)
    assert rel(got, full[tuple(pts.T)]) <= 1e-14


def test_points_match_continuum_gaussian_3d():
    # sigma >= 3 dx; every packet more than 7.5 sigma inside its box and inside the magnified box at t
    shape, dx, lam, t, moh = (48, 56, 56), (0.5, 0.4, 0.4), (3, 4, 5), 5.0, 1.0
    a, abar = oracle.default_offsets(shape, dx, lam)
    packets = [(0.2, 1.5, 0.3), (-0.4, 1.2, -0.2), (0.1, 1.2, 0.5)]  # x0, sigma, k0 per axis
    axes_in = [a[j] + np.arange(shape[j]) * dx[j] for j in range(3)]
    axes_out = [abar[j] + np.arange(shape[j]) * lam[j] * dx[j] for j in range(3)]
    f = [lambda xx, tt, p=p: gaussian_packet(xx, p[0], p[1], p[2], tt, 1 / moh) for p in packets]
    psi = np.einsum("i,j,k->ijk", f[0](axes_in[0], 0), f[1](axes_in[1], 0), f[2](axes_in[2], 0))
    pts = np.concatenate([_random_points(shape, 30, 7),
                          np.stack([np.full(10, s // 2) for s in shape], axis=1) + _random_points((3, 3, 3), 10, 8) - 1])
    got = oracle.expand_points(psi, pts, dx, moh, t, lam)
    ref = np.array([f[0](axes_out[0][p[0]], t) * f[1](axes_out[1][p[1]], t) * f[2](axes_out[2][p[2]], t)
                    for p in pts])
    peak = np.abs(f[0](axes_out[0], t)).max() * np.abs(f[1](axes_out[1], t)).max() * np.abs(f[2](axes_out[2], t)).max()
    assert np.max(np.abs(got - ref)) <= 1e-10 * peak


def _points_axes_swapped(psi, points, dx, moh, t, lam):
    """expand_points with the per-axis kernel rows taken from the wrong axis' index (planted)."""
    d = psi.ndim
    mats = oracle.propagator._matrices(psi.shape, dx, lam, t, moh, None, None)
    out = np.empty(len(points), dtype=np.complex128)
    for i, p in enumerate(points):
        x = psi
        for j in range(d - 1, -1, -1):
            x = np.tensordot(x, mats[j][p[d - 1 - j]], axes=([j], [0]))
        out[i] = x
    return out


def test_planted_axis_swap_in_point_evaluation_is_caught():
    shape, lam, dx, t, moh = (6, 6, 6), (2, 3, 2), (1.0, 0.8, 1.1), 2.5, 1.0
    psi = rand_field(shape, 31)
    a, abar = oracle.default_offsets(shape, dx, lam)
    pts = _random_points(shape, 20, 9)
    ref = brute_force(psi, dx, moh, t, lam, a, abar)[tuple(pts.T)]
    assert rel(oracle.expand_points(psi, pts, dx, moh, t, lam), ref) <= 1e-13
    assert rel(_points_axes_swapped(psi, pts, dx, moh, t, lam), ref) > 1e-3


# ---------------------------------------------------------------------------------------------
# Column density (section 6): image = integral over one axis of rho on the magnified grid
# ---------------------------------------------------------------------------------------------

# Three product Gaussian packets; the summed axis' packet is normalised, so its integral
# over the magnified axis is 1 at any time (free flight conserves the norm).
COL_SHAPE, COL_DX, COL_LAM, COL_T = (48, 40, 48), (0.5, 0.5, 0.4), (4, 4, 6), 6.0
COL_PACKETS = [(0.3, 1.5, 0.3), (-0.3, 1.5, -0.4), (0.2, 1.2, 0.9)]


def _product_gaussian(shape, dx, lam, t, packets):
    a, abar = oracle.default_offsets(shape, dx, lam)
    f = [lambda xx, tt, p=p: gaussian_packet(xx, p[0], p[1], p[2], tt, 1.0) for p in packets]
    d = len(shape)
    axes_in = [a[j] + np.arange(shape[j]) * dx[j] for j in range(d)]
    axes_out = [abar[j] + np.arange(shape[j]) * lam[j] * dx[j] for j in range(d)]
    psi = f[0](axes_in[0], 0)
    for j in range(1, d):
        psi = np.multiply.outer(psi, f[j](axes_in[j], 0))
    out_density = [np.abs(f[j](axes_out[j], t)) ** 2 for j in range(d)]
    return psi, out_density


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_column_image_of_product_gaussian_is_closed_form_density(axis):
    psi, dens = _product_gaussian(COL_SHAPE, COL_DX, COL_LAM, COL_T, COL_PACKETS)
    rho = oracle.density(oracle.expand(psi, COL_DX, 1.0, COL_T, COL_LAM))
    img = oracle.column_density(rho, axis, COL_LAM, COL_DX)
    rest = [dens[j] for j in range(3) if j != axis]
    ref = np.multiply.outer(rest[0], rest[1])
    assert img.shape == ref.shape
    assert np.max(np.abs(img - ref)) <= 1e-9 * ref.max()


def test_column_image_2d_axis1():
    shape, dx, lam, t = (40, 48), (0.5, 0.4), (4, 6), 6.0
    psi, dens = _product_gaussian(shape, dx, lam, t, COL_PACKETS[:2])
    rho = oracle.density(oracle.expand(psi, dx, 1.0, t, lam))
    img = oracle.column_density(rho, 1, lam, dx)
    assert np.max(np.abs(img - dens[0])) <= 1e-9 * dens[0].max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_column_image_at_t0_is_weighted_sum_of_subsampled_input(axis):
    # eq. (vacuum) at t = 0 with integer offsets: Psibar[nbar] = Psi[k] with k = (delta + lam nbar) taken
    # modulo the padded length lam M when k < M, zero elsewhere (the padded lattice is periodic); the
    # image sums the subsampled input density times the output spacing.
    shape, lam, dx = (9, 7, 8), (2, 3, 2), (0.5, 0.7, 1.1)
    shift = (-4, 3, 0)
    psi = rand_field(shape, 41)
    a = -0.5 * np.asarray(shape) * np.asarray(dx)
    abar = a + np.asarray(shift) * np.asarray(dx)
    rho = oracle.density(oracle.expand(psi, dx, 1.0, 0.0, lam, a, abar))
    img = oracle.column_density(rho, axis, lam, dx)
    sub = np.zeros(shape)
    for nb in np.ndindex(*shape):
        k = tuple((shift[j] + lam[j] * nb[j]) % (lam[j] * shape[j]) for j in range(3))
        if all(0 <= k[j] < shape[j] for j in range(3)):
            sub[nb] = abs(psi[k]) ** 2
    ref = sub.sum(axis=axis) * lam[axis] * dx[axis]
    assert np.max(np.abs(img - ref)) <= 1e-13 * ref.max()


@pytest.mark.parametrize("mutation", ["input_spacing", "wrong_axis", "mean"])
def test_planted_mistakes_in_column_density_are_caught(mutation):
    psi, dens = _product_gaussian(COL_SHAPE, COL_DX, COL_LAM, COL_T, COL_PACKETS)
    rho = oracle.density(oracle.expand(psi, COL_DX, 1.0, COL_T, COL_LAM))
    axis = 0
    ref = np.multiply.outer(dens[1], dens[2])
    if mutation == "input_spacing":      # the input spacing instead of the output spacing lam dz
        bad = rho.sum(axis=axis) * COL_DX[axis]
    elif mutation == "wrong_axis":       # the weight of another axis
        bad = rho.sum(axis=axis) * COL_LAM[2] * COL_DX[2]
    else:                                # a mean instead of an integral
        bad = rho.mean(axis=axis)
    assert np.max(np.abs(bad - ref)) > 1e-3 * ref.max()
