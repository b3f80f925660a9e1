"""Seeded synthetic initial fields and problem parameters.

The paper's own inputs are samples of a stochastic Gross-Pitaevskii simulation
(section 3) and the output of a 3D GPE conversion phase (section 6); none of
them is available, so every workload here is a synthetic stand-in with the
shape, length scales and structure of those states: a dark-soliton cloud in
1D, an elongated phase-fluctuating quasicondensate in 2D, the two-cloud
interferometer of eq. (3dic) in 3D, an ensemble of Thomas-Fermi clouds with
planar dark solitons, and a batch of 2D fields for fitting.

All fields are produced in complex128 on the host from
``numpy.random.default_rng(SeedSequence(...))``; a run in single precision
casts them to complex64 afterwards. Units: hbar = m = 1.

Nothing in this module evaluates the propagator.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Workload:
    """One expansion problem: initial fields plus lattice and flight parameters."""

    name: str
    fields: List[np.ndarray]          # complex128 arrays, C order, last axis contiguous
    dx: Tuple[float, ...]
    lam: Tuple[int, ...]
    t: float
    m_over_hbar: float = 1.0
    dtype: str = "c128"               # "c128" (plain FP64) or "c64" (FP32 data, FP64 phases)
    column_axis: Optional[int] = None  # axis summed for a density image, if any
    extra: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(self.fields[0].shape)

    def cast(self, arr: np.ndarray) -> np.ndarray:
        return arr.astype(np.complex64 if self.dtype == "c64" else np.complex128)


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.default_rng(seed)
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


def centred_coords(m: int, dx: float) -> np.ndarray:
    """Lattice positions x = a + n dx with a = -m dx / 2 (x = 0 at n = m/2)."""
    return (-0.5 * m + np.arange(m)) * dx


def gaussian_random_field(rng: np.random.Generator, shape: Sequence[int], corr_len: float,
                          std: float, dx: float = 1.0) -> np.ndarray:
    """Real Gaussian random field with covariance ~ exp(-r^2 / (2 corr_len^2)).

    White noise is filtered in Fourier space by exp(-k^2 corr_len^2 / 4) and the
    result is shifted to zero mean and rescaled to exactly the requested sample
    standard deviation.
    """
    white = rng.standard_normal(tuple(shape))
    spec = np.fft.fftn(white)
    k2 = np.zeros(tuple(shape))
    for ax, m in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(m, d=dx)
        sh = [1] * len(shape)
        sh[ax] = m
        k2 = k2 + (k ** 2).reshape(sh)
    field = np.fft.ifftn(spec * np.exp(-k2 * corr_len ** 2 / 4.0)).real
    field = field - field.mean()
    s = field.std()
    if s > 0:
        field = field * (std / s)
    return field


def random_field(shape: Sequence[int], seed, scale: float = 1.0) -> np.ndarray:
    """Complex standard-normal field (used for small property and parity cases)."""
    rng = _rng(seed)
    return scale * (rng.standard_normal(tuple(shape)) + 1j * rng.standard_normal(tuple(shape)))


def soliton_gaussian_1d(m: int, dx: float, seed, width: float = 5.0,
                        soliton_width: float = 1.0, xs_range: float = 10.0) -> np.ndarray:
    """Gaussian envelope of the given width times one dark soliton tanh((x - x_s)/w)."""
    rng = _rng(seed)
    xs = rng.uniform(-xs_range, xs_range)
    x = centred_coords(m, dx)
    return (np.exp(-x ** 2 / (2.0 * width ** 2)) * np.tanh((x - xs) / soliton_width)).astype(np.complex128)


def thomas_fermi_phase_2d(shape: Tuple[int, int], radii: Tuple[float, float], seed,
                          corr_len: float = 4.0, phase_std: float = 1.0, dx: float = 1.0) -> np.ndarray:
    """Elongated Thomas-Fermi amplitude times exp(i theta) with theta a Gaussian random field.

    ``shape`` is (My, Mx); ``radii`` is (R_y, R_x).
    """
    rng = _rng(seed)
    my, mx = shape
    y = centred_coords(my, dx)[:, None]
    x = centred_coords(mx, dx)[None, :]
    amp = np.sqrt(np.maximum(0.0, 1.0 - (x / radii[1]) ** 2 - (y / radii[0]) ** 2))
    theta = gaussian_random_field(rng, shape, corr_len, phase_std, dx)
    return amp * np.exp(1j * theta)


def two_cloud_3d(shape: Tuple[int, int, int], seed, sep: float = 12.0, sigma_t: float = 3.0,
                 sigma_ax: float = 150.0, corr_len: float = 32.0, phase_std: float = 1.0,
                 dx: float = 1.0) -> np.ndarray:
    """Two parallel elongated Gaussian clouds along x separated along y (cf. eq. (3dic)).

    ``shape`` is (Mz, My, Mx). The clouds carry phases +phi(x)/2 and -phi(x)/2,
    with phi a 1-D Gaussian random field along x.
    """
    rng = _rng(seed)
    mz, my, mx = shape
    z = centred_coords(mz, dx)[:, None, None]
    y = centred_coords(my, dx)[None, :, None]
    x = centred_coords(mx, dx)[None, None, :]
    phi = gaussian_random_field(rng, (mx,), corr_len, phase_std, dx)[None, None, :]
    out = np.zeros(shape, dtype=np.complex128)
    for sgn in (+1.0, -1.0):
        env = np.exp(-((y - sgn * sep / 2.0) ** 2 + z ** 2) / (2.0 * sigma_t ** 2)
                     - x ** 2 / (2.0 * sigma_ax ** 2))
        out += env * np.exp(1j * sgn * phi / 2.0)
    return out


def ensemble_member_3d(shape: Tuple[int, int, int], seed, mean_solitons: float = 3.0,
                       soliton_width: float = 2.0, corr_len: float = 4.0, phase_std: float = 0.5,
                       dx: float = 1.0) -> np.ndarray:
    """Thomas-Fermi cloud with Poisson-distributed planar dark solitons and thermal phase noise.

    ``shape`` is (Mz, My, Mx) with x the long axis: R_perp = M_perp/4, R_ax = 0.35 M_ax.
    """
    rng = _rng(seed)
    mz, my, mx = shape
    z = centred_coords(mz, dx)[:, None, None]
    y = centred_coords(my, dx)[None, :, None]
    x = centred_coords(mx, dx)[None, None, :]
    rz, ry, rx = mz * dx / 4.0, my * dx / 4.0, 0.35 * mx * dx
    amp = np.sqrt(np.maximum(0.0, 1.0 - (x / rx) ** 2 - (y / ry) ** 2 - (z / rz) ** 2))
    nsol = rng.poisson(mean_solitons)
    xk = rng.uniform(-0.7 * rx, 0.7 * rx, size=nsol)
    sol = np.ones((1, 1, mx))
    for xs in xk:
        sol = sol * np.tanh((x - xs) / soliton_width)
    theta = gaussian_random_field(rng, shape, corr_len, phase_std, dx)
    return amp * sol * np.exp(1j * theta)


# --------------------------------------------------------------------------------------
# The five workloads. Lattice spacing 1 and hbar = m = 1 unless stated; flight times are
# chosen so that the expanded cloud stays inside the magnified box.
# --------------------------------------------------------------------------------------

def make_c1(seed: int = 0) -> Workload:
    """1D soliton cloud, N=1024, dx=0.1, t=50, magnification 10, plain FP64."""
    f = soliton_gaussian_1d(1024, 0.1, seed)
    return Workload("c1_1d_soliton", [f], (0.1,), (10,), 50.0, dtype="c128")


def make_c2(seed: int = 1) -> Workload:
    """2D 512x512 elongated quasicondensate (aspect 8:1), magnification 32 per axis, FP32 data."""
    f = thomas_fermi_phase_2d((512, 512), (25.0, 200.0), seed, corr_len=4.0, phase_std=1.0)
    return Workload("c2_2d_quasicondensate_512", [f], (1.0, 1.0), (32, 32), 2000.0, dtype="c64")


def make_c3(seed: int = 2) -> Workload:
    """3D two-cloud interferometer 64x64x1024, magnification (50, 50, 5), column image along z."""
    f = two_cloud_3d((64, 64, 1024), seed)
    return Workload("c3_3d_interferometer", [f], (1.0, 1.0, 1.0), (50, 50, 5), 800.0,
                    dtype="c64", column_axis=0)


C4_SHAPES = ((32, 32, 256), (48, 48, 384), (64, 64, 512))


def make_c4(n: int = 768, seed: int = 3, members: Optional[Sequence[int]] = None) -> Workload:
    """Ragged ensemble: realization i has shape C4_SHAPES[i % 3]; magnification 40 per axis."""
    seqs = np.random.SeedSequence(seed).spawn(n)
    idx = range(n) if members is None else members
    fields = [ensemble_member_3d(C4_SHAPES[i % 3], seqs[i]) for i in idx]
    return Workload("c4_ragged_ensemble", fields, (1.0, 1.0, 1.0), (40, 40, 40), 400.0,
                    dtype="c64", extra={"members": list(idx)})


def _c4_member_c64(args):
    i, n, seed = args
    seqs = np.random.SeedSequence(seed).spawn(n)
    return ensemble_member_3d(C4_SHAPES[i % 3], seqs[i]).astype(np.complex64)


def c4_fields_c64(idx: Sequence[int], n: int = 768, seed: int = 3, workers: int = 1) -> List[np.ndarray]:
    """The complex64 fields of realizations ``idx`` of the ragged ensemble (same values as
    ``make_c4`` cast to complex64), generated by ``workers`` forked processes. Call it before the
    process touches the GPU."""
    jobs = [(int(i), n, seed) for i in idx]
    if workers <= 1 or len(jobs) < 2:
        return [_c4_member_c64(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_c4_member_c64, jobs, chunksize=max(1, len(jobs) // (4 * workers)))


def make_c5(n: int = 64, seed: int = 4, hidden_seed: int = 5) -> Workload:
    """Batch of 2D 256x256 fields for fitting, magnification 20 per axis; hidden fields give targets."""
    seqs = np.random.SeedSequence(seed).spawn(n)
    hid = np.random.SeedSequence(hidden_seed).spawn(n)
    fields = [thomas_fermi_phase_2d((256, 256), (12.5, 100.0), s) for s in seqs]
    hidden = [thomas_fermi_phase_2d((256, 256), (12.5, 100.0), s) for s in hid]
    return Workload("c5_2d_fit_batch", fields, (1.0, 1.0), (20, 20), 600.0, dtype="c64",
                    extra={"hidden": hidden})


WORKLOADS: Dict[str, Callable[..., Workload]] = {
    "c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5,
}


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
