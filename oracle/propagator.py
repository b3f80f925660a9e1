"""ORACLE -- test infrastructure, not part of the product (see ``oracle/__init__``).

Plain FP64 CPU evaluation of the finite-time free-flight expansion onto the
magnified grid, written from the definition the prescription (FF) reaches
exactly (sections 5.1-5.2):

* Lattices (section 2.1, eq. (xj); section 5.2): input x_j = a_j + n_j dx_j,
  n_j = 0..M_j-1, L_j = M_j dx_j; output xbar_j = abar_j + nbar_j lam_j dx_j,
  nbar_j = 0..M_j-1 (eq. (wbx)).
* Vacuum outside the input box (eq. (vacuum)), so the k-space field on the fine
  lattice of spacing dk_j / lam_j is a plain sum over the small lattice
  (eqs. (ex1)-(ex3)); free evolution multiplies by exp(-i hbar t k^2 / 2m)
  (eqs. (free0), (time)); the return sum (eq. (ex4)) is evaluated at the coarse
  points xbar (eq. (ex5)).
* Combining the three sums gives, per axis, the kernel
  G_j(r) = 1/(lam_j M_j) sum_{l in F_j} exp(i kappa_l r - i hbar t kappa_l^2 / 2m),
  kappa_l = 2 pi l / (lam_j L_j), F_j the lam_j M_j fine wave numbers centred on
  zero with the Nyquist value negative (eq. (kj) on the fine lattice, which
  also reproduces the odd-M umklapp rule of section 5.2).

Default offsets (readings of the paper where it leaves them free): the input
box is centred on zero, a_j = -L_j / 2 (as for the large lattice of section 3),
and the magnified box is centred on the same point, abar_j = a_j + (1 - lam_j) L_j / 2.
"""

from __future__ import annotations

import ctypes
import functools
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_gtable.so")
_lib = None


def _load():
    global _lib
    if _lib is None and os.path.exists(_LIB_PATH):
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_gtable.restype = ctypes.c_int
        lib.oracle_gtable.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


def have_c_kernel() -> bool:
    return _load() is not None


def build_c_kernel(verbose: bool = False) -> str:
    """Compile ``gtable.c`` with gcc into ``oracle/liboracle_gtable.so``."""
    import subprocess
    src = os.path.join(_HERE, "gtable.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB_PATH


# ----------------------------------------------------------------------------------------
# Offsets and the per-axis kernel G_j
# ----------------------------------------------------------------------------------------

def default_offsets(shape: Sequence[int], dx: Sequence[float], lam: Sequence[int],
                    a: Optional[Sequence[float]] = None,
                    abar: Optional[Sequence[float]] = None) -> Tuple[np.ndarray, np.ndarray]:
    shape = np.asarray(shape, dtype=np.int64)
    dx = np.asarray(dx, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.int64)
    L = shape * dx
    a_out = -0.5 * L if a is None else np.asarray(a, dtype=np.float64).copy()
    abar_out = a_out + (1.0 - lam) * L / 2.0 if abar is None else np.asarray(abar, dtype=np.float64).copy()
    return a_out, abar_out


def gtable_longdouble(M: int, lam: int, delta: float, t: float, m_over_hbar: float, dx: float,
                      s_min: int, count: int) -> np.ndarray:
    """Same sum as ``gtable.c`` in numpy long double (slow; tiny sizes and cross-checks)."""
    N = lam * M
    l = np.arange(-(N // 2), -(N // 2) + N, dtype=np.int64)
    pi = np.arccos(np.longdouble(-1))
    beta = pi * (np.longdouble(t) / np.longdouble(m_over_hbar)) / (np.longdouble(N) * np.longdouble(dx)) ** 2
    di = int(np.rint(delta))
    df = np.longdouble(delta) - np.longdouble(di)
    out = np.empty(count, dtype=np.complex128)
    lq = (l.astype(np.longdouble) * l.astype(np.longdouble))
    lf = l.astype(np.longdouble) * df / np.longdouble(N)
    for i in range(count):
        s = s_min + i + di
        k = np.mod(np.mod(l, N) * (s % N), N)
        ph = k.astype(np.longdouble) / np.longdouble(N) + lf - beta * lq
        ph = ph - np.rint(ph)
        ang = 2 * pi * ph
        out[i] = complex(np.cos(ang).sum() / N, np.sin(ang).sum() / N)
    return out


def gtable(M: int, lam: int, delta: float, t: float, m_over_hbar: float, dx: float,
           s_min: int, count: int) -> np.ndarray:
    """G(s_min + i), i < count, as complex128 (C kernel if built, else long double numpy)."""
    lib = _load()
    if lib is None:
        return gtable_longdouble(M, lam, delta, t, m_over_hbar, dx, s_min, count)
    re = np.empty(count, dtype=np.float64)
    im = np.empty(count, dtype=np.float64)
    rc = lib.oracle_gtable(int(M), int(lam), float(delta), float(t), float(m_over_hbar), float(dx),
                           int(s_min), int(count),
                           re.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           im.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_gtable rejected its arguments")
    return re + 1j * im


@functools.lru_cache(maxsize=64)
def _axis_matrix_cached(M: int, lam: int, dx: float, a: float, abar: float, t: float,
                        m_over_hbar: float) -> np.ndarray:
    delta = (abar - a) / dx
    s_min = -(M - 1)
    count = (lam + 1) * (M - 1) + 1
    tab = gtable(M, lam, delta, t, m_over_hbar, dx, s_min, count)
    nbar = np.arange(M)[:, None]
    n = np.arange(M)[None, :]
    G = tab[lam * nbar - n - s_min]
    G.setflags(write=False)
    return G


def axis_matrix(M: int, lam: int, dx: float, a: float, abar: float, t: float,
                m_over_hbar: float) -> np.ndarray:
    """Dense M x M matrix G[nbar, n] = G(lam*nbar - n) of one axis."""
    return _axis_matrix_cached(int(M), int(lam), float(dx), float(a), float(abar), float(t),
                               float(m_over_hbar))


def _matrices(shape, dx, lam, t, m_over_hbar, a, abar):
    a, abar = default_offsets(shape, dx, lam, a, abar)
    return [axis_matrix(shape[j], lam[j], dx[j], a[j], abar[j], t, m_over_hbar)
            for j in range(len(shape))]


def _apply(mats, x):
    for j, G in enumerate(mats):
        x = np.moveaxis(np.tensordot(G, x, axes=([1], [j])), 0, j)
    return x


# ----------------------------------------------------------------------------------------
# Public oracle entry points
# ----------------------------------------------------------------------------------------

def expand(psi: np.ndarray, dx, m_over_hbar: float, t: float, lam, a=None, abar=None) -> np.ndarray:
    """Expanded field on the magnified grid (complex128), same shape as ``psi``."""
    psi = np.asarray(psi).astype(np.complex128)
    d = psi.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    return _apply(_matrices(psi.shape, dx, lam, t, m_over_hbar, a, abar), psi)


def expand_adjoint(y: np.ndarray, dx, m_over_hbar: float, t: float, lam, a=None, abar=None) -> np.ndarray:
    """Hermitian adjoint of ``expand`` applied to a field on the magnified grid."""
    y = np.asarray(y).astype(np.complex128)
    d = y.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    mats = [G.conj().T for G in _matrices(y.shape, dx, lam, t, m_over_hbar, a, abar)]
    return _apply(mats, y)


def expand_points(psi: np.ndarray, points: np.ndarray, dx, m_over_hbar: float, t: float, lam,
                  a=None, abar=None) -> np.ndarray:
    """Expanded field at selected output indices ``points`` (shape [K, d]) only."""
    psi = np.asarray(psi).astype(np.complex128)
    d = psi.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    mats = _matrices(psi.shape, dx, lam, t, m_over_hbar, a, abar)
    points = np.atleast_2d(np.asarray(points, dtype=np.int64))
    out = np.empty(points.shape[0], dtype=np.complex128)
    for i, p in enumerate(points):
        x = psi
        for j in range(d - 1, -1, -1):
            x = np.tensordot(x, mats[j][p[j]], axes=([j], [0]))
        out[i] = x
    return out


def density(psibar: np.ndarray) -> np.ndarray:
    """rho = |Psibar|^2 (section 2: the measured quantity)."""
    return psibar.real ** 2 + psibar.imag ** 2


def column_density(rho: np.ndarray, axis: int, lam, dx) -> np.ndarray:
    """Density image integrated along one axis of the magnified grid (section 6: rho(x,y) = int dz |Psi|^2).

    The integral is the sum over the output samples times their spacing lam_j dx_j.
    """
    d = rho.ndim
    lam = np.broadcast_to(lam, (d,))
    dx = np.broadcast_to(dx, (d,))
    return rho.sum(axis=axis) * (float(lam[axis]) * float(dx[axis]))


def loss_and_grad(psi: np.ndarray, tau: np.ndarray, dx, m_over_hbar: float, t: float, lam,
                  a=None, abar=None):
    """L = sum (|U psi|^2 - tau)^2 and its gradient dL/dRe + i dL/dIm = U^H (4 (rho - tau) U psi)."""
    pb = expand(psi, dx, m_over_hbar, t, lam, a, abar)
    rho = density(pb)
    r = rho - tau
    loss = float((r * r).sum())
    grad = expand_adjoint(4.0 * r * pb, dx, m_over_hbar, t, lam, a, abar)
    return loss, grad


def direct_nd(psi: np.ndarray, dx, m_over_hbar: float, t: float, lam, a=None, abar=None) -> np.ndarray:
    """Full d-dimensional direct sum without the per-axis factorisation (tiny grids only).

    Psibar[nbar] = 1/(lam M) sum_n Psi[n] sum_{l vector} exp(2 pi i sum_j [l_j (s_j + delta_j)/N_j - beta_j l_j^2]),
    all phases accumulated in long double before a single exponential per term.
    """
    psi = np.asarray(psi).astype(np.complex128)
    d = psi.ndim
    shape = psi.shape
    dx = np.broadcast_to(np.asarray(dx, dtype=np.float64), (d,))
    lam = np.broadcast_to(np.asarray(lam, dtype=np.int64), (d,))
    a, abar = default_offsets(shape, dx, lam, a, abar)
    pi = np.arccos(np.longdouble(-1))
    N = [int(lam[j] * shape[j]) for j in range(d)]
    ls = [np.arange(-(Nj // 2), -(Nj // 2) + Nj, dtype=np.int64) for Nj in N]
    grids = np.meshgrid(*ls, indexing="ij")
    lvec = [g.reshape(-1).astype(np.longdouble) for g in grids]
    beta = [pi * (np.longdouble(t) / np.longdouble(m_over_hbar)) / (np.longdouble(N[j]) * np.longdouble(dx[j])) ** 2
            for j in range(d)]
    delta = [np.longdouble((abar[j] - a[j]) / dx[j]) for j in range(d)]
    Ntot = int(np.prod(N))
    out = np.zeros(shape, dtype=np.complex128)
    in_idx = list(np.ndindex(*shape))
    for nbar in np.ndindex(*shape):
        re = np.longdouble(0)
        im = np.longdouble(0)
        for n in in_idx:
            ph = np.zeros(lvec[0].shape, dtype=np.longdouble)
            for j in range(d):
                s = np.longdouble(int(lam[j]) * nbar[j] - n[j])
                ph = ph + lvec[j] * (s + delta[j]) / np.longdouble(N[j]) - beta[j] * lvec[j] * lvec[j]
            ph = ph - np.rint(ph)
            ang = 2 * pi * ph
            c = np.cos(ang).sum()
            s_ = np.sin(ang).sum()
            v = psi[n]
            re += np.longdouble(v.real) * c - np.longdouble(v.imag) * s_
            im += np.longdouble(v.real) * s_ + np.longdouble(v.imag) * c
        out[nbar] = complex(re / Ntot, im / Ntot)
    return out


# ----------------------------------------------------------------------------------------
# Other spectra (section 7.4, generalisations): exp(-i t omega_k) in place of the
# free-particle phase, for a dispersion that is a sum over axes, omega_k = sum_j omega_j(k_j).
# ----------------------------------------------------------------------------------------

def fine_wavenumbers(M: int, lam: int, dx: float) -> np.ndarray:
    """kappa_l = 2 pi l / (lam M dx) for the lam M fine wave numbers l, ascending from -floor(lam M / 2)."""
    N = int(lam) * int(M)
    l = np.arange(-(N // 2), -(N // 2) + N, dtype=np.float64)
    return 2.0 * np.pi * l / (N * float(dx))


def gtable_phase(M: int, lam: int, delta: float, phase: np.ndarray, s_min: int, count: int) -> np.ndarray:
    """G(s) = 1/(lam M) sum_l exp(2 pi i l (s + delta) / (lam M) - i phase_l), s = s_min + i.

    ``phase[i]`` is t * omega(kappa_l) in radians for l = i - floor(lam M / 2).
    The integer part of l (s + delta) is reduced exactly modulo lam M in int64,
    the rest of the phase is accumulated in long double.
    """
    N = int(lam) * int(M)
    phase = np.asarray(phase, dtype=np.float64)
    if phase.shape != (N,):
        raise ValueError(f"phase must hold lam*M = {N} values")
    l = np.arange(-(N // 2), -(N // 2) + N, dtype=np.int64)
    pi = np.arccos(np.longdouble(-1))
    di = int(np.rint(delta))
    df = np.longdouble(delta) - np.longdouble(di)
    rest = l.astype(np.longdouble) * df / np.longdouble(N) - phase.astype(np.longdouble) / (2 * pi)
    out = np.empty(count, dtype=np.complex128)
    for i in range(count):
        s = s_min + i + di
        k = np.mod(np.mod(l, N) * (s % N), N)
        ph = k.astype(np.longdouble) / np.longdouble(N) + rest
        ph = ph - np.rint(ph)
        ang = 2 * pi * ph
        out[i] = complex(np.cos(ang).sum() / N, np.sin(ang).sum() / N)
    return out


def axis_matrix_phase(M: int, lam: int, dx: float, a: float, abar: float, phase: np.ndarray) -> np.ndarray:
    """Dense M x M matrix G[nbar, n] = G(lam*nbar - n) of one axis for a tabulated spectrum."""
    delta = (abar - a) / dx
    s_min = -(M - 1)
    count = (lam + 1) * (M - 1) + 1
    tab = gtable_phase(M, lam, delta, phase, s_min, count)
    nbar = np.arange(M)[:, None]
    n = np.arange(M)[None, :]
    return tab[lam * nbar - n - s_min]


def _matrices_phase(shape, dx, lam, t, m_over_hbar, a, abar, phases):
    a, abar = default_offsets(shape, dx, lam, a, abar)
    mats = []
    for j in range(len(shape)):
        if phases is None or phases[j] is None:
            mats.append(axis_matrix(shape[j], lam[j], dx[j], a[j], abar[j], t, m_over_hbar))
        else:
            mats.append(axis_matrix_phase(shape[j], lam[j], dx[j], a[j], abar[j], phases[j]))
    return mats


def expand_dispersion(psi: np.ndarray, dx, lam, phases, m_over_hbar: float = 1.0, t: float = 0.0,
                      a=None, abar=None) -> np.ndarray:
    """Expansion with the spectrum t*omega_j tabulated per axis (``phases[j]``, see ``gtable_phase``).

    An axis whose entry is None keeps the free-particle phase hbar t k^2 / 2m.
    """
    psi = np.asarray(psi).astype(np.complex128)
    d = psi.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    return _apply(_matrices_phase(psi.shape, dx, lam, t, m_over_hbar, a, abar, phases), psi)


def expand_dispersion_adjoint(y: np.ndarray, dx, lam, phases, m_over_hbar: float = 1.0, t: float = 0.0,
                              a=None, abar=None) -> np.ndarray:
    """Hermitian adjoint of ``expand_dispersion``."""
    y = np.asarray(y).astype(np.complex128)
    d = y.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    mats = [G.conj().T for G in _matrices_phase(y.shape, dx, lam, t, m_over_hbar, a, abar, phases)]
    return _apply(mats, y)


# ----------------------------------------------------------------------------------------
# Two fields (section 7.4, generalisations): positive-P pairs psi, psi^+.
# ----------------------------------------------------------------------------------------

def expand_pair(psi: np.ndarray, psi_plus: np.ndarray, dx, m_over_hbar: float, t: float, lam,
                a=None, abar=None):
    """Free flight of a positive-P pair onto the magnified grid.

    psi follows the free Schroedinger equation (kernel G), psi^+ the conjugate one
    (kernel conj(G), elementwise), as the fields standing for the annihilation and
    creation operators do. Returns (psibar, psibar_plus, n) with the density
    estimator n = psibar_plus * psibar (complex).
    """
    psi = np.asarray(psi).astype(np.complex128)
    psi_plus = np.asarray(psi_plus).astype(np.complex128)
    if psi.shape != psi_plus.shape:
        raise ValueError("psi and psi_plus must have the same shape")
    d = psi.ndim
    dx = tuple(float(v) for v in np.broadcast_to(dx, (d,)))
    lam = tuple(int(v) for v in np.broadcast_to(lam, (d,)))
    mats = _matrices(psi.shape, dx, lam, t, m_over_hbar, a, abar)
    pb = _apply(mats, psi)
    pbp = _apply([G.conj() for G in mats], psi_plus)
    return pb, pbp, pbp * pb


# ----------------------------------------------------------------------------------------
# Far-field estimate (section 2.3, eqs. (farfieldk), (FT), (Psiwtm)): the comparator the
# finite-time expansion replaces.
# ----------------------------------------------------------------------------------------

def far_field(psi: np.ndarray, dx, m_over_hbar: float, t: float, lam, a=None, abar=None):
    """Far-field amplitude and density on the magnified output lattice.

    rho_ff(r) = (m / hbar t)^d |Psi~(m r / hbar t)|^2 (eq. (farfieldk)) with the norm-preserving
    transform of eq. (FT) evaluated directly (not on the DFT grid) at kappa = m r / (hbar t) from the
    lattice sum of eq. (Psiwtm): Psi~(kappa) = dV / (2 pi)^(d/2) sum_n Psi_n exp(-i kappa . x_n).
    r runs over the output points xbar_j = abar_j + nbar_j lam_j dx_j. Returns (amp, rho) with
    amp = (m / hbar t)^(d/2) Psi~(m r / hbar t) (the estimate carries no phase information beyond
    this), rho = |amp|^2. Phases are accumulated in long double before one exponential.
    """
    psi = np.asarray(psi).astype(np.complex128)
    d = psi.ndim
    if t == 0:
        raise ValueError("the far-field estimate needs t != 0")
    dx = np.broadcast_to(np.asarray(dx, dtype=np.float64), (d,))
    lam = np.broadcast_to(np.asarray(lam, dtype=np.int64), (d,))
    a, abar = default_offsets(psi.shape, dx, lam, a, abar)
    scale = np.longdouble(m_over_hbar) / np.longdouble(t)
    mats = []
    for j in range(d):
        M = psi.shape[j]
        x = np.longdouble(a[j]) + np.arange(M, dtype=np.longdouble) * np.longdouble(dx[j])
        xb = np.longdouble(abar[j]) + np.arange(M, dtype=np.longdouble) * np.longdouble(lam[j] * dx[j])
        ph = -(scale * xb)[:, None] * x[None, :]
        two_pi = 2 * np.arccos(np.longdouble(-1))
        ph = ph - two_pi * np.rint(ph / two_pi)
        mats.append((np.cos(ph) + 1j * np.sin(ph)).astype(np.complex128))
    amp = _apply(mats, psi)
    dV = float(np.prod(dx))
    amp = amp * (float(abs(scale)) ** (d / 2.0)) * dV / (2.0 * np.pi) ** (d / 2.0)
    return amp, density(amp)
