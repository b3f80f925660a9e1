"""Pins of the oracle's positive-P pair expansion (CPU only).

For the two fields of a positive-P simulation (section 7.4) psi^+ evolves with the
complex-conjugate free kernel. The pins tie ``oracle.expand_pair`` to facts
outside its own arithmetic:

* psi^+ = conj(psi) is the classical (Glauber-P-like) limit: psibar^+ must be
  conj(psibar) and the density estimator psibar^+ psibar must be |psibar|^2;
* for an integer offset delta the conjugate kernel is the free kernel run
  backwards in time (the fine wave-number set is symmetric modulo lam M), so
  psibar^+ equals the free-flight oracle at -t, itself pinned by brute force;
* the total of the estimator over the lam shifted output grids equals
  sum psi^+ psi at t = 0 (the conserved particle number of the pair);
* a planted mistake (psi^+ propagated with the unconjugated kernel) fails the
  time-reversal pin.
"""

import numpy as np

import oracle


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_conjugate_pair_reduces_to_classical_density():
    shape, lam, dx, t = (10, 12), (3, 2), (1.0, 0.5), 17.0
    psi = rand_field(shape, 1)
    pb, pbp, n = oracle.expand_pair(psi, psi.conj(), dx, 1.0, t, lam)
    ref = oracle.expand(psi, dx, 1.0, t, lam)
    assert rel(pb, ref) <= 1e-14
    assert rel(pbp, ref.conj()) <= 1e-14
    assert rel(n, np.abs(ref) ** 2) <= 1e-14


def test_psi_plus_runs_backwards_in_time():
    shape, lam, dx, t, moh = (9, 14), (4, 3), (0.5, 1.0), 23.0, 1.4
    psi = rand_field(shape, 2)
    psi_plus = rand_field(shape, 3)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = a + np.round((abar - a) / np.asarray(dx)) * np.asarray(dx)  # integer delta
    _, pbp, _ = oracle.expand_pair(psi, psi_plus, dx, moh, t, lam, a, abar)
    back = oracle.expand(psi_plus, dx, moh, -t, lam, a, abar)
    assert rel(pbp, back) <= 1e-13
    # planted mistake: psi^+ taken with the forward kernel
    fwd = oracle.expand(psi_plus, dx, moh, t, lam, a, abar)
    assert rel(fwd, back) > 1e-2


def test_estimator_total_is_conserved_over_shifted_grids():
    shape, lam, dx, t = (6, 5), (3, 2), (1.0, 0.5), 7.0
    psi = rand_field(shape, 4)
    psi_plus = rand_field(shape, 5)
    a, abar0 = oracle.default_offsets(shape, dx, lam)
    total = 0.0 + 0.0j
    for s0 in range(lam[0]):
        for s1 in range(lam[1]):
            abar = abar0 + np.array([s0 * dx[0], s1 * dx[1]])
            total += oracle.expand_pair(psi, psi_plus, dx, 1.0, t, lam, a, abar)[2].sum()
    expect = (psi_plus * psi).sum()
    assert abs(total - expect) <= 1e-13 * np.sum(np.abs(psi) * np.abs(psi_plus))
