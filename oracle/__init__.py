"""ORACLE -- test infrastructure, not part of the product.

A plain, slow, obviously correct CPU evaluation of what the free-flight
expansion computes, used only by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``. The product library never imports, links or
calls anything here, and nothing here imports the product package.

Definition (sections 5.1-5.2; eqs. (vacuum), (ex1)-(ex5), (iDFTbar), (FF)):
the expanded field on the magnified grid is the discrete free propagator of
the vacuum-padded, lam_j-times-larger periodic lattice, sampled at the coarse
output points,

    Psibar[nbar] = sum_n Psi[n] prod_j G_j(xbar_{nbar_j} - x_{n_j}),

with G_j the 1-D kernel tabulated by ``oracle/gtable.c``. The kernel factorises
over axes because the free dispersion hbar k^2 / 2m is a sum over axes
(eq. (free0)). No FFT is used anywhere in the oracle.
"""

from .propagator import (  # noqa: F401
    axis_matrix,
    build_c_kernel,
    column_density,
    default_offsets,
    density,
    direct_nd,
    expand,
    expand_adjoint,
    expand_dispersion,
    expand_pair,
    expand_dispersion_adjoint,
    fine_wavenumbers,
    gtable_phase,
    expand_points,
    far_field,
    gtable,
    gtable_longdouble,
    loss_and_grad,
    have_c_kernel,
)
