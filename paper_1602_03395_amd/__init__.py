"""MI355X (gfx950) implementation of the finite-time free-flight expansion onto a
magnified grid: the sum-of-FFTs prescription (FF) of arXiv:1602.03395,
section 5.2, as hand-written HIP kernels behind the C ABI of ``include/fx.h``.

Importing the package loads ``libfx.so`` from this directory and fails if it
is missing; build it with ``python paper_1602_03395_amd/build.py``.
"""

from . import _lib  # noqa: F401  (loads libfx.so, raises if absent)
from .api import (  # noqa: F401
    Batch,
    ExpandDensity,
    Plan,
    column_density,
    expand,
    expand_adjoint,
    expand_batch,
    expand_density,
    fine_wavenumbers,
    get_plan,
    real_dtype,
)

__all__ = ["Plan", "Batch", "expand_batch", "expand", "expand_adjoint", "expand_density", "ExpandDensity", "column_density", "get_plan",
           "fine_wavenumbers", "real_dtype"]
