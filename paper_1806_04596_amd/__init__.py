"""MI355X (gfx950) HyperSARA primal-dual hot path.

The compute lives in ``libhypersara.so`` (hand-written HIP kernels behind a C
ABI declared in ``include/hypersara.h``).  This package only marshals
arguments: there is no CPU fallback, and every entry point raises if the
library is missing or no HIP device is present.
"""
from ._lib import HSError, load  # noqa: F401
from .problem import Problem, density_precond, visibility_order, daubechies_filter  # noqa: F401

__all__ = ["Problem", "HSError", "load", "density_precond", "visibility_order", "daubechies_filter"]
