"""MI355X-native coupled multigrid for the generalized Stokes problem
(Takacs, "A robust multigrid method for the time-dependent Stokes problem").

The solver lives in the HIP library libstokesmg.so (C ABI in
include/stokesmg.h); this package is its thin Python front end.
"""
from .solver import Batch, Hierarchy, SolveInfo  # noqa: F401

__all__ = ["Batch", "Hierarchy", "SolveInfo"]
