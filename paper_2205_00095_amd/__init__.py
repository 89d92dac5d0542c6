"""MI355X-native DG special-relativistic hydrodynamics hot path (Glines et al.).

The arithmetic lives in the gfx950 HIP library ``libdgsrhd.so`` (C ABI in
include/dgsrhd.h); this package holds the ctypes binding (argument marshalling
only), the adjoint autograd function and the seeded workload generator.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "Solver", "build"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
