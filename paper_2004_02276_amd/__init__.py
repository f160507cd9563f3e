"""MI355X-native right-hand side and low-storage RK3 step of the compressible
Navier-Stokes equations, after "STREAmS" (arXiv 2004.02276).

The numerics live in the HIP library libcdns.so (C ABI in include/cdns.h);
this package only marshals arguments.  Importing `Solver` loads the library
and fails if it has not been built.
"""
from ._binding import CDNS_FP32_FLUX, CDNS_FP64, CdnsError, load  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name in ("Batch", "Server"):
        from . import serve
        return getattr(serve, name)
    raise AttributeError(name)
