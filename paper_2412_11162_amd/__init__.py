"""MI355X-native FFT-accelerated PML-BIE solver for axisymmetric two-layer
acoustic scattering (Wang & Lu, arXiv 2412.11162).

The work is done by the HIP library ``libpmlbie.so`` (C ABI in
``include/pmlbie.h``); :mod:`.solver` is a thin marshalling layer that uses
PyTorch only for device memory and streams.
"""

from ._binding import LIB_PATH, load  # noqa: F401

__all__ = ["LIB_PATH", "load", "Solver", "PmlbieError"]


def __getattr__(name):
    if name in ("Solver", "PmlbieError", "from_workload"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
