"""ParaDiag-II all-at-once time-parallel solver for MI355X (gfx950).

The compute path is the HIP library libparadiag.so (C ABI in
include/paradiag.h); this package only marshals torch tensors into it.
"""

from ._lib import ParaDiagError, load  # noqa: F401

__all__ = ["ParaDiag", "ParaDiagOC", "ParaDiagSolve", "ParaDiagError", "load", "host_plan"]


def __getattr__(name):
    # torch is imported lazily so that `build` works without it
    if name in ("ParaDiag", "ParaDiagOC", "ParaDiagSolve", "host_plan", "SolveResult"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
