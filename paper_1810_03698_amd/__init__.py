"""MI355X-native boundary-integral Poisson-Boltzmann solver with polarisable
point multipoles.

The computation runs in the HIP library ``libpbmp.so`` (C-ABI in
``include/pbmp.h``); ``pbmp`` is its ctypes binding and ``autograd`` wraps
solve/backward as a ``torch.autograd.Function``.
"""

from . import pbmp
from .pbmp import Solver, load, PbmpError


def solvation_energy(*args, **kwargs):
    """Differentiable solvation energy (see autograd.solvation_energy)."""
    from .autograd import solvation_energy as f
    return f(*args, **kwargs)


__all__ = ["pbmp", "Solver", "load", "PbmpError", "solvation_energy"]
