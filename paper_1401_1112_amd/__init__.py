"""MI355X-native level-by-level implicit diffusion solve for adaptive time-stepping
on oct-based AMR grids (Commercon, Debout & Teyssier 2014).

The compute path is the HIP library ``libamrfld.so`` (C ABI in include/amrfld.h);
this package holds its ctypes binding and a small convenience wrapper.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    AmrfldError, load, BC_DIRICHLET, BC_NEUMANN, BC_ROBIN, FP64, MIXED, K_CONST, K_LP, K_MINERBO,
    K_POWER,
    OK, E_INVALID, E_STATE, E_NOMEM, E_DEVICE, E_NOCONV, E_NONFINITE,
)
from .solver import HierarchySolver  # noqa: F401
