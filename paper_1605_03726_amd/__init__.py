"""MI355X (gfx950) engine for the lattice walk of pSpatiocyte.

The walk runs in hand-written HIP kernels behind the C ABI of libpsc.so
(include/psc.h); `psc` is its ctypes binding.
"""
from . import psc  # noqa: F401
from .psc import Lattice, PscError, lattice_from_workload  # noqa: F401
