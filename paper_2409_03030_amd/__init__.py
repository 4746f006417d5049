"""MI355X (gfx950) Wilson-Dirac operator and CG on D^dag D.

The compute path is the HIP library ``libwdirac.so`` (C ABI in
``include/wdirac.h``); ``wdirac`` is its ctypes binding.
"""

from . import wdirac  # noqa: F401
from .wdirac import (  # noqa: F401
    EO, F16, F32, F64, FULL, Lattice, Server, WDError, default_params, solve_batch,
)
