"""CPU oracle for the Wilson-Dirac operator and CG on D^dagger D.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  See ``wilson.py``.
"""

from .wilson import *  # noqa: F401,F403
from .wilson import GAMMA, GAMMA5, ONE4  # noqa: F401
from .propagator import point_propagator, pion_correlator, residual_D, solve_D  # noqa: F401
from .force import fermion_action, fermion_force, momentum_update, pseudofermion_heatbath  # noqa: F401
from .force import force_from_solutions, traceless_antihermitian  # noqa: F401
