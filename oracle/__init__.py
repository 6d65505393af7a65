"""Plain FP64 CPU oracle for the all-at-once CQM Galerkin BEM single-layer solve,
its compressed form and time marching, and the Calderon operators K, K' and D.

TEST INFRASTRUCTURE ONLY. This package exists to check the GPU library. Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path (the C-ABI library and its Python binding) never
does, and shares no code with it.

Everything here is written for a reader holding the paper (Seibel, "Boundary
Element Methods for the Wave Equation based on Hierarchical Matrices and
Adaptive Cross Approximation"): each function cites the section or equation it
follows. The arithmetic is plain NumPy/SciPy in float64/complex128, with no
blocking or reordering beyond what the definitions state.
"""
from .cqm import *  # noqa: F401,F403
from .compress import *  # noqa: F401,F403
from .marching import *  # noqa: F401,F403
from . import calderon  # noqa: F401
from . import marching  # noqa: F401
from . import hypersingular  # noqa: F401
