"""MI355X library for time-domain single-layer BEM by convolution quadrature.

The compute path is the HIP/C++ shared library lib/libcqm.so (C ABI declared in
include/cqm.h); this package is only its Python binding.  It never falls back
to a CPU implementation: if the library is missing, importing the binding's
entry points raises.
"""
from .cqm import *  # noqa: F401,F403
