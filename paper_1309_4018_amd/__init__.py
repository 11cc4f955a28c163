"""MI355X-native treecode boundary-element Poisson-Boltzmann solver.

The compute path is libpbtc.so (HIP C++ for gfx950, C interface in
include/pbtc.h); ``lib`` is its ctypes binding and ``autograd`` wraps a solve
as a differentiable torch function.
"""

from . import lib  # noqa: F401

__all__ = ["lib"]
