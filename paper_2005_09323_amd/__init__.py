"""MI355X ensemble lattice-Boltzmann with GKTL / AMS rare-event sampling.

A D2Q9 lattice-BGK channel flow past a square (paper Section 2, Appendix A)
is advanced for a whole ensemble of trajectories by hand-written gfx950 HIP
kernels behind the C ABI of ``include/lbm.h``; ``native`` binds it with
ctypes and ``ensemble`` wraps it around torch-owned device memory.
"""
from . import native  # noqa: F401
