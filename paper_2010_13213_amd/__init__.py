"""MI355X-native lattice Green's function (LGF) Poisson solver.

The solver itself lives in liblgf.so (HIP kernels for gfx950 behind the C
ABI of include/lgf.h); ``lgf`` is its ctypes binding and ``inputs`` builds
seeded synthetic supports and sources.
"""
from . import inputs  # noqa: F401
