"""MI355X-native vertical-extrapolation multigrid PCG for the P1 Poisson
equation on thin tetrahedral domains (Kramer, Cotter & Pain).

The solver runs in libvemg.so (host setup in C++, hot path in HIP kernels for
gfx950); this package is a thin ctypes binding over its C ABI (include/vemg.h)
that passes PyTorch device tensors as raw pointers.
"""
from ._lib import (  # noqa: F401
    Solver, Server, VemgError, load_library, library_path, OP_A, OP_PRECOND, OP_ET, OP_E,
    OP_VCYCLE_S, OP_VCYCLE_ABAR, OP_GS_FWD, OP_GS_COARSE, OP_COARSEST, STATUS,
)
