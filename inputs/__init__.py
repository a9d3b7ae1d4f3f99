"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates meshes and nodal field values only.  It holds none of
the solver's arithmetic (no assembly, no extrapolation, no multigrid, no
Krylov method): both the CPU oracle and the GPU library receive what it
produces and do all method computations themselves.
"""
from .mesh import box_mesh, graded_mesh, Mesh  # noqa: F401
from .fields import manufactured_u, manufactured_f, fourier_field  # noqa: F401
