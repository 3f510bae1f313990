"""Seeded synthetic inputs (meshes and manufactured problems).

This package is shared by the oracle and the HIP library's tests and
benchmark.  It holds input data only: element maps, connectivity and the
analytic data f, g, u_exact of the manufactured problems.  It contains none
of the discretisation's arithmetic.
"""
from .mesh import Mesh, box_mesh  # noqa: F401
