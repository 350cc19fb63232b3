"""Seeded synthetic inputs: meshes, stencils and initial fields.

Shared by the library's tests, its benchmark and its oracle; holds none of
the reconstruction method's arithmetic.
"""
from .mesh import Mesh, TRI, QUAD, TET, PYR, PRISM, HEX, quad_tri_2d, hex_3d  # noqa: F401
from .stencil import Stencils, build_stencils, n_unknowns, cell_centroids  # noqa: F401
