"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the DG method: it builds tetrahedral
meshes (vertex ids and coordinates), analytic initial fields in primitive
variables, and seeded random arrays. Both sides consume these inputs and do
everything else on their own.
"""
from .mesh import TetMesh, kuhn_cube  # noqa: F401
from . import fields  # noqa: F401
