"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *produces inputs*: a jittered tetrahedral cube mesh in the
form a mesh file would hold (vertex coordinates, tetrahedra, tagged boundary
triangles) and the per-cell initial fields of the benchmark problems.  It holds
none of the finite-volume method's arithmetic (no volumes, normals, stencils,
fluxes or solver steps); each side computes those itself.
"""
from .meshgen import CubeMesh, jittered_cube, BOUNDARY_TAGS
from .fields import (gaussian_field, rotating_velocity, mms_source,
                     mms_exact, problem_fields, batch_recipe, BatchMember)

__all__ = ["CubeMesh", "jittered_cube", "BOUNDARY_TAGS",
           "gaussian_field", "rotating_velocity", "mms_source", "mms_exact",
           "problem_fields", "batch_recipe", "BatchMember"]
