"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This package builds triangulated polyhedral surfaces (the input of the
capacity problem, Section 2.1 of the paper: conforming triangulations of a
closed polyhedral boundary into plane triangles), refines them with newest
vertex bisection (Fig. "nvb", Algorithm step (iv)) and draws seeded request
streams, and builds the barycentric refinement of a mesh (the common
refinement of the mesh and its dual, Section 2.1).  It contains none of the method's arithmetic (no quadrature, no
integral operator, no solver), so both sides can use it without sharing any
computation.
"""

from .meshes import (  # noqa: F401
    Mesh,
    box,
    convex_hull,
    cube,
    cube12,
    fichera48,
    icosphere,
    mesh_topology_ok,
    min_angle_deg,
    voxel_union,
)
from .nvb import (  # noqa: F401
    init_reference_edges,
    refine_nvb,
    refine_to_size,
    refine_uniform,
)
from .requests import Request, request_stream  # noqa: F401
from .dual import SON_VERTEX, barycentric, vertex_incidence  # noqa: F401
