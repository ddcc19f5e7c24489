"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This package only *generates inputs*: skeleton meshes, the triangle
quadrature rule, chart-node coordinates on the standard simplex, per-triangle
smoothing widths and target points.  It holds none of the level-set
arithmetic (quadrature-node placement, the smoothed-indicator kernel,
pseudonormals, Newton updates): the HIP library and the CPU oracle each do
that on their own.

Every generator is deterministic given its seed (numpy ``default_rng``,
PCG64).
"""
from .rules import dunavant6, chart_nodes_45, chart_nodes
from .meshes import (cube_mesh, icosphere, geodesic_sphere, star_surface,
                     bumpy_sphere, graded_torus, mesh_check, triangle_diameters,
                     refine_1to4, refine_1to4_quadratic, torus_mesh, quadratic_from_flat)
from .targets import (box_targets, shell_targets, surface_offset_targets,
                      bbox_targets)
from . import configs

__all__ = [
    "dunavant6", "chart_nodes_45", "chart_nodes", "cube_mesh", "icosphere",
    "geodesic_sphere", "star_surface", "bumpy_sphere", "graded_torus", "mesh_check",
    "triangle_diameters", "refine_1to4", "refine_1to4_quadratic", "torus_mesh", "quadratic_from_flat", "box_targets", "shell_targets",
    "surface_offset_targets", "bbox_targets", "configs",
]
