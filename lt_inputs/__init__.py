"""Seeded synthetic inputs for the light-tracing hot path.

This package builds scenes (triangles grouped into planar rectangular patches
that carry texel grids), luminaires and painted irradiance targets.  It is the
only code shared by the CPU oracle and the GPU path, and it holds none of the
method's arithmetic: no emission sampling, no intersection, no splatting, no
derivatives.  Everything it returns is plain geometry, parameters and target
values, fixed by a seed.
"""
from .scenes import (  # noqa: F401
    PATCH_DTYPE, LIGHT_DTYPE, Scene, Lights, SceneBuilder,
    box_room, office, room_set, building_floor, plane_scene, closed_box,
    painted_target, texel_centers, perturb_params, random_scene_tiny, crossing_slivers,
)
