"""Seeded synthetic scene generators shared by the oracle, the tests and the bench.

This module only builds inputs: rest meshes (hexahedral grids split into
tetrahedra, voxelised spheres and tori), their boundary surfaces, per-tet
material fields, planes, prescribed-vertex schedules and initial states.  It
holds none of the solver's arithmetic (no energy, no gradient, no distance,
no candidate test), so both sides that consume it stay independent.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
Positions are float64 ``(n, 3)`` row-major, indices int32, tets positively
oriented (``det[X1-X0, X2-X0, X3-X0] > 0``).
"""
from .mesh import (hex_grid, surface_of, voxel_mesh, merge_meshes, Scene,
                   rotation_matrix)
from .configs import (cube_scene, twisted_bar_scene, stacked_bars_scene, twist_targets, pile_scene,
                      packed_pile_scene,
                      batched_scenes, pack_batch, diff_bar_scene, small_contact_scene,
                      tiny_scene)

__all__ = [
    "hex_grid", "surface_of", "voxel_mesh", "merge_meshes", "Scene",
    "rotation_matrix", "cube_scene", "twisted_bar_scene", "stacked_bars_scene", "twist_targets",
    "pile_scene", "packed_pile_scene", "batched_scenes", "pack_batch", "diff_bar_scene", "small_contact_scene",
    "tiny_scene",
]
