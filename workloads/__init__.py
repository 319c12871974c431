"""Seeded synthetic workloads for LSNIF queries.

This package makes the *inputs* of the query path and nothing else: procedural
meshes, their surface voxelisation (the offline asset step of the method,
paper Sec. 3.1), the level resolutions, hash-table features, MLP weights and
ray batches.  It holds none of the query path's arithmetic (no DDA, no
encoding, no MLP, no decode), so that the CPU oracle and the GPU library can
both consume it without sharing any of the computation they are compared on.
"""

from .rng import streams
from .meshes import icosphere, uv_sphere, displaced_sphere, torus, box_soup
from .voxelize import voxelize, pack_bits, unpack_bits, tri_box_overlap
from .objects import LsnifObject, level_resolutions, make_object
from .rays import (sphere_to_box_rays, pinhole_rays, shadow_rays, diffuse_rays,
                   balanced_rays, ray_array)
from . import configs

__all__ = [
    "streams", "icosphere", "uv_sphere", "displaced_sphere", "torus", "box_soup",
    "voxelize", "pack_bits", "unpack_bits", "tri_box_overlap",
    "LsnifObject", "level_resolutions", "make_object",
    "sphere_to_box_rays", "pinhole_rays", "shadow_rays", "diffuse_rays",
    "balanced_rays", "ray_array", "configs",
]
