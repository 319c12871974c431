"""The named workloads.

* ``c1``: plain FP32, one icosphere object (1280 triangles), 4096 rays.
* ``c2``: 200k-triangle noise-displaced sphere at V = 128, 16 levels of 2**19
  entries, 1024 x 1024 pinhole primary rays plus 1M shadow rays.
* ``c3``: c2's object and weights, 4M cosine-distributed bounce rays.

The paper's own scenes are not available; these procedural objects and ray
distributions stand in for them (primary, shadow and diffuse-bounce rays,
paper Sec. 4 and 6).
"""

import hashlib
import os

import numpy as np

from .meshes import icosphere, displaced_sphere
from .objects import make_object, level_resolutions
from .rays import sphere_to_box_rays, pinhole_rays, shadow_rays, diffuse_rays
from .rng import streams, RAYS, GEOMETRY
from .voxelize import voxelize

_CACHE = os.environ.get("LSNIF_WORKLOAD_CACHE",
                        os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_cache"))


def _cached_voxels(key, verts, tris, V, bmin, bmax):
    """Voxelisation is the slow part of building c2; keep it on disk between runs."""
    h = hashlib.sha1(key.encode() + verts.tobytes() + tris.tobytes()).hexdigest()[:16]
    path = os.path.join(_CACHE, f"occ_{h}.npy")
    if os.path.exists(path):
        return np.load(path)
    occ = voxelize(verts, tris, V, np.asarray(bmin, np.float64), np.asarray(bmax, np.float64))
    try:
        os.makedirs(_CACHE, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npy"
        np.save(tmp, occ)
        os.replace(tmp, path)
    except OSError:
        pass
    return occ


def c1_object(seed=0):
    verts, tris = icosphere(3)
    R = level_resolutions(4, 64, 8)
    return make_object(verts, tris, V=32, bmin=[-1.1] * 3, bmax=[1.1] * 3, L=8, F=2,
                       log2_T=14, R=R, H=18, n_hidden=3, width=64, n_mat=4, seed=seed,
                       name="c1-icosphere")


def c1(seed=0, n_rays=4096):
    obj = c1_object(seed)
    rays = sphere_to_box_rays(streams(seed)[RAYS], n_rays)
    return {"name": "c1", "objects": [obj], "rays": rays}


def c2_mesh(seed=1):
    return displaced_sphere(streams(seed)[GEOMETRY], 400, 250, amplitude=0.1, frequency=4.0)


def c2_object(seed=1):
    verts, tris = c2_mesh(seed)
    V, bmin, bmax = 128, [-1.2] * 3, [1.2] * 3
    occ = _cached_voxels(f"c2-{seed}-{V}", verts, tris, V, bmin, bmax)
    R = level_resolutions(16, 2048, 16)
    return make_object(verts, tris, V=V, bmin=bmin, bmax=bmax, L=16, F=2, log2_T=19, R=R,
                       H=18, n_hidden=3, width=64, n_mat=4, seed=seed, name="c2-displaced-sphere",
                       occ=occ)


C2_LIGHT = (2.0, 3.0, 4.0)


def c2_rays(seed=1, side=1024, n_shadow=1 << 20):
    verts, tris = c2_mesh(seed)
    prim = pinhole_rays(side, side, eye=(0.0, 0.0, 3.0), look_at=(0.0, 0.0, 0.0),
                        up=(0.0, 1.0, 0.0), vfov_deg=50.0)
    shad = shadow_rays(streams(seed)[RAYS], verts, tris, n_shadow, C2_LIGHT)
    return np.concatenate([prim, shad])


def c2(seed=1, side=1024, n_shadow=1 << 20):
    return {"name": "c2", "objects": [c2_object(seed)],
            "rays": c2_rays(seed, side, n_shadow)}


def c3_rays(seed=1, n=1 << 22, ray_seed=3):
    verts, tris = c2_mesh(seed)
    return diffuse_rays(streams(ray_seed)[RAYS], verts, tris, n)


def c3(seed=1, n=1 << 22):
    return {"name": "c3", "objects": [c2_object(seed)], "rays": c3_rays(seed, n)}


def subsample(rays, n, seed=12345):
    """A uniform, seeded subset of a ray batch (kept in original order)."""
    if n >= len(rays):
        return rays
    idx = np.sort(np.random.Generator(np.random.PCG64(seed)).choice(len(rays), n, replace=False))
    return rays[idx]
