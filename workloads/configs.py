"""The named workloads.

* ``c1``: plain FP32, one icosphere object (1280 triangles), 4096 rays.
* ``c2``: 200k-triangle noise-displaced sphere at V = 128, 16 levels of 2**19
  entries, 1024 x 1024 pinhole primary rays plus 1M shadow rays.
* ``c3``: c2's object and weights, 4M cosine-distributed bounce rays.
* ``p1``: the paper's default object shape (Sec. 5.1) on c1's icosphere: V = 32,
  two face-aligned levels (R = 64, 128) of 2**17 entries x 3 features, a
  2 x 128 leaky-ReLU MLP with the albedo head and 4 materials, H = 18; and its
  low-quality variant (width 64, H = 10); 1M rays from the enclosing sphere.

The paper's own scenes are not available; these procedural objects and ray
distributions stand in for them (primary, shadow and diffuse-bounce rays,
paper Sec. 4 and 6).
"""

import hashlib
import os

import numpy as np

from .meshes import icosphere, displaced_sphere
from .objects import make_object, level_resolutions, LEAKY_RELU
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


def paper_object(seed=0, width=128, H=18):
    """The paper's default object shape (width 128, H = 18) or its low-quality variant
    (width 64, H = 10), with seeded features and weights on c1's icosphere."""
    verts, tris = icosphere(3)
    return make_object(verts, tris, V=32, bmin=[-1.1] * 3, bmax=[1.1] * 3, L=2, F=3, log2_T=17,
                       R=[64, 128], H=H, n_hidden=2, width=width, n_mat=4, has_albedo=1,
                       act=LEAKY_RELU, leaky_slope=0.01, seed=seed,
                       name=f"p1-icosphere-w{width}-h{H}")


def p1_rays(seed=0, n_rays=1 << 20):
    return sphere_to_box_rays(streams(seed)[RAYS], n_rays)


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


# ----------------------------------------------------------------------------- c4
C4_OBJECTS = 64
C4_TOTAL_RAYS = 1 << 24


def c4_ray_counts(n_objects=C4_OBJECTS, total=C4_TOTAL_RAYS, lo=1e3, hi=1e6, seed=4):
    """Per-object ray counts: the mid-quantiles of a power law p(n) ~ n^-beta truncated to
    [lo, hi], beta solved so that the rounded counts sum to `total`; assigned to objects by a
    seeded permutation."""
    from scipy.optimize import brentq

    def counts(beta):
        q = (np.arange(n_objects) + 0.5) / n_objects
        e = 1.0 - beta
        return (lo ** e + q * (hi ** e - lo ** e)) ** (1.0 / e)

    beta = brentq(lambda b: counts(b).sum() - total, 0.05, 0.99)
    c = np.round(counts(beta)).astype(np.int64)
    c[-1] += total - c.sum()
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(n_objects)
    return c[perm], beta


def c4_object_params(i, seed_base=100):
    """Shape, triangle count, V, L and log2_T of c4 object i (seeded per object)."""
    rng = streams(seed_base + i)[GEOMETRY]
    kind = ("torus", "displaced-sphere", "box-soup")[i % 3]
    n_tris = int(round(np.exp(rng.uniform(np.log(1e3), np.log(5e5)))))
    V = int(rng.choice([32, 64, 128, 256]))
    L = int(rng.integers(8, 17))
    log2_T = int(rng.integers(14, 20))
    return kind, n_tris, V, L, log2_T, rng


def c4_mesh(i, seed_base=100):
    from .meshes import torus, box_soup
    kind, n_tris, V, L, log2_T, rng = c4_object_params(i, seed_base)
    if kind == "torus":
        verts, tris = torus(n_tris)
    elif kind == "displaced-sphere":
        stacks = max(int(round((n_tris / 4.0) ** 0.5)), 3)
        verts, tris = displaced_sphere(rng, slices=2 * stacks, stacks=stacks, amplitude=0.1)
    else:
        verts, tris = box_soup(rng, n_tris)
    return verts, tris


def c4_object(i, seed_base=100):
    kind, n_tris, V, L, log2_T, _ = c4_object_params(i, seed_base)
    verts, tris = c4_mesh(i, seed_base)
    s = float(np.abs(verts).max()) * 1.05
    bmin, bmax = [-s] * 3, [s] * 3
    occ = _cached_voxels(f"c4-{seed_base}-{i}-{V}", verts, tris, V, bmin, bmax)
    R = level_resolutions(16, 16 * V, L)
    return make_object(verts, tris, V=V, bmin=bmin, bmax=bmax, L=L, F=2, log2_T=log2_T, R=R,
                       H=18, n_hidden=3, width=64, n_mat=4, seed=seed_base + i,
                       name=f"c4-{i}-{kind}-{len(tris)}tri-V{V}-L{L}-T{log2_T}", occ=occ)


def c4(n_objects=C4_OBJECTS, total=C4_TOTAL_RAYS, scale=1.0, seed_base=100):
    """64 objects with power-law ray counts (16,777,216 pairs at scale 1).

    Rays of object k are in its object space: half from its AABB's bounding sphere toward
    the centre, half leaving its surface (balanced sampling).  ``scale`` shrinks every
    ray count (for tests).  Returns objects, rays (all objects concatenated, object-major)
    and the object index of each ray.
    """
    from .rays import balanced_rays
    counts, beta = c4_ray_counts(n_objects, total)
    counts = np.maximum((counts * scale).astype(np.int64), 1)
    objects, rays, owner = [], [], []
    for i in range(n_objects):
        obj = c4_object(i, seed_base)
        verts, tris = c4_mesh(i, seed_base)
        r = balanced_rays(streams(seed_base + i)[RAYS], verts, tris, int(counts[i]),
                          obj.bmin.astype(np.float64), obj.bmax.astype(np.float64))
        objects.append(obj)
        rays.append(r)
        owner.append(np.full(len(r), i, np.uint32))
    return {"name": "c4", "objects": objects, "rays": np.concatenate(rays),
            "owner": np.concatenate(owner), "counts": counts, "beta": beta}


# ----------------------------------------------------------------------------- c5
def c5_instances(objects, seed=5, spacing=3.0):
    """c4's objects as instances on an 8 x 8 grid with seeded yaw and scale in [0.8, 1.2].

    Returns [(object index, world_to_object 3x4)] and the world-space AABBs."""
    rng = streams(seed)[GEOMETRY]
    insts, boxes = [], []
    n = len(objects)
    side = int(np.ceil(np.sqrt(n)))
    for k, obj in enumerate(objects):
        i, j = k % side, k // side
        c = np.array([spacing * i - spacing * (side - 1) / 2, 0.0, spacing * j - spacing * (side - 1) / 2])
        th = rng.uniform(0, 2 * np.pi)
        s = rng.uniform(0.8, 1.2)
        Rm = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
        A = Rm.T / s                      # world -> object
        b = -A @ c
        insts.append((k, np.concatenate([A, b[:, None]], 1).astype(np.float32)))
        corners = np.array([[x, y, z] for x in obj.bmin[[0]].tolist() + obj.bmax[[0]].tolist()
                            for y in obj.bmin[[1]].tolist() + obj.bmax[[1]].tolist()
                            for z in obj.bmin[[2]].tolist() + obj.bmax[[2]].tolist()], np.float64)
        w = (s * (Rm @ corners.T)).T + c
        boxes.append((w.min(0), w.max(0)))
    return insts, boxes


def ray_box_pairs(rays, boxes, chunk=1 << 17):
    """Brute-force broad phase: every (ray, instance) whose slab interval overlaps
    [tmin, tmax] with positive length; sorted by instance, then ray."""
    lo = np.array([b[0] for b in boxes], np.float32)     # (k, 3)
    hi = np.array([b[1] for b in boxes], np.float32)
    pr, pi = [], []
    for s in range(0, len(rays), chunk):
        r = rays[s:s + chunk]
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            inv = (np.float32(1.0) / r[:, 3:6])
            tn = np.maximum(r[:, 6:7], np.full((len(r), 1), -np.inf, np.float32))
            tn = np.broadcast_to(tn, (len(r), len(boxes))).copy()
            tf = np.broadcast_to(r[:, 7:8], (len(r), len(boxes))).copy()
            for a in range(3):
                t0 = (lo[None, :, a] - r[:, a:a + 1]) * inv[:, a:a + 1]
                t1 = (hi[None, :, a] - r[:, a:a + 1]) * inv[:, a:a + 1]
                np.maximum(tn, np.nan_to_num(np.minimum(t0, t1), nan=-np.inf), out=tn)
                np.minimum(tf, np.nan_to_num(np.maximum(t0, t1), nan=np.inf), out=tf)
        ray_i, inst_i = np.nonzero(tn < tf)
        pr.append(ray_i + s)
        pi.append(inst_i)
    pr, pi = np.concatenate(pr).astype(np.uint32), np.concatenate(pi).astype(np.uint32)
    order = np.lexsort((pr, pi))
    return pr[order], pi[order]


def _instance_surface(rng, meshes, insts, n):
    """World-space area-uniform points on randomly chosen instances, with world normals."""
    from .rays import surface_points
    k = rng.integers(0, len(insts), n)
    P = np.empty((n, 3))
    N = np.empty((n, 3))
    for idx in np.unique(k):
        sel = np.nonzero(k == idx)[0]
        verts, tris = meshes[insts[idx][0]]
        p, nrm = surface_points(rng, verts, tris, len(sel))
        m = insts[idx][1].astype(np.float64)
        A, b = m[:, :3], m[:, 3]
        Ainv = np.linalg.inv(A)
        P[sel] = (p - b) @ Ainv.T
        nw = nrm @ A                                   # normals go with A^T
        N[sel] = nw / np.linalg.norm(nw, axis=1, keepdims=True)
    return P, N


C5_LIGHT = (5.0, 20.0, -5.0)


def c5_pool(objects, n_secondary=3 << 20, side=1024, seed=5):
    """Rays a path tracer over the c5 scene would ask about, in world space.

    Rays [0, side^2) are the primary rays of a pinhole camera in row-major
    pixel order; the rest are secondary: half cosine-weighted bounces leaving
    instance surfaces, half shadow rays from instance surfaces toward a point
    light (tmax = distance)."""
    from .rays import pinhole_rays, ray_array, _cosine_about
    insts, boxes = c5_instances(objects, seed)
    meshes = [c4_mesh(i) for i in range(len(objects))]
    prim = pinhole_rays(side, side, eye=(0.0, 18.0, -22.0), look_at=(0.0, 0.0, 0.0),
                        up=(0.0, 1.0, 0.0), vfov_deg=50.0)
    rng = streams(seed)[RAYS]
    half = n_secondary // 2
    P, N = _instance_surface(rng, meshes, insts, half)
    bounce = ray_array(P + 1e-4 * N, _cosine_about(rng, N))
    P, N = _instance_surface(rng, meshes, insts, n_secondary - half)
    o = P + 1e-4 * N
    to = np.asarray(C5_LIGHT)[None] - o
    dist = np.linalg.norm(to, axis=1)
    shadow = ray_array(o, to / dist[:, None], 0.0, dist)
    sec = np.concatenate([bounce, shadow])
    sec = sec[rng.permutation(len(sec))]
    return {"rays": np.concatenate([prim, sec]), "n_primary": side * side, "insts": insts, "boxes": boxes}


def c5_requests(n_primary, n_total, n_requests=2000, lo=256, hi=1 << 21, seed=6):
    """Request windows of the pool: size log-uniform in [lo, hi], depth uniform in 1..4.
    Depth 1 draws from the primary region, depths 2-4 from the secondary region."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_requests):
        n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        depth = int(rng.integers(1, 5))
        if depth == 1:
            n = min(n, n_primary)
            s = int(rng.integers(0, n_primary - n + 1))
        else:
            n = min(n, n_total - n_primary)
            s = n_primary + int(rng.integers(0, n_total - n_primary - n + 1))
        out.append((s, n, depth))
    return out
