"""Training batches: rays with reference signals from ray casting the true mesh.

The reference of a training ray is the nearest intersection of the ray with the
object's triangles (the paper takes it from BVH ray casting, Sec. 5.2; here a
brute-force float64 Moeller-Trumbore test over every triangle stands in, which
gives the same nearest hit).  At the hit: the distance t along the ray, the
triangle's unit normal (the mesh's outward orientation), a material index and
an albedo.  The synthetic meshes carry no materials, so each triangle gets one
from the octant of its centroid (x > 0, y > 0: 4 materials, modulo n_mat), and
each material a seeded albedo colour.
"""
import numpy as np

from .meshes import face_normals
from .rng import streams, RAYS


def ray_cast(verts, tris, rays, chunk=2048):
    """Nearest hit of each ray with the triangles in [tmin, tmax]: (hit, t, tri)."""
    v = np.asarray(verts, np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    e1, e2 = b - a, c - a
    n = len(rays)
    hit = np.zeros(n, bool)
    t_best = np.full(n, np.inf)
    tri_best = np.full(n, -1, np.int64)
    for s in range(0, n, chunk):
        r = np.asarray(rays[s:s + chunk], np.float64)
        o, d = r[:, None, 0:3], r[:, None, 3:6]
        tmin, tmax = r[:, 6:7], r[:, 7:8]
        p = np.cross(d, e2[None])
        det = np.sum(e1[None] * p, axis=2)
        ok = np.abs(det) > 1e-14
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tv = o - a[None]
        u = np.sum(tv * p, axis=2) * inv
        q = np.cross(tv, e1[None])
        w = np.sum(d * q, axis=2) * inv
        t = np.sum(e2[None] * q, axis=2) * inv
        good = ok & (u >= 0) & (w >= 0) & (u + w <= 1) & (t >= tmin) & (t <= tmax)
        t = np.where(good, t, np.inf)
        k = np.argmin(t, axis=1)
        tk = t[np.arange(len(r)), k]
        h = np.isfinite(tk)
        hit[s:s + chunk] = h
        t_best[s:s + chunk] = tk
        tri_best[s:s + chunk] = np.where(h, k, -1)
    return hit, t_best, tri_best


def materials_of(verts, tris, n_mat):
    cen = np.asarray(verts, np.float64)[tris].mean(axis=1)
    return ((cen[:, 0] > 0).astype(np.int64) + 2 * (cen[:, 1] > 0).astype(np.int64)) % n_mat


def _cast_part(args):
    return ray_cast(*args)


def ray_cast_parallel(verts, tris, rays, workers):
    """ray_cast over `workers` processes (spawned: they import numpy and this module only)."""
    if workers <= 1 or len(rays) < 8192:
        return ray_cast(verts, tris, rays)
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    parts = np.array_split(np.arange(len(rays)), workers * 4)
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_cast_part, [(verts, tris, rays[p]) for p in parts]))
    return tuple(np.concatenate([r[i] for r in res]) for i in range(3))


def targets(verts, tris, rays, n_mat, seed=0, workers=1):
    """Reference signals of a ray batch as a dict of arrays (hit, t, n, albedo, material)."""
    hit, t, tri = ray_cast_parallel(verts, tris, rays, workers)
    fn, _ = face_normals(np.asarray(verts, np.float64), tris)
    mats = materials_of(verts, tris, n_mat)
    colours = np.random.default_rng(seed).uniform(0.05, 0.95, size=(n_mat, 3))
    k = np.where(hit, tri, 0)
    n = np.where(hit[:, None], fn[k], 0.0)
    m = np.where(hit, mats[k], 0)
    return {"hit": hit.astype(np.uint32), "t": np.where(hit, t, 0.0).astype(np.float32),
            "n": n.astype(np.float32), "albedo": np.where(hit[:, None], colours[m], 0.0).astype(np.float32),
            "material": m.astype(np.int32)}


def batch(mesh, obj, n_rays, seed=0, workers=1):
    """A training batch for ``obj`` (built from ``mesh`` = (verts, tris)): the balanced rays of
    Sec. 5.2 and their reference signals."""
    from .rays import balanced_rays
    verts, tris = mesh
    rays = balanced_rays(streams(seed)[RAYS], verts, tris, n_rays, obj.bmin, obj.bmax)
    return rays, targets(verts, tris, rays, obj.n_mat, seed, workers)
