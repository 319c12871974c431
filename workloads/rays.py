"""Ray batches.

A batch is a float32 array of shape (n, 8): origin (3), direction (3), tmin,
tmax, matching the 32-byte ``lsnif_ray`` record.  Directions are unit length.
"""

import numpy as np

from .meshes import face_normals


def ray_array(o, d, tmin=0.0, tmax=np.inf):
    n = len(o)
    r = np.empty((n, 8), dtype=np.float32)
    r[:, 0:3] = o
    r[:, 3:6] = d
    r[:, 6] = tmin
    r[:, 7] = tmax
    return r


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def sphere_to_box_rays(rng, n, radius=2.0, half_box=1.0):
    """Origins uniform on a sphere (normalised Gaussians), aimed at a uniform point of a cube."""
    o = _normalize(rng.standard_normal((n, 3))) * radius
    target = rng.uniform(-half_box, half_box, size=(n, 3))
    return ray_array(o, _normalize(target - o))


def pinhole_rays(width, height, eye, look_at, up, vfov_deg):
    """One primary ray per pixel centre, row-major from the top-left pixel."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = _normalize(np.asarray(look_at, dtype=np.float64) - eye)
    right = _normalize(np.cross(fwd, np.asarray(up, dtype=np.float64)))
    upv = np.cross(right, fwd)
    th = np.tan(np.radians(vfov_deg) / 2.0)
    aspect = width / height
    j, i = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    sx = ((i + 0.5) / width * 2.0 - 1.0) * th * aspect
    sy = (1.0 - (j + 0.5) / height * 2.0) * th
    d = fwd[None] + sx.reshape(-1, 1) * right[None] + sy.reshape(-1, 1) * upv[None]
    return ray_array(np.broadcast_to(eye, d.shape), _normalize(d))


def surface_points(rng, verts, tris, n):
    """Area-uniform points on a mesh with their outward face normals."""
    nrm, area = face_normals(verts, tris)
    cdf = np.cumsum(area)
    t = np.searchsorted(cdf, rng.uniform(0.0, cdf[-1], n), side="right")
    t = np.minimum(t, len(tris) - 1)
    u1, u2 = rng.uniform(size=n), rng.uniform(size=n)
    s = np.sqrt(u1)
    b0, b1, b2 = 1.0 - s, s * (1.0 - u2), s * u2
    v = verts[tris[t]]
    p = b0[:, None] * v[:, 0] + b1[:, None] * v[:, 1] + b2[:, None] * v[:, 2]
    return p, nrm[t]


def _cosine_about(rng, nrm):
    """Cosine-weighted hemisphere directions about unit normals (Malley's method)."""
    n = len(nrm)
    u1, u2 = rng.uniform(size=n), rng.uniform(size=n)
    r, phi = np.sqrt(u1), 2.0 * np.pi * u2
    local = np.stack([r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))], 1)
    helper = np.where(np.abs(nrm[:, :1]) > 0.9, [[0.0, 1.0, 0.0]], [[1.0, 0.0, 0.0]])
    t = _normalize(np.cross(helper, nrm))
    b = np.cross(nrm, t)
    return _normalize(local[:, :1] * t + local[:, 1:2] * b + local[:, 2:3] * nrm)


def shadow_rays(rng, verts, tris, n, light, eps=1e-4):
    """From area-uniform surface points (offset eps along the normal) toward a point light.

    ``tmax`` is the distance to the light, so an occluder beyond it does not count.
    """
    p, nrm = surface_points(rng, verts, tris, n)
    o = p + eps * nrm
    to = np.asarray(light, dtype=np.float64)[None] - o
    dist = np.linalg.norm(to, axis=1)
    return ray_array(o, to / dist[:, None], 0.0, dist)


def diffuse_rays(rng, verts, tris, n, eps=1e-4):
    """Cosine-distributed bounce rays leaving area-uniform surface points."""
    p, nrm = surface_points(rng, verts, tris, n)
    return ray_array(p + eps * nrm, _cosine_about(rng, nrm))


def balanced_rays(rng, verts, tris, n, bmin, bmax, eps=1e-4):
    """Half from the AABB's bounding sphere toward its centre, half from the surface.

    The outside half samples origins uniformly on the bounding sphere and
    directions cosine-weighted about the inward normal; the surface half leaves
    area-uniform surface points with cosine-weighted directions about the face
    normal (the balanced sampling of paper Sec. 5.2, with surface points taken
    directly from the mesh rather than from a first ray cast).
    """
    bmin = np.asarray(bmin, dtype=np.float64)
    bmax = np.asarray(bmax, dtype=np.float64)
    c = 0.5 * (bmin + bmax)
    rad = 0.5 * np.linalg.norm(bmax - bmin)
    n_out = n // 2
    u = _normalize(rng.standard_normal((n_out, 3)))
    o_out = c + rad * u
    d_out = _cosine_about(rng, -u)
    inside = diffuse_rays(rng, verts, tris, n - n_out, eps)
    out = ray_array(o_out, d_out)
    return np.concatenate([out, inside])
