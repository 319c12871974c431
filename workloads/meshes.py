"""Procedural triangle meshes (float64 vertices, int64 triangle indices).

All meshes are wound counter-clockwise seen from outside, so that
``cross(v1 - v0, v2 - v0)`` points outwards.
"""

import numpy as np


def icosphere(subdivisions: int = 3, radius: float = 1.0):
    """Icosahedron split ``subdivisions`` times into 4, midpoints pushed to the sphere.

    Subdivision 3 gives 20 * 4**3 = 1280 triangles.
    """
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdivisions):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        new = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new
    return np.array(verts) * radius, np.array(faces, dtype=np.int64)


def uv_sphere(slices: int, stacks: int):
    """Unit latitude/longitude sphere with poles on +-y.

    ``2 * slices`` cap triangles plus ``2 * slices * (stacks - 2)`` band triangles.
    """
    theta = np.pi * np.arange(1, stacks) / stacks            # polar angle of the rings
    phi = 2.0 * np.pi * np.arange(slices) / slices
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    ring = np.stack([st * np.cos(phi)[None, :], np.broadcast_to(ct, (stacks - 1, slices)),
                     -st * np.sin(phi)[None, :]], axis=-1).reshape(-1, 3)
    verts = np.concatenate([[[0.0, 1.0, 0.0]], ring, [[0.0, -1.0, 0.0]]])
    north, south = 0, len(verts) - 1

    def vid(r, s):
        return 1 + r * slices + (s % slices)

    s = np.arange(slices)
    tris = [np.stack([np.full(slices, north), vid(0, s), vid(0, s + 1)], 1)]
    for r in range(stacks - 2):
        a, b, c, d = vid(r, s), vid(r + 1, s), vid(r + 1, s + 1), vid(r, s + 1)
        tris.append(np.stack([a, b, c], 1))
        tris.append(np.stack([a, c, d], 1))
    last = stacks - 2
    tris.append(np.stack([np.full(slices, south), vid(last, s + 1), vid(last, s)], 1))
    return verts, np.concatenate(tris).astype(np.int64)


def _perlin_permutation(rng):
    p = rng.permutation(256).astype(np.int64)
    return np.concatenate([p, p])


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _grad(h, x, y, z):
    h = h & 15
    u = np.where(h < 8, x, y)
    v = np.where(h < 4, y, np.where((h == 12) | (h == 14), x, z))
    return np.where(h & 1, -u, u) + np.where(h & 2, -v, v)


def perlin3(p, perm):
    """Improved gradient noise (Perlin 2002) at points ``p`` (n, 3)."""
    fl = np.floor(p)
    X, Y, Z = [(fl[:, i].astype(np.int64) & 255) for i in range(3)]
    x, y, z = [p[:, i] - fl[:, i] for i in range(3)]
    u, v, w = _fade(x), _fade(y), _fade(z)
    A = perm[X] + Y
    AA, AB = perm[A] + Z, perm[A + 1] + Z
    B = perm[X + 1] + Y
    BA, BB = perm[B] + Z, perm[B + 1] + Z

    def lerp(t, a, b):
        return a + t * (b - a)

    return lerp(w,
                lerp(v, lerp(u, _grad(perm[AA], x, y, z), _grad(perm[BA], x - 1, y, z)),
                     lerp(u, _grad(perm[AB], x, y - 1, z), _grad(perm[BB], x - 1, y - 1, z))),
                lerp(v, lerp(u, _grad(perm[AA + 1], x, y, z - 1), _grad(perm[BA + 1], x - 1, y, z - 1)),
                     lerp(u, _grad(perm[AB + 1], x, y - 1, z - 1), _grad(perm[BB + 1], x - 1, y - 1, z - 1))))


def displaced_sphere(rng, slices: int = 400, stacks: int = 250, amplitude: float = 0.1,
                     frequency: float = 4.0):
    """UV sphere whose vertices move radially by ``amplitude * noise(frequency * p)``."""
    verts, tris = uv_sphere(slices, stacks)
    perm = _perlin_permutation(rng)
    r = 1.0 + amplitude * perlin3(frequency * verts, perm)
    return verts * r[:, None], tris


def torus(n_tris: int, major: float = 0.7, minor: float = 0.25):
    """Torus around +y with about ``n_tris`` triangles (2 per quad)."""
    quads = max(n_tris // 2, 8)
    nv = max(int(round((quads * minor / major) ** 0.5)), 3)
    nu = max(quads // nv, 3)
    u = 2.0 * np.pi * np.arange(nu) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, Vv = np.meshgrid(u, v, indexing="ij")
    rr = major + minor * np.cos(Vv)
    verts = np.stack([rr * np.cos(U), minor * np.sin(Vv), -rr * np.sin(U)], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = i * nv + j
    b = ((i + 1) % nu) * nv + j
    c = ((i + 1) % nu) * nv + (j + 1) % nv
    d = i * nv + (j + 1) % nv
    tris = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                           np.stack([a, c, d], -1).reshape(-1, 3)])
    return verts, tris.astype(np.int64)


def _box_faces(lo, hi, n):
    """Six faces of an axis-aligned box, each an n x n grid of quads, wound outwards."""
    verts, tris = [], []
    g = np.linspace(0.0, 1.0, n + 1)
    for axis in range(3):
        for side in (0, 1):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            P = np.zeros((n + 1, n + 1, 3))
            P[..., axis] = hi[axis] if side else lo[axis]
            P[..., a1] = lo[a1] + (hi[a1] - lo[a1]) * g[:, None]
            P[..., a2] = lo[a2] + (hi[a2] - lo[a2]) * g[None, :]
            base = sum(len(v) for v in verts)
            verts.append(P.reshape(-1, 3))
            i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
            a = base + i * (n + 1) + j
            b = a + (n + 1)
            c = b + 1
            d = a + 1
            t1, t2 = np.stack([a, b, c], -1), np.stack([a, c, d], -1)
            if not side:
                t1, t2 = t1[..., ::-1], t2[..., ::-1]
            tris += [t1.reshape(-1, 3), t2.reshape(-1, 3)]
    return np.concatenate(verts), np.concatenate(tris)


def box_soup(rng, n_tris: int, n_boxes: int = 6, extent: float = 0.9):
    """Union of random axis-aligned boxes (overlapping, not merged: a polygon soup)."""
    n = max(int(round((n_tris / (12.0 * n_boxes)) ** 0.5)), 1)
    verts, tris, off = [], [], 0
    for _ in range(n_boxes):
        c = rng.uniform(-0.5 * extent, 0.5 * extent, 3)
        h = rng.uniform(0.1, 0.45, 3) * extent
        v, t = _box_faces(c - h, c + h, n)
        verts.append(v)
        tris.append(t + off)
        off += len(v)
    return np.concatenate(verts), np.concatenate(tris).astype(np.int64)


def face_normals(verts, tris):
    """Unit outward face normals and face areas."""
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    ln = np.linalg.norm(n, axis=1)
    return n / np.maximum(ln, 1e-300)[:, None], 0.5 * ln
