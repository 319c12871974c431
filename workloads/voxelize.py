"""Surface voxelisation (the offline asset step of paper Sec. 3.1).

Only the surface polygons are voxelised and nothing is assumed about topology,
so any polygon soup works.  A voxel is occupied when its *closed* box overlaps
a triangle, decided in float64 with the separating-axis test of
Akenine-Moller (2001): three box axes, the triangle normal and the nine
edge-by-axis cross products.  Closed boxes make the result conservative: a
triangle that only touches a voxel face marks both neighbours.

Occupancy is returned as a flat bit array with bit ``x + V*(y + V*z)``,
packed least-significant-bit first into ``uint32`` words.
"""

import numpy as np


def tri_box_overlap(center, half, v0, v1, v2):
    """Vectorised closed triangle/box overlap.

    ``center`` (n, 3), ``half`` (3,) or (n, 3) and triangle vertices (n, 3)
    each, float64.  Returns a bool array (n,).
    """
    half = np.broadcast_to(np.asarray(half, dtype=np.float64), center.shape)
    a0, a1, a2 = v0 - center, v1 - center, v2 - center
    ok = np.ones(len(center), dtype=bool)
    # box face normals: triangle bounding box against the box
    for k in range(3):
        lo = np.minimum(np.minimum(a0[:, k], a1[:, k]), a2[:, k])
        hi = np.maximum(np.maximum(a0[:, k], a1[:, k]), a2[:, k])
        ok &= ~((lo > half[:, k]) | (hi < -half[:, k]))
    edges = (a1 - a0, a2 - a1, a0 - a2)
    # triangle plane
    nrm = np.cross(edges[0], edges[1])
    dist = np.einsum("ij,ij->i", nrm, a0)
    rad = np.einsum("ij,ij->i", np.abs(nrm), half)
    ok &= ~(np.abs(dist) > rad)
    # nine cross-product axes
    for e in edges:
        for k in range(3):
            axis = np.zeros_like(e)
            # unit vector u_k cross e
            k1, k2 = (k + 1) % 3, (k + 2) % 3
            axis[:, k1] = -e[:, k2]
            axis[:, k2] = e[:, k1]
            p0 = np.einsum("ij,ij->i", axis, a0)
            p1 = np.einsum("ij,ij->i", axis, a1)
            p2 = np.einsum("ij,ij->i", axis, a2)
            r = np.einsum("ij,ij->i", np.abs(axis), half)
            lo = np.minimum(np.minimum(p0, p1), p2)
            hi = np.maximum(np.maximum(p0, p1), p2)
            ok &= ~((lo > r) | (hi < -r))
    return ok


def pack_bits(occ_flat):
    """Bool array of length V**3 -> uint32 words, LSB first."""
    n = occ_flat.size
    words = np.zeros((n + 31) // 32, dtype=np.uint32)
    idx = np.nonzero(occ_flat)[0]
    np.bitwise_or.at(words, idx >> 5, (np.uint32(1) << (idx & 31).astype(np.uint32)))
    return words


def unpack_bits(words, n):
    idx = np.arange(n)
    return ((words[idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(bool)


def voxelize(verts, tris, V, bmin, bmax, chunk=200_000):
    """Occupancy of the V**3 closed voxels of the box [bmin, bmax] touched by any triangle.

    Candidates are the voxels whose index range covers the triangle's bounding
    box (widened by a hair so that exact ties are never dropped); each
    candidate is then decided by :func:`tri_box_overlap`.
    Returns packed uint32 words.
    """
    bmin = np.asarray(bmin, dtype=np.float64)
    bmax = np.asarray(bmax, dtype=np.float64)
    vs = (bmax - bmin) / V
    half = 0.5 * vs
    occ = np.zeros(V ** 3, dtype=bool)
    tv = verts[tris]                                  # (n, 3, 3)
    lo = (tv.min(axis=1) - bmin) / vs
    hi = (tv.max(axis=1) - bmin) / vs
    ilo = np.clip(np.ceil(lo - 1e-9).astype(np.int64) - 1, 0, V - 1)
    ihi = np.clip(np.floor(hi + 1e-9).astype(np.int64), 0, V - 1)
    span = ihi - ilo + 1
    span = np.where(np.any((hi < 0) | (lo > V), axis=1)[:, None], 0, span)
    counts = span.prod(axis=1)
    tri_ids = np.repeat(np.arange(len(tris)), counts)
    # enumerate the candidate voxels of each triangle
    starts = np.repeat(np.cumsum(counts) - counts, counts)
    local = np.arange(tri_ids.size) - starts
    for s in range(0, tri_ids.size, chunk):
        t = tri_ids[s:s + chunk]
        q = local[s:s + chunk]
        sx, sy = span[t, 0], span[t, 1]
        kx = ilo[t, 0] + q % sx
        ky = ilo[t, 1] + (q // sx) % sy
        kz = ilo[t, 2] + q // (sx * sy)
        center = bmin + (np.stack([kx, ky, kz], 1) + 0.5) * vs
        hit = tri_box_overlap(center, half, tv[t, 0], tv[t, 1], tv[t, 2])
        occ[(kx + V * (ky + V * kz))[hit]] = True
    return pack_bits(occ)


def voxelize_brute(verts, tris, V, bmin, bmax):
    """Every voxel against every triangle; only for tiny meshes (test pin)."""
    bmin = np.asarray(bmin, dtype=np.float64)
    bmax = np.asarray(bmax, dtype=np.float64)
    vs = (bmax - bmin) / V
    k = np.arange(V ** 3)
    kk = np.stack([k % V, (k // V) % V, k // (V * V)], 1)
    center = bmin + (kk + 0.5) * vs
    occ = np.zeros(V ** 3, dtype=bool)
    for tri in tris:
        v = verts[tri]
        n = len(center)
        occ |= tri_box_overlap(center, 0.5 * vs, np.broadcast_to(v[0], (n, 3)),
                               np.broadcast_to(v[1], (n, 3)), np.broadcast_to(v[2], (n, 3)))
    return pack_bits(occ)
