"""Brute-force definitions used to pin the oracle (test helpers, numpy only).

``voxel_list`` slab-tests every voxel of the grid on its own, with the
per-axis plane function t = (k - o) / d (as a float32 product with the
reciprocal) and no walk at all, then sorts the survivors by entry parameter.
It is an independent route to the voxel list that the walk must reproduce.
"""

import numpy as np

f32 = np.float32


def to_voxel_space(ray, bmin, bmax, V):
    s = (f32(V) / (bmax.astype(f32) - bmin.astype(f32))).astype(f32)
    o = ((ray[0:3].astype(f32) - bmin.astype(f32)) * s).astype(f32)
    d = (ray[3:6].astype(f32) * s).astype(f32)
    return o, d


def voxel_list(ray, occ_bool, V, bmin, bmax, H):
    """Every occupied voxel with a positive-length overlap of [ta, tb], in entry order."""
    ray = np.asarray(ray, dtype=f32)
    if np.any(np.isnan(ray)) or np.any(np.isinf(ray[:6])) or not np.any(ray[3:6] != 0) \
            or ray[6] > ray[7]:
        return None
    o, d = to_voxel_space(ray, np.asarray(bmin), np.asarray(bmax), V)
    with np.errstate(divide="ignore", over="ignore"):
        inv = (f32(1.0) / d).astype(f32)
    moving = (d != 0) & np.isfinite(inv)
    if not moving.any():
        return None
    k = np.arange(V + 1, dtype=f32)
    planes = [((k - o[a]) * inv[a]).astype(f32) if moving[a] else None for a in range(3)]
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if moving[a]:
            lo, hi = planes[a][0], planes[a][V]
            t0 = max(t0, min(lo, hi))
            t1 = min(t1, max(lo, hi))
        elif not (0 <= o[a] <= V):
            return {"ta": None, "tb": None, "vox": []}
    ta, tb = f32(max(t0, ray[6])), f32(t1)
    if not ta < tb:
        return {"ta": ta, "tb": tb, "vox": []}
    idx = np.arange(V)
    ent, ext = [], []
    cells = []
    for a in range(3):
        if moving[a]:
            p = planes[a]
            en = np.where(d[a] > 0, p[idx], p[idx + 1])
            ex = np.where(d[a] > 0, p[idx + 1], p[idx])
            ent.append(en)
            ext.append(ex)
            cells.append(idx)
        else:
            c = min(int(np.floor(o[a])), V - 1)
            ent.append(np.array([-np.inf], dtype=f32))
            ext.append(np.array([np.inf], dtype=f32))
            cells.append(np.array([c]))
    X, Y, Z = np.meshgrid(np.arange(len(cells[0])), np.arange(len(cells[1])),
                          np.arange(len(cells[2])), indexing="ij")
    E = np.stack([ent[0][X], ent[1][Y], ent[2][Z]], -1)
    Q = np.stack([ext[0][X], ext[1][Y], ext[2][Z]], -1)
    in_axis = E.argmax(-1)          # first maximum: lowest axis on ties
    out_axis = Q.argmin(-1)
    # the value comes from that axis (this fixes the sign of a zero on ties)
    tin = np.take_along_axis(E, in_axis[..., None], -1)[..., 0]
    tout = np.take_along_axis(Q, out_axis[..., None], -1)[..., 0]
    cx, cy, cz = cells[0][X], cells[1][Y], cells[2][Z]
    occ = occ_bool[cx + V * (cy + V * cz)]
    keep = occ & (np.minimum(tout, tb) > np.maximum(tin, ta))
    sel = np.nonzero(keep.ravel())[0]
    order = np.argsort(tin.ravel()[sel], kind="stable")
    sel = sel[order][: H // 2]
    vox = [((int(cx.ravel()[s]), int(cy.ravel()[s]), int(cz.ravel()[s])), f32(tin.ravel()[s]),
            f32(tout.ravel()[s]), int(in_axis.ravel()[s]), int(out_axis.ravel()[s])) for s in sel]
    return {"ta": ta, "tb": tb, "vox": vox, "o": o, "d": d}


def recheck_sets(ray, occ_bool, V, bmin, bmax):
    """For the float64 grazing recheck: the occupied voxels that must be listed (float32
    overlap of positive length, not grazing) and those that may be listed (those, plus
    grazing voxels whose float64 overlap has positive length).  Every voxel of the grid is
    tested on its own, in float32 with the plane function and in float64 with divisions."""
    ray = np.asarray(ray, dtype=f32)
    o, d = to_voxel_space(ray, np.asarray(bmin), np.asarray(bmax), V)
    with np.errstate(divide="ignore", over="ignore"):
        inv = (f32(1.0) / d).astype(f32)
    moving = (d != 0) & np.isfinite(inv)
    k32 = np.arange(V + 1, dtype=f32)
    k64 = np.arange(V + 1, dtype=np.float64)
    t0, t1, g0, g1 = -np.inf, np.inf, -np.inf, np.inf
    E32, X32, E64, X64 = [], [], [], []
    for a in range(3):
        if moving[a]:
            p32 = ((k32 - o[a]) * inv[a]).astype(f32)
            p64 = (k64 - np.float64(o[a])) / np.float64(d[a])
            t0, t1 = max(t0, min(p32[0], p32[V])), min(t1, max(p32[0], p32[V]))
            g0, g1 = max(g0, min(p64[0], p64[V])), min(g1, max(p64[0], p64[V]))
            lo32, hi32 = np.minimum(p32[:-1], p32[1:]), np.maximum(p32[:-1], p32[1:])
            lo64, hi64 = np.minimum(p64[:-1], p64[1:]), np.maximum(p64[:-1], p64[1:])
        else:
            c = min(int(np.floor(o[a])), V - 1)
            inside = np.arange(V) == c
            lo32 = np.where(inside, -np.inf, np.inf).astype(f32)
            hi32 = np.where(inside, np.inf, -np.inf).astype(f32)
            lo64, hi64 = lo32.astype(np.float64), hi32.astype(np.float64)
        E32.append(lo32); X32.append(hi32); E64.append(lo64); X64.append(hi64)
    ta, tb = f32(max(t0, ray[6])), f32(t1)
    ta64, tb64 = max(g0, np.float64(ray[6])), g1
    X, Y, Z = np.meshgrid(np.arange(V), np.arange(V), np.arange(V), indexing="ij")
    tin = np.maximum(np.maximum(E32[0][X], E32[1][Y]), E32[2][Z]).astype(f32)
    tout = np.minimum(np.minimum(X32[0][X], X32[1][Y]), X32[2][Z]).astype(f32)
    lo, hi = np.maximum(tin, ta), np.minimum(tout, tb)
    q = f32(2.0 ** -16)
    with np.errstate(invalid="ignore", over="ignore"):
        flag = ((hi - lo).astype(f32) <= q * np.maximum(f32(1), np.abs(tin))) | \
               (f32(tb - ta) <= q * max(f32(1), abs(ta)))
    in64 = np.maximum(np.maximum(E64[0][X], E64[1][Y]), E64[2][Z])
    out64 = np.minimum(np.minimum(X64[0][X], X64[1][Y]), X64[2][Z])
    pos64 = np.minimum(out64, tb64) > np.maximum(in64, ta64)
    occ = occ_bool[X + V * (Y + V * Z)]
    # a voxel with a positive float32 overlap is visited by the walk: listed when it is not
    # grazing, or when it is and its float64 overlap is positive too; a grazing voxel the
    # float32 test gives no length may be visited (ties) and is then listed iff float64 says so
    must = occ & (hi > lo) & (~flag | pos64)
    may = must | (occ & flag & pos64)
    cell = lambda m: {(int(x), int(y), int(z)) for x, y, z in zip(X[m], Y[m], Z[m])}
    return {"ta": ta, "tb": tb, "must": cell(must), "may": cell(may), "must_grazing": cell(must & flag),
            "cand": bool(ta < tb)}
