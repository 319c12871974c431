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
