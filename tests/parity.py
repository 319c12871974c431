"""Comparison helpers between the HIP path and the oracle (test helpers).

Tolerances (applied by the GPU tests):

* voxel lists, boundary points, grid slots and interpolation weights: bit-exact.
* float32 path: encoding within 1e-6 of the largest |feature|; raw network
  outputs within ``fp32_logit_bound``; visibility equal on every candidate
  ray whose oracle occlusion logit clears that bound; hit t within 1e-5
  relative (of max(|t|, tb - ta)); normal angle within 1e-4 rad on >= 99.99 %
  of hits, and on every hit within 1e-4 rad or its perturbation bound
  |dn| / |n| (a nearly-zero normal head has an ill-conditioned direction).
* FP16 / BF16 matrix-core path: visibility agreement >= 99.9 % of candidate
  rays, hit t within 1e-3 relative; normal angle within 1e-2 rad on >= 99.9 %
  of hits, and on every hit within 1e-2 rad or its perturbation bound.
* Angles are atan2(|a x b|, a . b), exact near zero.
"""

import numpy as np


def gpu_query(L, ctx, oid, rays_np, debug=False, obj=None, stream=None):
    """Run a query through the C ABI; return numpy results (and debug arrays)."""
    import torch
    rays = torch.from_numpy(np.ascontiguousarray(rays_np, np.float32)).cuda()
    n = rays.shape[0]
    out = torch.empty((max(n, 1), 6), dtype=torch.float32, device="cuda")
    res = {}
    if debug:
        H, Lv, F = obj.H, obj.L, obj.F
        od = obj.out_dim
        bufs = {"count": torch.empty(n, dtype=torch.int32, device="cuda"),
                "tatb": torch.empty((n, 2), dtype=torch.float32, device="cuda"),
                "vox_ijk": torch.empty((n, H // 2, 3), dtype=torch.int32, device="cuda"),
                "vox_t": torch.empty((n, H // 2, 2), dtype=torch.float32, device="cuda"),
                "vox_axis": torch.empty((n, H // 2, 2), dtype=torch.int8, device="cuda"),
                "points": torch.empty((n, H, 3), dtype=torch.float32, device="cuda"),
                "slots": torch.empty((n, H, Lv, 8), dtype=torch.int32, device="cuda"),
                "weights": torch.empty((n, H, Lv, 3), dtype=torch.float32, device="cuda"),
                "enc": torch.zeros((n, H * Lv * F), dtype=torch.float32, device="cuda"),
                "out": torch.empty((n, od), dtype=torch.float32, device="cuda")}
        L.lsnif_query_debug(ctx, oid, rays, out, bufs, stream)
        torch.cuda.synchronize()
        for k, v in bufs.items():
            res[k] = v.cpu().numpy()
        res["slots"] = res["slots"].view(np.uint32)
    else:
        L.lsnif_query(ctx, oid, rays, out, stream)
        torch.cuda.synchronize()
    o = out[:n].cpu().numpy()
    res["hit"] = o[:, 0].view(np.uint32).copy()
    res["t"] = o[:, 1].copy()
    res["normal"] = o[:, 2:5].copy()
    res["material"] = o[:, 5].view(np.int32).copy()
    return res


def angle(a, b):
    """Angle in radians between the rows of ``a`` and ``b``, as atan2(|a x b|, a . b) in
    float64: accurate near 0, where arccos of the dot product of two float32 unit
    vectors would report sqrt(2 |1 - |n|^2|) ~ 4e-4 rad for identical vectors.  A zero
    vector against a nonzero one is pi apart; two zero vectors agree."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, 1))
    za, zb = ~np.any(a != 0, 1), ~np.any(b != 0, 1)
    return np.where(za != zb, np.pi, np.where(za & zb, 0.0, ang))


def output_bound(obj, enc_or, u):
    """Forward-error bound of every network output for unit roundoff ``u``, shape (n, outputs).

    Per layer k with n_k inputs, the computed product differs from the exact
    one by at most gamma(n_k) |W_k| |x_k| (plus the rounding of x_k itself
    when activations are stored in a narrow type); propagate |W| |x| through
    the network in float64 and scale by the accumulated relative error.
    """
    x = np.abs(enc_or.T)
    Ws = [np.abs(w.astype(np.float64)) for w in obj.weights]
    rel = 0.0
    for w in Ws:
        n = w.shape[1]
        rel = rel + (n + 2) * u
        x = w @ x
    return (rel * x).T.astype(np.float64)


def logit_bound(obj, enc_or, u):
    return output_bound(obj, enc_or, u)[:, 0]


def compare_hits(g, o, tatb, enc_or, out_or, obj, u, t_rel, n_ang, vis_min):
    """Visibility agreement and hit errors of GPU results ``g`` against oracle ``o``."""
    cand = o["count"] > 0
    ob = output_bound(obj, enc_or, u)
    bound = ob[:, 0]
    z = out_or[:, 0]
    agree = (g["hit"] == o["hit"])
    stats = {"candidates": int(cand.sum()),
             "vis_agree_cand": float(agree[cand].mean()) if cand.any() else 1.0,
             "vis_agree_all": float(agree.mean())}
    confident = cand & (np.abs(z) > bound)
    stats["vis_agree_confident"] = float(agree[confident].mean()) if confident.any() else 1.0
    both = (g["hit"] == 1) & (o["hit"] == 1)
    if both.any():
        scale = np.maximum(np.abs(o["t"][both]), tatb[both, 1] - tatb[both, 0])
        terr = np.abs(g["t"][both].astype(np.float64) - o["t"][both]) / scale
        ang = angle(g["normal"][both], o["normal"][both])
        # the direction of a nearly-zero normal head is ill-conditioned: allow the
        # angle its perturbation bound |dn| / |n| where that exceeds the tolerance
        nmag = np.linalg.norm(out_or[both, 2:5], axis=1)
        nerr = np.linalg.norm(ob[both, 2:5], axis=1)
        allowed = np.maximum(n_ang, 4.0 * nerr / np.maximum(nmag, 1e-300))
        stats.update({"t_rel_max": float(terr.max()), "t_rel_p999": float(np.quantile(terr, 0.999)),
                      "normal_ang_max": float(ang.max()),
                      "normal_ang_p999": float(np.quantile(ang, 0.999)),
                      "normal_within_tol": float((ang <= n_ang).mean()),
                      "normal_within_bound": float((ang <= allowed).mean()),
                      "material_agree": float((g["material"][both] == o["material"][both]).mean())})
    else:
        stats.update({"t_rel_max": 0.0, "t_rel_p999": 0.0, "normal_ang_max": 0.0,
                      "normal_ang_p999": 0.0, "normal_within_tol": 1.0, "normal_within_bound": 1.0,
                      "material_agree": 1.0})
    stats["ok"] = (stats["vis_agree_cand"] >= vis_min and stats["vis_agree_confident"] == 1.0
                   and stats["t_rel_max"] <= t_rel and stats["normal_within_bound"] == 1.0
                   and stats["normal_within_tol"] >= vis_min)
    return stats


def to_object_f32(m, rays):
    """World rays mapped into an instance's object space the way the oracle's pair query
    maps them: x = A x + b and d = A d, each row as ((m0 x + m1 y) + m2 z) + m3 in float32
    (numpy float32 products and sums round once each, with no fused multiply-add).  An
    invalid world ray (a NaN anywhere, an infinite origin or direction, a zero direction,
    tmin > tmax) stays invalid: its mapped origin is NaN."""
    m = np.asarray(m, np.float32).reshape(3, 4)
    r = np.ascontiguousarray(rays, np.float32)
    out = r.copy()
    with np.errstate(invalid="ignore", over="ignore"):
        for a in range(3):
            out[:, a] = ((m[a, 0] * r[:, 0] + m[a, 1] * r[:, 1]) + m[a, 2] * r[:, 2]) + m[a, 3]
            out[:, 3 + a] = (m[a, 0] * r[:, 3] + m[a, 1] * r[:, 4]) + m[a, 2] * r[:, 5]
    valid = (~np.any(np.isnan(r), 1) & np.all(np.isfinite(r[:, :6]), 1) & np.any(r[:, 3:6] != 0, 1)
             & ~(r[:, 6] > r[:, 7]))
    out[~valid, 0] = np.nan
    return out


def pair_reference(oracle, objs, insts, rays, pr, pi, u):
    """The oracle's pairs, one by one: every pair's voxel count, occlusion logit and its
    forward-error bound (unit roundoff ``u``), hit distance over [ta, tb] (also for pairs
    that miss), and normal-head magnitude and bound; plus the nearest hit per ray.

    Each pair is answered by ``oracle.query`` on the ray mapped into its instance's
    object space (``to_object_f32``); the nearest hit over those answers is checked
    against ``oracle.query_pairs`` bit for bit, so the pairs are exactly the ones the
    oracle's own pair query saw."""
    rays = np.ascontiguousarray(rays, np.float32)
    pr = np.asarray(pr, np.int64)
    pi = np.asarray(pi, np.int64)
    n, npairs = len(rays), len(pr)
    P = {"count": np.zeros(npairs, np.int32), "hit": np.zeros(npairs, np.uint32),
         "t": np.full(npairs, np.inf, np.float32), "z": np.zeros(npairs), "zb": np.zeros(npairs),
         "t_any": np.full(npairs, np.inf), "nmag": np.zeros(npairs), "nerr": np.zeros(npairs)}
    for i in np.unique(pi):
        sel = np.nonzero(pi == i)[0]
        k, m = insts[i]
        obj = objs[k]
        o = oracle.query(obj, to_object_f32(m, rays[pr[sel]]), debug=True)
        ob = output_bound(obj, o["enc"], u)
        P["count"][sel], P["hit"][sel], P["t"][sel] = o["count"], o["hit"], o["t"]
        P["z"][sel], P["zb"][sel] = o["out"][:, 0], ob[:, 0]
        ta, tb = o["tatb"][:, 0].astype(np.float64), o["tatb"][:, 1].astype(np.float64)
        P["t_any"][sel] = np.where(o["count"] > 0, ta + (tb - ta) / (1.0 + np.exp(-o["out"][:, 1])), np.inf)
        P["nmag"][sel] = np.linalg.norm(o["out"][:, 2:5], axis=1)
        P["nerr"][sel] = np.linalg.norm(ob[:, 2:5], axis=1)
    # nearest hit per ray, ties to the lowest instance (the oracle's rule)
    order = np.lexsort((pi, P["t"]))
    best = np.full(n, -1, np.int64)
    hits = order[P["hit"][order] == 1]
    first = np.unique(pr[hits], return_index=True)
    best[first[0]] = hits[first[1]]
    ref = oracle.query_pairs(objs, insts, rays, pr.astype(np.uint32), pi.astype(np.uint32))
    won = best >= 0
    assert np.array_equal(won.astype(np.uint32), ref["hit"]), "per-pair answers disagree with query_pairs"
    assert np.array_equal(P["t"][best[won]].view(np.uint32), ref["t"][won].view(np.uint32))
    P.update({"pr": pr, "pi": pi, "best": best, "ref": ref, "n": n})
    return P


def compare_pairs(g, P, t_rel, n_ang, vis_min):
    """Nearest-hit results ``g`` of the HIP pair query against ``pair_reference``.

    * Visibility: agreement over the rays with a candidate pair (a pair whose walk finds
      an occupied voxel) >= ``vis_min``, and 100 % on the rays whose every candidate
      pair's logit clears its bound ("confident").
    * Hit t within ``t_rel`` relative, and the normal within ``n_ang`` rad (or the
      winning pair's perturbation bound), on the rays both sides call hits whose winner
      is clear: every other candidate pair either misses confidently or lies more than
      4 ``t_rel`` behind the winner, so no rounding can change which pair wins.  At
      least a ``vis_min`` fraction of those normals must be within ``n_ang`` itself.
    """
    o, pr, n = P["ref"], P["pr"], P["n"]
    cand_pair = P["count"] > 0
    cand = np.zeros(n, bool)
    np.logical_or.at(cand, pr[cand_pair], True)
    unsure = np.zeros(n, bool)
    np.logical_or.at(unsure, pr[cand_pair & ~(np.abs(P["z"]) > P["zb"])], True)
    conf = cand & ~unsure
    best = P["best"]
    t_win = np.full(n, np.inf)
    t_win[best >= 0] = P["t"][best[best >= 0]]
    is_best = np.zeros(len(pr), bool)
    is_best[best[best >= 0]] = True
    harmless = (P["z"] < -P["zb"]) | (P["t_any"] > t_win[pr] * (1 + 4 * t_rel))
    blocked = np.zeros(n, bool)
    np.logical_or.at(blocked, pr[cand_pair & ~is_best & ~harmless], True)
    agree = g["hit"] == o["hit"]
    st = {"candidate_rays": int(cand.sum()), "candidate_pairs": int(cand_pair.sum()),
          "vis_agree_cand": float(agree[cand].mean()) if cand.any() else 1.0,
          "vis_agree_all": float(agree.mean()),
          "confident_rays": int(conf.sum()),
          "vis_agree_confident": float(agree[conf].mean()) if conf.any() else 1.0}
    both = (g["hit"] == 1) & (o["hit"] == 1) & ~blocked
    if both.any():
        tt = o["t"][both].astype(np.float64)
        terr = np.abs(g["t"][both].astype(np.float64) - tt) / np.maximum(np.abs(tt), 1e-30)
        ang = angle(g["normal"][both], o["normal"][both])
        w = best[both]
        allowed = np.maximum(n_ang, 4.0 * P["nerr"][w] / np.maximum(P["nmag"][w], 1e-300))
        st.update({"t_rel_max": float(terr.max()), "t_rel_p999": float(np.quantile(terr, 0.999)),
                   "normal_ang_max": float(ang.max()),
                   "normal_ang_p999": float(np.quantile(ang, 0.999)),
                   "normal_within_tol": float((ang <= n_ang).mean()),
                   "normal_within_bound": float((ang <= allowed).mean()),
                   "material_agree": float((g["material"][both] == o["material"][both]).mean()),
                   "hits_compared": int(both.sum())})
    else:
        st.update({"t_rel_max": 0.0, "t_rel_p999": 0.0, "normal_ang_max": 0.0, "normal_ang_p999": 0.0,
                   "normal_within_tol": 1.0, "normal_within_bound": 1.0, "material_agree": 1.0,
                   "hits_compared": 0})
    st["ok"] = (st["vis_agree_cand"] >= vis_min and st["vis_agree_confident"] == 1.0
                and st["t_rel_max"] <= t_rel and st["normal_within_bound"] == 1.0
                and st["normal_within_tol"] >= vis_min)
    return st
