"""Comparison helpers between the HIP path and the oracle (test helpers).

Tolerances (applied by the GPU tests):

* voxel lists, boundary points, grid slots and interpolation weights: bit-exact.
* float32 path: encoding within 1e-6 of the largest |feature|; raw network
  outputs within ``fp32_logit_bound``; visibility equal on every candidate
  ray whose oracle occlusion logit clears that bound; hit t within 1e-5
  relative (of max(|t|, tb - ta)); normal angle within 1e-4 rad, or within
  its perturbation bound |dn| / |n| for a nearly-zero normal head.
* FP16 / BF16 matrix-core path: visibility agreement >= 99.9 % of candidate
  rays, hit t within 1e-3 relative; normal angle within 1e-2 rad or its
  perturbation bound.
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
        dots = np.clip(np.sum(g["normal"][both].astype(np.float64) * o["normal"][both], 1), -1, 1)
        ang = np.arccos(dots)
        # the direction of a nearly-zero normal head is ill-conditioned: allow the
        # angle its perturbation bound |dn| / |n| where that exceeds the tolerance
        nmag = np.linalg.norm(out_or[both, 2:5], axis=1)
        nerr = np.linalg.norm(ob[both, 2:5], axis=1)
        allowed = np.maximum(n_ang, 4.0 * nerr / np.maximum(nmag, 1e-300))
        stats.update({"t_rel_max": float(terr.max()), "t_rel_p999": float(np.quantile(terr, 0.999)),
                      "normal_ang_max": float(ang.max()),
                      "normal_ang_p999": float(np.quantile(ang, 0.999)),
                      "normal_within_bound": float((ang <= allowed).mean()),
                      "material_agree": float((g["material"][both] == o["material"][both]).mean())})
    else:
        stats.update({"t_rel_max": 0.0, "t_rel_p999": 0.0, "normal_ang_max": 0.0,
                      "normal_ang_p999": 0.0, "normal_within_bound": 1.0, "material_agree": 1.0})
    stats["ok"] = (stats["vis_agree_cand"] >= vis_min and stats["vis_agree_confident"] == 1.0
                   and stats["t_rel_max"] <= t_rel and stats["normal_within_bound"] == 1.0)
    return stats
