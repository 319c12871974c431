"""Throughput of batched LSNIF queries on one MI355X.

Workload: the 200k-triangle noise-displaced sphere (V = 128, 16 levels of
2^19 entries, 2 features, 576 -> 64 -> 64 -> 64 -> 9 MLP) queried with
2,097,152 rays (1024 x 1024 pinhole primary rays and 1M shadow rays).  One
step is one query of the whole batch, inputs resident in HBM.  The headline
path stores features in FP16 and runs the MLP on the matrix cores (FP16
operands, FP32 accumulation); the plain FP32 path (vector ALU) is timed
beside it.

Prints one JSON line: Mrays/s, per-launch p50/p99 latency from HIP events,
the roofline of the query kernel (algorithmic gather bytes per launch over
its mean duration, against the 8 TB/s HBM peak), and the CPU oracle timed on
a bounded sample of the same rays.
"""

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_FP16_PEAK_TFLOPS = 2500.0
MFMA_FP32_PEAK_TFLOPS = 157.3
KERNEL = "k_query_mma<_Float16, _Float16, F=2, WIDTH=64, KBM=2, PAIRS=false, HOT=false>"


KERNEL_SOURCES = ("lsnif_device.hpp", "lsnif_kernels.hpp", "lsnif_launch.hpp", "k_mma_f16.hip",
                  "lsnif_host.hip")


def kernel_source_hash():
    """Hash of the sources that fix the timed kernel's code and its data layout in HBM."""
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_21627_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def tuning_key(t):
    """A tuning as the comma list that `--tuning` takes."""
    return ",".join(str(int(t[k])) for k in ("sort_bits", "pair_bits", "hot_lds_bytes", "walk_chunks", "persistent"))


def kernel_label(tuning):
    """The timed query kernel: the persistent grid is a kernel of its own."""
    return KERNEL.replace("k_query_mma<", "k_query_mma_persist<") if tuning.get("persistent") else KERNEL


def stored_traffic(workload, tuning):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it was taken with
    the same tuning at the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload, {}).get(tuning_key(tuning))
    if not rec or rec.get("src_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_calls(L, ctx, call, steps, warmup):
    """Time `call(stream)` on torch's current stream: wall clock over `steps` calls, per-call
    HIP event latency, and the library's own per-query sort (or pair preparation), walk-kernel
    and query-kernel times."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        call(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    L.lsnif_profile_read(ctx)
    L.lsnif_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        call(stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.lsnif_profile_enable(ctx, False)
    sort_ms, walk_ms, kern_ms, k = L.lsnif_profile_read(ctx)
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    per = lambda x: x / k if k else None
    return wall, lat, per(sort_ms), per(walk_ms), per(kern_ms)


def time_path(L, ctx, oid, rays, out, steps, warmup):
    return time_calls(L, ctx, lambda s: L.lsnif_query(ctx, oid, rays, out, s), steps, warmup)


def point_counts(L, ctx, oid, rays, out, H, chunk=1 << 19):
    """Boundary points of one launch: (all points, fresh points, candidate rays).

    All points are every ray's 2 x voxels (the unit of the per-point byte count).  A
    voxel's entry point that equals the previous voxel's exit point bit for bit, on the
    same face axis, is the same point with the same features; the query kernel reuses
    them and gathers nothing for it.  Fresh points are the others: the points whose
    features must be fetched.  Counted from the debug query's voxel axes and points."""
    import torch
    n = rays.shape[0]
    allp = fresh = cand = 0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        m = b - a
        cnt = torch.empty(m, dtype=torch.int32, device="cuda")
        axis = torch.empty((m, H // 2, 2), dtype=torch.int8, device="cuda")
        pts = torch.empty((m, H, 3), dtype=torch.float32, device="cuda")
        L.lsnif_query_debug(ctx, oid, rays[a:b], out[a:b], {"count": cnt, "vox_axis": axis, "points": pts})
        torch.cuda.synchronize()
        c = cnt.clamp(min=0)
        pb = pts.view(torch.int32)
        same = (pb[:, 2::2] == pb[:, 1:-1:2]).all(-1) & (axis[:, 1:, 0] == axis[:, :-1, 1])
        j = torch.arange(1, H // 2, device="cuda")
        dup = same & (2 * j[None, :] < c[:, None])
        allp += int(c.sum().item())
        fresh += int(c.sum().item()) - int(dup.sum().item())
        cand += int((c > 0).sum().item())
        del cnt, axis, pts
    return allp, fresh, cand


def cpu_baseline(obj, rays_np, sample):
    import oracle
    import workloads as W
    sub = W.configs.subsample(rays_np, sample, seed=2024)
    oracle.query(obj, sub[:1024])          # load and warm the library
    t0 = time.perf_counter()
    oracle.query(obj, sub)
    dt = time.perf_counter() - t0
    return {"value": len(sub) / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{len(sub)} of the {len(rays_np)} rays (uniform, seed 2024), "
                      f"float32 walk + float64 encoding/MLP, OpenMP, {dt:.2f} s wall"}


def mlp_flops(obj, points, cand):
    """Algorithmic MLP FLOPs of a launch: the input layer over each ray's own points only
    (the zero-filled rest of the input vector contributes nothing), the other layers once
    per candidate ray."""
    w0 = obj.weights[0]
    per_point = w0.shape[0] * obj.L * obj.F          # one point's L x F inputs into the first layer
    rest = sum(w.shape[0] * w.shape[1] for w in obj.weights[1:])
    return 2.0 * (per_point * points + rest * cand)


def bytes_per_point(obj, feat_bytes=2):
    """Algorithmic gather bytes of one boundary point: 4 corners on levels aligned with the
    voxel faces, 8 elsewhere, F features each."""
    return sum(4 if int(R) % obj.V == 0 else 8 for R in obj.R) * obj.F * feat_bytes


def bench_c4(L, steps, warmup, tune=True):
    """64 objects, 16,777,216 (ray, object) pairs with power-law counts, one pair query per step
    (identity instances), timed as direct calls and as replays of a captured graph."""
    import torch
    import workloads as W
    print("[bench] generating the c4 workload (64 objects, 16M pairs)", file=sys.stderr, flush=True)
    d = W.configs.c4()
    objs, rays_np, owner, counts = d["objects"], d["rays"], d["owner"], d["counts"]
    n = len(rays_np)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        eye = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
        inst = torch.from_numpy(L.instances_array([(i, eye) for i in ids])).cuda()
        rays = torch.from_numpy(rays_np).cuda()
        pr = torch.arange(n, dtype=torch.int32, device="cuda")
        pi = torch.from_numpy(owner.astype(np.int32)).cuda()
        out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        tuning = L.lsnif_autotune_pairs(ctx, rays, pr, pi, inst, out) if tune else L.lsnif_get_tuning(ctx, ids[0])
        print(f"[bench] timing c4 direct ({tuning}): {warmup} warmup + {steps} steps", file=sys.stderr, flush=True)
        wall_d, lat_d, prep_ms, walk_ms, kern_ms = time_calls(
            L, ctx, lambda st: L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out, st), steps, warmup)
        g = L.lsnif_graph_pairs(ctx, rays, pr, pi, inst, out)
        try:
            print(f"[bench] timing c4 graph replays", file=sys.stderr, flush=True)
            wall_g, lat_g, _, _, _ = time_calls(L, ctx, lambda st: L.lsnif_graph_launch(g, st), steps, warmup)
        finally:
            L.lsnif_graph_destroy(g)
        # algorithmic gather bytes: the fresh boundary points of each object's rays
        m = int(counts.max())
        tmp = torch.empty((m, 6), dtype=torch.float32, device="cuda")
        alg, all_b, pts, fresh, cand, flops, off = 0, 0, 0, 0, 0, 0.0, 0
        for k, o in enumerate(objs):
            c = int(counts[k])
            p, f, cd = point_counts(L, ctx, ids[k], rays[off:off + c], tmp[:c], o.H)
            alg += f * bytes_per_point(o)
            all_b += p * bytes_per_point(o)
            pts += p
            fresh += f
            cand += cd
            flops += mlp_flops(o, p, cd)
            off += c
    finally:
        L.lsnif_destroy(ctx)
    val = lambda wall: n / (wall / steps) / 1e6
    return {
        "workload": "c4: 64 objects (tori, displaced spheres, box soups; 1k-500k triangles; V 32-256; "
                    "8-16 levels x 2^14-2^19 entries x 2 fp16 features; MLP 3x64 fp16), 16,777,216 "
                    "(ray, object) pairs, power-law counts 1,189-977,190 per object, one pair query",
        "pairs": n, "objects": len(objs), "tuning": tuning,
        "launches": steps,
        "direct": {"value": val(wall_d), "unit": "Mpairs/s", "ms_per_step": wall_d * 1e3 / steps,
                   "p50_ms": float(np.percentile(lat_d, 50)), "p99_ms": float(np.percentile(lat_d, 99)),
                   "prepare_ms": prep_ms, "walk_ms": walk_ms, "kernel_ms": kern_ms},
        "graph": {"value": val(wall_g), "unit": "Mpairs/s", "ms_per_step": wall_g * 1e3 / steps,
                  "p50_ms": float(np.percentile(lat_g, 50)), "p99_ms": float(np.percentile(lat_g, 99))},
        "roofline": {"bound": "hbm", "alg_bytes_per_launch": alg, "fresh_points_per_launch": fresh,
                     "achieved": alg / (kern_ms * 1e-3) / 1e9 if kern_ms else None, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if kern_ms else None,
                     "points_per_launch": pts, "all_points_bytes_per_launch": all_b,
                     "frac_all_points": all_b / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if kern_ms else None,
                     "candidate_pairs": cand, "mlp_flops_per_launch": flops,
                     "mfma_frac": flops / (kern_ms * 1e-3) / 1e12 / MFMA_FP16_PEAK_TFLOPS if kern_ms else None},
    }


def bench_c5(L, n_requests, seed=7):
    """Serving: requests from a path tracer over c4's 64 objects as 8 x 8 instances (primary
    tiles, diffuse bounces, shadow rays), sizes log-uniform in [256, 2M] rays.  First every
    request is submitted at once (closed loop: the sustained rate); then requests arrive as a
    Poisson process at 0.7x that rate, and p50/p99 are taken from submit to completion."""
    import torch
    import workloads as W
    from paper_2504_21627_amd.serving import RequestSet
    print("[bench] generating the c5 scene and ray pool", file=sys.stderr, flush=True)
    objs = [W.configs.c4_object(i) for i in range(64)]
    pool = W.configs.c5_pool(objs)
    rays = pool["rays"]
    windows = W.configs.c5_requests(pool["n_primary"], len(rays), n_requests=n_requests)
    total = sum(n for _, n, _ in windows)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        insts = [(ids[k], m) for k, m in pool["insts"]]
        # the broad phase of the whole pool on the device; its pairs feed the requests
        print("[bench] device broad phase of the c5 pool", file=sys.stderr, flush=True)
        rays_d = torch.from_numpy(rays).cuda()
        inst_d = torch.from_numpy(L.instances_array(insts)).cuda()
        cap = 2 * len(rays)
        while True:
            pr_d = torch.empty(cap, dtype=torch.int32, device="cuda")
            pi_d = torch.empty(cap, dtype=torch.int32, device="cuda")
            try:
                n_pairs = L.lsnif_broad_phase(ctx, rays_d, inst_d, pr_d, pi_d)
                break
            except L.LsnifError as e:
                if e.status != L.LSNIF_E_NOMEM:
                    raise
                cap = L.lsnif_last_pair_count
        bp_ms = []
        for _ in range(6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.lsnif_broad_phase(ctx, rays_d, inst_d, pr_d, pi_d)
            torch.cuda.synchronize()
            bp_ms.append((time.perf_counter() - t0) * 1e3)
        pr, pi = pr_d[:n_pairs].cpu().numpy(), pi_d[:n_pairs].cpu().numpy()
        # the whole pool as one scene query (broad phase + pair query)
        out_d = torch.empty((len(rays), 6), dtype=torch.float32, device="cuda")
        # the pair tuning of every object, timed on the pool's pairs; the scene query, the
        # wavefront loop and the serving loop all run with it
        print("[bench] autotuning the c5 pair query", file=sys.stderr, flush=True)
        tuning = L.lsnif_autotune_pairs(ctx, rays_d, pr_d[:n_pairs], pi_d[:n_pairs], inst_d, out_d)
        sc_ms = []
        for _ in range(6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.lsnif_query_scene(ctx, rays_d, inst_d, out_d)
            torch.cuda.synchronize()
            sc_ms.append((time.perf_counter() - t0) * 1e3)
        # a wavefront path tracer over the same scene: the primary image, then depth - 1 diffuse
        # bounces, each one lsnif_query_scene of the previous hits' bounce rays (lsnif_bounce)
        depth = 4
        prim = rays_d[:pool["n_primary"]]
        nxt = torch.empty((len(prim), 8), dtype=torch.float32, device="cuda")
        par = torch.empty(len(prim), dtype=torch.int32, device="cuda")
        hits = torch.empty((len(prim), 6), dtype=torch.float32, device="cuda")
        bufs = [torch.empty_like(nxt), torch.empty_like(nxt)]

        def trace():
            cur, counts = prim, []
            for b in range(depth):
                m = cur.shape[0]
                counts.append(m)
                if m == 0:
                    break
                L.lsnif_query_scene(ctx, cur, inst_d, hits[:m])
                if b + 1 < depth:
                    k = L.lsnif_bounce(ctx, cur, hits[:m], 17, b + 1, 1e-4, bufs[b % 2], par)
                    cur = bufs[b % 2][:k]
            return counts
        tr_ms = []
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            counts = trace()
            torch.cuda.synchronize()
            tr_ms.append((time.perf_counter() - t0) * 1e3)
        del out_d, pr_d, pi_d, nxt, hits, bufs
        rs = RequestSet(L, rays, pr, pi, insts, windows)
        torch.cuda.synchronize()
        cfg = dict(max_inflight=8, hbm_budget=4 << 30, n_streams=4, merge_rays=1 << 21)

        def run(arrivals):
            L.lsnif_serve_start(ctx, **cfg)
            try:
                t0 = time.perf_counter()
                tickets = []
                for j in range(len(windows)):
                    if arrivals is not None:
                        dt = t0 + arrivals[j] - time.perf_counter()
                        if dt > 0:
                            time.sleep(dt)
                    tickets.append(L.lsnif_serve_submit(ctx, rs.request(j)))
                for t in tickets:
                    if L.lsnif_serve_wait(ctx, t) != L.LSNIF_OK:
                        raise RuntimeError("a serving request failed")
                wall = time.perf_counter() - t0
                st = L.lsnif_serve_stats_get(ctx)
            finally:
                L.lsnif_serve_stop(ctx)
            return wall, st

        print("[bench] c5 warm-up", file=sys.stderr, flush=True)
        for j in range(min(16, len(windows))):
            L.lsnif_query_pairs(ctx, rs.rays_of(j), rs.pr[j], rs.pi[j], rs.inst, rs.outs[j])
        torch.cuda.synchronize()
        print(f"[bench] c5 closed loop: {len(windows)} requests, {total} rays", file=sys.stderr, flush=True)
        wall_c, st_c = run(None)
        sustained = total / wall_c
        lam = 0.7 * sustained / (total / len(windows))          # requests per second
        arrivals = np.cumsum(np.random.Generator(np.random.PCG64(seed)).exponential(1.0 / lam, len(windows)))
        arrivals -= arrivals[0]
        print(f"[bench] c5 Poisson arrivals at {lam:.1f} requests/s", file=sys.stderr, flush=True)
        wall_p, st_p = run(arrivals)
    finally:
        L.lsnif_destroy(ctx)
    return {
        "workload": "c5: c4's 64 objects as 8x8 instances, 1024x1024 primary pool + 3M secondary "
                    f"(diffuse, shadow) rays, {len(windows)} requests of 256-2M rays, depth 1-4, "
                    "fp16, 4 GiB in-flight budget, 8 slots, 4 streams, requests merged up to 8M rays per launch",
        "requests": len(windows), "rays": total, "pairs_per_ray": len(pr) / len(rays), "tuning": tuning,
        "broad_phase": {"where": "device (lsnif_broad_phase)", "pool_rays": len(rays), "pairs": int(n_pairs),
                        "ms": float(np.median(bp_ms[1:])),
                        "mrays_s": len(rays) / float(np.median(bp_ms[1:])) / 1e3},
        "wavefront": {"what": f"1024x1024 primary rays, then {depth - 1} diffuse bounces from the hits: "
                              "one lsnif_query_scene per depth, lsnif_bounce between",
                      "rays_per_depth": counts, "ms": float(np.median(tr_ms[1:])),
                      "value": sum(counts) / float(np.median(tr_ms[1:])) / 1e3, "unit": "Mrays/s"},
        "scene_query": {"what": "the whole pool in one lsnif_query_scene (broad phase + pair query)",
                        "value": len(rays) / float(np.median(sc_ms[1:])) / 1e3, "unit": "Mrays/s",
                        "ms": float(np.median(sc_ms[1:]))},
        "closed_loop": {"value": sustained / 1e6, "unit": "Mrays/s", "wall_s": wall_c,
                        "p50_ms": st_c["p50_ms"], "p99_ms": st_c["p99_ms"],
                        "ws_bytes_peak": st_c["ws_bytes_peak"]},
        "poisson": {"rate_req_s": lam, "offered_mrays_s": 0.7 * sustained / 1e6,
                    "value": total / wall_p / 1e6, "unit": "Mrays/s", "wall_s": wall_p,
                    "p50_ms": st_p["p50_ms"], "p99_ms": st_p["p99_ms"], "max_ms": st_p["max_ms"]},
    }


def bench_small(L, reps=200):
    """Per-call latency of small batches on the c2 object (FP16): a consumer that queries a
    few rays at a time, like an intersection shader calling one LSNIF per ray, against the
    batched path.  Each size is queried `reps` times on one stream; HIP events per call."""
    import torch
    import workloads as W
    obj = W.configs.c2_object()
    rays_all = W.configs.subsample(W.configs.c2_rays(), 1 << 16, seed=77)
    rays = torch.from_numpy(rays_all).cuda()
    out = torch.empty((len(rays_all), 6), dtype=torch.float32, device="cuda")
    ctx = L.lsnif_create(0)
    res = {"workload": "c2's object (FP16), batches of 1..65,536 rays drawn from c2's ray mix"}
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        for n in (1, 32, 256, 4096, 65536):
            wall, lat, _, _, _ = time_calls(L, ctx, lambda st: L.lsnif_query(ctx, oid, rays[:n], out, st), reps, 10)
            res[str(n)] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                           "mrays_s": n * reps / wall / 1e6}
    finally:
        L.lsnif_destroy(ctx)
    return res


def bench_c1(L, reps=200):
    """c1: the plain FP32 path on the icosphere object (8 levels, 2^14 entries, 288-64-64-64-9
    MLP) and its 4,096 rays; latency-bound (16 blocks of 256 rays cannot fill 256 compute
    units), so p50/p99 per launch over `reps` launches and Mrays/s, with the oracle on the
    same 4,096 rays."""
    import torch
    import oracle
    import workloads as W
    c = W.configs.c1()
    obj, rays_np = c["objects"][0], c["rays"]
    n = len(rays_np)
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        wall, lat, _, _, kern_ms = time_path(L, ctx, oid, rays, out, reps, 10)
        # the same query captured once and replayed: the launches leave the host as one graph
        g = L.lsnif_graph_query(ctx, oid, rays, out)
        try:
            wall_g, lat_g, _, _, _ = time_calls(L, ctx, lambda st: L.lsnif_graph_launch(g, st), reps, 10)
        finally:
            L.lsnif_graph_destroy(g)
    finally:
        L.lsnif_destroy(ctx)
    oracle.query(obj, rays_np[:256])
    t0 = time.perf_counter()
    for _ in range(5):
        oracle.query(obj, rays_np)
    dt = (time.perf_counter() - t0) / 5
    return {"workload": "c1: icosphere (1,280 triangles), V=32, 8 levels x 2^14 entries x 2 fp32 features, "
                        "MLP 288-64-64-64-9 fp32, 4,096 rays",
            "path": "fp32 features, fp32 vector-ALU MLP, one wave per ray (k_query_lat)",
            "rays": n, "launches": reps, "value": n * reps / wall / 1e6, "unit": "Mrays/s",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "kernel_ms": kern_ms,
            "graph": {"value": n * reps / wall_g / 1e6, "unit": "Mrays/s", "p50_ms": float(np.percentile(lat_g, 50)),
                      "p99_ms": float(np.percentile(lat_g, 99))},
            "roofline": "not meaningful: 4,096 waves of a few microseconds each (latency-bound)",
            "cpu_baseline": {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
                             "kind": "oracle", "sample": "all 4,096 rays, mean of 5 runs"}}


def bench_c3(L, steps, warmup):
    """c3: c2's object queried with 4,194,304 incoherent diffuse bounce rays in every MLP x
    feature precision (FP32 / BF16 / FP16 / FP8-e4m3 MLP with FP32 accumulation, FP16 / BF16
    features, plus FP32 / FP32).  Per combination: Mrays/s, p50/p99 per launch, the query
    kernel's gather roofline (fresh points x bytes per point over its mean time).  The
    oracle is timed once on a sample (its arithmetic is float64 whatever the GPU's types)."""
    import torch
    import oracle
    import workloads as W
    print("[bench] generating the c3 workload", file=sys.stderr, flush=True)
    obj = W.configs.c2_object()
    rays_np = W.configs.c3_rays()
    n = len(rays_np)
    scales = (oracle.act_amax(obj, rays_np[:65536]) / 448.0).astype(np.float32)
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    res = {"workload": "c3: c2's object, 4,194,304 cosine-weighted diffuse bounce rays from its surface",
           "rays": n, "launches": steps, "fp8_act_scale": [float(x) for x in scales], "combos": {}}
    ctx = L.lsnif_create(0)
    try:
        combos = [("fp32", "fp32")] + [(f, m) for m in ("fp32", "bf16", "fp16", "fp8") for f in ("fp16", "bf16")]
        pts = None
        for feat, mlp in combos:
            oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp, fp8_act_scale=scales if mlp == "fp8" else None))
            tuning = L.lsnif_autotune(ctx, oid, rays, out)
            iso = dict(tuning, walk_chunks=1)
            print(f"[bench] c3 {feat}/{mlp} ({tuning})", file=sys.stderr, flush=True)
            wall, lat, _, _, _ = time_path(L, ctx, oid, rays, out, steps, warmup)
            L.lsnif_set_tuning(ctx, oid, *iso.values())
            _, _, _, _, kern_ms = time_path(L, ctx, oid, rays, out, max(steps // 4, 5), warmup)
            if pts is None:
                pts = point_counts(L, ctx, oid, rays, out, obj.H)
            L.lsnif_release(ctx, oid)
            bpp = bytes_per_point(obj, 4 if feat == "fp32" else 2)
            gbs = pts[1] * bpp / (kern_ms * 1e-3) / 1e9
            res["combos"][f"mlp={mlp} feat={feat}"] = {
                "value": n * steps / wall / 1e6, "unit": "Mrays/s", "tuning": tuning,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "kernel_ms": kern_ms,
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS, "alg_bytes_per_launch": pts[1] * bpp}}
        res["points_per_launch"], res["fresh_points_per_launch"], res["candidate_rays"] = pts
    finally:
        L.lsnif_destroy(ctx)
    sub = W.configs.subsample(rays_np, 1 << 19, seed=2024)
    oracle.query(obj, sub[:1024])
    t0 = time.perf_counter()
    oracle.query(obj, sub)
    dt = time.perf_counter() - t0
    res["cpu_baseline"] = {"value": len(sub) / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
                           "kind": "oracle", "sample": f"{len(sub)} of the {n} rays (uniform, seed 2024), "
                                                       f"float32 walk + float64 encoding/MLP, {dt:.2f} s wall"}
    return res


def bench_p1(L, steps, warmup, tune):
    """The paper's default object shape (width-128 leaky-ReLU MLP, albedo head, F = 3, two
    face-aligned levels) and its low-quality variant (width 64, H = 10), FP16 features and
    MLP, 1M rays from the enclosing sphere."""
    import torch
    import workloads as W
    rays_np = W.configs.p1_rays()
    n = len(rays_np)
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    res = {"workload": "p1: c1's icosphere as the paper's default object shape (V=32, levels R=64,128 "
                       "face-aligned, 2^17 entries x 3 fp16 features, H=18, MLP 108-128-128-12 leaky ReLU, "
                       "albedo head, 4 materials) and its low-quality variant (width 64, H=10); 1,048,576 "
                       "rays from the enclosing sphere", "rays": n, "launches": steps}
    ctx = L.lsnif_create(0)
    try:
        for name, width, H in (("default", 128, 18), ("low_quality", 64, 10)):
            obj = W.configs.paper_object(width=width, H=H)
            oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
            tuning = L.lsnif_autotune(ctx, oid, rays, out) if tune else L.lsnif_get_tuning(ctx, oid)
            print(f"[bench] timing p1 {name} ({tuning}): {warmup} warmup + {steps} steps", file=sys.stderr,
                  flush=True)
            wall, lat, sort_ms, walk_ms, kern_ms = time_path(L, ctx, oid, rays, out, steps, warmup)
            res[name] = {"width": width, "H": H, "value": n / (wall / steps) / 1e6, "unit": "Mrays/s",
                         "ms_per_step": wall * 1e3 / steps, "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "sort_ms": sort_ms, "walk_ms": walk_ms,
                         "kernel_ms": kern_ms, "tuning": tuning}
            L.lsnif_release(ctx, oid)
    finally:
        L.lsnif_destroy(ctx)
    return res


# FLOPs of one training ray on a fully connected network: forward, weight gradients and input
# gradients are one multiply-add per weight each
def train_flops_per_ray(obj):
    return 3 * 2 * sum(int(w.shape[0]) * int(w.shape[1]) for w in obj.weights)


def t1_batch(n=1 << 18, extra=4, held_out=1 << 16):
    """The training batches: generated before the GPU is touched (the ray cast runs in spawned
    worker processes).  The timed batch, `extra` further training batches of n / 4 rays and a
    held-out batch, each from its own ray seed."""
    import workloads as W
    from workloads import train as WT
    obj = W.configs.paper_object(seed=0)
    print(f"[bench] generating the t1 training batches ({n} + {extra} x {n // 4} + {held_out} rays, ray casting)",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    mesh = W.icosphere(3)
    rays_np, tg = WT.batch(mesh, obj, n, seed=31, workers=8)
    more = [WT.batch(mesh, obj, n // 4, seed=32 + i, workers=8) for i in range(extra)]
    test = WT.batch(mesh, obj, held_out, seed=99, workers=8)
    return obj, rays_np, tg, time.perf_counter() - t0, more, test


def t1_quality(L, ctx, oid, tr, obj, batches, test, steps):
    """Train on, cycling over the batches, then score the object on the held-out rays against
    the ray-cast references: visibility, hit distance and normal of the FP32 query, and the
    FP16 query of the trained parameters against the FP32 one."""
    import torch
    dev = [(torch.from_numpy(r).cuda(), torch.from_numpy(L.targets_array(t["hit"], t["t"], t["n"], t["material"],
                                                                          t["albedo"])).cuda()) for r, t in batches]
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for k in range(steps):
        r, t = dev[k % len(dev)]
        L.lsnif_train_step(tr, r, t, loss)
    rays_np, tg = test
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
    L.lsnif_query(ctx, oid, rays, out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    hit = g[:, 0].view(np.uint32) == 1
    ref = tg["hit"] == 1
    both = hit & ref
    t_err = np.abs(g[both, 1] - tg["t"][both]) / np.maximum(np.abs(tg["t"][both]), 1e-6)
    cosang = np.clip(np.sum(g[both, 2:5] * tg["n"][both], axis=1), -1, 1)
    tab, Ws, _, _, n_steps = L.lsnif_trainer_read(tr, obj)
    import dataclasses
    trained = dataclasses.replace(obj, tables=tab, weights=Ws)
    oid16 = L.lsnif_build(ctx, L.ObjectDesc(trained, "fp16", "fp16"))
    out16 = torch.empty_like(out)
    L.lsnif_query(ctx, oid16, rays, out16)
    torch.cuda.synchronize()
    hit16 = out16.cpu().numpy()[:, 0].view(np.uint32) == 1
    L.lsnif_release(ctx, oid16)
    return {"adam_steps": int(n_steps), "held_out_rays": len(rays_np), "reference_hits": int(ref.sum()),
            "visibility_accuracy": float((hit == ref).mean()), "hit_recall": float(both.sum() / max(ref.sum(), 1)),
            "hit_precision": float(both.sum() / max(hit.sum(), 1)),
            "t_rel_err_median": float(np.median(t_err)) if both.any() else None,
            "normal_err_median_rad": float(np.median(np.arccos(cosang))) if both.any() else None,
            "fp16_vs_fp32_visibility": float((hit16 == hit).mean()), "last_batch_loss": float(loss.item())}


def bench_t1(L, steps, warmup, data, cpu=True, quality_steps=400):
    """Training (Sec. 5.2, 5.3): the paper's default object shape with FP32 parameters, one
    batch of 2^18 balanced rays with references from ray casting its mesh, Adam at lr 0.01."""
    import torch
    obj, rays_np, tg, gen_s, more, test = data
    n = len(rays_np)
    res = {"workload": "t1: training the paper's default object shape (c1's icosphere, V=32, levels R=64,128, "
                       "2^17 x 3 fp32 features, H=18, MLP 108-128-128-12 leaky ReLU, albedo head, 4 materials); "
                       "batches of 262,144 balanced rays (half from the enclosing sphere, half from the "
                       "surface) with references from ray casting the mesh; Adam lr 0.01",
           "rays_per_step": n, "reference_hits": int(tg["hit"].sum()), "batch_gen_s": gen_s}
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        tr = L.lsnif_trainer_create(ctx, oid)
        try:
            rays = torch.from_numpy(rays_np).cuda()
            tgt = torch.from_numpy(L.targets_array(tg["hit"], tg["t"], tg["n"], tg["material"],
                                                   tg["albedo"])).cuda()
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            L.lsnif_train_step(tr, rays, tgt, loss)
            torch.cuda.synchronize()
            loss_first = float(loss.item())
            for _ in range(warmup):
                L.lsnif_train_step(tr, rays, tgt, loss)
            print(f"[bench] timing t1: {warmup} warmup + {steps} steps", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                L.lsnif_train_step(tr, rays, tgt, loss)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            flops = train_flops_per_ray(obj) * n
            # the same steps again with the library's phase events: layer products and scatter
            L.lsnif_profile_enable(ctx, True)
            for _ in range(steps):
                L.lsnif_train_step(tr, rays, tgt, loss)
            prod_ms, scat_ms, k = L.lsnif_train_profile_read(tr)
            L.lsnif_profile_enable(ctx, False)
            prod_ms, scat_ms = prod_ms / k, scat_ms / k
            cnt = torch.empty(n, dtype=torch.int32, device="cuda")
            tmp = torch.empty((n, 6), dtype=torch.float32, device="cuda")
            L.lsnif_query_debug(ctx, oid, rays, tmp, {"count": cnt})
            torch.cuda.synchronize()
            points = int(cnt.clamp(min=0).sum().item())
            corners = sum(4 if int(R) % obj.V == 0 else 8 for R in obj.R)
            scat_bytes = points * obj.F * 4 * (obj.L + corners)   # read d loss/d x, add to every corner
            res.update({"value": n / ms / 1e3, "unit": "Mrays/s trained", "ms_per_step": ms,
                        "steps": steps, "warmup": warmup, "gflop_per_step": flops / 1e9,
                        "layer_tflops": flops / ms / 1e9, "loss_step1": loss_first,
                        "loss_last": float(loss.item()), "adam_steps": 2 * steps + warmup + 1,
                        "roofline": {
                            "products": {"bound": "mfma", "achieved": flops / prod_ms / 1e9,
                                         "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                         "frac": flops / prod_ms / 1e9 / MFMA_FP32_PEAK_TFLOPS,
                                         "ms_per_step": prod_ms, "flop_per_step": flops,
                                         "what": "forward and backward layer products (fp32 matrix cores), "
                                                 "with the weight-gradient partial sums"},
                            "scatter": {"bound": "hbm", "achieved": scat_bytes / scat_ms / 1e6,
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": scat_bytes / scat_ms / 1e6 / HBM_PEAK_GBS,
                                        "ms_per_step": scat_ms, "bytes_per_step": scat_bytes,
                                        "points_per_step": points,
                                        "what": "k_train_enc<true>: per boundary point, read its L x F encoding "
                                                "gradients and add F floats to each of its corners "
                                                "(4 on face-aligned levels, 8 elsewhere)"}}})
            if quality_steps:
                print("[bench] t1: training on to score held-out rays", file=sys.stderr, flush=True)
                res["trained"] = t1_quality(L, ctx, oid, tr, obj, [(rays_np, tg)] + list(more), test, quality_steps)
        finally:
            L.lsnif_trainer_destroy(tr)
    finally:
        L.lsnif_destroy(ctx)
    if cpu:
        import oracle
        import oracle.train as OT
        m = 16384
        sub = rays_np[:m]
        tsub = {k: v[:m] for k, v in tg.items()}
        OT.train_grads(obj, sub[:256], {k: v[:256] for k, v in tsub.items()})   # load and warm
        t0 = time.perf_counter()
        g = OT.train_grads(obj, sub, tsub)
        OT.adam(obj.tables, g["gtab"], 0.0, 0.0, 1)
        for k, w in enumerate(obj.weights):
            OT.adam(w, g["gW"][k], 0.0, 0.0, 1)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": m / dt / 1e6, "unit": "Mrays/s trained", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"one step on the first {m} rays of the batch "
                                                           f"(the C query oracle on {oracle.num_threads()} OpenMP "
                                                           f"threads for the walk and encoding, then float64 numpy, "
                                                           f"mostly one thread, for the rest), {dt:.2f} s wall"}
    return res


def bench_c2(L, args):
    """The headline: the c2 batch through the FP16 matrix-core path and the plain FP32 path."""
    import torch
    import workloads as W
    print("[bench] generating the c2 workload", file=sys.stderr, flush=True)
    obj = W.configs.c2_object()
    rays_np = W.configs.c2_rays()
    n = len(rays_np)
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    ctx = L.lsnif_create(0)
    paths = {}
    for name, feat, mlp in (("fp16", "fp16", "fp16"), ("fp32", "fp32", "fp32")):
        if args.only and name != args.only:
            continue
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
        if args.tuning:
            L.lsnif_set_tuning(ctx, oid, *[int(x) for x in args.tuning.split(",")])
        tuning = (L.lsnif_autotune(ctx, oid, rays, out) if not (args.no_tune or args.tuning)
                  else L.lsnif_get_tuning(ctx, oid))
        print(f"[bench] timing the {name} path ({tuning}): {args.warmup} warmup + {args.steps} steps",
              file=sys.stderr, flush=True)
        wall, lat, sort_ms, walk_ms, kern_ms = time_path(L, ctx, oid, rays, out, args.steps, args.warmup)
        iso = tuning
        if tuning["walk_chunks"] > 1:
            # with the walk running ahead on a side stream the kernels overlap; the roofline
            # takes the query kernel alone, from steps that walk the whole batch first
            iso = dict(tuning, walk_chunks=1)
            L.lsnif_set_tuning(ctx, oid, *iso.values())
            print(f"[bench] timing the {name} kernels one after another ({iso})", file=sys.stderr, flush=True)
            _, _, sort_ms, walk_ms, kern_ms = time_path(L, ctx, oid, rays, out, max(args.steps // 4, 5),
                                                        args.warmup)
            L.lsnif_set_tuning(ctx, oid, *tuning.values())
        ub_ms = None
        if name == "fp16":
            # the gather ceiling: the same batch through the kernel that only gathers (SURVEY's
            # ub_gather), with the walk of the whole batch first as for the roofline's kernel time
            L.lsnif_set_tuning(ctx, oid, *iso.values())
            sums = torch.empty(n, dtype=torch.float32, device="cuda")
            _, _, _, _, ub_ms = time_calls(L, ctx, lambda st: L.lsnif_gather_ceiling(ctx, oid, rays, sums, st),
                                           max(args.steps // 4, 5), args.warmup)
            L.lsnif_set_tuning(ctx, oid, *tuning.values())
            del sums
        pts, fresh, cand = point_counts(L, ctx, oid, rays, out, obj.H)
        paths[name] = {"wall": wall, "lat": lat, "points": pts, "fresh": fresh, "cand": cand, "sort_ms": sort_ms,
                       "ub_ms": ub_ms,
                       "walk_ms": walk_ms, "kern_ms": kern_ms, "feat_bytes": 2 if feat == "fp16" else 4,
                       "tuning": tuning, "tuning_isolated": iso}
        L.lsnif_release(ctx, oid)
    L.lsnif_destroy(ctx)

    head = paths.get("fp16") or paths["fp32"]
    ms_per_step = head["wall"] * 1e3 / args.steps
    mean_ms = float(head["kern_ms"])      # query kernel alone, HIP events on its stream
    bpp = bytes_per_point(obj, head["feat_bytes"])
    alg_bytes = head["fresh"] * bpp                # fresh points only: the bytes that must move
    all_bytes = head["points"] * bpp               # every boundary point, repeats included
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    flops = mlp_flops(obj, head["points"], head["cand"])
    rec = {
        "metric": "Mrays/s LSNIF queries (FP16 MFMA vs FP32 plain) + p50/p99 batch latency",
        "value": n / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "p50_ms": float(np.percentile(head["lat"], 50)),
        "p99_ms": float(np.percentile(head["lat"], 99)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp16" if "fp16" in paths else "fp32",
        "tuning": head["tuning"],
        "data": "synthetic",
        "config": {"workload": "c2: 200k-triangle noise-displaced sphere, V=128, 16 levels x 2^19 "
                               "entries x 2 features, MLP 576-64-64-64-9, 1024x1024 pinhole primary "
                               "rays + 1048576 shadow rays",
                   "rays": n, "path": "fp16 features, fp16 MFMA MLP, fp32 accumulation"
                   if "fp16" in paths else "fp32 features, fp32 vector-ALU MLP"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic("c2-fp16", head["tuning_isolated"]) if "fp16" in paths else None,
                     "kernel": kernel_label(head["tuning_isolated"]) if "fp16" in paths else "k_query_f32",
                     "alg_bytes_per_launch": alg_bytes, "fresh_points_per_launch": head["fresh"],
                     "bytes_per_point": bpp, "mean_kernel_ms": mean_ms,
                     "points_per_launch": head["points"], "all_points_bytes_per_launch": all_bytes,
                     "frac_all_points": all_bytes / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "mean_sort_ms": float(head["sort_ms"]), "mean_walk_ms": float(head["walk_ms"]),
                     "tuning": head["tuning_isolated"],
                     "ub_gather_ms": head["ub_ms"],
                     "ub_gather_gbs": alg_bytes / (head["ub_ms"] * 1e-3) / 1e9 if head["ub_ms"] else None,
                     "mlp_flops_per_launch": flops,
                     "frac_of_ub_gather": head["ub_ms"] / mean_ms if head["ub_ms"] else None,
                     "mfma_tflops": flops / (mean_ms * 1e-3) / 1e12,
                     "mfma_frac": flops / (mean_ms * 1e-3) / 1e12 / MFMA_FP16_PEAK_TFLOPS},
    }
    if "fp32" in paths:
        p = paths["fp32"]
        rec["fp32_plain"] = {"value": n / (p["wall"] / args.steps) / 1e6, "unit": "Mrays/s", "tuning": p["tuning"],
                             "p50_ms": float(np.percentile(p["lat"], 50)),
                             "p99_ms": float(np.percentile(p["lat"], 99))}
        if "fp16" in paths:
            rec["fp16_over_fp32"] = rec["value"] / rec["fp32_plain"]["value"]
    return rec, obj, rays_np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--only", choices=["fp16", "fp32"], default=None,
                    help="time one path only (for profiling)")
    ap.add_argument("--legs", default="c2,c4,c5,p1,small,t1,c1,c3",
                    help="comma list: c2 (headline), c4 (batched objects), c5 (serving), "
                         "p1 (the paper's default object shape), small (latency of small batches), "
                         "t1 (training steps), c1 (latency of the small FP32 config), "
                         "c3 (precision sweep on incoherent rays)")
    ap.add_argument("--c5-requests", type=int, default=2000)
    ap.add_argument("--t1-quality-steps", type=int, default=400,
                    help="t1: further training steps before scoring held-out rays (0: skip the scoring)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tuning (no autotuner)")
    ap.add_argument("--tuning", default=None,
                    help="sort_bits,pair_bits,hot_lds_bytes[,walk_chunks] for the c2 object instead of the "
                         "autotuner (profiling runs repeat the tuning the autotuner chose)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first copy a device buffer of this size (MiB): the copy of known size "
                         "against which rocprofv3's FETCH_SIZE/WRITE_SIZE counters are scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library has no multi-GPU "
              "path.", file=sys.stderr)
        sys.exit(2)

    legs = set(args.legs.split(","))
    t1_data = t1_batch() if "t1" in legs else None

    import torch
    import workloads as W
    from paper_2504_21627_amd import lsnif as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_ref_mib:
        src = torch.ones(args.copy_ref_mib << 18, dtype=torch.float32, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    if "c2" in legs:
        rec, obj, rays_np = bench_c2(L, args)
    else:
        rec = {"metric": "Mrays/s LSNIF queries (FP16 MFMA vs FP32 plain) + p50/p99 batch latency",
               "legs": sorted(legs), "note": "headline (c2) leg not run"}
    if "c4" in legs:
        # p50 / p99 over the same number of whole-batch launches as the headline (200 by default)
        rec["batched_c4"] = bench_c4(L, args.steps, min(args.warmup, 3), not args.no_tune)
    if "c5" in legs:
        rec["serving_c5"] = bench_c5(L, args.c5_requests)
    if "small" in legs:
        rec["small_batches"] = bench_small(L)
    if "c1" in legs:
        rec["latency_c1"] = bench_c1(L)
    if "c3" in legs:
        rec["precision_c3"] = bench_c3(L, max(args.steps // 10, 10), min(args.warmup, 3))
    if "p1" in legs:
        rec["paper_default_p1"] = bench_p1(L, args.steps, min(args.warmup, 3), not args.no_tune)
    if "t1" in legs:
        rec["training_t1"] = bench_t1(L, max(args.steps // 10, 5), min(args.warmup, 3), t1_data, not args.no_cpu,
                                      args.t1_quality_steps)
    if not args.no_cpu and "c2" in legs:
        print("[bench] timing the oracle on a CPU sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(obj, rays_np, args.cpu_sample)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
