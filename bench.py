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
KERNEL = "k_query_mma<_Float16, _Float16, 2, 64>"


def kernel_source_hash():
    h = hashlib.sha1()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2504_21627_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload)
    if not rec or rec.get("src_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_path(L, ctx, oid, rays, out, steps, warmup):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        L.lsnif_query(ctx, oid, rays, out, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        L.lsnif_query(ctx, oid, rays, out, stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    return wall, lat


def points_per_launch(L, ctx, oid, rays, out):
    import torch
    n = rays.shape[0]
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    L.lsnif_query_debug(ctx, oid, rays, out, {"count": cnt})
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()
    return int(np.maximum(c, 0).sum()), int((c > 0).sum())


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--only", choices=["fp16", "fp32"], default=None,
                    help="time one path only (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); every box here has one GPU "
              "and this build runs no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2504_21627_amd import lsnif as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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
        print(f"[bench] timing the {name} path: {args.warmup} warmup + {args.steps} steps",
              file=sys.stderr, flush=True)
        wall, lat = time_path(L, ctx, oid, rays, out, args.steps, args.warmup)
        pts, cand = points_per_launch(L, ctx, oid, rays, out)
        paths[name] = {"wall": wall, "lat": lat, "points": pts, "cand": cand,
                       "feat_bytes": 2 if feat == "fp16" else 4}
        L.lsnif_release(ctx, oid)
    L.lsnif_destroy(ctx)

    head = paths.get("fp16") or paths["fp32"]
    ms_per_step = head["wall"] * 1e3 / args.steps
    mean_ms = float(head["lat"].mean())
    # algorithmic gather bytes per boundary point: 4 corners on levels aligned with the
    # voxel faces, 8 elsewhere, F features each
    corners = sum(4 if int(R) % obj.V == 0 else 8 for R in obj.R)
    bytes_per_point = corners * obj.F * head["feat_bytes"]
    alg_bytes = head["points"] * bytes_per_point
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    macs = sum(w.shape[0] * w.shape[1] for w in obj.weights)
    flops = 2.0 * macs * head["cand"]
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
        "data": "synthetic",
        "config": {"workload": "c2: 200k-triangle noise-displaced sphere, V=128, 16 levels x 2^19 "
                               "entries x 2 features, MLP 576-64-64-64-9, 1024x1024 pinhole primary "
                               "rays + 1048576 shadow rays",
                   "rays": n, "path": "fp16 features, fp16 MFMA MLP, fp32 accumulation"
                   if "fp16" in paths else "fp32 features, fp32 vector-ALU MLP"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("c2-fp16"),
                     "kernel": KERNEL if "fp16" in paths else "k_query_f32",
                     "alg_bytes_per_launch": alg_bytes, "points_per_launch": head["points"],
                     "bytes_per_point": bytes_per_point, "mean_kernel_ms": mean_ms,
                     "mfma_tflops": flops / (mean_ms * 1e-3) / 1e12,
                     "mfma_frac": flops / (mean_ms * 1e-3) / 1e12 / MFMA_FP16_PEAK_TFLOPS},
    }
    if "fp32" in paths:
        p = paths["fp32"]
        rec["fp32_plain"] = {"value": n / (p["wall"] / args.steps) / 1e6, "unit": "Mrays/s",
                             "p50_ms": float(np.percentile(p["lat"], 50)),
                             "p99_ms": float(np.percentile(p["lat"], 99))}
        if "fp16" in paths:
            rec["fp16_over_fp32"] = rec["value"] / rec["fp32_plain"]["value"]
    if not args.no_cpu:
        print("[bench] timing the oracle on a CPU sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(obj, rays_np, args.cpu_sample)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
