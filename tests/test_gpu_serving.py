"""Serving on the GPU: continuous batching gives each request the answer it gets alone."""

import time

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import compare_pairs, pair_reference

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


@pytest.fixture(scope="module")
def scene():
    objs = [W.configs.c4_object(i) for i in range(16)]
    insts, boxes = W.configs.c5_instances(objs, seed=5)
    pool = W.configs.c5_pool(objs, n_secondary=1 << 17, side=256, seed=5)
    rays = pool["rays"]
    pr, pi = W.configs.ray_box_pairs(rays, boxes)
    windows = W.configs.c5_requests(pool["n_primary"], len(rays), n_requests=40, lo=256, hi=1 << 15, seed=7)
    return objs, insts, rays, pr, pi, windows


def bits(t):
    return t.cpu().numpy().view(np.uint32)


def test_serving_matches_alone(L, scene):
    import torch
    from paper_2504_21627_amd.serving import RequestSet
    objs, insts, rays, pr, pi, windows = scene
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        insts_dev = [(ids[k], m) for k, m in insts]
        rs = RequestSet(L, rays, pr, pi, insts_dev, windows)
        # alone: each request by itself through the direct call
        alone = []
        for j in range(len(windows)):
            out = torch.empty_like(rs.outs[j])
            L.lsnif_query_pairs(ctx, rs.rays_of(j), rs.pr[j], rs.pi[j], rs.inst, out)
            alone.append(out)
        torch.cuda.synchronize()
        # in the mix: all submitted at once to the serving loop, 4 streams, 6 slots
        L.lsnif_serve_start(ctx, max_inflight=6, hbm_budget=256 << 20, n_streams=4)
        tickets = [L.lsnif_serve_submit(ctx, rs.request(j)) for j in range(len(windows))]
        for t in tickets:
            assert L.lsnif_serve_wait(ctx, t, 60_000_000_000) == L.LSNIF_OK
        st = L.lsnif_serve_stats_get(ctx)
        L.lsnif_serve_stop(ctx)
        print({k: st[k] for k in ("completed", "rays_completed", "p50_ms", "p99_ms", "ws_bytes_peak")})
        assert st["completed"] == len(windows) and st["failed"] == 0
        for j in range(len(windows)):
            assert np.array_equal(bits(alone[j]), bits(rs.outs[j])), j
        # and the answers agree with the oracle on 24 requests, at the FP16 pair bars
        for j in range(24):
            s, n, _ = windows[j]
            pr_j = rs.pr[j].cpu().numpy().astype(np.uint32)
            pi_j = rs.pi[j].cpu().numpy().astype(np.uint32)
            o = rs.outs[j].cpu().numpy()
            g = {"hit": o[:, 0].view(np.uint32), "t": o[:, 1], "normal": o[:, 2:5],
                 "material": o[:, 5].view(np.int32)}
            st = compare_pairs(g, pair_reference(oracle, objs, insts, rays[s:s + n], pr_j, pi_j, 2.0 ** -11),
                               1e-3, 1e-2, 0.999)
            print(j, n, st["candidate_rays"], st["vis_agree_cand"], st["t_rel_max"], st["normal_ang_max"])
            assert st["ok"], (j, st)
    finally:
        L.lsnif_destroy(ctx)


def test_serving_budget_and_overlap(L, scene):
    """A budget that fits one large request at a time still completes everything; several
    small requests overlap (more than one in flight at once)."""
    import torch
    from paper_2504_21627_amd.serving import RequestSet
    objs, insts, rays, pr, pi, windows = scene
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        rs = RequestSet(L, rays, pr, pi, [(ids[k], m) for k, m in insts], windows)
        L.lsnif_serve_start(ctx, max_inflight=8, hbm_budget=48 << 20, n_streams=4)
        tickets = [L.lsnif_serve_submit(ctx, rs.request(j)) for j in range(len(windows))]
        peak_inflight = 0
        while True:
            s = L.lsnif_serve_stats_get(ctx)
            peak_inflight = max(peak_inflight, s["inflight"])
            if s["completed"] + s["failed"] >= len(windows):
                break
            time.sleep(0.0002)
        for t in tickets:
            assert L.lsnif_serve_wait(ctx, t) == L.LSNIF_OK
        s = L.lsnif_serve_stats_get(ctx)
        L.lsnif_serve_stop(ctx)
        assert s["ws_bytes_peak"] <= 48 << 20
        assert peak_inflight >= 2
    finally:
        L.lsnif_destroy(ctx)


def test_serving_tuning_change_while_queued(L, scene):
    """A request queued behind a long one is sized again when it is admitted: its object's
    tuning (a finer coherence sort, hence more sort bins in the workspace) changes after
    submit and before admission, and the answer still equals the direct query's."""
    import torch
    objs, insts, rays, pr, pi, windows = scene
    obj = objs[0]
    rng = np.random.default_rng(12)
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        base = L.lsnif_get_tuning(ctx, oid)
        coarse = dict(base, sort_bits=1)
        fine = dict(base, sort_bits=6)
        L.lsnif_set_tuning(ctx, oid, *coarse.values())
        big = torch.from_numpy(W.sphere_to_box_rays(rng, 1 << 21, radius=3.0, half_box=1.0)).cuda()
        small = torch.from_numpy(W.sphere_to_box_rays(rng, 1 << 16, radius=3.0, half_box=1.0)).cuda()
        out_big = torch.empty((big.shape[0], 6), device="cuda")
        out_small = torch.empty((small.shape[0], 6), device="cuda")
        L.lsnif_serve_start(ctx, max_inflight=1, hbm_budget=512 << 20, n_streams=1)
        t1 = L.lsnif_serve_submit(ctx, L.make_request(rays=big, out=out_big, object_id=oid))
        t2 = L.lsnif_serve_submit(ctx, L.make_request(rays=small, out=out_small, object_id=oid))
        L.lsnif_set_tuning(ctx, oid, *fine.values())
        assert L.lsnif_serve_wait(ctx, t1) == L.LSNIF_OK
        assert L.lsnif_serve_wait(ctx, t2) == L.LSNIF_OK
        st = L.lsnif_serve_stats_get(ctx)
        L.lsnif_serve_stop(ctx)
        assert st["completed"] == 2 and st["failed"] == 0
        ref = torch.empty_like(out_small)
        L.lsnif_query(ctx, oid, small, ref)
        torch.cuda.synchronize()
        assert np.array_equal(ref.cpu().numpy().view(np.uint32), out_small.cpu().numpy().view(np.uint32))
    finally:
        L.lsnif_destroy(ctx)


@pytest.mark.parametrize("merge_max", [32, 1])
def test_serving_merged_launches(L, scene, merge_max):
    """Small requests submitted together share launches (merge_max 32; 1 turns merging
    off): single-object requests on two objects, interleaved so only neighbours with the
    same object merge, and pair requests, one of which names a ray past its own rays and
    an instance past the array.  Every answer equals the request's direct call bit for
    bit, and with merging on there are fewer launches than requests."""
    import torch
    objs, insts, rays, pr, pi, windows = scene
    rng = np.random.default_rng(31)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs[:2]]
        inst = torch.from_numpy(L.instances_array([(ids[k % 2], m) for k, m in insts[:4]])).cuda()
        reqs, refs = [], []
        for j in range(24):
            n = int(rng.integers(1, 3000))
            r = torch.from_numpy(W.sphere_to_box_rays(rng, n, radius=3.0, half_box=1.0)).cuda()
            out = torch.full((n, 6), 7.0, device="cuda")
            ref = torch.empty_like(out)
            if j < 12:
                oid = ids[(j // 3) % 2]          # runs of three requests per object
                reqs.append((L.make_request(rays=r, out=out, object_id=oid), r, out))
                L.lsnif_query(ctx, oid, r, ref)
            else:
                m = 2 * n
                p_r = torch.from_numpy(rng.integers(0, n, m).astype(np.int32)).cuda()
                p_i = torch.from_numpy(rng.integers(0, 4, m).astype(np.int32)).cuda()
                if j == 15:
                    p_r[0] = n + 5              # no such ray in this request: dropped
                    p_i[1] = 9                  # no such instance: dropped
                reqs.append((L.make_request(rays=r, out=out, pair_ray=p_r, pair_inst=p_i, inst=inst), r, out,
                             p_r, p_i))
                L.lsnif_query_pairs(ctx, r, p_r, p_i, inst, ref)
            refs.append(ref)
        torch.cuda.synchronize()
        L.lsnif_serve_start(ctx, max_inflight=2, hbm_budget=256 << 20, n_streams=2, merge_max=merge_max)
        tickets = [L.lsnif_serve_submit(ctx, q[0]) for q in reqs]
        for t in tickets:
            assert L.lsnif_serve_wait(ctx, t, 60_000_000_000) == L.LSNIF_OK
        st = L.lsnif_serve_stats_get(ctx)
        L.lsnif_serve_stop(ctx)
        print(merge_max, {k: st[k] for k in ("completed", "launches", "p50_ms", "p99_ms")})
        assert st["completed"] == len(reqs) and st["failed"] == 0
        if merge_max == 1:
            assert st["launches"] == len(reqs)
        else:
            assert st["launches"] < len(reqs)
        for j, (q, ref) in enumerate(zip(reqs, refs)):
            assert np.array_equal(bits(q[2]), bits(ref)), j
    finally:
        L.lsnif_destroy(ctx)
