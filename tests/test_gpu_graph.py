"""Captured HIP graphs replay exactly what the direct calls compute.

Each graph is replayed several times with eager device work and
synchronisations between the replays (the output buffer is overwritten in
between), and every replay is compared bit for bit with the direct call.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


def bits(t):
    return t.cpu().numpy().view(np.uint32)


def test_graph_query_replays(L):
    import torch
    obj = W.configs.c2_object()
    # above the sort threshold, and 782 tiles: with walk_chunks 4, 3 walk ranges of at least 256
    # tiles run ahead on the context's side stream, and the capture records that fork and join
    rays_np = W.configs.subsample(W.configs.c2_rays(), 200000, seed=3)
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        L.lsnif_set_tuning(ctx, oid, 5, 4, 0, 4)
        rays = torch.from_numpy(rays_np).cuda()
        ref = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
        L.lsnif_query(ctx, oid, rays, ref)
        torch.cuda.synchronize()
        want = bits(ref)
        out = torch.empty_like(ref)
        g = L.lsnif_graph_query(ctx, oid, rays, out)
        try:
            for rep in range(4):
                out.fill_(float("nan"))
                torch.cuda.synchronize()
                L.lsnif_graph_launch(g)
                torch.cuda.synchronize()
                assert np.array_equal(bits(out), want), rep
                # eager library work between replays
                L.lsnif_query(ctx, oid, rays[:5000], ref[:5000])
                torch.cuda.synchronize()
        finally:
            L.lsnif_graph_destroy(g)
    finally:
        L.lsnif_destroy(ctx)


def test_graph_pairs_replays_and_goes_stale(L):
    import torch
    d = W.configs.c4(n_objects=6, total=6 * 200000, scale=0.05)
    objs, rays_np, owner = d["objects"], d["rays"], d["owner"]
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        for i in ids:
            L.lsnif_set_tuning(ctx, i, 5, 4, 0, 4)   # the walk runs ahead in 4 ranges
        eye = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
        inst = torch.from_numpy(L.instances_array([(i, eye) for i in ids])).cuda()
        rays = torch.from_numpy(rays_np).cuda()
        pr = torch.arange(len(rays_np), dtype=torch.int32, device="cuda")
        pi = torch.from_numpy(owner.astype(np.int32)).cuda()
        ref = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
        L.lsnif_query_pairs(ctx, rays, pr, pi, inst, ref)
        torch.cuda.synchronize()
        want = bits(ref)
        assert (want[:, 0] == 1).sum() > 100
        out = torch.empty_like(ref)
        g = L.lsnif_graph_pairs(ctx, rays, pr, pi, inst, out)
        try:
            for rep in range(4):
                out.fill_(float("nan"))
                torch.cuda.synchronize()
                L.lsnif_graph_launch(g)
                torch.cuda.synchronize()
                assert np.array_equal(bits(out), want), rep
                L.lsnif_query_pairs(ctx, rays[:1000], pr[:1000], pi[:1000], inst, ref[:1000])
                torch.cuda.synchronize()
            # building another object invalidates the graph
            extra = L.lsnif_build(ctx, L.ObjectDesc(objs[0], "fp16", "fp16"))
            with pytest.raises(L.LsnifError):
                L.lsnif_graph_launch(g)
            L.lsnif_release(ctx, extra)
        finally:
            L.lsnif_graph_destroy(g)
    finally:
        L.lsnif_destroy(ctx)
