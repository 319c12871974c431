"""Tuning parameters change speed, never results; the autotuner returns a valid choice."""

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


def test_single_object_tunings_agree(L):
    import torch
    obj = W.configs.c2_object()
    # 300,000 rays = 1,172 tiles: up to 4 walk ranges of at least 256 tiles each
    rays_np = W.configs.subsample(W.configs.c2_rays(), 300000, seed=8)
    ctx = L.lsnif_create(0)
    try:
        rays = torch.from_numpy(rays_np).cuda()
        for feat, mlp in (("fp16", "fp16"), ("fp32", "fp32")):
            oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
            ref = None
            for sb, hot, ch in ((5, 40960, 1), (0, 0, 4), (3, 20480, 2), (4, 0, 16), (6, 0, 3)):
                L.lsnif_set_tuning(ctx, oid, sb, 4, hot, ch)
                assert L.lsnif_get_tuning(ctx, oid) == {"sort_bits": sb, "pair_bits": 4, "hot_lds_bytes": hot,
                                                        "walk_chunks": ch}
                out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
                L.lsnif_query(ctx, oid, rays, out)
                torch.cuda.synchronize()
                if ref is None:
                    ref = bits(out)
                else:
                    assert np.array_equal(bits(out), ref), (feat, sb, hot, ch)
            out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
            best = L.lsnif_autotune(ctx, oid, rays, out)
            print(feat, "autotuned", best, flush=True)
            assert best["sort_bits"] in (0, 4, 5, 6) and best["hot_lds_bytes"] in (0, 20480, 40960)
            assert best["walk_chunks"] in (1, 2, 4, 8)
            assert L.lsnif_get_tuning(ctx, oid) == best
            L.lsnif_query(ctx, oid, rays, out)
            torch.cuda.synchronize()
            assert np.array_equal(bits(out), ref)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 7, 4, 0)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 5, 4, 0, 17)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 5, 6, 0)
            L.lsnif_release(ctx, oid)
    finally:
        L.lsnif_destroy(ctx)


def test_pair_tunings_agree(L):
    import torch
    d = W.configs.c4(n_objects=6, total=6 * 200000, scale=0.1)
    objs, rays_np, owner = d["objects"], d["rays"], d["owner"]
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        eye = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
        inst = torch.from_numpy(L.instances_array([(i, eye) for i in ids])).cuda()
        rays = torch.from_numpy(rays_np).cuda()
        pr = torch.arange(len(rays_np), dtype=torch.int32, device="cuda")
        pi = torch.from_numpy(owner.astype(np.int32)).cuda()
        ref = None
        # pb None: the objects alternate between the finest and a coarse grouping
        for pb, hot, ch in ((4, 40960, 1), (2, 0, 4), (3, 20480, 16), (5, 0, 1), (1, 0, 2), (None, 0, 1)):
            for k, i in enumerate(ids):
                L.lsnif_set_tuning(ctx, i, 5, pb if pb is not None else (5 if k % 2 else 2), hot, ch)
            out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
            L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out)
            torch.cuda.synchronize()
            if ref is None:
                ref = bits(out)
                assert (ref[:, 0] == 1).sum() > 100
            else:
                assert np.array_equal(bits(out), ref), (pb, hot, ch)
        out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
        best = L.lsnif_autotune_pairs(ctx, rays, pr, pi, inst, out)
        print("pairs autotuned", best, flush=True)
        assert best["pair_bits"] in (2, 3, 4, 5) and best["walk_chunks"] in (1, 2, 4, 8)
        L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out)
        torch.cuda.synchronize()
        assert np.array_equal(bits(out), ref)
    finally:
        L.lsnif_destroy(ctx)
