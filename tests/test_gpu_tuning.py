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
            for sb, hot, ch, pe in ((5, 40960, 1, 0), (0, 0, 4, 0), (3, 20480, 2, 1), (4, 0, 16, 0), (6, 0, 3, 1),
                                    (5, 0, 1, 1), (0, 40960, 1, 1), (7, 0, 1, 0), (7, 20480, 2, 1)):
                L.lsnif_set_tuning(ctx, oid, sb, 4, hot, ch, pe)
                assert L.lsnif_get_tuning(ctx, oid) == {"sort_bits": sb, "pair_bits": 4, "hot_lds_bytes": hot,
                                                        "walk_chunks": ch, "persistent": pe}
                out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
                L.lsnif_query(ctx, oid, rays, out)
                torch.cuda.synchronize()
                if ref is None:
                    ref = bits(out)
                else:
                    assert np.array_equal(bits(out), ref), (feat, sb, hot, ch, pe)
            out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
            best = L.lsnif_autotune(ctx, oid, rays, out)
            print(feat, "autotuned", best, flush=True)
            assert best["sort_bits"] in (0, 4, 5, 6, 7) and best["hot_lds_bytes"] in (0, 20480, 40960)
            assert best["walk_chunks"] in (1, 2, 4, 8) and best["persistent"] in (0, 1)
            assert L.lsnif_get_tuning(ctx, oid) == best
            L.lsnif_query(ctx, oid, rays, out)
            torch.cuda.synchronize()
            assert np.array_equal(bits(out), ref)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 8, 4, 0)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 5, 4, 0, 17)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 5, 7, 0)
            with pytest.raises(L.LsnifError):
                L.lsnif_set_tuning(ctx, oid, 5, 4, 0, 1, 2)
            L.lsnif_release(ctx, oid)
    finally:
        L.lsnif_destroy(ctx)


@pytest.mark.parametrize("n", [8192, 8193, 10241, 65535])
def test_radix_sorted_batches_ragged(L, n):
    """Batches just above the sort threshold and across partial 2,048-ray blocks of the
    radix passes (one, two and three passes: sort_bits 1, 4, 7) answer every ray as the
    unsorted batch does, bit for bit."""
    import torch
    obj = W.configs.c2_object()
    rays_np = W.configs.subsample(W.configs.c2_rays(), n, seed=19)
    ctx = L.lsnif_create(0)
    try:
        rays = torch.from_numpy(rays_np).cuda()
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        ref = None
        for sb in (0, 1, 4, 7):
            L.lsnif_set_tuning(ctx, oid, sb, 4, 0)
            out = torch.full((n, 6), float("nan"), dtype=torch.float32, device="cuda")
            L.lsnif_query(ctx, oid, rays, out)
            torch.cuda.synchronize()
            if ref is None:
                ref = bits(out)
                assert (ref[:, 0] == 1).sum() > n // 10
            else:
                assert np.array_equal(bits(out), ref), (n, sb)
        print(f"{n} rays: sorted in 1, 2 and 3 passes as unsorted", flush=True)
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
        # a pair (fine, coarse): the objects alternate between two groupings
        for pb, hot, ch, pe in ((4, 40960, 1, 0), (2, 0, 4, 0), (3, 20480, 16, 1), (5, 0, 1, 1), (1, 0, 2, 0),
                                ((5, 2), 0, 1, 0), (4, 0, 1, 1), ((5, 2), 40960, 2, 1), (6, 0, 1, 0),
                                ((6, 3), 20480, 1, 1), ((6, 5), 0, 2, 0)):
            for k, i in enumerate(ids):
                L.lsnif_set_tuning(ctx, i, 5, pb if isinstance(pb, int) else pb[k % 2 == 0], hot, ch, pe)
            out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
            L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out)
            torch.cuda.synchronize()
            if ref is None:
                ref = bits(out)
                assert (ref[:, 0] == 1).sum() > 100
            else:
                assert np.array_equal(bits(out), ref), (pb, hot, ch, pe)
        out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
        best = L.lsnif_autotune_pairs(ctx, rays, pr, pi, inst, out)
        print("pairs autotuned", best, flush=True)
        assert best["pair_bits"] in (2, 3, 4, 5, 6) and best["walk_chunks"] in (1, 2, 4, 8)
        L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out)
        torch.cuda.synchronize()
        assert np.array_equal(bits(out), ref)
    finally:
        L.lsnif_destroy(ctx)


def test_autotune_cache_round_trip(L, tmp_path):
    """lsnif_autotune writes its winner to the context's cache file; a second context with
    the same file starts the same object with the cached parameters, without timing; an
    entry edited in the file is what the next context applies; a context without the
    cache keeps the defaults."""
    import json
    import torch
    obj = W.configs.c1_object()
    rays_np = W.sphere_to_box_rays(np.random.default_rng(21), 200_000, radius=2.0, half_box=1.0)
    path = str(tmp_path / "tune.json")
    rays = torch.from_numpy(rays_np).cuda()
    out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
    ctx = L.lsnif_create(0, autotune_cache=path)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        default = L.lsnif_get_tuning(ctx, oid)
        won = L.lsnif_autotune(ctx, oid, rays, out)
    finally:
        L.lsnif_destroy(ctx)
    data = json.load(open(path))
    assert data["lsnif_autotune_cache"] == 1
    (key, entry), = data["entries"].items()
    assert key.startswith("gfx950 V=32 L=8 F=2 log2_T=14 H=18 width=64 feat=fp16 mlp=fp16"), key
    assert entry == won
    ctx = L.lsnif_create(0, autotune_cache=path)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        assert L.lsnif_get_tuning(ctx, oid) == won
        other = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))   # another key: defaults
        assert L.lsnif_get_tuning(ctx, other) == default
    finally:
        L.lsnif_destroy(ctx)
    edited = {"sort_bits": 2, "pair_bits": 5, "hot_lds_bytes": 20480, "walk_chunks": 3, "persistent": 1}
    data["entries"][key] = edited
    json.dump(data, open(path, "w"))
    ctx = L.lsnif_create(0, autotune_cache=path)
    plain = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        assert L.lsnif_get_tuning(ctx, oid) == edited
        a = torch.empty_like(out)
        L.lsnif_query(ctx, oid, rays, a)
        pid = L.lsnif_build(plain, L.ObjectDesc(obj, "fp16", "fp16"))
        assert L.lsnif_get_tuning(plain, pid) == default
        b = torch.empty_like(out)
        L.lsnif_query(plain, pid, rays, b)
        torch.cuda.synchronize()
        assert np.array_equal(bits(a), bits(b))     # parameters change speed, never results
    finally:
        L.lsnif_destroy(ctx)
        L.lsnif_destroy(plain)
