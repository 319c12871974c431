"""The device broad phase and the scene query (Sec. 4) against the oracle's broad phase
and against the pair query given the host's world-box pairs."""

import numpy as np
import pytest

import oracle
from tests.parity import compare_pairs, pair_reference
import workloads as W
from tests.scene import small_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


@pytest.fixture(scope="module")
def scene():
    return small_scene()


def bits(t):
    return t.cpu().numpy().view(np.uint32)


def setup(L, ctx, objs, insts, rays):
    import torch
    ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
    inst = torch.from_numpy(L.instances_array([(ids[k], m) for k, m in insts])).cuda()
    return ids, inst, torch.from_numpy(rays).cuda()


def test_broad_phase_matches_oracle(L, scene):
    import torch
    objs, insts, boxes, rays_np = scene
    want_r, want_i = oracle.broad_phase(objs, insts, rays_np)
    ctx = L.lsnif_create(0)
    try:
        ids, inst, rays = setup(L, ctx, objs, insts, rays_np)
        cap = len(want_r) + 100
        pr = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        pi = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        n = L.lsnif_broad_phase(ctx, rays, inst, pr, pi)
        torch.cuda.synchronize()
        assert n == len(want_r)
        assert np.array_equal(pr[:n].cpu().numpy().astype(np.uint32), want_r)
        assert np.array_equal(pi[:n].cpu().numpy().astype(np.uint32), want_i)
        assert (pr[n:] == -1).all()
        # too small a buffer: nothing written, the count reported
        small = torch.full((10,), -1, dtype=torch.int32, device="cuda")
        with pytest.raises(L.LsnifError) as e:
            L.lsnif_broad_phase(ctx, rays, inst, small, small.clone())
        assert e.value.status == L.LSNIF_E_NOMEM and L.lsnif_last_pair_count == n
        assert (small == -1).all()
        # no instances; an instance naming no built object; no rays
        none = torch.empty((0, 13), dtype=torch.int32, device="cuda")
        assert L.lsnif_broad_phase(ctx, rays, none, pr, pi) == 0
        ghost = inst[:2].clone()
        ghost[1, 0] = 999
        got = L.lsnif_broad_phase(ctx, rays, ghost, pr, pi)
        torch.cuda.synchronize()
        assert got == int((want_i == 0).sum()) and (pi[:got] == 0).all()
        assert L.lsnif_broad_phase(ctx, rays[:0], inst, pr, pi) == 0
    finally:
        L.lsnif_destroy(ctx)


@pytest.mark.parametrize("n_inst", [40, 256, 257])
def test_broad_phase_many_instances(L, scene, n_inst):
    """Instance bit masks over several words (40, and 256: the most the masks serve) and the
    repeated tests beyond them (257): the pairs are the oracle's, an instance naming no built
    object (index 37) giving none."""
    import torch
    objs, insts, boxes, rays_np = scene
    rays_np = rays_np[::3]
    many = [insts[k % len(insts)] for k in range(n_inst)]
    want_r, want_i = oracle.broad_phase(objs, many, rays_np)
    keep = want_i != 37
    want_r, want_i = want_r[keep], want_i[keep]
    ctx = L.lsnif_create(0)
    try:
        ids, inst, rays = setup(L, ctx, objs, many, rays_np)
        inst[37, 0] = 999
        cap = len(want_r) + 100
        pr = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        pi = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        for _ in range(2):   # the second call reuses the workspace and its stale masks
            n = L.lsnif_broad_phase(ctx, rays, inst, pr, pi)
            torch.cuda.synchronize()
            assert n == len(want_r)
            assert np.array_equal(pr[:n].cpu().numpy().astype(np.uint32), want_r)
            assert np.array_equal(pi[:n].cpu().numpy().astype(np.uint32), want_i)
            assert (pr[n:] == -1).all()
        print(f"{n_inst} instances: {n} pairs", flush=True)
    finally:
        L.lsnif_destroy(ctx)


def test_scene_query_equals_pairs_query(L, scene):
    """lsnif_query_scene answers every ray as the pair query does given the host's (looser)
    world-box pairs, bit for bit, and agrees with the oracle's pair query."""
    import torch
    objs, insts, boxes, rays_np = scene
    ctx = L.lsnif_create(0)
    try:
        ids, inst, rays = setup(L, ctx, objs, insts, rays_np)
        n = len(rays_np)
        got = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        L.lsnif_query_scene(ctx, rays, inst, got)
        hr, hi = W.configs.ray_box_pairs(rays_np, boxes)
        ref = torch.empty_like(got)
        L.lsnif_query_pairs(ctx, rays, torch.from_numpy(hr.astype(np.int32)).cuda(),
                            torch.from_numpy(hi.astype(np.int32)).cuda(), inst, ref)
        torch.cuda.synchronize()
        g, r = bits(got), bits(ref)
        assert np.array_equal(g, r)
        assert (g[:, 0] == 1).sum() > 100
        pr, pi = oracle.broad_phase(objs, insts, rays_np)
        h = got.cpu().numpy()
        res = {"hit": h[:, 0].view(np.uint32), "t": h[:, 1], "normal": h[:, 2:5], "material": h[:, 5].view(np.int32)}
        st = compare_pairs(res, pair_reference(oracle, objs, insts, rays_np, pr, pi, 2.0 ** -11), 1e-3, 1e-2, 0.999)
        print(st)
        assert st["ok"], st
    finally:
        L.lsnif_destroy(ctx)


def test_bounce_matches_oracle(L, scene):
    """Bounce rays from the scene query's hits: the same parents, bit-identical origins and
    directions within a few float32 ulps of the oracle's (the device's and libm's cos and sin
    differ in the last bits)."""
    import torch
    objs, insts, boxes, rays_np = scene
    ctx = L.lsnif_create(0)
    try:
        ids, inst, rays = setup(L, ctx, objs, insts, rays_np)
        n = len(rays_np)
        hits = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        L.lsnif_query_scene(ctx, rays, inst, hits)
        torch.cuda.synchronize()
        h = hits.cpu().numpy()
        hit = h[:, 0].view(np.uint32).copy()
        assert hit.sum() > 100
        nxt = torch.full((n, 8), float("nan"), dtype=torch.float32, device="cuda")
        par = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        m = L.lsnif_bounce(ctx, rays, hits, 3, 1, 1e-4, nxt, par)
        torch.cuda.synchronize()
        want, wpar = oracle.bounce(rays_np, hit, h[:, 1], h[:, 2:5], 3, 1, 1e-4)
        assert m == len(want)
        assert np.array_equal(par[:m].cpu().numpy().astype(np.uint32), wpar)
        g = nxt[:m].cpu().numpy()
        assert np.array_equal(g[:, :3].view(np.uint32), want[:, :3].view(np.uint32))
        # |lx|, |ly| <= 1 carry the two libraries' cos/sin differences (a few ulps, ~2.4e-7
        # each), and the basis products and the two sums of each component add four
        # roundings of values <= 1: 8e-7 bounds the component difference
        assert np.abs(g[:, 3:6] - want[:, 3:6]).max() <= 8e-7
        assert np.array_equal(g[:, 6:].view(np.uint32), want[:, 6:].view(np.uint32))
        assert torch.isnan(nxt[m:]).all()
        small = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
        with pytest.raises(L.LsnifError) as e:
            L.lsnif_bounce(ctx, rays, hits, 3, 1, 1e-4, small, par[:4].clone())
        assert e.value.status == L.LSNIF_E_NOMEM and L.lsnif_last_pair_count == m
    finally:
        L.lsnif_destroy(ctx)
