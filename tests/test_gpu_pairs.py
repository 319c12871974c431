"""Instanced pair queries on the GPU against the oracle's nearest-hit definition."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import compare_pairs, pair_reference

# unit roundoff and bars per MLP precision: (u, hit-t relative, normal angle rad, visibility)
BARS = {"fp32": (2.0 ** -24, 1e-5, 1e-4, 0.9999), "fp16": (2.0 ** -11, 1e-3, 1e-2, 0.999)}

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


def random_instances(rng, n_inst, n_obj, spread=1.5):
    out = []
    for k in range(n_inst):
        ang = rng.uniform(0, 2 * np.pi)
        sc = rng.uniform(0.8, 1.2)
        A = np.array([[np.cos(ang), 0, -np.sin(ang)], [0, 1, 0], [np.sin(ang), 0, np.cos(ang)]]) / sc
        t = rng.uniform(-spread, spread, 3)
        out.append((k % n_obj, np.concatenate([A, t[:, None]], 1).astype(np.float32)))
    return out


def run_pairs(L, ctx, ids, insts, rays, pr, pi):
    import torch
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).cuda()
    inst_arr = L.instances_array([(ids[o], m) for o, m in insts])
    out = torch.empty((len(rays), 6), dtype=torch.float32, device="cuda")
    L.lsnif_query_pairs(ctx, dev(rays, np.float32), dev(pr, np.int32), dev(pi, np.int32),
                        dev(inst_arr, np.int32), out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return {"hit": o[:, 0].view(np.uint32), "t": o[:, 1], "normal": o[:, 2:5],
            "material": o[:, 5].view(np.int32)}


@pytest.mark.parametrize("mlp", ["fp32", "fp16"])
def test_pairs_random_instances(L, mlp):
    """Every ray against every instance of two objects under random rigid transforms."""
    rng = np.random.default_rng(5)
    objs = [W.configs.c1_object(0), W.configs.c1_object(1)]
    insts = random_instances(rng, 6, 2, spread=1.2)
    rays = W.sphere_to_box_rays(np.random.default_rng(9), 3000, radius=3.5, half_box=1.5)
    n = len(rays)
    pr = np.repeat(np.arange(n), len(insts)).astype(np.uint32)
    pi = np.tile(np.arange(len(insts)), n).astype(np.uint32)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, mlp, mlp)) for o in objs]
        g = run_pairs(L, ctx, ids, insts, rays, pr, pi)
    finally:
        L.lsnif_destroy(ctx)
    u, t_rel, n_ang, vis = BARS[mlp]
    st = compare_pairs(g, pair_reference(oracle, objs, insts, rays, pr, pi, u), t_rel, n_ang, vis)
    print(f"pairs {mlp}: {st}")
    assert st["hits_compared"] > 200
    assert st["ok"], st
    if mlp == "fp32":
        assert st["material_agree"] > 0.999
    assert np.all(g["material"][g["hit"] == 0] == -1)


def c4_identity_pairs(objs, owner):
    ident = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    return [(k, ident) for k in range(len(objs))], np.arange(len(owner), dtype=np.uint32), owner.astype(np.uint32)


def test_pairs_multi_object_batch(L):
    """A scaled-down c4 batch: 64 objects of different sizes, one pair per ray, FP16 MFMA."""
    c = W.configs.c4(scale=0.002)
    objs, rays, owner = c["objects"], c["rays"], c["owner"]
    insts, pr, pi = c4_identity_pairs(objs, owner)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        g = run_pairs(L, ctx, ids, insts, rays, pr, pi)
        # a second call with the pairs shuffled gives the same answers bit for bit
        perm = np.random.default_rng(3).permutation(len(pr))
        g2 = run_pairs(L, ctx, ids, insts, rays, pr[perm], pi[perm])
    finally:
        L.lsnif_destroy(ctx)
    for k in ("hit", "t", "normal", "material"):
        assert np.array_equal(g[k].view(np.uint32), g2[k].view(np.uint32)), k
    u, t_rel, n_ang, vis = BARS["fp16"]
    st = compare_pairs(g, pair_reference(oracle, objs, insts, rays, pr, pi, u), t_rel, n_ang, vis)
    print(f"c4 x0.002: {len(rays)} rays: {st}")
    assert st["ok"], st


@pytest.mark.timeout(600)
def test_c4_full_size_sampled(L):
    """The full c4 launch (64 objects, 16,777,216 pairs, one pair query under the autotuned
    tuning), checked on 8,192 rays drawn with a fixed seed: each sampled ray's result of
    the whole launch against the oracle, at the FP16 bars."""
    import torch
    print("c4 full: generating the workload", flush=True)
    c = W.configs.c4()
    objs, rays_np, owner = c["objects"], c["rays"], c["owner"]
    n = len(rays_np)
    assert n == 16_777_216
    insts, pr_np, pi_np = c4_identity_pairs(objs, owner)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        inst = torch.from_numpy(L.instances_array([(ids[k], m) for k, m in insts])).cuda()
        rays = torch.from_numpy(rays_np).cuda()
        pr = torch.from_numpy(pr_np.astype(np.int32)).cuda()
        pi = torch.from_numpy(pi_np.astype(np.int32)).cuda()
        out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        print("c4 full: autotuning", flush=True)
        tuning = L.lsnif_autotune_pairs(ctx, rays, pr, pi, inst, out)
        print(f"c4 full: launch under {tuning}", flush=True)
        out.fill_(0.0)
        L.lsnif_query_pairs(ctx, rays, pr, pi, inst, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
    finally:
        L.lsnif_destroy(ctx)
    sample = np.sort(np.random.default_rng(2025).choice(n, 8192, replace=False))
    g = {"hit": o[sample, 0].view(np.uint32), "t": o[sample, 1], "normal": o[sample, 2:5],
         "material": o[sample, 5].view(np.int32)}
    print("c4 full: oracle on the sample", flush=True)
    u, t_rel, n_ang, vis = BARS["fp16"]
    sub = np.arange(len(sample), dtype=np.uint32)
    st = compare_pairs(g, pair_reference(oracle, objs, insts, rays_np[sample], sub, pi_np[sample], u),
                       t_rel, n_ang, vis)
    print(f"c4 full, 8192 sampled rays: {st}", flush=True)
    assert st["candidate_rays"] > 2000
    assert st["ok"], st


def test_pairs_objects_without_pairs(L):
    """Objects with no pairs between objects with pairs, and dropped pairs, in shuffled
    order: the sorted keys' object bounds leave the empty objects no tiles and every other
    object its own, so the answers are the oracle's."""
    rng = np.random.default_rng(23)
    objs = [W.configs.c1_object(s) for s in range(4)]
    insts = [(o, m) for o, m in random_instances(rng, 8, 4, spread=1.0) if o in (0, 3)]
    rays = W.sphere_to_box_rays(np.random.default_rng(29), 2500, radius=3.5, half_box=1.5)
    n = len(rays)
    pr = np.repeat(np.arange(n), len(insts)).astype(np.uint32)
    pi = np.tile(np.arange(len(insts)), n).astype(np.uint32)
    perm = rng.permutation(len(pr))
    pr, pi = pr[perm], pi[perm]
    bad = np.array([len(insts) + 3] * 50, np.uint32)     # instances that do not exist: dropped
    pr_all = np.concatenate([pr, rng.integers(0, n, 50).astype(np.uint32)])
    pi_all = np.concatenate([pi, bad])
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        g = run_pairs(L, ctx, ids, insts, rays, pr_all, pi_all)
    finally:
        L.lsnif_destroy(ctx)
    u, t_rel, n_ang, vis = BARS["fp16"]
    st = compare_pairs(g, pair_reference(oracle, objs, insts, rays, pr, pi, u), t_rel, n_ang, vis)
    print(f"pairs with empty objects: {st}", flush=True)
    assert st["hits_compared"] > 100
    assert st["ok"], st


def test_pairs_edge_cases(L):
    """No pairs, pairs naming missing rays/instances/objects, and mixed kernel classes."""
    import torch
    obj = W.configs.c1_object()
    rays = W.configs.c1()["rays"][:100]
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        ident = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
        insts = [(0, ident)]
        g = run_pairs(L, ctx, [oid], insts, rays, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
        assert g["hit"].sum() == 0 and np.all(g["material"] == -1)
        pr = np.array([0, 1, 500, 2], np.uint32)        # ray 500 does not exist
        pi = np.array([0, 7, 0, 0], np.uint32)          # instance 7 does not exist
        g = run_pairs(L, ctx, [oid], insts, rays, pr, pi)
        o = oracle.query_pairs([obj], insts, rays, np.array([0, 2], np.uint32), np.array([0, 0], np.uint32))
        assert np.array_equal(g["hit"][[0, 2]], o["hit"][[0, 2]]) and g["hit"][1] == 0
        g = run_pairs(L, ctx, [oid + 100], insts, rays, np.arange(100, dtype=np.uint32),
                      np.zeros(100, np.uint32))        # unknown object id
        assert g["hit"].sum() == 0
        L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        with pytest.raises(L.LsnifError):
            run_pairs(L, ctx, [oid], insts, rays, np.arange(100, dtype=np.uint32), np.zeros(100, np.uint32))
    finally:
        L.lsnif_destroy(ctx)
