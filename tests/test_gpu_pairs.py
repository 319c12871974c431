"""Instanced pair queries on the GPU against the oracle's nearest-hit definition."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import output_bound

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


def compare(g, o, vis_min, t_rel):
    agree = g["hit"] == o["hit"]
    cand = (o["hit"] == 1) | (g["hit"] == 1)
    frac = agree[cand].mean() if cand.any() else 1.0
    both = (g["hit"] == 1) & (o["hit"] == 1)
    terr = np.abs(g["t"][both].astype(np.float64) - o["t"][both]) / np.maximum(np.abs(o["t"][both]), 1e-3)
    return frac, (terr.max() if both.any() else 0.0), both.sum()


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
    o = oracle.query_pairs(objs, insts, rays, pr, pi)
    frac, terr, nboth = compare(g, o, 0, 0)
    print(f"pairs {mlp}: agreement {frac:.5f}, t rel err {terr:.2e}, hits {nboth}")
    assert nboth > 200
    assert frac >= (0.9999 if mlp == "fp32" else 0.995)
    assert terr <= (1e-5 if mlp == "fp32" else 1e-3)
    same = (g["hit"] == 1) & (o["hit"] == 1) & (np.abs(g["t"] - o["t"]) <= 1e-5 * np.abs(o["t"]))
    if mlp == "fp32":
        assert np.allclose(g["normal"][same], o["normal"][same], atol=5e-3)
        assert (g["material"][same] == o["material"][same]).mean() > 0.999
    assert np.all(g["material"][g["hit"] == 0] == -1)


def test_pairs_multi_object_batch(L):
    """A scaled-down c4 batch: 64 objects of different sizes, one pair per ray, FP16 MFMA."""
    c = W.configs.c4(scale=0.002)
    objs, rays, owner = c["objects"], c["rays"], c["owner"]
    ident = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    insts = [(k, ident) for k in range(len(objs))]
    pr = np.arange(len(rays), dtype=np.uint32)
    pi = owner.astype(np.uint32)
    ctx = L.lsnif_create(0)
    try:
        ids = [L.lsnif_build(ctx, L.ObjectDesc(o, "fp16", "fp16")) for o in objs]
        g = run_pairs(L, ctx, ids, insts, rays, pr, pi)
        # a second call with the pairs shuffled gives the same answers bit for bit
        perm = np.random.default_rng(3).permutation(len(pr))
        g2 = run_pairs(L, ctx, ids, insts, rays, pr[perm], pi[perm])
    finally:
        L.lsnif_destroy(ctx)
    for k in ("hit", "t", "material"):
        assert np.array_equal(g[k].view(np.uint32), g2[k].view(np.uint32)), k
    o = oracle.query_pairs(objs, insts, rays, pr, pi)
    frac, terr, nboth = compare(g, o, 0, 0)
    print(f"c4 x0.002: {len(rays)} rays, agreement {frac:.5f}, t rel err {terr:.2e}, hits {nboth}")
    assert frac >= 0.995 and terr <= 1e-3


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
