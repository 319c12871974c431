"""Parity of the HIP query path (through the C ABI) with the CPU oracle."""

import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import gpu_query, compare_hits, output_bound

pytestmark = pytest.mark.gpu

U = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


@pytest.fixture(scope="module")
def ctx(L):
    c = L.lsnif_create(0)
    yield c
    L.lsnif_destroy(c)


@pytest.fixture(scope="module")
def c1():
    return W.configs.c1()


@pytest.fixture(scope="module")
def c2_small():
    c = W.configs.c2()
    rays = W.configs.subsample(c["rays"], 12_000, seed=5)
    return {"objects": c["objects"], "rays": rays, "full": c["rays"]}


def bitwise_equal(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def check_intermediates(g, o, obj):
    """Voxel lists, points, slots and weights must equal the oracle's bit for bit."""
    assert np.array_equal(g["count"], o["count"])
    cand = o["count"] > 0
    assert bitwise_equal(g["tatb"][cand], o["tatb"][cand])
    assert np.array_equal(g["vox_ijk"], o["vox_ijk"])
    assert np.array_equal(g["vox_axis"], o["vox_axis"])
    m = o["vox_ijk"][..., 0] >= 0
    assert bitwise_equal(g["vox_t"][m], o["vox_t"][m])
    hm = np.arange(obj.H)[None, :] < np.maximum(o["count"], 0)[:, None]
    assert bitwise_equal(g["points"][hm], o["points"][hm])
    assert np.array_equal(g["slots"][hm], o["slots"][hm])
    assert bitwise_equal(g["weights"][hm], o["weights"][hm])


def enc_compare(g_enc, o_enc, obj, count, rel):
    ge = g_enc   # [n][H * L * F], as the oracle's
    scale = np.abs(o_enc).max()
    err = np.abs(ge - o_enc).max() / scale
    assert err <= rel, err
    return err


@pytest.mark.parametrize("feat,mlp", [("fp32", "fp32")])
def test_c1_fp32_parity(L, ctx, c1, feat, mlp):
    obj, rays = c1["objects"][0], c1["rays"]
    _say(f"c1 {feat}/{mlp}: {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
        enc_compare(g["enc"], o["enc"], obj, o["count"], 1e-6)
        cand = o["count"] > 0
        zerr = np.abs(g["out"][cand] - o["out"][cand]).max() / np.abs(o["out"][cand]).max()
        assert zerr < 1e-5, zerr
        st = compare_hits(g, o, o["tatb"], o["enc"], o["out"], obj, U["fp32"], 1e-5, 1e-4, 0.9999)
        _say(str(st))
        assert st["ok"], st
    finally:
        L.lsnif_release(ctx, oid)


def test_small_batch_wave_per_ray(L, ctx, c1):
    """FP32 batches of at most 8,192 rays run one wave per ray.  c1's 4,096 rays: voxel
    counts exact, raw outputs and hits against the oracle at the c1 bar; then the same
    rays three times over (12,288 rays, the ray-per-lane kernel) and 1 and 7 of them (a
    partly filled workgroup) give the same hits bit for bit."""
    import torch
    obj, rays = c1["objects"][0], c1["rays"]
    n = len(rays)
    _say(f"small batch: {n} rays, one wave each")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
    try:
        t = torch.from_numpy(np.ascontiguousarray(rays, np.float32)).cuda()
        out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        bufs = {"count": torch.empty(n, dtype=torch.int32, device="cuda"),
                "tatb": torch.empty((n, 2), dtype=torch.float32, device="cuda"),
                "out": torch.empty((n, obj.out_dim), dtype=torch.float32, device="cuda")}
        L.lsnif_query_debug(ctx, oid, t, out, bufs)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in bufs.items()}
        h = out.cpu().numpy()
        g.update(hit=h[:, 0].view(np.uint32).copy(), t=h[:, 1].copy(), normal=h[:, 2:5].copy(),
                 material=h[:, 5].view(np.int32).copy())
        o = oracle.query(obj, rays, debug=True)
        assert np.array_equal(g["count"], o["count"])
        cand = o["count"] > 0
        zerr = np.abs(g["out"][cand] - o["out"][cand]).max() / np.abs(o["out"][cand]).max()
        assert zerr < 1e-5, zerr
        st = compare_hits(g, o, o["tatb"], o["enc"], o["out"], obj, U["fp32"], 1e-5, 1e-4, 0.9999)
        _say(str(st))
        assert st["ok"], st
        def same(a, b, m):
            for k in ("hit", "t", "normal", "material"):
                assert np.array_equal(np.ascontiguousarray(a[k]).view(np.uint8),
                                      np.ascontiguousarray(b[k][:m]).view(np.uint8)), k
        big = gpu_query(L, ctx, oid, np.concatenate([rays] * 3))
        for k in range(3):
            same({key: v[k * n:(k + 1) * n] for key, v in big.items()}, g, n)
        for m in (1, 7):
            same(gpu_query(L, ctx, oid, rays[:m]), g, m)
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("feat,mlp", [("fp16", "fp16"), ("bf16", "bf16"), ("fp32", "bf16"), ("fp16", "fp8")])
def test_small_batch_matrix_core(L, ctx, c2_small, feat, mlp):
    """Matrix-core objects' batches of at most 8,192 rays run one wave per ray, each of the
    32 columns of every product holding that ray: on c2's object (16 levels, two K blocks)
    4,096 rays give the raw outputs and hits that the same rays get three times over
    (12,288 rays, k_query_mma), bit for bit, with the per-layer FP8 scales fixed."""
    import torch
    obj = c2_small["objects"][0]
    rays = c2_small["rays"][:4096]
    n = len(rays)
    _say(f"small batch, {feat}/{mlp}: {n} rays against {3 * n}")
    scale = [1.0 / 64.0] * (obj.n_hidden + 1) if mlp == "fp8" else None
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp, fp8_act_scale=scale))
    try:
        def run(r):
            m = len(r)
            t = torch.from_numpy(np.ascontiguousarray(r, np.float32)).cuda()
            out = torch.empty((m, 6), dtype=torch.float32, device="cuda")
            raw = torch.empty((m, obj.out_dim), dtype=torch.float32, device="cuda")
            L.lsnif_query_debug(ctx, oid, t, out, {"out": raw})
            torch.cuda.synchronize()
            return out.cpu().numpy(), raw.cpu().numpy()
        small_out, small_raw = run(rays)
        big_out, big_raw = run(np.concatenate([rays] * 3))
        for k in range(3):
            assert np.array_equal(big_out[k * n:(k + 1) * n].view(np.uint32), small_out.view(np.uint32)), k
            assert np.array_equal(big_raw[k * n:(k + 1) * n].view(np.uint32), small_raw.view(np.uint32)), k
        assert (small_out[:, 0].view(np.uint32) == 1).sum() > 100   # hits to compare
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("feat,mlp", [("fp16", "fp16"), ("bf16", "bf16"), ("fp32", "fp16")])
def test_c1_mma_parity(L, ctx, c1, feat, mlp):
    obj, rays = c1["objects"][0], c1["rays"]
    _say(f"c1 {feat}/{mlp}: {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
        u = max(U[feat], U[mlp])
        enc_compare(g["enc"], o["enc"], obj, o["count"], 4 * u)
        st = compare_hits(g, o, o["tatb"], o["enc"], o["out"], obj, u, 1e-3 if mlp == "fp16" else 1e-2,
                          1e-2 if mlp == "fp16" else 1e-1, 0.999 if mlp == "fp16" else 0.99)
        _say(str(st))
        assert st["ok"], st
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("feat,mlp", [("fp32", "fp32"), ("fp16", "fp16")])
def test_c2_subset_parity(L, ctx, c2_small, feat, mlp):
    obj, rays = c2_small["objects"][0], c2_small["rays"]
    _say(f"c2 subset {feat}/{mlp}: {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
        u = max(U[feat], U[mlp])
        enc_compare(g["enc"], o["enc"], obj, o["count"], 1e-6 if mlp == "fp32" else 4 * u)
        st = compare_hits(g, o, o["tatb"], o["enc"], o["out"], obj, u, 1e-5 if mlp == "fp32" else 1e-3,
                          1e-4 if mlp == "fp32" else 1e-2, 0.9999 if mlp == "fp32" else 0.999)
        _say(str(st))
        assert st["ok"], st
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("feat,mlp", [("fp32", "fp32"), ("fp16", "fp16")])
def test_c2_full_size_sampled(L, ctx, c2_small, feat, mlp):
    """The full 2M-ray batch in one launch; a seeded sample of rays checked against the oracle."""
    obj, rays = c2_small["objects"][0], c2_small["full"]
    _say(f"c2 full {feat}/{mlp}: {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, rays)
        idx = np.sort(np.random.default_rng(77).choice(len(rays), 6000, replace=False))
        idx = np.concatenate([idx, [0, len(rays) // 2 - 1, len(rays) // 2, len(rays) - 1]])
        o = oracle.query(obj, rays[idx], debug=True)
        gs = {k: v[idx] for k, v in g.items()}
        u = max(U[feat], U[mlp])
        st = compare_hits(gs, o, o["tatb"], o["enc"], o["out"], obj, u, 1e-5 if mlp == "fp32" else 1e-3,
                          1e-4 if mlp == "fp32" else 1e-2, 0.9999 if mlp == "fp32" else 0.999)
        _say(str(st))
        assert st["ok"], st
        # rays outside the sample obey the invariants: a hit has t within its AABB segment
        h = g["hit"] == 1
        assert np.all(np.isfinite(g["t"][h])) and np.all(np.isinf(g["t"][~h]))
        assert np.all(g["material"][~h] == -1)
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("mlp", ["fp32", "fp16"])
def test_edge_cases(L, ctx, c1, mlp):
    """Empty batch, a single ray, a ragged tail, invalid rays, an empty grid."""
    import torch
    obj = c1["objects"][0]
    feat = "fp32" if mlp == "fp32" else "fp16"
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        empty = torch.empty((0, 8), dtype=torch.float32, device="cuda")
        L.lsnif_query(ctx, oid, empty, torch.empty((1, 6), device="cuda"))
        rays = c1["rays"]
        for n in (1, 63, 257, 1000):
            g = gpu_query(L, ctx, oid, rays[:n])
            full = gpu_query(L, ctx, oid, rays[:1024])
            for k in ("hit", "t", "normal", "material"):
                assert bitwise_equal(g[k], full[k][:n]), (n, k)
        bad = np.array([[np.nan, 0, 0, 1, 0, 0, 0, np.inf], [0, 0, 0, 0, 0, 0, 0, np.inf],
                        [0, 0, 0, 1, 0, 0, 2, 1], [np.inf, 0, 0, 1, 0, 0, 0, np.inf],
                        [-3, 0, 0, 1, 0, 0, 0, 0.5]], np.float32)
        g = gpu_query(L, ctx, oid, bad)
        assert g["hit"].sum() == 0 and np.all(g["material"] == -1)
    finally:
        L.lsnif_release(ctx, oid)
    empty_obj = W.configs.c1_object()
    empty_obj.occ = np.zeros_like(empty_obj.occ)
    oid = L.lsnif_build(ctx, L.ObjectDesc(empty_obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, c1["rays"])
        assert g["hit"].sum() == 0
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("feat,mlp", [("fp32", "fp32"), ("fp16", "fp16")])
def test_gather_ceiling_sums(L, ctx, c1, c2_small, feat, mlp):
    """The gather-ceiling kernel runs the query's walk and encoding: each ray's summed
    features equal the sum of the oracle's encoding row, within the feature type's rounding."""
    import torch
    for obj, rays in ((c1["objects"][0], c1["rays"]), (c2_small["objects"][0], c2_small["rays"][:6000])):
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
        try:
            sums = torch.full((len(rays),), float("nan"), dtype=torch.float32, device="cuda")
            L.lsnif_gather_ceiling(ctx, oid, torch.from_numpy(rays).cuda(), sums)
            torch.cuda.synchronize()
            o = oracle.query(obj, rays, debug=True)
            want, scale = o["enc"].sum(1), np.abs(o["enc"]).sum(1)
            got = sums.cpu().numpy().astype(np.float64)
            tol = (1e-5 if feat == "fp32" else 4 * U[feat]) * scale + 1e-30
            bad = np.abs(got - want) > tol
            assert not bad.any(), (int(bad.sum()), float(np.abs(got - want)[bad].max()))
            assert (np.abs(want) > 0).sum() > 100
        finally:
            L.lsnif_release(ctx, oid)


def test_width_limits_rejected(L, ctx):
    """Width 128 runs on the matrix cores for at most 32 inputs per point (2 K blocks);
    widths other than 64 and 128 have no kernel."""
    from tests.test_oracle_pins import tiny_object
    occ = np.ones(16 ** 3, bool)
    wide = tiny_object(16, occ, L=9, F=3, log2_T=10, R=[16 + 8 * i for i in range(9)], H=4, width=128,
                       n_hidden=1)
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_build(ctx, L.ObjectDesc(wide, "fp16", "fp16"))
    assert e.value.status == L.LSNIF_E_INVALID and "width 128" in L.lsnif_last_error()
    oid = L.lsnif_build(ctx, L.ObjectDesc(wide, "fp32", "fp32"))   # the FP32 path has no such limit
    L.lsnif_release(ctx, oid)
    odd = tiny_object(16, occ, L=2, F=2, log2_T=10, R=[16, 32], H=4, width=96, n_hidden=1)
    with pytest.raises(L.LsnifError):
        L.lsnif_build(ctx, L.ObjectDesc(odd, "fp32", "fp32"))


def test_level_beyond_offset_range_rejected(L, ctx):
    """The gathers address a level with 32-bit byte offsets: 2^30 entries of two fp32
    features (8 GiB a level) are refused before any table is read or allocated."""
    d = L.ObjectDesc(W.configs.c1_object(), "fp32", "fp32")
    d.d.log2_T = 30
    with pytest.raises(L.LsnifError) as e:
        L.lsnif_build(ctx, d)
    assert e.value.status == L.LSNIF_E_INVALID and "4 GiB" in L.lsnif_last_error()


def test_batch_invariance(L, ctx, c1):
    """A ray's result does not depend on its neighbours: shuffled batches agree bit for bit."""
    obj, rays = c1["objects"][0], c1["rays"]
    for feat, mlp in (("fp32", "fp32"), ("fp16", "fp16")):
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
        try:
            a = gpu_query(L, ctx, oid, rays)
            perm = np.random.default_rng(1).permutation(len(rays))
            b = gpu_query(L, ctx, oid, rays[perm])
            inv = np.argsort(perm)
            for k in ("hit", "t", "normal", "material"):
                assert bitwise_equal(a[k], b[k][inv]), k
        finally:
            L.lsnif_release(ctx, oid)


def test_linear_exactness_on_gpu(L, ctx):
    """A dense level holding A v + b interpolates A x + b on the GPU (float32 rounding)."""
    from tests.test_oracle_pins import tiny_object, adversarial_rays
    V, R, F = 8, 12, 2
    side = R + 1
    rng = np.random.default_rng(7)
    A = np.round(rng.uniform(-1, 1, (F, 3)) * 64) / 64
    b = np.round(rng.uniform(-1, 1, F) * 64) / 64
    v = np.arange(side ** 3)
    verts = np.stack([v % side, (v // side) % side, v // (side * side)], 1)
    tab = np.zeros((1, 1 << 12, F), np.float32)
    tab[0, : side ** 3] = (verts @ A.T + b).astype(np.float32)
    occ = np.random.default_rng(8).uniform(size=V ** 3) < 0.5
    obj = tiny_object(V, occ, L=1, F=F, log2_T=12, R=[R], tables=tab, H=18, width=64, n_hidden=3)
    rays = adversarial_rays(np.random.default_rng(9), V, 200)
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        n = 0
        for i in range(len(rays)):
            for h in range(max(g["count"][i], 0)):
                x = np.clip((g["points"][i, h] * (np.float32(R) / np.float32(V))).astype(np.float32), 0, R)
                want = A @ x.astype(np.float64) + b
                got = g["enc"][i, h * F:(h + 1) * F]
                assert np.allclose(got, want, rtol=0, atol=2e-5 * max(1.0, np.abs(want).max())), (got, want)
                n += 1
        assert n > 500
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("mlp", ["fp32", "fp16"])
def test_debug_buffer_subsets(L, ctx, c1, mlp):
    """Any subset of the debug buffers may be passed; a count-only call matches a full one."""
    import torch
    obj, rays_np = c1["objects"][0], c1["rays"]
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, mlp, mlp))
    try:
        full = gpu_query(L, ctx, oid, rays_np, debug=True, obj=obj)
        rays = torch.from_numpy(rays_np).cuda()
        out = torch.empty((len(rays_np), 6), dtype=torch.float32, device="cuda")
        for keys in (("count",), ("tatb",), ("out",), ("count", "out")):
            bufs = {}
            if "count" in keys:
                bufs["count"] = torch.full((len(rays_np),), -7, dtype=torch.int32, device="cuda")
            if "tatb" in keys:
                bufs["tatb"] = torch.zeros((len(rays_np), 2), dtype=torch.float32, device="cuda")
            if "out" in keys:
                bufs["out"] = torch.zeros((len(rays_np), obj.out_dim), dtype=torch.float32, device="cuda")
            L.lsnif_query_debug(ctx, oid, rays, out, bufs)
            torch.cuda.synchronize()
            for k, v in bufs.items():
                assert bitwise_equal(v.cpu().numpy(), full[k]), (keys, k)
    finally:
        L.lsnif_release(ctx, oid)


@pytest.mark.parametrize("mlp", ["fp32", "fp16"])
def test_grazing_recheck_parity(L, ctx, mlp):
    """With the float64 grazing recheck on, voxel lists, points and slots equal the oracle's
    bit for bit on rays aimed at lattice edges, and some lists differ from the float32 ones."""
    import dataclasses
    from tests.test_oracle_pins import tiny_object, edge_grazing_rays
    V = 8
    rng = np.random.default_rng(7)
    occ = rng.uniform(size=V ** 3) < 0.8
    base = tiny_object(V, occ, H=48, L=2, F=2, R=[V, 2 * V], log2_T=10, width=64, n_hidden=3,
                       bmin=(0, 0, 0), bmax=(V, V, V), seed=3)
    rays = edge_grazing_rays(rng, V, 2048)
    feat = "fp32" if mlp == "fp32" else "fp16"
    counts = {}
    for recheck in (0, 1):
        obj = dataclasses.replace(base, grazing_recheck=recheck)
        _say(f"grazing recheck={recheck} {feat}/{mlp}: {len(rays)} rays")
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
        try:
            g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
            o = oracle.query(obj, rays, debug=True)
            check_intermediates(g, o, obj)
            counts[recheck] = o["vox_ijk"].copy()
        finally:
            L.lsnif_release(ctx, oid)
    changed = np.any(counts[0] != counts[1], axis=(1, 2)).sum()
    assert changed >= 20, changed


@pytest.mark.parametrize("width,H", [(128, 18), (64, 10), (64, 18)])
@pytest.mark.parametrize("feat,mlp", [("fp32", "fp32"), ("fp16", "fp16"), ("fp16", "bf16")])
def test_paper_shaped_object_parity(L, ctx, c1, feat, mlp, width, H):
    """An object shaped like the paper's default (Sec. 5.1): V = 32 surface voxels, two
    face-aligned hashed levels (R = 64, 128; 2^17 entries) of 3 features, a 2-hidden-layer
    leaky-ReLU MLP and the albedo head (8 + 4 outputs): width 128 with H = 18 points (the
    paper's default), width 64 with H = 10 (its low-quality variant, Sec. 6.4), and width
    64 with H = 18.  Exercises the F = 3 gathers, the 4-corner collapse on both levels,
    leaky ReLU, the albedo outputs, the width-128 kernels and the shorter point cap."""
    from tests.test_oracle_pins import tiny_object
    base = c1["objects"][0]
    occ = np.unpackbits(base.occ.view(np.uint8), bitorder="little").astype(bool)[: base.V ** 3]
    obj = tiny_object(base.V, occ, L=2, F=3, log2_T=17, R=[64, 128], H=H, width=width, n_hidden=2,
                      n_mat=4, has_albedo=1, act=1, bmin=tuple(base.bmin), bmax=tuple(base.bmax), seed=21)
    obj.tables *= np.float32(1e-2)
    assert obj.out_dim == 12
    rays = c1["rays"]
    _say(f"paper-shaped object {feat}/{mlp} width {width} H {H}: {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, feat, mlp))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
        u = max(U[feat], U[mlp])
        enc_compare(g["enc"], o["enc"], obj, o["count"], 1e-6 if mlp == "fp32" else 4 * u)
        cand = o["count"] > 0
        ob = output_bound(obj, o["enc"], u)
        # every raw output (albedo logits included) within its forward-error bound (x4 slack)
        err = np.abs(g["out"][cand].astype(np.float64) - o["out"][cand])
        assert np.all(err <= 4 * ob[cand] + 1e-30), float((err / np.maximum(ob[cand], 1e-30)).max())
        # hit-t, normal-angle and visibility bars by the MLP type's unit roundoff, as for c1
        t_rel, n_ang, vis = {"fp32": (1e-5, 1e-4, 0.9999), "fp16": (1e-3, 1e-2, 0.999),
                             "bf16": (1e-2, 1e-1, 0.99)}[mlp]
        st = compare_hits(g, o, o["tatb"], o["enc"], o["out"], obj, u, t_rel, n_ang, vis)
        _say(str(st))
        assert st["ok"], st
    finally:
        L.lsnif_release(ctx, oid)


def sparse_blobs(rng, V, n_blobs):
    occ3 = np.zeros((V, V, V), bool)
    for _ in range(n_blobs):
        cx, cy, cz = rng.integers(0, V, 3)
        r = int(rng.integers(1, 4))
        sl = (slice(max(cx - r, 0), cx + r), slice(max(cy - r, 0), cy + r), slice(max(cz - r, 0), cz + r))
        occ3[sl] = rng.uniform(size=occ3[sl].shape) < 0.7
    return occ3.transpose(2, 1, 0).ravel()          # bit x + V (y + V z)


@pytest.mark.parametrize("V", [16, 32, 64])
def test_sparse_grid_walk_parity(L, ctx, V):
    """Grids that are mostly empty bricks (the walk crosses an empty 4x4x4 brick in one step):
    voxel lists, points and slots equal the oracle's bit for bit on adversarial rays."""
    from tests.test_oracle_pins import tiny_object, adversarial_rays
    rng = np.random.default_rng(40 + V)
    occ = sparse_blobs(rng, V, max(2, V // 8))
    obj = tiny_object(V, occ, H=48, L=2, F=2, R=[V, 2 * V], log2_T=12, width=64, n_hidden=1, seed=V)
    rays = adversarial_rays(rng, V, n_random=1500)
    _say(f"sparse grid V={V}: {occ.sum()} occupied voxels, {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
        assert (o["count"] > 0).sum() > 100
    finally:
        L.lsnif_release(ctx, oid)


def test_large_sparse_object_walk_parity(L, ctx):
    """A V = 256 c4 object (mostly empty bricks) with its own balanced rays: bit-exact lists."""
    obj = W.configs.c4_object(3)
    assert obj.V == 256
    from workloads.rays import balanced_rays
    from workloads.rng import streams, RAYS
    verts, tris = W.configs.c4_mesh(3)
    rays = balanced_rays(streams(777)[RAYS], verts, tris, 3000, obj.bmin.astype(np.float64),
                         obj.bmax.astype(np.float64))
    _say(f"c4 object 3 (V={obj.V}): {len(rays)} rays")
    oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
    try:
        g = gpu_query(L, ctx, oid, rays, debug=True, obj=obj)
        o = oracle.query(obj, rays, debug=True)
        check_intermediates(g, o, obj)
    finally:
        L.lsnif_release(ctx, oid)
