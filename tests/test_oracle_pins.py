"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a
brute-force all-voxel slab test, closed forms (linear functions interpolate
exactly; vertices are reproduced exactly), the analytic +-identity network,
BLAS matrix products, and invariants (rays that meet no occupied voxel miss).
"""

import numpy as np
import pytest

import oracle
import workloads as W
from workloads.objects import LsnifObject, make_weights
from tests.bruteforce import voxel_list, recheck_sets

f32 = np.float32
HASH_PRIMES = (1, 2654435761, 805459861)   # Mueller et al. 2022, Eq. 4


def tiny_object(V, occ_bool, *, L=1, F=2, log2_T=10, R=None, H=18, weights=None, tables=None,
                bmin=(-1.0, -1.0, -1.0), bmax=(1.0, 1.0, 1.0), seed=0, width=8, n_hidden=2,
                n_mat=4, has_albedo=0, act=0):
    rng = np.random.default_rng(seed)
    if R is None:
        R = [V] * L
    T = 1 << log2_T
    if tables is None:
        tables = rng.uniform(-1, 1, (L, T, F)).astype(f32)
    if weights is None:
        dims = [H * L * F] + [width] * n_hidden + [5 + 3 * has_albedo + n_mat]
        weights = make_weights(rng, dims)
    return LsnifObject(bmin=np.asarray(bmin, f32), bmax=np.asarray(bmax, f32), V=V,
                       occ=W.pack_bits(occ_bool), L=L, F=F, log2_T=log2_T,
                       R=np.asarray(R, np.int32), tables=tables, H=H, weights=weights,
                       act=act, n_mat=n_mat, has_albedo=has_albedo)


def adversarial_rays(rng, V, n_random=300):
    """Random rays plus rays along axes, through edges and corners, along faces and from inside."""
    rays = []
    for _ in range(n_random):
        o = rng.uniform(-2, 2, 3)
        tgt = rng.uniform(-1, 1, 3)
        d = tgt - o
        rays.append([*o, *(d / np.linalg.norm(d)), 0.0, np.inf])
    g = 2.0 / V                        # voxel size in object space for a [-1,1] box
    for _ in range(n_random // 3):
        # origin on a lattice point, direction with zeros / equal components
        o = -1.0 + g * rng.integers(-2, V + 3, 3).astype(float)
        d = rng.integers(-2, 3, 3).astype(float)
        if not d.any():
            d[rng.integers(3)] = 1.0
        rays.append([*o, *d, 0.0, np.inf])
        # inside the grid, random direction, tmin inside the segment
        o2 = rng.uniform(-1, 1, 3)
        d2 = rng.standard_normal(3)
        rays.append([*o2, *d2, rng.uniform(-0.5, 0.5), np.inf])
        # along a face plane: one coordinate on a lattice plane with zero direction
        o3 = rng.uniform(-1.5, 1.5, 3)
        a = rng.integers(3)
        o3[a] = -1.0 + g * rng.integers(0, V + 1)
        d3 = rng.standard_normal(3)
        d3[a] = 0.0
        rays.append([*o3, *d3, 0.0, np.inf])
    # exact diagonals through corners
    for s in [(1, 1, 1), (1, -1, 1), (-1, -1, -1), (1, 1, 0), (0, 1, 1), (1, 0, 0)]:
        s = np.asarray(s, float)
        rays.append([*(-1.5 * s + 1e-9 * 0), *s, 0.0, np.inf])
        rays.append([*(-2.0 * s), *s, 0.0, np.inf])
    return np.asarray(rays, dtype=f32)


@pytest.mark.parametrize("V", [1, 2, 4, 8, 16])
def test_walk_equals_bruteforce(V):
    """The voxel walk lists exactly the voxels the all-voxel slab test keeps, bit for bit."""
    rng = np.random.default_rng(100 + V)
    occ = rng.uniform(size=V ** 3) < 0.35
    H = 2 * V * 3 if V <= 16 else 18
    H = min(H, 96)
    obj = tiny_object(V, occ, H=H, L=1, F=1, width=2, n_hidden=1)
    rays = adversarial_rays(rng, V)
    r = oracle.query(obj, rays, debug=True)
    for i, ray in enumerate(rays):
        ref = voxel_list(ray, occ, V, obj.bmin, obj.bmax, H)
        if ref is None:
            assert r["count"][i] == -1
            continue
        vox = ref["vox"]
        assert r["count"][i] == 2 * len(vox), (i, ray)
        for j, (ijk, tin, tout, ia, oa) in enumerate(vox):
            assert tuple(r["vox_ijk"][i, j]) == ijk, (i, j)
            assert r["vox_t"][i, j, 0].tobytes() == tin.tobytes()
            assert r["vox_t"][i, j, 1].tobytes() == tout.tobytes()
            assert tuple(r["vox_axis"][i, j]) == (ia, oa)
        if ref["ta"] is not None and len(vox) > 0:
            assert r["tatb"][i, 0] == ref["ta"] and r["tatb"][i, 1] == ref["tb"]


def test_walk_cap_takes_first_voxels():
    """With more occupied voxels than H/2 only the first H/2 along the ray are kept."""
    V = 16
    occ = np.ones(V ** 3, bool)
    obj = tiny_object(V, occ, H=6, L=1, F=1, width=2, n_hidden=1)
    ray = np.array([[-2.0, 0.03, 0.01, 1.0, 0.0, 0.0, 0.0, np.inf]], f32)
    r = oracle.query(obj, ray, debug=True)
    assert r["count"][0] == 6
    assert [tuple(v) for v in r["vox_ijk"][0]] == [(0, 8, 8), (1, 8, 8), (2, 8, 8)]


def test_axis_ray_crosses_V_cells():
    """An axis-parallel ray through the interior of a full grid crosses exactly V cells."""
    V = 8
    occ = np.ones(V ** 3, bool)
    obj = tiny_object(V, occ, H=2 * V, L=1, F=1, width=2, n_hidden=1)
    ray = np.array([[0.1, -3.0, 0.37, 0.0, 1.0, 0.0, 0.0, np.inf]], f32)
    r = oracle.query(obj, ray, debug=True)
    assert r["count"][0] == 2 * V
    assert [v[1] for v in r["vox_ijk"][0]] == list(range(V))


def test_points_on_boundaries_of_occupied_voxels():
    """Every point lies on a face of its voxel (integer coordinate on the crossing axis) and inside it."""
    c = W.configs.c1()
    obj = c["objects"][0]
    r = oracle.query(obj, c["rays"][:1000], debug=True)
    occ = W.unpack_bits(obj.occ, obj.V ** 3)
    V = obj.V
    for i in range(1000):
        for h in range(max(r["count"][i], 0)):
            j = h // 2
            ijk = r["vox_ijk"][i, j]
            p = r["points"][i, h]
            assert occ[ijk[0] + V * (ijk[1] + V * ijk[2])]
            assert np.all(p >= ijk) and np.all(p <= ijk + 1)
            face = r["vox_axis"][i, j, h & 1]
            assert p[face] == np.floor(p[face]) and p[face] in (ijk[face], ijk[face] + 1)


def test_dense_level_linear_exactness():
    """A dense level whose table holds A v + b interpolates A x + b exactly (float64 rounding)."""
    V, R, F = 8, 12, 3
    side = R + 1
    assert side ** 3 <= 1 << 12
    rng = np.random.default_rng(7)
    # coefficients on a dyadic grid so that float32 stores A v + b exactly
    A = np.round(rng.uniform(-1, 1, (F, 3)) * 64) / 64
    b = np.round(rng.uniform(-1, 1, F) * 64) / 64
    v = np.arange(side ** 3)
    verts = np.stack([v % side, (v // side) % side, v // (side * side)], 1)
    lin = verts @ A.T + b
    tab = np.zeros((1, 1 << 12, F), f32)
    tab[0, : side ** 3] = lin.astype(f32)
    assert np.all(tab[0, : side ** 3].astype(np.float64) == lin)
    occ = np.random.default_rng(8).uniform(size=V ** 3) < 0.5
    obj = tiny_object(V, occ, L=1, F=F, log2_T=12, R=[R], tables=tab, H=18)
    rays = adversarial_rays(np.random.default_rng(9), V, 200)
    r = oracle.query(obj, rays, debug=True)
    n = 0
    for i in range(len(rays)):
        for h in range(max(r["count"][i], 0)):
            # level coordinate as the method forms it: float32 product, clamped to [0, R]
            x = np.clip((r["points"][i, h] * (f32(R) / f32(V))).astype(f32), 0, R).astype(np.float64)
            want = A @ x + b
            got = r["enc"][i, h * F:(h + 1) * F]
            assert np.allclose(got, want, rtol=0, atol=1e-12), (got, want, x)
            n += 1
    assert n > 500


def test_vertices_reproduced_and_partition_of_unity():
    """At a grid vertex the feature equals that vertex's entry; the 8 weights sum to one."""
    V, R, F = 4, 8, 2
    rng = np.random.default_rng(3)
    occ = np.ones(V ** 3, bool)
    ones = np.ones((1, 1 << 12, F), f32)
    obj = tiny_object(V, occ, L=1, F=F, log2_T=12, R=[R], tables=ones, H=8)
    rays = adversarial_rays(rng, V, 100)
    r = oracle.query(obj, rays, debug=True)
    m = r["count"] > 0
    for i in np.nonzero(m)[0]:
        c = r["count"][i]
        assert np.allclose(r["enc"][i, : c * F], 1.0, rtol=0, atol=1e-15)
    # axis-parallel ray through lattice-aligned coordinates: points land on vertices
    tab = rng.uniform(-1, 1, (1, 1 << 12, F)).astype(f32)
    obj = tiny_object(V, occ, L=1, F=F, log2_T=12, R=[R], tables=tab, H=8)
    ray = np.array([[-2.0, -1.0 + 2.0 * 3 / 8, -1.0 + 2.0 * 5 / 8, 1, 0, 0, 0, np.inf]], f32)
    r = oracle.query(obj, ray, debug=True)
    side = R + 1
    for h in range(r["count"][0]):
        p = r["points"][0, h] * f32(R / V)
        vx, vy, vz = (int(round(x)) for x in p)
        assert np.all(p == np.round(p))
        slot = vx + side * (vy + side * vz)
        assert np.array_equal(r["enc"][0, h * F:(h + 1) * F], tab[0, slot].astype(np.float64))


def test_dense_slots_are_a_bijection():
    """Dense levels map the (R+1)^3 vertices one to one onto [0, (R+1)^3)."""
    V, R = 4, 6
    occ = np.ones(V ** 3, bool)
    obj = tiny_object(V, occ, L=1, F=1, log2_T=10, R=[R], H=8)
    rays = adversarial_rays(np.random.default_rng(5), V, 400)
    r = oracle.query(obj, rays, debug=True)
    side = R + 1
    seen = {}
    for i in range(len(rays)):
        for h in range(max(r["count"][i], 0)):
            x = np.clip(r["points"][i, h] * f32(R / V), 0, R)
            base = np.minimum(np.floor(x), R - 1).astype(int)
            for c in range(8):
                v = tuple(base + [(c >> k) & 1 for k in range(3)])
                s = int(r["slots"][i, h, 0, c])
                assert 0 <= s < side ** 3
                assert seen.setdefault(v, s) == s
    vals = list(seen.values())
    assert len(set(vals)) == len(vals)


def test_hashed_slots_follow_published_hash():
    """Hashed levels: slots xor-decompose per axis with the published primes, x-neighbours
    differ exactly as their coordinates do, and the origin vertex maps to slot 0."""
    V, R, log2_T = 4, 64, 8
    T = 1 << log2_T
    occ = np.ones(V ** 3, bool)
    obj = tiny_object(V, occ, L=1, F=1, log2_T=log2_T, R=[R], H=8)
    rays = adversarial_rays(np.random.default_rng(6), V, 200)
    rays = np.concatenate([rays, np.array([[-1.0 - 1e-3, -1.0, -1.0, 1, 1e-3, 1e-3, 0, np.inf]], f32)])
    r = oracle.query(obj, rays, debug=True)
    n = 0
    for i in range(len(rays)):
        for h in range(max(r["count"][i], 0)):
            x = np.clip(r["points"][i, h] * f32(R / V), 0, R)
            base = np.minimum(np.floor(x), R - 1).astype(np.int64)
            s = r["slots"][i, h, 0].astype(np.int64)
            for c in range(8):
                v = base + [(c >> k) & 1 for k in range(3)]
                parts = [(int(v[k]) * HASH_PRIMES[k]) % (1 << 32) for k in range(3)]
                assert s[c] == (parts[0] ^ parts[1] ^ parts[2]) % T
            assert s[1] ^ s[0] == ((base[0] + 1) ^ base[0]) % T
            if np.all(base == 0):
                assert s[0] == 0 and s[1] == 1 and s[2] == HASH_PRIMES[1] % T
                assert s[4] == HASH_PRIMES[2] % T
            n += 1
    assert n > 100


def test_aligned_level_face_weight_is_binary():
    """On a level with R a multiple of V the crossing-axis weight is exactly 0 or 1, so only the
    4 corners of the face matter (the sparse-grid claim of Sec. 3.2)."""
    V, R = 8, 32
    occ = np.random.default_rng(1).uniform(size=V ** 3) < 0.4
    obj = tiny_object(V, occ, L=1, F=2, log2_T=10, R=[R], H=18)
    rays = adversarial_rays(np.random.default_rng(2), V, 300)
    r = oracle.query(obj, rays, debug=True)
    n = 0
    for i in range(len(rays)):
        for h in range(max(r["count"][i], 0)):
            face = r["vox_axis"][i, h // 2, h & 1]
            w = r["weights"][i, h, 0, face]
            assert w == 0.0 or w == 1.0
            n += 1
    assert n > 300


def test_mlp_matches_blas():
    """The float64 loop network equals numpy's BLAS product chain to 1e-12."""
    c = W.configs.c1()
    obj = c["objects"][0]
    r = oracle.query(obj, c["rays"][:512], debug=True)
    x = r["enc"].T
    Ws = [w.astype(np.float64) for w in obj.weights]
    for k, Wk in enumerate(Ws):
        x = Wk @ x
        if k < len(Ws) - 1:
            x = np.maximum(x, 0.0)
    m = r["count"] > 0
    got = r["out"][m]
    want = x.T[m]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15 * np.abs(want).max())
    assert np.all(r["out"][~m] == 0)


def test_leaky_relu_network_matches_blas():
    V = 8
    occ = np.random.default_rng(4).uniform(size=V ** 3) < 0.5
    obj = tiny_object(V, occ, L=2, F=2, R=[4, 8], H=10, width=16, n_hidden=2, act=1)
    obj.leaky_slope = 0.01
    rays = adversarial_rays(np.random.default_rng(4), V, 200)
    r = oracle.query(obj, rays, debug=True)
    x = r["enc"].T
    for k, w in enumerate(obj.weights):
        x = w.astype(np.float64) @ x
        if k < len(obj.weights) - 1:
            x = np.where(x > 0, x, np.float64(np.float32(0.01)) * x)
    m = r["count"] > 0
    assert np.allclose(r["out"][m], x.T[m], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("act", [0, 1])
def test_layer_inputs_and_act_amax(act):
    """oracle.layer_inputs ends in the C oracle's own raw outputs (1e-12), for ReLU and leaky
    ReLU; act_amax takes each layer's largest |input| over the candidate rays, so its first
    entry is the largest |encoding| and the others are positive (ReLU outputs of a
    Kaiming-initialised network on nonzero encodings)."""
    V = 8
    occ = np.random.default_rng(7).uniform(size=V ** 3) < 0.5
    obj = tiny_object(V, occ, L=2, F=2, R=[4, 8], H=10, width=16, n_hidden=2, act=act)
    obj.leaky_slope = 0.01
    rays = adversarial_rays(np.random.default_rng(7), V, 200)
    r = oracle.query(obj, rays, debug=True)
    m = r["count"] > 0
    xs, out = oracle.layer_inputs(obj, r["enc"][m])
    assert len(xs) == len(obj.weights)
    assert [x.shape[1] for x in xs] == [w.shape[1] for w in obj.weights]
    assert np.allclose(out, r["out"][m], rtol=1e-12, atol=1e-13 * np.abs(r["out"][m]).max())
    amax = oracle.act_amax(obj, rays, chunk=97)
    assert amax[0] == np.abs(r["enc"][m]).max()
    assert np.all(amax > 0)
    assert np.allclose(amax, [np.abs(x).max() for x in xs], rtol=0, atol=0)


def test_miss_invariants():
    """No occupied voxel on the ray -> miss, whatever the weights; zero network -> miss."""
    V = 8
    empty = np.zeros(V ** 3, bool)
    obj = tiny_object(V, empty)
    rays = adversarial_rays(np.random.default_rng(11), V, 200)
    r = oracle.query(obj, rays)
    assert r["hit"].sum() == 0 and np.all(r["count"] <= 0)
    assert np.all(np.isinf(r["t"])) and np.all(r["material"] == -1)
    # one occupied voxel; rays that pass beside it miss even with a network biased to "hit"
    one = np.zeros(V ** 3, bool)
    one[3 + V * (3 + V * 3)] = True
    obj = tiny_object(V, one, L=1, F=1, H=4, width=2, n_hidden=1,
                      weights=[np.ones((2, 4), f32), np.ones((9, 2), f32)],
                      tables=np.ones((1, 1 << 10, 1), f32))
    side_rays = np.array([[-2, 0.9, 0.9, 1, 0, 0, 0, np.inf], [-2, -0.9, 0.3, 1, 0, 0, 0, np.inf],
                          [0.0, -2, 0.9, 0, 1, 0, 0, np.inf]], f32)
    r = oracle.query(obj, side_rays)
    assert r["hit"].sum() == 0
    through = np.array([[-2, -0.1, -0.1, 1, 0, 0, 0, np.inf]], f32)   # voxel 3 spans [-0.25, 0)
    r = oracle.query(obj, through)
    assert r["count"][0] == 2 and r["hit"][0] == 1
    # zero weights: logit 0 is not > 0, so a miss
    obj0 = tiny_object(V, np.ones(V ** 3, bool), weights=make_zero_weights(18 * 1 * 2, 8, 9))
    r = oracle.query(obj0, rays)
    assert r["hit"].sum() == 0


def make_zero_weights(i, w, o):
    return [np.zeros((w, i), f32), np.zeros((w, w), f32), np.zeros((o, w), f32)]


def test_invalid_rays_miss():
    V = 4
    obj = tiny_object(V, np.ones(V ** 3, bool))
    bad = np.array([[np.nan, 0, 0, 1, 0, 0, 0, np.inf], [0, 0, 0, 0, 0, 0, 0, np.inf],
                    [0, 0, 0, 1, 0, 0, 2, 1], [np.inf, 0, 0, 1, 0, 0, 0, np.inf],
                    [0, 0, 0, 1, np.inf, 0, 0, np.inf], [0, 0, 0, 1, 0, 0, np.nan, np.inf]], f32)
    r = oracle.query(obj, bad)
    assert np.all(r["count"] == -1) and r["hit"].sum() == 0


def identity_network(L, F, H, width=8, n_mat=4):
    """+-identity construction: normal head = point 0's first three features,
    occlusion logit = their sum, t logit = 0, material logit k = feature k (k < 3), -sum for k = 3."""
    in_dim = H * L * F
    W1 = np.zeros((width, in_dim), f32)
    for a in range(3):
        W1[a, a] = 1.0
        W1[3 + a, a] = -1.0
    W2 = np.eye(width, dtype=f32)
    out = np.zeros((5 + n_mat, width), f32)
    out[0, 0:3] = 1.0
    out[0, 3:6] = -1.0
    for a in range(3):
        out[2 + a, a] = 1.0
        out[2 + a, 3 + a] = -1.0
        out[5 + a, a] = 1.0
        out[5 + a, 3 + a] = -1.0
    out[8, 0:3] = -1.0
    return [W1, W2, out]


def test_end_to_end_identity_network():
    """One dense level with R = V and table[v] = v: the network returns the first entry point.

    The expected normal is normalize(entry point of the first occupied voxel), the hit
    distance is the midpoint of [ta, tb], the material is the largest coordinate -- all
    derived from the brute-force voxel list, with no oracle intermediate."""
    V = 8
    R = V
    side = R + 1
    v = np.arange(side ** 3)
    tab = np.zeros((1, 1 << 10, 3), f32)
    tab[0, : side ** 3] = np.stack([v % side, (v // side) % side, v // (side * side)], 1)
    rng = np.random.default_rng(21)
    occ = rng.uniform(size=V ** 3) < 0.3
    obj = tiny_object(V, occ, L=1, F=3, log2_T=10, R=[R], H=6, tables=tab,
                      weights=identity_network(1, 3, 6))
    rays = adversarial_rays(rng, V, 300)
    r = oracle.query(obj, rays)
    checked = 0
    for i, ray in enumerate(rays):
        ref = voxel_list(ray, occ, V, obj.bmin, obj.bmax, 6)
        if ref is None or not ref["vox"]:
            assert r["hit"][i] == 0
            continue
        ijk, tin, tout, ia, oa = ref["vox"][0]
        o, d = ref["o"], ref["d"]
        p = np.empty(3)
        for b in range(3):
            if b == ia:
                p[b] = ijk[b] if d[b] > 0 else ijk[b] + 1
            else:
                p[b] = np.clip(f32(o[b] + f32(tin * d[b])), ijk[b], ijk[b] + 1)
        if p.sum() <= 0 or ray[7] < ref["ta"]:
            continue
        t_mid = np.float64(ref["ta"]) + 0.5 * (np.float64(ref["tb"]) - np.float64(ref["ta"]))
        assert r["hit"][i] == 1
        assert np.allclose(r["normal"][i], p / np.linalg.norm(p), atol=1e-6)
        assert r["t"][i] == np.float32(t_mid)
        assert r["material"][i] == int(np.argmax(p))
        checked += 1
    assert checked > 100


def test_decode_semantics_c1():
    """Hit iff points > 0, occlusion logit > 0 and t <= tmax; t inside [ta, tb]; unit normals."""
    c = W.configs.c1()
    r = oracle.query(c["objects"][0], c["rays"])
    out, cnt = r["out"], r["count"]
    expect = (cnt > 0) & (out[:, 0] > 0)
    assert np.array_equal(r["hit"].astype(bool), expect)       # tmax = inf here
    h = r["hit"] == 1
    ta, tb = r["tatb"][h, 0], r["tatb"][h, 1]
    assert np.all(r["t"][h] >= ta * (1 - 1e-6)) and np.all(r["t"][h] <= tb * (1 + 1e-6))
    assert np.allclose(np.linalg.norm(r["normal"][h], axis=1), 1.0, atol=1e-6)
    assert np.array_equal(r["material"][h], np.argmax(out[h, 5:9], axis=1))
    assert np.all(r["material"][~h] == -1) and np.all(np.isinf(r["t"][~h]))


def test_tmax_filters_hits():
    c = W.configs.c1()
    rays = c["rays"].copy()
    r0 = oracle.query(c["objects"][0], rays)
    h = r0["hit"] == 1
    rays[:, 7] = r0["t"] - 1e-3
    rays[~h, 7] = np.inf
    r1 = oracle.query(c["objects"][0], rays)
    assert r1["hit"][h].sum() == 0
    assert np.array_equal(r1["hit"][~h], r0["hit"][~h])


def test_pairs_nearest_hit_matches_bruteforce():
    """Nearest hit over instances equals the min over per-instance single-object queries."""
    V = 8
    rng = np.random.default_rng(31)
    objs = [tiny_object(V, rng.uniform(size=V ** 3) < 0.3, seed=s, L=2, F=2, R=[4, 8], H=8)
            for s in range(2)]
    insts = []
    for k in range(5):
        ang = rng.uniform(0, 2 * np.pi)
        sc = rng.uniform(0.8, 1.2)
        A = np.array([[np.cos(ang), 0, -np.sin(ang)], [0, 1, 0], [np.sin(ang), 0, np.cos(ang)]]) / sc
        t = rng.uniform(-0.5, 0.5, 3)
        insts.append((k % 2, np.concatenate([A, t[:, None]], 1).astype(f32)))
    rays = adversarial_rays(rng, V, 200)
    n = len(rays)
    pr = np.repeat(np.arange(n), len(insts)).astype(np.uint32)
    pi = np.tile(np.arange(len(insts)), n).astype(np.uint32)
    r = oracle.query_pairs(objs, insts, rays, pr, pi)
    best_t = np.full(n, np.inf, f32)
    best_i = np.full(n, -1)
    for k, (oi, m) in enumerate(insts):
        A, b = m[:, :3], m[:, 3]
        ro = rays.copy()
        for a in range(3):
            ro[:, a] = ((A[a, 0] * rays[:, 0] + A[a, 1] * rays[:, 1]) + A[a, 2] * rays[:, 2]) + b[a]
            ro[:, 3 + a] = (A[a, 0] * rays[:, 3] + A[a, 1] * rays[:, 4]) + A[a, 2] * rays[:, 5]
        q = oracle.query(objs[oi], ro)
        better = (q["hit"] == 1) & (q["t"] < best_t)
        best_t[better] = q["t"][better]
        best_i[better] = k
    assert np.array_equal(r["winner"], best_i)
    assert np.array_equal(r["t"][best_i >= 0], best_t[best_i >= 0])
    assert np.all(r["hit"] == (best_i >= 0))


def edge_grazing_rays(rng, V, n):
    """Rays aimed within 1e-7.5 .. 1e-5 voxels of a lattice edge inside the grid (object space is
    voxel space here), so float32 and float64 can disagree on the cells at the edge."""
    rays = []
    for _ in range(n):
        p = rng.integers(1, V, 3).astype(np.float64)
        p[rng.integers(3)] = rng.uniform(0.5, V - 0.5)
        p += rng.choice([-1, 1], 3) * 10 ** rng.uniform(-7.5, -5, 3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        o = p - rng.uniform(1.5, 3) * V * d
        rays.append([*o, *d, 0.0, np.inf])
    return np.asarray(rays, f32)


def test_grazing_recheck_against_bruteforce():
    """Optional float64 recheck of grazing voxels (off by default): against the all-voxel test
    in float32 and float64, every listed voxel is allowed and every required one is listed,
    in walk order; the recheck changes some lists, a walk that ignored it would fail, and so
    would one that dropped every grazing voxel."""
    V = 8
    rng = np.random.default_rng(7)
    occ = rng.uniform(size=V ** 3) < 0.8
    obj = tiny_object(V, occ, H=48, L=1, F=1, width=2, n_hidden=1, bmin=(0, 0, 0), bmax=(V, V, V))
    rays = edge_grazing_rays(rng, V, 3000)
    off = oracle.query(obj, rays, debug=True)
    obj.grazing_recheck = 1
    on = oracle.query(obj, rays, debug=True)
    changed = fp32_fails = grazing_required = 0
    for i, ray in enumerate(rays):
        s = recheck_sets(ray, occ, V, obj.bmin, obj.bmax)
        n = on["count"][i] // 2
        listed = [tuple(int(x) for x in v) for v in on["vox_ijk"][i, :n]]
        assert len(set(listed)) == len(listed), i
        assert set(listed) >= s["must"] and set(listed) <= s["may"], i
        assert np.all(np.diff(on["vox_t"][i, :n, 0]) >= 0), i
        n0 = off["count"][i] // 2
        l32 = {tuple(int(x) for x in v) for v in off["vox_ijk"][i, :n0]}
        fp32_fails += not (l32 >= s["must"] and l32 <= s["may"])
        changed += l32 != set(listed)
        grazing_required += len(s["must_grazing"])
    assert changed >= 50 and fp32_fails >= 10 and grazing_required >= 50


def vertex_table(R, F=3, log2_T=10):
    """One dense level whose entry for vertex (x, y, z) holds (x, y, z): the interpolated
    feature at a point is the point itself (in level units, which are voxel units for R = V)."""
    side = R + 1
    v = np.arange(side ** 3)
    tab = np.zeros((1, 1 << log2_T, F), f32)
    tab[0, : side ** 3, :3] = np.stack([v % side, (v // side) % side, v // (side * side)], 1)
    return tab


def first_entry_point(ref):
    """Entry point of the first listed voxel of a brute-force voxel list (voxel units): the
    crossing axis snapped to the face plane, the others clamped into the voxel."""
    ijk, tin, _, ia, _ = ref["vox"][0]
    o, d = ref["o"], ref["d"]
    p = np.empty(3)
    for b in range(3):
        if b == ia:
            p[b] = ijk[b] if d[b] > 0 else ijk[b] + 1
        else:
            p[b] = np.clip(f32(o[b] + f32(tin * d[b])), ijk[b], ijk[b] + 1)
    return p


def map_rays(rays, m):
    """World rays into an instance's object space, x = A x + b row by row in float32."""
    A, b = m[:, :3], m[:, 3]
    ro = rays.copy()
    for a in range(3):
        ro[:, a] = ((A[a, 0] * rays[:, 0] + A[a, 1] * rays[:, 1]) + A[a, 2] * rays[:, 2]) + b[a]
        ro[:, 3 + a] = (A[a, 0] * rays[:, 3] + A[a, 1] * rays[:, 4]) + A[a, 2] * rays[:, 5]
    return ro


def test_pairs_world_normal_is_inverse_transpose():
    """Sec. 4: the winning pair's normal returns to world space.  A normal is a covector, so
    with x_obj = A x_world + b it maps as normalize(A^T n_obj).  The +-identity network makes
    n_obj = normalize(first entry point) in closed form from the brute-force voxel list; A is a
    rotation times a non-uniform scale times a shear, so A n_obj would differ on almost every
    ray."""
    V = 8
    rng = np.random.default_rng(41)
    occ = rng.uniform(size=V ** 3) < 0.3
    obj = tiny_object(V, occ, L=1, F=3, log2_T=10, R=[V], H=6, tables=vertex_table(V),
                      weights=identity_network(1, 3, 6))
    c, s = np.cos(0.7), np.sin(0.7)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    A = rot @ np.diag([1.3, 0.7, 1.1]) @ np.array([[1.0, 0.4, 0.0], [0.0, 1.0, -0.3], [0.0, 0.0, 1.0]])
    m = np.concatenate([A, np.array([[0.1], [-0.2], [0.05]])], 1).astype(f32)
    Af = m[:, :3].astype(np.float64)
    rays = adversarial_rays(rng, V, 300)
    n = len(rays)
    r = oracle.query_pairs([obj], [(0, m)], rays, np.arange(n, dtype=np.uint32),
                           np.zeros(n, np.uint32))
    ro = map_rays(rays, m)
    checked = discriminating = 0
    for i in range(n):
        ref = voxel_list(ro[i], occ, V, obj.bmin, obj.bmax, 6)
        if ref is None or not ref["vox"]:
            assert r["hit"][i] == 0
            continue
        p = first_entry_point(ref)
        if p.sum() <= 0 or ro[i, 7] < ref["ta"]:
            continue
        assert r["hit"][i] == 1 and r["winner"][i] == 0
        n_obj = p / np.linalg.norm(p)
        want = Af.T @ n_obj
        want /= np.linalg.norm(want)
        assert np.allclose(r["normal"][i], want, atol=2e-6), (i, r["normal"][i], want)
        wrong = Af @ n_obj
        wrong /= np.linalg.norm(wrong)
        discriminating += np.abs(wrong - want).max() > 1e-2
        checked += 1
    assert checked > 100 and discriminating > 0.9 * checked


def test_local_hit_distance_sigmoid_direction():
    """Sec. 5.3: the hit distance is predicted on the ray's AABB interval [ta, tb] as
    t = ta + sigmoid(z_t) (tb - ta), so a positive logit moves the hit toward tb.  Here the
    t logit is k (p_x - p_y) for the first entry point p (known in closed form), which takes
    both signs; sigmoid(-z) or 1 - sigmoid(z) would put t on the other side of the midpoint."""
    V = 8
    rng = np.random.default_rng(43)
    occ = rng.uniform(size=V ** 3) < 0.3
    net = identity_network(1, 3, 6)
    k = 0.6
    net[2][1, :] = 0.0
    net[2][1, 0], net[2][1, 3] = k, -k          # +k x+ - k x-  = k p_x
    net[2][1, 1], net[2][1, 4] = -k, k          # -k y+ + k y-  = -k p_y
    obj = tiny_object(V, occ, L=1, F=3, log2_T=10, R=[V], H=6, tables=vertex_table(V), weights=net)
    rays = adversarial_rays(rng, V, 400)
    r = oracle.query(obj, rays)
    pos = neg = 0
    for i, ray in enumerate(rays):
        ref = voxel_list(ray, occ, V, obj.bmin, obj.bmax, 6)
        if ref is None or not ref["vox"]:
            continue
        p = first_entry_point(ref)
        if p.sum() <= 0 or ray[7] < ref["ta"]:
            continue
        z = k * (p[0] - p[1])
        ta, tb = np.float64(ref["ta"]), np.float64(ref["tb"])
        want = ta + (tb - ta) / (1.0 + np.exp(-z))
        assert r["hit"][i] == 1
        assert abs(np.float64(r["t"][i]) - want) <= 1e-6 * max(abs(want), tb - ta), (i, r["t"][i], want)
        if abs(z) > 0.3:
            flipped = ta + (tb - ta) / (1.0 + np.exp(z))
            assert abs(flipped - want) > 1e-3 * (tb - ta)
            pos += z > 0
            neg += z < 0
    assert pos > 30 and neg > 30
