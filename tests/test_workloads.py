"""Synthetic workloads: mesh construction, voxelisation against brute force, seeding."""

import numpy as np

import workloads as W
from workloads.meshes import face_normals
from workloads.voxelize import voxelize_brute


def test_icosphere_counts_and_radius():
    v, t = W.icosphere(3)
    assert t.shape == (1280, 3)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)


def test_uv_sphere_counts():
    v, t = W.uv_sphere(400, 250)
    assert t.shape[0] == 199_200


def test_meshes_wound_outwards():
    for v, t in [W.icosphere(2), W.uv_sphere(24, 12)]:
        n, _ = face_normals(v, t)
        assert np.all(np.einsum("ij,ij->i", n, v[t].mean(1)) > 0)


def test_voxelize_matches_bruteforce():
    """Bounding-box-culled SAT voxelisation equals testing every voxel against every triangle."""
    rng = np.random.default_rng(0)
    cases = [(W.icosphere(1), 8, [-1.1] * 3, [1.1] * 3),
             (W.torus(300), 8, [-1.0] * 3, [1.0] * 3),
             (W.box_soup(rng, 200, n_boxes=2), 6, [-0.6] * 3, [0.6] * 3),
             # a mesh whose vertices sit exactly on voxel faces
             ((np.array([[0, 0, 0], [0.5, 0, 0], [0, 0.5, 0]], float), np.array([[0, 1, 2]])),
              4, [-1.0] * 3, [1.0] * 3)]
    for (v, t), V, lo, hi in cases:
        fast = voxelize(v, t, V, lo, hi)
        slow = voxelize_brute(v, t, V, np.array(lo), np.array(hi))
        assert np.array_equal(fast, slow)


def voxelize(v, t, V, lo, hi):
    return W.voxelize(v, t, V, np.array(lo, float), np.array(hi, float))


def test_vertex_voxels_occupied_and_shell():
    v, t = W.icosphere(3)
    V = 32
    lo, hi = np.array([-1.1] * 3), np.array([1.1] * 3)
    occ = W.unpack_bits(voxelize(v, t, V, lo, hi), V ** 3)
    vs = (hi - lo) / V
    k = np.clip(np.floor((v - lo) / vs).astype(int), 0, V - 1)
    assert np.all(occ[k[:, 0] + V * (k[:, 1] + V * k[:, 2])])
    idx = np.nonzero(occ)[0]
    c = lo + (np.stack([idx % V, (idx // V) % V, idx // (V * V)], 1) + 0.5) * vs
    r = np.linalg.norm(c, axis=1)
    assert np.all(np.abs(r - 1.0) <= np.sqrt(3) * vs[0])


def test_pack_roundtrip():
    rng = np.random.default_rng(3)
    b = rng.uniform(size=1000) < 0.3
    assert np.array_equal(W.unpack_bits(W.pack_bits(b), 1000), b)


def test_seeded_reproducible():
    a = W.configs.c1()
    b = W.configs.c1()
    assert np.array_equal(a["rays"], b["rays"])
    assert np.array_equal(a["objects"][0].tables, b["objects"][0].tables)
    assert all(np.array_equal(x, y) for x, y in zip(a["objects"][0].weights, b["objects"][0].weights))


def test_level_resolutions():
    assert list(W.level_resolutions(4, 64, 8)) == [4, 6, 9, 13, 20, 29, 43, 64]
    assert list(W.level_resolutions(16, 2048, 16)) == [16, 22, 31, 42, 58, 81, 111, 154, 213, 294,
                                                      406, 562, 776, 1072, 1482, 2048]


def test_ray_batches_well_formed():
    c = W.configs.c1()
    r = c["rays"]
    assert r.shape == (4096, 8) and r.dtype == np.float32
    assert np.allclose(np.linalg.norm(r[:, 3:6], axis=1), 1.0, atol=1e-6)
    assert np.allclose(np.linalg.norm(r[:, 0:3], axis=1), 2.0, atol=1e-5)
