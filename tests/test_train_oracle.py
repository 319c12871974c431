"""Pins of the training oracle (paper Sec. 5.2, 5.3) against what does not depend on it.

- the reference signals: a ray cast of the icosphere against the sphere it approximates;
- the loss: its closed form when every weight is zero (all outputs 0);
- the gradient: central finite differences of the batch loss, per table entry and weight;
- Adam: its closed form for the first steps from zero moments (Kingma and Ba 2015);
- rays with no listed voxel add nothing; a few steps lower the loss.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.train as OT
import workloads as W
from workloads import train as WT


@pytest.fixture(scope="module")
def mesh():
    return W.icosphere(3)


@pytest.fixture(scope="module")
def paper():
    return W.configs.paper_object(seed=3)


def test_ray_cast_matches_the_sphere(mesh):
    verts, tris = mesh
    # the icosphere's vertices lie on the unit sphere; its faces within 1 - cos(half edge angle)
    rng = np.random.default_rng(0)
    d = rng.standard_normal((500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = -3.0 * d
    rays = W.ray_array(o, d)
    hit, t, tri = WT.ray_cast(verts, tris, rays)
    assert hit.all()
    assert np.all(t >= 2.0 - 1e-12) and np.all(t <= 2.0 + 0.02)
    # rays that pass the sphere at distance 1.5 from its centre miss
    side = np.cross(d, [0.3, 0.5, 0.8])
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    hit2, _, _ = WT.ray_cast(verts, tris, W.ray_array(o + 1.5 * side, d))
    assert not hit2.any()
    # a ray starting past the surface going outward misses (convex mesh)
    hit3, _, _ = WT.ray_cast(verts, tris, W.ray_array(1.01 * d, d))
    assert not hit3.any()


def test_targets(mesh, paper):
    rays, tg = WT.batch(mesh, paper, 400, seed=1)
    h = tg["hit"] == 1
    # outside half: cosine-weighted toward the centre from radius 1.1 sqrt(3), the unit sphere
    # subtends sin^2 = 1 / 3.63 of that distribution (about 55 of 200); the surface half leaves
    # a convex mesh and never hits
    assert 30 < h.sum() < 90 and not h[200:].any()
    assert np.allclose(np.linalg.norm(tg["n"][h], axis=1), 1.0, atol=1e-6)
    assert set(np.unique(tg["material"][h])) <= set(range(paper.n_mat))
    # every hit lies on the unit sphere up to the faceting
    p = rays[h, 0:3].astype(np.float64) + tg["t"][h, None] * rays[h, 3:6]
    r = np.linalg.norm(p, axis=1)
    assert np.all(r > 0.98) and np.all(r < 1.0 + 1e-5)


def zero_weights(obj):
    return dataclasses.replace(obj, weights=[np.zeros_like(w) for w in obj.weights])


@pytest.mark.parametrize("which", ["paper", "c1"])
def test_loss_closed_form_at_zero_weights(mesh, paper, which):
    obj = paper if which == "paper" else W.configs.c1_object()
    obj = zero_weights(obj)
    rays, tg = WT.batch(mesh, obj, 300, seed=2)
    g = OT.train_grads(obj, rays, tg)
    q = oracle.query(obj, rays)
    act = q["count"] > 0
    y = (tg["hit"] == 1) & act
    ta, tb = q["tatb"][:, 0].astype(np.float64), q["tatb"][:, 1].astype(np.float64)
    tau = np.clip((tg["t"] - ta) / np.where(act, tb - ta, 1.0), 0, 1)
    per = np.log(2.0) + y * (np.abs(0.5 - tau) + 1.0 + np.log(obj.n_mat))
    if obj.has_albedo:
        per = per + y * np.mean((0.5 - tg["albedo"].astype(np.float64)) ** 2 / 0.51 ** 2, axis=1)
    want = np.sum(np.where(act, per, 0.0)) / len(rays)
    assert abs(g["loss"] - want) <= 1e-12 * want
    assert act.sum() > 100 and y.sum() > 20


def test_forward_matches_the_query_oracle(mesh, paper):
    rays, tg = WT.batch(mesh, paper, 200, seed=4)
    g = OT.train_grads(paper, rays, tg)
    q = oracle.query(paper, rays)
    assert np.allclose(g["z"], q["out"], rtol=0, atol=1e-12)


def _fd(obj, rays, tg, which, idx, h, den):
    """Central difference of the batch loss in parameter idx of `which` ('tab' or layer k), the
    albedo term's denominators held at the base point's values `den` (the loss treats them as
    constants)."""
    vals = []
    deltas = []
    for sgn in (+1, -1):
        if which == "tab":
            t = obj.tables.copy()
            x = float(t[idx])
            t[idx] = np.float32(x + sgn * h)
            deltas.append(float(t[idx]) - x)
            o = dataclasses.replace(obj, tables=t)
        else:
            ws = [w.copy() for w in obj.weights]
            x = float(ws[which][idx])
            ws[which][idx] = np.float32(x + sgn * h)
            deltas.append(float(ws[which][idx]) - x)
            o = dataclasses.replace(obj, weights=ws)
        vals.append(OT.batch_loss(o, rays, tg, den))
    return (vals[0] - vals[1]) / (deltas[0] - deltas[1])


@pytest.mark.parametrize("which", ["paper", "c1"])
def test_gradient_matches_finite_differences(mesh, paper, which):
    obj = paper if which == "paper" else W.configs.c1_object()
    rays, tg = WT.batch(mesh, obj, 160, seed=5)
    g = OT.train_grads(obj, rays, tg)
    # table entries: the largest gradients, plus one of each level
    flat = np.abs(g["gtab"]).ravel()
    picks = list(np.argsort(flat)[-4:])
    for l in range(obj.L):
        lvl = np.abs(g["gtab"][l]).ravel()
        picks.append(l * lvl.size + int(np.argmax(lvl)))
    for p in picks:
        idx = np.unravel_index(p, g["gtab"].shape)
        fd = _fd(obj, rays, tg, "tab", idx, 1e-6, g["albedo_den"])
        assert abs(fd - g["gtab"][idx]) <= 2e-4 * abs(g["gtab"][idx]) + 1e-10, (idx, fd, g["gtab"][idx])
    # weights: the largest gradient of each layer and one random entry
    rng = np.random.default_rng(1)
    for k, gw in enumerate(g["gW"]):
        for idx in (np.unravel_index(int(np.argmax(np.abs(gw))), gw.shape),
                    tuple(int(rng.integers(0, s)) for s in gw.shape)):
            fd = _fd(obj, rays, tg, k, idx, 1e-5, g["albedo_den"])
            assert abs(fd - gw[idx]) <= 2e-4 * abs(gw[idx]) + 1e-9, (k, idx, fd, gw[idx])


def test_inactive_rays_add_nothing(mesh, paper):
    rays, tg = WT.batch(mesh, paper, 150, seed=6)
    g1 = OT.train_grads(paper, rays, tg)
    # 50 rays pointing away from the object: no listed voxel
    far = W.ray_array(np.tile([[5.0, 0.0, 0.0]], (50, 1)), np.tile([[1.0, 0.0, 0.0]], (50, 1)))
    rays2 = np.concatenate([rays, far])
    tg2 = {k: np.concatenate([v, np.zeros((50,) + v.shape[1:], v.dtype)]) for k, v in tg.items()}
    tg2["hit"][150:] = 1   # even a reference hit changes nothing without a listed voxel
    g2 = OT.train_grads(paper, rays2, tg2)
    s = 150.0 / 200.0
    assert abs(g2["loss"] - s * g1["loss"]) <= 1e-12 * g1["loss"]
    # equal up to the summation order of the products (rounding of float64 sums)
    assert np.allclose(g2["gtab"], s * g1["gtab"], rtol=1e-9, atol=1e-12 * np.abs(g1["gtab"]).max())
    for a, b in zip(g2["gW"], g1["gW"]):
        assert np.allclose(a, s * b, rtol=1e-9, atol=1e-12 * np.abs(b).max())


def test_adam_closed_form():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(1000)
    g = rng.standard_normal(1000) * 10.0 ** rng.uniform(-6, 1, 1000)
    g[:10] = 0.0
    lr, eps = 0.01, 1e-8
    m = v = np.zeros(1000)
    # step 1 from zero moments: the bias corrections give m_hat = g, v_hat = g^2
    p1, m, v = OT.adam(p0, g, m, v, 1, lr=lr, eps=eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    assert np.array_equal(p1[:10], p0[:10])
    # step 2 with the same gradient: again m_hat = g, v_hat = g^2
    p2, m, v = OT.adam(p1, g, m, v, 2, lr=lr, eps=eps)
    assert np.allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    # a gradient that flips sign at step 2: m_hat = (0.09 g - 0.1 g) / 0.19, v_hat = g^2
    q1, m, v = OT.adam(p0, g, np.zeros(1000), np.zeros(1000), 1, lr=lr, eps=eps)
    q2, _, _ = OT.adam(q1, -g, m, v, 2, lr=lr, eps=eps)
    mh = (0.9 * 0.1 * g - 0.1 * g) / (1 - 0.81)
    assert np.allclose(q2, q1 - lr * mh / (np.abs(g) + eps), rtol=1e-10, atol=1e-15)


def test_steps_lower_the_loss(mesh):
    obj = W.configs.paper_object(seed=7)
    rays, tg = WT.batch(mesh, obj, 256, seed=8)
    tab = obj.tables.astype(np.float64)
    ws = [w.astype(np.float64) for w in obj.weights]
    mt, vt = np.zeros_like(tab), np.zeros_like(tab)
    mw = [np.zeros_like(w) for w in ws]
    vw = [np.zeros_like(w) for w in ws]
    losses = []
    for t in range(1, 7):
        cur = dataclasses.replace(obj, tables=tab.astype(np.float32), weights=[w.astype(np.float32) for w in ws])
        g = OT.train_grads(cur, rays, tg)
        losses.append(g["loss"])
        tab, mt, vt = OT.adam(tab, g["gtab"], mt, vt, t)
        for k in range(len(ws)):
            ws[k], mw[k], vw[k] = OT.adam(ws[k], g["gW"][k], mw[k], vw[k], t)
    assert all(b < a for a, b in zip(losses, losses[1:])) and losses[-1] < 0.8 * losses[0], losses
