"""The oracle's diffuse bounce rays (the consumer side of a wavefront path tracer)."""

import numpy as np

import oracle


def hits_on_plane(n_rays, seed=0, flip=False):
    """Rays from z = 2 toward the plane z = 0 (normal +z, or -z when flipped so that it
    faces along the ray); every third ray misses."""
    rng = np.random.default_rng(seed)
    o = np.concatenate([rng.uniform(-1, 1, (n_rays, 2)), np.full((n_rays, 1), 2.0)], 1)
    d = np.concatenate([rng.uniform(-0.3, 0.3, (n_rays, 2)), np.full((n_rays, 1), -1.0)], 1)
    rays = np.concatenate([o, d, np.zeros((n_rays, 1)), np.full((n_rays, 1), np.inf)], 1).astype(np.float32)
    t = (2.0 / 1.0) * np.ones(n_rays, np.float32)        # o_z + t d_z = 0
    hit = (np.arange(n_rays) % 3 != 2).astype(np.uint32)
    nz = -1.0 if flip else 1.0
    normal = np.tile(np.array([0.0, 0.0, nz], np.float32), (n_rays, 1))
    return rays, hit, t, normal


def test_bounce_geometry():
    rays, hit, t, normal = hits_on_plane(3000)
    eps = 1e-3
    nxt, par = oracle.bounce(rays, hit, t, normal, seed=5, bounce_index=1, eps=eps)
    assert np.array_equal(par, np.nonzero(hit)[0])            # compacted, in order
    x = rays[par, :3].astype(np.float64) + t[par, None] * rays[par, 3:6].astype(np.float64)
    # the new origin sits eps above the plane, on the side the ray came from
    assert np.allclose(nxt[:, :3] - x, [[0, 0, eps]], atol=1e-6)
    d = nxt[:, 3:6].astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-6)
    assert np.all(d[:, 2] >= 0.0)
    assert np.all(nxt[:, 6] == 0.0) and np.all(np.isinf(nxt[:, 7]))
    # a normal facing along the ray is turned around: the same rays leave upward
    nxt2, _ = oracle.bounce(rays, hit, t, -normal, seed=5, bounce_index=1, eps=eps)
    assert np.array_equal(nxt2, nxt)


def test_bounce_is_cosine_distributed():
    """cos(theta) about the normal has density 2 cos(theta) sin(theta): E[cos] = 2/3,
    E[cos^2] = 1/2; the azimuth is uniform."""
    n = 300_000
    rays, hit, t, normal = hits_on_plane(n, seed=1)
    hit[:] = 1
    nxt, _ = oracle.bounce(rays, hit, t, normal, seed=9, bounce_index=2, eps=1e-4)
    c = nxt[:, 5].astype(np.float64)
    se = 1 / np.sqrt(n)
    assert abs(c.mean() - 2 / 3) < 5 * se and abs((c * c).mean() - 0.5) < 5 * se
    az = np.arctan2(nxt[:, 4], nxt[:, 3])
    assert abs(np.cos(az).mean()) < 5 * se * 2 and abs(np.sin(az).mean()) < 5 * se * 2
    # P(cos <= x) = x^2
    for x in (0.25, 0.5, 0.75):
        assert abs((c <= x).mean() - x * x) < 5 * se


def test_bounce_seeds():
    rays, hit, t, normal = hits_on_plane(500)
    a, _ = oracle.bounce(rays, hit, t, normal, seed=1, bounce_index=1, eps=1e-4)
    b, _ = oracle.bounce(rays, hit, t, normal, seed=1, bounce_index=1, eps=1e-4)
    c, _ = oracle.bounce(rays, hit, t, normal, seed=1, bounce_index=2, eps=1e-4)
    d, _ = oracle.bounce(rays, hit, t, normal, seed=2, bounce_index=1, eps=1e-4)
    assert np.array_equal(a, b)
    assert (a[:, 3:6] != c[:, 3:6]).any(axis=1).mean() > 0.99
    assert (a[:, 3:6] != d[:, 3:6]).any(axis=1).mean() > 0.99
    none, par = oracle.bounce(rays, np.zeros_like(hit), t, normal, seed=1, bounce_index=1, eps=1e-4)
    assert len(none) == 0 and len(par) == 0
