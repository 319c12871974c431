"""The oracle's broad phase (Sec. 4): which (ray, instance) pairs the narrow phase can hit."""

import numpy as np

import oracle
import workloads as W
from tests.scene import small_scene


def test_oracle_broad_phase_closed_form():
    """One object (AABB [-1.1, 1.1]^3) as an instance at the origin and one moved by +10 in x:
    the pairs follow from where each ray's segment crosses the two boxes."""
    obj = W.configs.c1_object()
    eye = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    moved = eye.copy()
    moved[0, 3] = -10.0                       # world -> object: x - 10
    inf = np.inf
    rays = np.array([[-5, 0, 0, 1, 0, 0, 0, inf],      # through both boxes
                     [-5, 0, 0, 1, 0, 0, 0, 8.0],      # stops before the second (t 13.9)
                     [0, -5, 0, 0, 1, 0, 0, inf],      # along y through the first only
                     [-5, 0, 0, 1, 0, 0, 7.0, inf],    # starts after the first (t 3.9 .. 6.1)
                     [-5, 3, 0, 1, 0, 0, 0, inf],      # passes above both
                     [np.nan, 0, 0, 1, 0, 0, 0, inf],  # invalid
                     [0, 0, 0, 0, 0, 0, 0, inf]],      # no direction
                    np.float32)
    pr, pi = oracle.broad_phase([obj], [(0, eye), (0, moved)], rays)
    assert list(zip(pr.tolist(), pi.tolist())) == [(0, 0), (0, 1), (1, 0), (2, 0), (3, 1)]
    # no instances, no rays
    pr, pi = oracle.broad_phase([obj], [], rays)
    assert len(pr) == 0 and len(pi) == 0
    pr, pi = oracle.broad_phase([obj], [(0, eye)], rays[:0])
    assert len(pr) == 0


def test_oracle_broad_phase_loses_nothing():
    """Against the host's world-box brute force (a superset: a box around each instance's
    transformed object box): every broad-phase pair is a padded-box pair, and the pairs it
    drops change no ray's nearest hit in the oracle's pair query."""
    objs, insts, boxes, rays = small_scene()
    pr, pi = oracle.broad_phase(objs, insts, rays)
    assert len(pr) > 500
    key = pr.astype(np.int64) * len(insts) + pi
    assert np.all(np.diff(key) > 0)                # sorted by ray, then instance, no repeats
    pad = [(lo - 1e-3 * (hi - lo), hi + 1e-3 * (hi - lo)) for lo, hi in boxes]
    hr, hi_ = W.configs.ray_box_pairs(rays, pad)
    host = set((hr.astype(np.int64) * len(insts) + hi_).tolist())
    assert set(key.tolist()) <= host
    hr0, hi0 = W.configs.ray_box_pairs(rays, boxes)
    assert len(hr0) > len(pr)                      # the world boxes are looser
    a = oracle.query_pairs(objs, insts, rays, pr, pi)
    b = oracle.query_pairs(objs, insts, rays, hr0, hi0)
    for k in ("hit", "t", "normal", "material", "winner"):
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), k
    assert a["hit"].sum() > 100
