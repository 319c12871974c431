"""A small instanced scene shared by the broad-phase tests: two c1-class objects as
nine instances on a 3 x 3 grid (seeded yaw and scale), camera rays from above, random
rays through the scene, and a few invalid or short rays."""

import numpy as np

import workloads as W
from workloads.rays import pinhole_rays


def small_scene(n_random=3000, side=48, seed=11):
    objs = [W.configs.c1_object(seed=0), W.configs.c1_object(seed=1)]
    grid = [objs[k % 2] for k in range(9)]
    insts, boxes = W.configs.c5_instances(grid, seed=seed)
    insts = [(k % 2, m) for k, m in insts]   # the instances name the two objects in turn
    cam = pinhole_rays(side, side, eye=(0.5, 7.0, -8.0), look_at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                       vfov_deg=55.0)
    rng = np.random.default_rng(seed)
    o = rng.uniform(-6, 6, (n_random, 3))
    d = rng.normal(size=(n_random, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rnd = np.concatenate([o, d, np.zeros((n_random, 1)), np.full((n_random, 1), np.inf)], 1)
    rnd[::7, 7] = rng.uniform(0.5, 4.0, len(rnd[::7]))     # short segments
    rnd[3::11, 6] = rng.uniform(0.5, 3.0, len(rnd[3::11]))  # late starts
    bad = np.array([[np.nan, 0, 0, 1, 0, 0, 0, np.inf], [0, 0, 0, 0, 0, 0, 0, np.inf],
                    [0, 0, 0, 1, 0, 0, 2, 1]])
    rays = np.concatenate([cam, rnd, bad]).astype(np.float32)
    return objs, insts, boxes, rays
