"""Seeded random streams.

Every workload draws from numpy's PCG64 through ``SeedSequence(seed).spawn``.
Children are assigned by role so that changing, say, the ray count never
changes the features or the weights:

* child 0: hash-table features
* child 1: MLP weights
* child 2: rays
* child 3: mesh noise, placement and other geometry randomness
"""

import numpy as np

FEATURES, WEIGHTS, RAYS, GEOMETRY = 0, 1, 2, 3


def streams(seed: int):
    """Return four independent generators ``[features, weights, rays, geometry]``."""
    children = np.random.SeedSequence(int(seed)).spawn(4)
    return [np.random.Generator(np.random.PCG64(c)) for c in children]
