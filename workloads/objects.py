"""LSNIF object bundles: voxels + hash-grid tables + MLP weights (paper Sec. 3.3, 5.1).

The weights and features are synthetic and untrained: features are uniform in
``[-feature_amp, feature_amp]`` and weights are Kaiming-normal
(``std = sqrt(2 / fan_in)``, He et al. 2015, as paper Sec. 5.1 initialises
them), drawn row-major per layer from the seeded weight stream.
"""

from dataclasses import dataclass, field

import numpy as np

from .rng import streams, FEATURES, WEIGHTS
from .voxelize import voxelize

RELU, LEAKY_RELU = 0, 1


def level_resolutions(r_min: int, r_max: int, levels: int):
    """Geometric level resolutions ``round(r_min * (r_max / r_min) ** (l / (L - 1)))``.

    Rounded to nearest in float64 (a floor would give 63 instead of 64 at the
    top of 4 -> 64 over 8 levels, because the power lands a hair below 64).
    """
    if levels == 1:
        return np.array([r_min], dtype=np.int32)
    b = (r_max / r_min) ** (1.0 / (levels - 1))
    return np.array([int(np.floor(r_min * b ** l + 0.5)) for l in range(levels)], dtype=np.int32)


@dataclass
class LsnifObject:
    """Host-side description of one LSNIF object (all arrays in numpy)."""
    bmin: np.ndarray                 # (3,) float32, object-space AABB
    bmax: np.ndarray                 # (3,) float32
    V: int                           # voxels per axis (power of two)
    occ: np.ndarray                  # uint32 words, bit x + V*(y + V*z), LSB first
    L: int                           # hash-grid levels
    F: int                           # features per entry
    log2_T: int                      # log2 of entries per level
    R: np.ndarray                    # (L,) int32 level resolutions (vertices 0..R)
    tables: np.ndarray               # (L, 2**log2_T, F) float32
    H: int                           # cap on boundary points per ray (even)
    weights: list = field(default_factory=list)   # float32 [out][in] per layer, no biases
    act: int = RELU
    leaky_slope: float = 0.01
    n_mat: int = 4
    has_albedo: int = 0
    name: str = ""
    grazing_recheck: int = 0         # 1: re-decide grazing voxels of the walk in float64

    @property
    def T(self):
        return 1 << self.log2_T

    @property
    def in_dim(self):
        return self.H * self.L * self.F

    @property
    def out_dim(self):
        return 5 + 3 * self.has_albedo + self.n_mat

    @property
    def n_hidden(self):
        return len(self.weights) - 1

    @property
    def width(self):
        return self.weights[0].shape[0]


def make_weights(rng, dims):
    """Kaiming-normal weights for the layer widths ``dims`` (input first)."""
    out = []
    for i in range(len(dims) - 1):
        fan_in, fan_out = dims[i], dims[i + 1]
        w = rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)
        out.append(w.astype(np.float32))
    return out


def make_object(verts, tris, *, V, bmin, bmax, L, F, log2_T, R, H=18, n_hidden=3,
                width=64, n_mat=4, has_albedo=0, act=RELU, leaky_slope=0.01,
                feature_amp=1e-2, seed=0, name="", occ=None):
    """Voxelise a mesh and attach seeded tables and weights."""
    bmin = np.asarray(bmin, dtype=np.float32)
    bmax = np.asarray(bmax, dtype=np.float32)
    if occ is None:
        occ = voxelize(verts, tris, V, bmin.astype(np.float64), bmax.astype(np.float64))
    rf, rw, _, _ = streams(seed)
    T = 1 << log2_T
    tables = rf.uniform(-feature_amp, feature_amp, size=(L, T, F)).astype(np.float32)
    out_dim = 5 + 3 * has_albedo + n_mat
    dims = [H * L * F] + [width] * n_hidden + [out_dim]
    weights = make_weights(rw, dims)
    return LsnifObject(bmin=bmin, bmax=bmax, V=V, occ=occ, L=L, F=F, log2_T=log2_T,
                       R=np.asarray(R, dtype=np.int32), tables=tables, H=H, weights=weights,
                       act=act, leaky_slope=leaky_slope, n_mat=n_mat, has_albedo=has_albedo,
                       name=name)
