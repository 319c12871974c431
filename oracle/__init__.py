"""Python access to the LSNIF query oracle (``lsnif_oracle.c``).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the GPU library.

``query(obj, rays)`` returns the oracle's per-ray results and, with
``debug=True``, every intermediate: slab interval, voxel list, boundary points,
grid slots and weights, the float64 encoding and the raw network outputs.
Objects are any value with the fields of ``workloads.LsnifObject``.
"""

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsnif_oracle.c")
_LIB = os.path.join(_HERE, "liblsnif_oracle.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build():
    """Compile the oracle with gcc (float32 steps must not be contracted into FMAs)."""
    tmp = _LIB + f".{os.getpid()}.tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)


class _Object(C.Structure):
    _fields_ = [("bmin", C.c_float * 3), ("bmax", C.c_float * 3), ("V", C.c_int32),
                ("occ", C.c_void_p), ("L", C.c_int32), ("F", C.c_int32), ("log2_T", C.c_int32),
                ("R", C.c_void_p), ("tables", C.c_void_p), ("H", C.c_int32),
                ("n_layers", C.c_int32), ("dims", C.c_void_p), ("W", C.c_void_p),
                ("act", C.c_int32), ("leaky_slope", C.c_float), ("n_mat", C.c_int32),
                ("has_albedo", C.c_int32), ("grazing_recheck", C.c_int32)]


class _Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("count", "tatb", "vox_ijk", "vox_t", "vox_axis",
                                           "points", "slots", "weights", "enc", "out", "hit",
                                           "t", "nrm", "material", "albedo")]


class _Instance(C.Structure):
    _fields_ = [("object", C.c_int32), ("m", C.c_float * 12)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        lib.oracle_query.argtypes = [C.POINTER(_Object), C.c_void_p, C.c_int64, C.POINTER(_Outputs)]
        lib.oracle_query.restype = C.c_int
        lib.oracle_query_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_query_pairs.restype = C.c_int
        lib.oracle_broad_phase.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
        lib.oracle_broad_phase.restype = C.c_int64
        lib.oracle_bounce.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_uint32,
                                      C.c_uint32, C.c_float, C.c_void_p, C.c_void_p]
        lib.oracle_bounce.restype = C.c_int64
        lib.oracle_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Bound:
    """A C view of one object; keeps every array it points to alive."""

    def __init__(self, obj):
        self.occ = np.ascontiguousarray(obj.occ, dtype=np.uint32)
        self.R = np.ascontiguousarray(obj.R, dtype=np.int32)
        self.tables = np.ascontiguousarray(obj.tables, dtype=np.float32)
        self.W = [np.ascontiguousarray(w, dtype=np.float32) for w in obj.weights]
        self.dims = np.array([self.W[0].shape[1]] + [w.shape[0] for w in self.W], dtype=np.int32)
        self.Wp = (C.c_void_p * len(self.W))(*[w.ctypes.data for w in self.W])
        s = _Object()
        s.bmin[:] = [float(x) for x in np.asarray(obj.bmin, np.float32)]
        s.bmax[:] = [float(x) for x in np.asarray(obj.bmax, np.float32)]
        s.V, s.L, s.F, s.log2_T, s.H = obj.V, obj.L, obj.F, obj.log2_T, obj.H
        s.occ, s.R, s.tables = _ptr(self.occ), _ptr(self.R), _ptr(self.tables)
        s.n_layers = len(self.W)
        s.dims = _ptr(self.dims)
        s.W = C.cast(self.Wp, C.c_void_p)
        s.act, s.leaky_slope = obj.act, obj.leaky_slope
        s.n_mat, s.has_albedo = obj.n_mat, obj.has_albedo
        s.grazing_recheck = int(getattr(obj, "grazing_recheck", 0))
        self.s = s


def num_threads():
    """Threads the oracle's OpenMP loops run on."""
    return _load().oracle_num_threads()


def query(obj, rays, debug=False, outputs=True):
    """Oracle results for a (n, 8) float32 ray batch against one object.

    Always returned: ``hit`` (uint32), ``t`` (float32, +inf on a miss),
    ``normal`` (n, 3), ``material`` (int32, -1 on a miss), ``albedo``,
    ``count`` (boundary points, -1 for an invalid ray), ``tatb`` and the raw
    float64 network outputs ``out``.  ``debug`` adds the voxel list
    (``vox_ijk``, ``vox_t``, ``vox_axis``), ``points``, ``slots``,
    ``weights`` and ``enc``.
    """
    lib = _load()
    b = _Bound(obj)
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    n = len(rays)
    H, L, F = obj.H, obj.L, obj.F
    od = b.dims[-1]
    r = {"count": np.empty(n, np.int32), "tatb": np.empty((n, 2), np.float32),
         "out": np.empty((n, od), np.float64), "hit": np.empty(n, np.uint32),
         "t": np.empty(n, np.float32), "normal": np.empty((n, 3), np.float32),
         "material": np.empty(n, np.int32), "albedo": np.empty((n, 3), np.float32)}
    if debug:
        r.update({"vox_ijk": np.empty((n, H // 2, 3), np.int32),
                  "vox_t": np.empty((n, H // 2, 2), np.float32),
                  "vox_axis": np.empty((n, H // 2, 2), np.int8),
                  "points": np.empty((n, H, 3), np.float32),
                  "slots": np.empty((n, H, L, 8), np.uint32),
                  "weights": np.empty((n, H, L, 3), np.float32),
                  "enc": np.empty((n, H * L * F), np.float64)})
    o = _Outputs()
    for k, name in [("count", "count"), ("tatb", "tatb"), ("out", "out"), ("hit", "hit"),
                    ("t", "t"), ("nrm", "normal"), ("material", "material"), ("albedo", "albedo"),
                    ("vox_ijk", "vox_ijk"), ("vox_t", "vox_t"), ("vox_axis", "vox_axis"),
                    ("points", "points"), ("slots", "slots"), ("weights", "weights"),
                    ("enc", "enc")]:
        if name in r:
            setattr(o, k, _ptr(r[name]))
    rc = lib.oracle_query(C.byref(b.s), _ptr(rays), n, C.byref(o))
    if rc != 0:
        raise RuntimeError(f"oracle_query failed ({rc})")
    return r


def _instances(instances):
    inst = (_Instance * max(len(instances), 1))()
    for i, (oi, m) in enumerate(instances):
        inst[i].object = int(oi)
        inst[i].m[:] = [float(x) for x in np.asarray(m, np.float32).reshape(12)]
    return inst


def broad_phase(objects, instances, rays):
    """The (ray, instance) pairs whose ray, in the instance's object space, the narrow
    phase's slab test makes a candidate (Sec. 4): ``(pair_ray, pair_inst)`` uint32 arrays
    listed by ray, then instance.  ``instances`` as for ``query_pairs``."""
    lib = _load()
    bound = [_Bound(o) for o in objects]
    objs = (_Object * len(bound))(*[b.s for b in bound])
    inst = _instances(instances)
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    n = len(rays)
    counts = np.empty(max(n, 1), np.uint32)
    total = lib.oracle_broad_phase(C.cast(objs, C.c_void_p), C.cast(inst, C.c_void_p), len(instances),
                                   _ptr(rays), n, _ptr(counts), None, None, 0)
    if total < 0:
        raise RuntimeError(f"oracle_broad_phase failed ({total})")
    pr, pi = np.empty(max(total, 1), np.uint32), np.empty(max(total, 1), np.uint32)
    got = lib.oracle_broad_phase(C.cast(objs, C.c_void_p), C.cast(inst, C.c_void_p), len(instances),
                                 _ptr(rays), n, _ptr(counts), _ptr(pr), _ptr(pi), total)
    if got != total:
        raise RuntimeError(f"oracle_broad_phase failed ({got})")
    return pr[:total], pi[:total]


def bounce(rays, hit, t, normal, seed, bounce_index, eps):
    """Diffuse bounce rays of the rays with a hit, in order: ``(next_rays (m, 8) float32,
    parent (m,) uint32)``.  ``hit``, ``t`` and ``normal`` as returned by ``query_pairs``."""
    lib = _load()
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    hit = np.ascontiguousarray(hit, dtype=np.uint32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    normal = np.ascontiguousarray(normal, dtype=np.float32)
    n = len(rays)
    m = int(hit[:n].astype(bool).sum())
    nxt, par = np.empty((max(m, 1), 8), np.float32), np.empty(max(m, 1), np.uint32)
    got = lib.oracle_bounce(_ptr(rays), _ptr(hit), _ptr(t), _ptr(normal), n, seed, bounce_index,
                            float(eps), _ptr(nxt), _ptr(par))
    if got != m:
        raise RuntimeError(f"oracle_bounce returned {got}, expected {m}")
    return nxt[:m], par[:m]


def query_pairs(objects, instances, rays, pair_ray, pair_inst):
    """Nearest hit per ray over (ray, instance) pairs.

    ``instances`` is a list of ``(object_index, world_to_object 3x4)``.
    Returns ``hit``, ``t``, ``normal`` (world space), ``material`` and the
    winning instance per ray (``winner``, -1 on a miss).
    """
    lib = _load()
    bound = [_Bound(o) for o in objects]
    objs = (_Object * len(bound))(*[b.s for b in bound])
    inst = _instances(instances)
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    pr = np.ascontiguousarray(pair_ray, dtype=np.uint32)
    pi = np.ascontiguousarray(pair_inst, dtype=np.uint32)
    n = len(rays)
    r = {"hit": np.empty(n, np.uint32), "t": np.empty(n, np.float32),
         "normal": np.empty((n, 3), np.float32), "material": np.empty(n, np.int32),
         "winner": np.empty(n, np.int32)}
    rc = lib.oracle_query_pairs(C.cast(objs, C.c_void_p), C.cast(inst, C.c_void_p), len(instances),
                                _ptr(rays), n, _ptr(pr), _ptr(pi), len(pr), _ptr(r["hit"]),
                                _ptr(r["t"]), _ptr(r["normal"]), _ptr(r["material"]),
                                _ptr(r["winner"]))
    if rc != 0:
        raise RuntimeError(f"oracle_query_pairs failed ({rc})")
    return r


def layer_inputs(obj, enc):
    """The input of every layer of the object's MLP (Sec. 5.1; bias-free layers, ReLU or
    leaky ReLU between them) for encodings ``enc`` (n, in_dim), in float64, and the raw
    outputs: ``([x_0 = enc, x_1, ..., x_last], out)``, each x_k of shape (n, dims_k).
    Each layer is one float64 matrix product (numpy), then the activation."""
    x = np.asarray(enc, np.float64)
    xs = [x]
    for k, w in enumerate(obj.weights):
        y = x @ np.asarray(w, np.float64).T
        if k + 1 < len(obj.weights):
            y = np.maximum(y, 0.0) if obj.act == 0 else np.where(y > 0.0, y, float(np.float32(obj.leaky_slope)) * y)
            xs.append(y)
        x = y
    return xs, x


def act_amax(obj, rays, chunk=16384):
    """Per-layer activation range for the FP8-e4m3 MLP's static scales (reading of the
    configs' "per-layer scale"): the largest |input| of each layer over a calibration
    batch of rays, in float64, from the oracle's own encodings.  Rays without a
    candidate voxel do not run the network and contribute nothing."""
    amax = np.zeros(len(obj.weights))
    for a in range(0, len(rays), chunk):
        o = query(obj, rays[a:a + chunk], debug=True)
        cand = o["count"] > 0
        if not cand.any():
            continue
        xs, _ = layer_inputs(obj, o["enc"][cand])
        amax = np.maximum(amax, [np.abs(x).max() for x in xs])
    return amax
