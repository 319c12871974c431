"""ctypes binding of the LSNIF HIP library (``liblsnif.so``), names as in lsnif.h.

Argument marshalling only: every step of a query runs in the library's HIP
kernels.  Device buffers are torch tensors on the GPU (passed by
``data_ptr()``) and streams are torch streams (passed by ``cuda_stream``).
The library must be built (``__graft_entry__.build()``); loading fails with
an error if it is not.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsnif.so")

LSNIF_OK, LSNIF_E_INVALID, LSNIF_E_NOMEM, LSNIF_E_DEVICE = 0, -1, -2, -3
LSNIF_E_BUSY, LSNIF_E_NOTFOUND, LSNIF_E_TIMEOUT, LSNIF_E_CANCELLED = -4, -5, -6, -7
LSNIF_FP32, LSNIF_FP16, LSNIF_BF16, LSNIF_FP8_E4M3 = 0, 1, 2, 3
LSNIF_RELU, LSNIF_LEAKY_RELU = 0, 1
DTYPES = {"fp32": LSNIF_FP32, "fp16": LSNIF_FP16, "bf16": LSNIF_BF16, "fp8": LSNIF_FP8_E4M3}

RAY_BYTES, HIT_BYTES = 32, 24


class LsnifError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lsnif error {status}: {msg}")
        self.status = status


class lsnif_ctx_desc(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget", C.c_uint64), ("autotune_cache", C.c_char_p)]


class lsnif_object_desc(C.Structure):
    _fields_ = [("aabb_min", C.c_float * 3), ("aabb_max", C.c_float * 3), ("V", C.c_int32),
                ("occupancy", C.c_void_p), ("L", C.c_int32), ("F", C.c_int32),
                ("log2_T", C.c_int32), ("R", C.c_void_p), ("tables", C.c_void_p),
                ("H", C.c_int32), ("n_hidden", C.c_int32), ("width", C.c_int32),
                ("act", C.c_int32), ("leaky_slope", C.c_float), ("n_mat", C.c_int32),
                ("has_albedo", C.c_int32), ("W", C.c_void_p), ("feat_dtype", C.c_int32),
                ("mlp_dtype", C.c_int32), ("fp8_act_scale", C.c_void_p),
                ("grazing_recheck", C.c_int32)]


class lsnif_tuning(C.Structure):
    _fields_ = [("sort_bits", C.c_int32), ("pair_bits", C.c_int32), ("hot_lds_bytes", C.c_int32),
                ("walk_chunks", C.c_int32), ("persistent", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lsnif_serve_cfg(C.Structure):
    _fields_ = [("max_inflight", C.c_uint32), ("hbm_budget", C.c_uint64), ("n_streams", C.c_uint32),
                ("max_queue", C.c_uint32), ("dry_run_ns_per_ray", C.c_uint64), ("merge_rays", C.c_uint32),
                ("merge_max", C.c_uint32)]


class lsnif_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("object_id", C.c_uint32), ("d_rays", C.c_void_p), ("n_rays", C.c_uint32),
                ("d_pair_ray", C.c_void_p), ("d_pair_inst", C.c_void_p), ("n_pairs", C.c_uint32),
                ("d_inst", C.c_void_p), ("n_inst", C.c_uint32), ("d_out", C.c_void_p),
                ("timeout_ns", C.c_int64)]


class lsnif_serve_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "admitted", "completed", "rejected", "cancelled",
                                           "timed_out", "failed", "queued", "inflight",
                                           "rays_completed", "ws_bytes_peak")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "elapsed_s")] + \
               [("launches", C.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


LSNIF_REQ_QUEUED, LSNIF_REQ_RUNNING, LSNIF_REQ_DONE = 0, 1, 2
LSNIF_REQ_SINGLE, LSNIF_REQ_PAIRS = 0, 1


class lsnif_adam_cfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


# lsnif_train_target as a numpy record: hit, t, n[3], albedo[3], material (36 bytes)
TRAIN_TARGET = np.dtype([("hit", np.uint32), ("t", np.float32), ("n", np.float32, 3),
                         ("albedo", np.float32, 3), ("material", np.int32)])


class lsnif_debug_bufs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("count", "tatb", "vox_ijk", "vox_t", "vox_axis",
                                           "points", "slots", "weights", "enc", "out", "act_amax")]


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"LSNIF HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    lib.lsnif_version.restype = C.c_int32
    lib.lsnif_last_error.restype = C.c_char_p
    lib.lsnif_create.argtypes = [C.POINTER(lsnif_ctx_desc), C.POINTER(C.c_void_p)]
    lib.lsnif_destroy.argtypes = [C.c_void_p]
    lib.lsnif_destroy.restype = None
    lib.lsnif_desc_bytes.argtypes = [C.POINTER(lsnif_object_desc), C.POINTER(C.c_uint64)]
    lib.lsnif_build.argtypes = [C.c_void_p, C.POINTER(lsnif_object_desc), C.POINTER(C.c_uint32)]
    lib.lsnif_release.argtypes = [C.c_void_p, C.c_uint32]
    lib.lsnif_object_bytes.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(C.c_uint64)]
    lib.lsnif_query.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_query_noalloc.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_query_debug.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                      C.POINTER(lsnif_debug_bufs), C.c_void_p]
    lib.lsnif_query_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                      C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_bounce.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_float,
                                 C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32), C.c_void_p]
    lib.lsnif_gather_ceiling.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_broad_phase.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                      C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32), C.c_void_p]
    lib.lsnif_query_scene.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                      C.c_void_p]
    lib.lsnif_serve_start.argtypes = [C.c_void_p, C.POINTER(lsnif_serve_cfg)]
    lib.lsnif_serve_submit.argtypes = [C.c_void_p, C.POINTER(lsnif_request), C.POINTER(C.c_uint64)]
    lib.lsnif_serve_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]
    lib.lsnif_serve_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int64]
    lib.lsnif_serve_cancel.argtypes = [C.c_void_p, C.c_uint64]
    lib.lsnif_serve_stats_get.argtypes = [C.c_void_p, C.POINTER(lsnif_serve_stats)]
    lib.lsnif_serve_stop.argtypes = [C.c_void_p]
    lib.lsnif_profile_enable.argtypes = [C.c_void_p, C.c_int32]
    lib.lsnif_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    lib.lsnif_graph_query.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                      C.POINTER(C.c_void_p)]
    lib.lsnif_graph_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                      C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.lsnif_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
    lib.lsnif_graph_destroy.argtypes = [C.c_void_p]
    lib.lsnif_graph_destroy.restype = None
    lib.lsnif_get_tuning.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(lsnif_tuning)]
    lib.lsnif_set_tuning.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(lsnif_tuning)]
    lib.lsnif_autotune.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                   C.POINTER(lsnif_tuning)]
    lib.lsnif_autotune_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                         C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                         C.POINTER(lsnif_tuning)]
    lib.lsnif_trainer_create.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(lsnif_adam_cfg), C.POINTER(C.c_void_p)]
    lib.lsnif_trainer_destroy.argtypes = [C.c_void_p]
    lib.lsnif_trainer_destroy.restype = None
    lib.lsnif_train_grads.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.lsnif_train_apply.argtypes = [C.c_void_p, C.c_void_p]
    lib.lsnif_trainer_read.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_uint64)]
    lib.lsnif_train_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                             C.POINTER(C.c_uint32)]
    for name in ("lsnif_create", "lsnif_desc_bytes", "lsnif_build", "lsnif_release",
                 "lsnif_object_bytes", "lsnif_query", "lsnif_query_debug", "lsnif_profile_enable",
                 "lsnif_profile_read", "lsnif_query_pairs", "lsnif_serve_start", "lsnif_serve_submit",
                 "lsnif_serve_poll", "lsnif_serve_wait", "lsnif_serve_cancel", "lsnif_serve_stats_get",
                 "lsnif_serve_stop", "lsnif_graph_query", "lsnif_graph_pairs", "lsnif_graph_launch",
                 "lsnif_get_tuning", "lsnif_set_tuning", "lsnif_autotune", "lsnif_autotune_pairs",
                 "lsnif_broad_phase", "lsnif_query_scene", "lsnif_gather_ceiling", "lsnif_bounce",
                 "lsnif_trainer_create", "lsnif_train_grads", "lsnif_train_step", "lsnif_train_apply",
                 "lsnif_trainer_read", "lsnif_train_profile_read", "lsnif_query_noalloc"):
        getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def _check(st):
    if st != LSNIF_OK:
        raise LsnifError(st, load().lsnif_last_error().decode(errors="replace"))


def lsnif_version():
    return load().lsnif_version()


def lsnif_last_error():
    return load().lsnif_last_error().decode(errors="replace")


def lsnif_create(device=0, hbm_budget=0, autotune_cache=None):
    d = lsnif_ctx_desc(device, hbm_budget, autotune_cache.encode() if autotune_cache else None)
    h = C.c_void_p()
    _check(load().lsnif_create(C.byref(d), C.byref(h)))
    return h


def lsnif_destroy(ctx):
    load().lsnif_destroy(ctx)


class ObjectDesc:
    """An ``lsnif_object_desc`` and the host arrays it points to (kept alive here)."""

    def __init__(self, obj, feat_dtype="fp32", mlp_dtype="fp32", fp8_act_scale=None):
        self.occ = np.ascontiguousarray(obj.occ, dtype=np.uint32)
        self.R = np.ascontiguousarray(obj.R, dtype=np.int32)
        self.tables = np.ascontiguousarray(obj.tables, dtype=np.float32)
        self.W = [np.ascontiguousarray(w, dtype=np.float32) for w in obj.weights]
        self.Wp = (C.c_void_p * len(self.W))(*[w.ctypes.data for w in self.W])
        self.scale = None if fp8_act_scale is None else np.ascontiguousarray(fp8_act_scale, np.float32)
        d = lsnif_object_desc()
        d.aabb_min[:] = [float(x) for x in np.asarray(obj.bmin, np.float32)]
        d.aabb_max[:] = [float(x) for x in np.asarray(obj.bmax, np.float32)]
        d.V, d.L, d.F, d.log2_T, d.H = obj.V, obj.L, obj.F, obj.log2_T, obj.H
        d.occupancy = self.occ.ctypes.data
        d.R = self.R.ctypes.data
        d.tables = self.tables.ctypes.data
        d.n_hidden = len(self.W) - 1
        d.width = self.W[0].shape[0]
        d.act, d.leaky_slope = obj.act, obj.leaky_slope
        d.n_mat, d.has_albedo = obj.n_mat, obj.has_albedo
        d.W = C.cast(self.Wp, C.c_void_p)
        d.feat_dtype = DTYPES[feat_dtype] if isinstance(feat_dtype, str) else feat_dtype
        d.mlp_dtype = DTYPES[mlp_dtype] if isinstance(mlp_dtype, str) else mlp_dtype
        d.fp8_act_scale = self.scale.ctypes.data if self.scale is not None else None
        d.grazing_recheck = int(getattr(obj, "grazing_recheck", 0))
        self.d = d


def lsnif_desc_bytes(desc: ObjectDesc):
    b = C.c_uint64()
    _check(load().lsnif_desc_bytes(C.byref(desc.d), C.byref(b)))
    return b.value


def lsnif_build(ctx, desc: ObjectDesc):
    oid = C.c_uint32()
    _check(load().lsnif_build(ctx, C.byref(desc.d), C.byref(oid)))
    return oid.value


def lsnif_release(ctx, object_id):
    _check(load().lsnif_release(ctx, object_id))


def lsnif_object_bytes(ctx, object_id):
    b = C.c_uint64()
    _check(load().lsnif_object_bytes(ctx, object_id, C.byref(b)))
    return b.value


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def lsnif_query(ctx, object_id, rays, out, stream=None):
    """Enqueue a query: ``rays`` (n, 8) float32 and ``out`` (n, 6) 4-byte device tensors."""
    n = rays.shape[0]
    assert rays.is_cuda and out.is_cuda and out.shape[0] >= n
    _check(load().lsnif_query(ctx, object_id, C.c_void_p(rays.data_ptr()), n,
                              C.c_void_p(out.data_ptr()), _stream_handle(stream)))


def lsnif_query_noalloc(ctx, object_id, rays, out, stream=None):
    """``lsnif_query`` with its workspace in the library's fixed per-device scratch array
    (``NOALLOC_SCRATCH_BYTES``); allocates nothing."""
    n = rays.shape[0]
    assert rays.is_cuda and out.is_cuda and out.shape[0] >= n
    _check(load().lsnif_query_noalloc(ctx, object_id, C.c_void_p(rays.data_ptr()), n,
                                      C.c_void_p(out.data_ptr()), _stream_handle(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20   # LSNIF_NOALLOC_SCRATCH_BYTES of include/lsnif.h


def lsnif_query_debug(ctx, object_id, rays, out, bufs: dict, stream=None):
    """Like ``lsnif_query`` and also fills the debug tensors given in ``bufs``."""
    b = lsnif_debug_bufs()
    for k, v in bufs.items():
        setattr(b, k, v.data_ptr() if v is not None else None)
    n = rays.shape[0]
    _check(load().lsnif_query_debug(ctx, object_id, C.c_void_p(rays.data_ptr()), n,
                                    C.c_void_p(out.data_ptr()), C.byref(b), _stream_handle(stream)))


def instances_array(instances):
    """Host array of ``lsnif_instance`` records (n, 13) int32 from [(object_id, 3x4 matrix)]."""
    a = np.zeros((len(instances), 13), np.int32)
    for i, (oid, m) in enumerate(instances):
        a[i, 0] = int(oid)
        a[i, 1:] = np.asarray(m, np.float32).reshape(12).view(np.int32)
    return a


def lsnif_query_pairs(ctx, rays, pair_ray, pair_inst, inst, out, stream=None):
    """Nearest hit per ray over pairs.  All arguments are device tensors: rays (n, 8) float32,
    pair_ray / pair_inst (m,) int32, inst (k, 13) int32 (see ``instances_array``),
    out (n, 6) 4-byte."""
    n, m, k = rays.shape[0], pair_ray.shape[0], inst.shape[0]
    assert pair_inst.shape[0] == m and out.shape[0] >= n
    _check(load().lsnif_query_pairs(ctx, C.c_void_p(rays.data_ptr()), n,
                                    C.c_void_p(pair_ray.data_ptr() if m else 0),
                                    C.c_void_p(pair_inst.data_ptr() if m else 0), m,
                                    C.c_void_p(inst.data_ptr() if k else 0), k,
                                    C.c_void_p(out.data_ptr()), _stream_handle(stream)))


def lsnif_bounce(ctx, rays, hits, seed, bounce, eps, next_rays, parent, stream=None):
    """Diffuse bounce rays of the rays with a hit, compacted into ``next_rays`` (m, 8) float32
    and ``parent`` (m,) int32 (device tensors, m = capacity); returns their number."""
    n, cap = rays.shape[0], next_rays.shape[0]
    assert hits.shape[0] >= n and parent.shape[0] == cap
    cnt = C.c_uint32()
    st = load().lsnif_bounce(ctx, C.c_void_p(rays.data_ptr() if n else 0), C.c_void_p(hits.data_ptr() if n else 0),
                             n, seed, bounce, eps, C.c_void_p(next_rays.data_ptr() if cap else 0),
                             C.c_void_p(parent.data_ptr() if cap else 0), cap, C.byref(cnt), _stream_handle(stream))
    global lsnif_last_pair_count
    lsnif_last_pair_count = cnt.value
    _check(st)
    return cnt.value


def lsnif_gather_ceiling(ctx, object_id, rays, sums, stream=None):
    """The query's gathers alone: sums[i] = ray i's summed interpolated features."""
    n = rays.shape[0]
    assert sums.shape[0] >= n
    _check(load().lsnif_gather_ceiling(ctx, object_id, C.c_void_p(rays.data_ptr()), n,
                                       C.c_void_p(sums.data_ptr()), _stream_handle(stream)))


def lsnif_broad_phase(ctx, rays, inst, pair_ray, pair_inst, stream=None):
    """Device broad phase: fills ``pair_ray`` / ``pair_inst`` (int32 device tensors, their
    length is the capacity) and returns the number of pairs; raises with status
    LSNIF_E_NOMEM when they do not fit (``lsnif_last_pair_count`` then has the count)."""
    n, k = rays.shape[0], inst.shape[0]
    cnt = C.c_uint32()
    cap = pair_ray.shape[0]
    assert pair_inst.shape[0] == cap
    st = load().lsnif_broad_phase(ctx, C.c_void_p(rays.data_ptr() if n else 0), n,
                                  C.c_void_p(inst.data_ptr() if k else 0), k,
                                  C.c_void_p(pair_ray.data_ptr() if cap else 0),
                                  C.c_void_p(pair_inst.data_ptr() if cap else 0), cap, C.byref(cnt),
                                  _stream_handle(stream))
    global lsnif_last_pair_count
    lsnif_last_pair_count = cnt.value
    _check(st)
    return cnt.value


lsnif_last_pair_count = 0


def lsnif_query_scene(ctx, rays, inst, out, stream=None):
    """World rays against instances: device broad phase, then the pair query."""
    n, k = rays.shape[0], inst.shape[0]
    assert out.shape[0] >= n
    _check(load().lsnif_query_scene(ctx, C.c_void_p(rays.data_ptr() if n else 0), n,
                                    C.c_void_p(inst.data_ptr() if k else 0), k, C.c_void_p(out.data_ptr()),
                                    _stream_handle(stream)))


def lsnif_get_tuning(ctx, object_id):
    t = lsnif_tuning()
    _check(load().lsnif_get_tuning(ctx, object_id, C.byref(t)))
    return t.as_dict()


def lsnif_set_tuning(ctx, object_id, sort_bits, pair_bits, hot_lds_bytes, walk_chunks=1, persistent=0):
    t = lsnif_tuning(sort_bits, pair_bits, hot_lds_bytes, walk_chunks, persistent)
    _check(load().lsnif_set_tuning(ctx, object_id, C.byref(t)))


def lsnif_autotune(ctx, object_id, rays, out):
    """Time the tuning candidates on this batch, keep the fastest for the object, return it."""
    t = lsnif_tuning()
    _check(load().lsnif_autotune(ctx, object_id, C.c_void_p(rays.data_ptr()), rays.shape[0],
                                 C.c_void_p(out.data_ptr()), C.byref(t)))
    return t.as_dict()


def lsnif_autotune_pairs(ctx, rays, pair_ray, pair_inst, inst, out):
    """Time the pair-query candidates on this batch, apply the fastest to every object, return it."""
    n, m, k = rays.shape[0], pair_ray.shape[0], inst.shape[0]
    t = lsnif_tuning()
    _check(load().lsnif_autotune_pairs(ctx, C.c_void_p(rays.data_ptr()), n, C.c_void_p(pair_ray.data_ptr()),
                                       C.c_void_p(pair_inst.data_ptr()), m, C.c_void_p(inst.data_ptr()), k,
                                       C.c_void_p(out.data_ptr()), C.byref(t)))
    return t.as_dict()


def lsnif_graph_query(ctx, object_id, rays, out):
    """Capture ``lsnif_query(ctx, object_id, rays, out)`` into a graph; returns its handle."""
    g = C.c_void_p()
    _check(load().lsnif_graph_query(ctx, object_id, C.c_void_p(rays.data_ptr()), rays.shape[0],
                                    C.c_void_p(out.data_ptr()), C.byref(g)))
    return g


def lsnif_graph_pairs(ctx, rays, pair_ray, pair_inst, inst, out):
    """Capture ``lsnif_query_pairs`` with these tensors into a graph; returns its handle."""
    n, m, k = rays.shape[0], pair_ray.shape[0], inst.shape[0]
    assert pair_inst.shape[0] == m and out.shape[0] >= n
    g = C.c_void_p()
    _check(load().lsnif_graph_pairs(ctx, C.c_void_p(rays.data_ptr()), n,
                                    C.c_void_p(pair_ray.data_ptr() if m else 0),
                                    C.c_void_p(pair_inst.data_ptr() if m else 0), m,
                                    C.c_void_p(inst.data_ptr() if k else 0), k,
                                    C.c_void_p(out.data_ptr()), C.byref(g)))
    return g


def lsnif_graph_launch(graph, stream=None):
    _check(load().lsnif_graph_launch(graph, _stream_handle(stream)))


def lsnif_graph_destroy(graph):
    load().lsnif_graph_destroy(graph)


def lsnif_serve_start(ctx, max_inflight=0, hbm_budget=0, n_streams=0, max_queue=0, dry_run_ns_per_ray=0,
                      merge_rays=0, merge_max=0):
    cfg = lsnif_serve_cfg(max_inflight, hbm_budget, n_streams, max_queue, dry_run_ns_per_ray, merge_rays, merge_max)
    _check(load().lsnif_serve_start(ctx, C.byref(cfg)))


def make_request(rays=None, out=None, object_id=0, pair_ray=None, pair_inst=None, inst=None,
                 n_rays=None, timeout_ns=0):
    """An ``lsnif_request`` from device tensors (or raw pointers with ``n_rays``, for dry runs)."""
    ptr = lambda t: (t.data_ptr() if hasattr(t, "data_ptr") else int(t)) if t is not None else None
    n = n_rays if n_rays is not None else rays.shape[0]
    r = lsnif_request()
    r.kind = LSNIF_REQ_SINGLE
    r.object_id = object_id
    r.d_rays, r.n_rays, r.d_out = ptr(rays), n, ptr(out)
    if pair_ray is not None:
        r.kind = LSNIF_REQ_PAIRS
        r.d_pair_ray, r.d_pair_inst = ptr(pair_ray), ptr(pair_inst)
        r.n_pairs = pair_ray.shape[0] if hasattr(pair_ray, "shape") else 0
        r.d_inst = ptr(inst)
        r.n_inst = inst.shape[0] if hasattr(inst, "shape") else 0
    r.timeout_ns = timeout_ns
    return r


def lsnif_serve_submit(ctx, req):
    t = C.c_uint64()
    _check(load().lsnif_serve_submit(ctx, C.byref(req), C.byref(t)))
    return t.value


def lsnif_serve_poll(ctx, ticket):
    st = C.c_int32()
    _check(load().lsnif_serve_poll(ctx, ticket, C.byref(st)))
    return st.value


def lsnif_serve_wait(ctx, ticket, timeout_ns=-1):
    """Final status of the request (0 = completed); raises on a wait timeout."""
    st = load().lsnif_serve_wait(ctx, ticket, timeout_ns)
    if st == LSNIF_E_TIMEOUT and lsnif_last_error().endswith("not finished"):
        raise LsnifError(st, lsnif_last_error())
    return st


def lsnif_serve_cancel(ctx, ticket):
    _check(load().lsnif_serve_cancel(ctx, ticket))


def lsnif_serve_stats_get(ctx):
    s = lsnif_serve_stats()
    _check(load().lsnif_serve_stats_get(ctx, C.byref(s)))
    return s.as_dict()


def lsnif_serve_stop(ctx):
    _check(load().lsnif_serve_stop(ctx))


def lsnif_profile_enable(ctx, on=True):
    _check(load().lsnif_profile_enable(ctx, 1 if on else 0))


def lsnif_profile_read(ctx):
    """(sort_ms, walk_ms, kernel_ms, queries) summed over the queries since the last read."""
    a, b, c, k = C.c_double(), C.c_double(), C.c_double(), C.c_uint64()
    _check(load().lsnif_profile_read(ctx, C.byref(a), C.byref(b), C.byref(c), C.byref(k)))
    return a.value, b.value, c.value, k.value


def hits_from(out):
    """Split an (n, 6) 4-byte result tensor into hit, t, normal, material (torch views)."""
    import torch
    i = out.view(torch.int32)
    return {"hit": i[:, 0], "t": out[:, 1], "normal": out[:, 2:5], "material": i[:, 5]}


def targets_array(hit, t, n, material, albedo=None):
    """Training targets as the (n, 9) 4-byte array lsnif_train_target expects."""
    m = len(hit)
    rec = np.zeros(m, TRAIN_TARGET)
    rec["hit"] = np.asarray(hit, np.uint32)
    rec["t"] = np.where(rec["hit"] == 1, np.asarray(t, np.float32), 0.0)
    rec["n"] = np.asarray(n, np.float32)
    if albedo is not None:
        rec["albedo"] = np.asarray(albedo, np.float32)
    rec["material"] = np.asarray(material, np.int32)
    return rec.view(np.float32).reshape(m, 9)


def lsnif_trainer_create(ctx, object_id, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
    cfg = lsnif_adam_cfg(lr, beta1, beta2, eps)
    h = C.c_void_p()
    _check(load().lsnif_trainer_create(ctx, object_id, C.byref(cfg), C.byref(h)))
    return h


def lsnif_trainer_destroy(tr):
    load().lsnif_trainer_destroy(tr)


def lsnif_train_grads(tr, rays, targets, loss, stream=None):
    """Gradients of one batch: ``rays`` (n, 8) float32, ``targets`` (n, 9) 4-byte, ``loss`` a
    device float32 tensor that receives the batch loss."""
    n = rays.shape[0]
    assert targets.shape[0] == n
    _check(load().lsnif_train_grads(tr, C.c_void_p(rays.data_ptr()), C.c_void_p(targets.data_ptr()), n,
                                    C.c_void_p(loss.data_ptr()), _stream_handle(stream)))


def lsnif_train_apply(tr, stream=None):
    _check(load().lsnif_train_apply(tr, _stream_handle(stream)))


def lsnif_train_step(tr, rays, targets, loss, stream=None):
    n = rays.shape[0]
    assert targets.shape[0] == n
    _check(load().lsnif_train_step(tr, C.c_void_p(rays.data_ptr()), C.c_void_p(targets.data_ptr()), n,
                                   C.c_void_p(loss.data_ptr()), _stream_handle(stream)))


def lsnif_train_profile_read(tr):
    """(layer-product ms, scatter ms, steps) summed over the steps timed since the last read."""
    a, b, k = C.c_double(), C.c_double(), C.c_uint32()
    _check(load().lsnif_train_profile_read(tr, C.byref(a), C.byref(b), C.byref(k)))
    return a.value, b.value, k.value


def lsnif_trainer_read(tr, obj):
    """Host copies: (tables, [W_k], grad_tables, [grad_W_k], steps), shaped like ``obj``'s."""
    tab = np.empty_like(np.asarray(obj.tables, np.float32))
    gtab = np.empty_like(tab)
    W = [np.empty_like(np.asarray(w, np.float32)) for w in obj.weights]
    gW = [np.empty_like(w) for w in W]
    Wp = (C.c_void_p * len(W))(*[w.ctypes.data for w in W])
    gWp = (C.c_void_p * len(gW))(*[w.ctypes.data for w in gW])
    steps = C.c_uint64()
    _check(load().lsnif_trainer_read(tr, C.c_void_p(tab.ctypes.data), C.cast(Wp, C.c_void_p),
                                     C.c_void_p(gtab.ctypes.data), C.cast(gWp, C.c_void_p), C.byref(steps)))
    return tab, W, gtab, gW, steps.value
