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
                ("mlp_dtype", C.c_int32), ("fp8_act_scale", C.c_void_p)]


class lsnif_debug_bufs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("count", "tatb", "vox_ijk", "vox_t", "vox_axis",
                                           "points", "slots", "weights", "enc", "out")]


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
    lib.lsnif_query_debug.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                      C.POINTER(lsnif_debug_bufs), C.c_void_p]
    for name in ("lsnif_create", "lsnif_desc_bytes", "lsnif_build", "lsnif_release",
                 "lsnif_object_bytes", "lsnif_query", "lsnif_query_debug"):
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


def lsnif_query_debug(ctx, object_id, rays, out, bufs: dict, stream=None):
    """Like ``lsnif_query`` and also fills the debug tensors given in ``bufs``."""
    b = lsnif_debug_bufs()
    for k, v in bufs.items():
        setattr(b, k, v.data_ptr() if v is not None else None)
    n = rays.shape[0]
    _check(load().lsnif_query_debug(ctx, object_id, C.c_void_p(rays.data_ptr()), n,
                                    C.c_void_p(out.data_ptr()), C.byref(b), _stream_handle(stream)))


def hits_from(out):
    """Split an (n, 6) 4-byte result tensor into hit, t, normal, material (torch views)."""
    import torch
    i = out.view(torch.int32)
    return {"hit": i[:, 0], "t": out[:, 1], "normal": out[:, 2:5], "material": i[:, 5]}
