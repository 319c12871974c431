/*
 * lsnif.h -- C ABI of the LSNIF query library for AMD Instinct MI355X (gfx950).
 *
 * The library answers ray queries against LSNIF objects (Fujieda, Kao, Harada,
 * "LSNIF: Locally-Subdivided Neural Intersection Function", 2025): a neural
 * stand-in for an object's bottom-level BVH made of a surface-occupancy voxel
 * grid, a sparse multiresolution hash grid and a small MLP (Sec. 3).  For each
 * ray it walks the occupied voxels the ray crosses (Sec. 3.1), encodes the
 * entry and exit points of each one with the hash grid (Sec. 3.2), runs the
 * MLP on the concatenated features, at most H points, zero filled (Sec. 5.1),
 * and decodes occlusion, hit distance, normal and material (Sec. 5.1, 5.3).
 * Instanced pair queries keep the nearest hit per ray (Sec. 4).
 *
 * Conventions shared by every call:
 *  - Every call returns an lsnif_status; LSNIF_OK is 0.  No exception crosses
 *    the ABI.  lsnif_last_error() returns a message for the calling thread's
 *    last failure (valid until that thread's next call).
 *  - Host pointers passed to lsnif_build are copied; the caller keeps them.
 *  - Query calls take DEVICE pointers and a hipStream_t (passed as void*;
 *    NULL = the null stream) and are asynchronous: the caller keeps the
 *    buffers alive until the stream has completed the work.
 *  - Per-ray problems (NaN or infinite origin/direction, zero direction,
 *    tmin > tmax) are not errors: such a ray is reported as a miss.
 *  - A context is used by one host thread at a time.
 */
#ifndef LSNIF_H
#define LSNIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lsnif_status;
enum {
    LSNIF_OK = 0,
    LSNIF_E_INVALID = -1,    /* inconsistent or out-of-range arguments */
    LSNIF_E_NOMEM = -2,      /* device allocation failed or the HBM budget is exceeded */
    LSNIF_E_DEVICE = -3,     /* a HIP runtime call failed */
    LSNIF_E_BUSY = -4,
    LSNIF_E_NOTFOUND = -5,   /* unknown object id */
    LSNIF_E_TIMEOUT = -6,
    LSNIF_E_CANCELLED = -7
};

/* Storage / arithmetic types of hash features and MLP weights. */
enum { LSNIF_FP32 = 0, LSNIF_FP16 = 1, LSNIF_BF16 = 2, LSNIF_FP8_E4M3 = 3 };
/* Hidden-layer activation (Sec. 5.1 uses leaky ReLU; ReLU also supported). */
enum { LSNIF_RELU = 0, LSNIF_LEAKY_RELU = 1 };

/* One ray, 32 bytes, in the object's space for lsnif_query and in world
 * space for lsnif_query_pairs.  The direction need not be unit length; the
 * reported t is in units of the direction given. */
typedef struct {
    float o[3];
    float d[3];
    float tmin;
    float tmax;
} lsnif_ray;

/* One result, 24 bytes.  On a miss: hit = 0, t = +inf, n = 0, material = -1. */
typedef struct {
    uint32_t hit;
    float t;          /* ray parameter of the predicted hit */
    float n[3];       /* unit normal (object space for lsnif_query, world space for pairs) */
    int32_t material; /* argmax of the material logits, lowest index on ties */
} lsnif_hit;

typedef struct lsnif_ctx lsnif_ctx;

typedef struct {
    int32_t device;          /* HIP device ordinal */
    uint64_t hbm_budget;     /* bytes the context may hold for objects; 0 = no limit */
    const char *autotune_cache; /* path of the tile-size cache, or NULL */
} lsnif_ctx_desc;

/*
 * One LSNIF object (Sec. 3.3, 5.1): voxels + sparse hash grid + MLP weights.
 *
 *  aabb_min/max   object-space box covered by the voxel grid.
 *  V              voxels per axis, a power of two in [1, 1024].
 *  occupancy      V^3 bits; voxel (x, y, z) is bit x + V*(y + V*z), packed
 *                 least-significant bit first into uint32 words.
 *  L, F, log2_T   levels, features per table entry, log2 of entries per level
 *                 (log2_T in [1, 30]).
 *  R              L level resolutions; level l has vertices 0..R[l] per axis
 *                 spanning the voxel grid.  A level whose (R+1)^3 vertices fit
 *                 in the table is indexed directly, otherwise through the
 *                 spatial hash of Mueller et al. 2022 (Eq. 4).
 *  tables         float32 [L][2^log2_T][F].
 *  H              cap on boundary points per ray (even, 2..64); a ray uses
 *                 the entry and exit point of its first H/2 occupied voxels.
 *  n_hidden,width hidden layers and their width (width 64 or 128).
 *  act, leaky_slope  hidden activation.
 *  n_mat, has_albedo output heads: [occlusion, t, normal x3, (albedo x3),
 *                 material x n_mat], so 5 + 3*has_albedo + n_mat outputs.
 *  W              n_hidden + 1 float32 row-major [out][in] matrices, no biases;
 *                 W[0] has H*L*F inputs.
 *  feat_dtype     type the tables are stored in on the device (FP32/FP16/BF16).
 *  mlp_dtype      MLP arithmetic: FP32 (vector ALU) or FP16/BF16/FP8_E4M3
 *                 (matrix cores, FP32 accumulation).
 *  fp8_act_scale  n_hidden + 1 activation scales for FP8 (else NULL).
 */
typedef struct {
    float aabb_min[3];
    float aabb_max[3];
    int32_t V;
    const uint32_t *occupancy;
    int32_t L, F, log2_T;
    const int32_t *R;
    const float *tables;
    int32_t H;
    int32_t n_hidden, width, act;
    float leaky_slope;
    int32_t n_mat, has_albedo;
    const float *const *W;
    int32_t feat_dtype, mlp_dtype;
    const float *fp8_act_scale;
} lsnif_object_desc;

/* Optional device buffers filled by lsnif_query_debug; any may be NULL. */
typedef struct {
    int32_t *count;      /* [n] boundary points used (2 per voxel); -1 = invalid ray */
    float *tatb;         /* [n][2] segment [max(aabb entry, tmin), aabb exit] */
    int32_t *vox_ijk;    /* [n][H/2][3] voxel list, -1 padded */
    float *vox_t;        /* [n][H/2][2] entry and exit parameter of each voxel */
    int8_t *vox_axis;    /* [n][H/2][2] entry and exit face axis */
    float *points;       /* [n][H][3] boundary points in voxel units */
    uint32_t *slots;     /* [n][H][L][8] table slot of each cell corner */
    float *weights;      /* [n][H][L][3] interpolation weights */
    float *enc;          /* [n][H*L*F] encoding as fed to the MLP (widened to fp32) */
    float *out;          /* [n][outputs] raw network outputs */
} lsnif_debug_bufs;

/* Context. */
lsnif_status lsnif_create(const lsnif_ctx_desc *desc, lsnif_ctx **out);
void lsnif_destroy(lsnif_ctx *ctx);
const char *lsnif_last_error(void);
/* Library version, for checks by the binding: major*10000 + minor*100 + patch. */
int32_t lsnif_version(void);

/* Validate a descriptor and report the device bytes an object built from it
 * occupies (voxels + tables in feat_dtype + weights in mlp_dtype, excluding
 * layout padding).  Host only; no device is touched.  The paper-default object
 * (V = 32, 2 levels of 2^17 entries x 3 FP16 features, 108->128->128->12 FP16
 * weights) gives 4 KiB + 1536 KiB + 62 KiB (Sec. 5.1). */
lsnif_status lsnif_desc_bytes(const lsnif_object_desc *desc, uint64_t *bytes);

/* Copy an object to the device; it stays resident until released. */
lsnif_status lsnif_build(lsnif_ctx *ctx, const lsnif_object_desc *desc, uint32_t *object_id);
lsnif_status lsnif_release(lsnif_ctx *ctx, uint32_t object_id);
/* Device bytes held by a built object (including layout padding). */
lsnif_status lsnif_object_bytes(lsnif_ctx *ctx, uint32_t object_id, uint64_t *bytes);

/* Query n rays (object space) against one object: out[i] answers rays[i]. */
lsnif_status lsnif_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays,
                         uint32_t n, lsnif_hit *d_out, void *stream);

/* Same query, also writing the intermediates of each step to the non-NULL
 * buffers of *dbg (device pointers; the struct itself is read on the host).
 * Uses a one-ray-per-lane kernel built from the same device functions. */
lsnif_status lsnif_query_debug(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays,
                               uint32_t n, lsnif_hit *d_out, const lsnif_debug_bufs *dbg,
                               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LSNIF_H */
