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

/* One instance of a built object, 52 bytes: the object's id and the row-major
 * 3x4 world-to-object matrix [A | b], x_obj = A x_world + b.  Rays are mapped
 * with d_obj = A d_world and not renormalised, so t is shared by both spaces;
 * normals return to world space as normalize(A^T n). */
typedef struct {
    uint32_t object_id;
    float world_to_object[12];
} lsnif_instance;

typedef struct lsnif_ctx lsnif_ctx;

typedef struct {
    int32_t device;          /* HIP device ordinal; -1 = a host-only context (serving dry runs) */
    uint64_t hbm_budget;     /* bytes the context may hold for objects; 0 = no limit */
    const char *autotune_cache; /* path of the autotune cache file, or NULL (see below) */
} lsnif_ctx_desc;

/* Autotune cache.  With a path, lsnif_create reads the file if it exists (a
 * missing file is an empty cache; an unreadable or malformed file, or an entry
 * out of lsnif_set_tuning's ranges, fails creation with LSNIF_E_INVALID), every
 * lsnif_build whose object matches an entry starts with that entry's launch
 * parameters instead of the defaults (no timing), and every successful
 * lsnif_autotune / lsnif_autotune_pairs records its winners (per object, the
 * object's whole lsnif_tuning after the call) and rewrites the file (a sibling
 * temporary file renamed over it).  JSON: {"lsnif_autotune_cache": 1,
 * "entries": {key: {"sort_bits", "pair_bits", "hot_lds_bytes", "walk_chunks",
 * "persistent"}}},
 * key = "<gfx arch> V=.. L=.. F=.. log2_T=.. H=.. width=.. feat=<dtype> mlp=<dtype>".
 * Launch parameters change speed only, never a result.  Contexts that share a
 * file and autotune concurrently keep the last writer's entries. */

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
 *  n_hidden,width hidden layers and their width; the query kernels are built
 *                 for widths 64 and 128 (the paper's), the matrix-core ones of
 *                 width 128 for at most 32 inputs per point (L x F, F = 3
 *                 counted as 4); lsnif_build returns LSNIF_E_INVALID otherwise,
 *                 lsnif_desc_bytes accounts any width.
 *  act, leaky_slope  hidden activation.
 *  n_mat, has_albedo output heads: [occlusion, t, normal x3, (albedo x3),
 *                 material x n_mat], so 5 + 3*has_albedo + n_mat outputs.
 *  W              n_hidden + 1 float32 row-major [out][in] matrices, no biases;
 *                 W[0] has H*L*F inputs.
 *  feat_dtype     type the tables are stored in on the device (FP32/FP16/BF16).
 *  mlp_dtype      MLP arithmetic: FP32 (vector ALU) or FP16/BF16/FP8_E4M3
 *                 (matrix cores, FP32 accumulation).
 *  fp8_act_scale  n_hidden + 1 activation scales for FP8 (else NULL): layer k's
 *                 input x is stored as e4m3(x / fp8_act_scale[k]); weights get a
 *                 per-layer scale amax|W_k| / 448 at build.  All e4m3 values
 *                 round to nearest even and saturate at +-448.
 *  grazing_recheck 0 (default) or 1: the walk lists a visited voxel when its
 *                 float32 slab interval overlaps [ta, tb] with positive length
 *                 (Sec. 3.1); with 1, a voxel whose float32 overlap is at most
 *                 2^-16 max(1, |entry|) long, or any voxel of a ray whose whole
 *                 segment [ta, tb] is that short, is instead listed iff its
 *                 float64 slab interval (computed from the same float32
 *                 voxel-space origin and direction) overlaps the float64
 *                 [ta, tb] with positive length.  t values stay float32.
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
    int32_t grazing_recheck;
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
    float *act_amax;     /* [n_hidden + 1] largest |input| of each MLP layer over the batch,
                            folded in with a maximum (FP32-MLP objects only); start it at 0.
                            act_amax / 448 are the FP8 activation scales of a calibration
                            batch. */
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

/* Direct calls (lsnif_query, _query_debug, _query_pairs, _query_scene,
 * _broad_phase, _bounce, _gather_ceiling) keep their scratch arrays in
 * workspaces of the context, grown on demand and reused by the next call: two
 * such calls enqueued on different streams must not overlap on the device
 * (order them, or use graphs or the serving loop, which own their
 * workspaces).  Calls on one stream are ordered by the stream. */

/* Query n rays (object space) against one object: out[i] answers rays[i].
 * Batches of at most 8,192 rays of a width-64 object with at most 16 levels
 * (FP32 features and MLP with F <= 3, or a matrix-core MLP with F = 2) run
 * one wave per ray instead of one ray per lane (lower latency); a ray's answer
 * is the same bits either way. */
lsnif_status lsnif_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays,
                         uint32_t n, lsnif_hit *d_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lsnif_query with the
 * same kernels and the same results, bit for bit, whose workspace (the
 * coherence sort's keys, ray indices and digit counters; the voxel counts and
 * lists) lives in a fixed device array of LSNIF_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends.  The call allocates nothing
 * (no hipMalloc or hipFree, no stream or event creation); the caller still
 * passes the rays and the output as for lsnif_query.
 *
 * Limit: the workspace of n rays is about (17.5 + 4 H/2) bytes per ray (the
 * sort's 16.5, the voxel count and lists; 53.5 bytes per ray at H = 18, so
 * about 1.25M rays); a batch that needs more returns LSNIF_E_INVALID, naming
 * the limit, and enqueues nothing.
 * Every call on one GPU shares that GPU's array, whatever its context:
 * allocation-free queries that may overlap on the device (different streams,
 * different contexts on the same device, threads) race on it, so order them
 * (one stream, or events).  The array keeps the last call's contents; the
 * kernels clear what must start at zero. */
#define LSNIF_NOALLOC_SCRATCH_BYTES (64u << 20)
lsnif_status lsnif_query_noalloc(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays,
                                 uint32_t n, lsnif_hit *d_out, void *stream);

/* Same query, also writing the intermediates of each step to the non-NULL
 * buffers of *dbg (device pointers; the struct itself is read on the host).
 * Uses a one-ray-per-lane kernel built from the same device functions. */
lsnif_status lsnif_query_debug(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays,
                               uint32_t n, lsnif_hit *d_out, const lsnif_debug_bufs *dbg,
                               void *stream);

/* Measurement aid: the gathers of lsnif_query alone.  Runs the same sort,
 * walk, boundary points and hash-grid encoding (Sec. 3.2) as the query, but
 * instead of the MLP writes d_sums[i] = the sum over ray i's boundary points,
 * levels and features of the interpolated features (0 for a ray with no
 * point).  Its kernel holds no MLP accumulators, so its time is a ceiling for
 * what the query kernel's gathers can take on the same batch.  d_sums: [n]
 * floats on the device; asynchronous on `stream`; timed by lsnif_profile_*. */
lsnif_status lsnif_gather_ceiling(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                                  float *d_sums, void *stream);

/* Nearest hit over (ray, instance) pairs (Sec. 4: the broad phase lists the
 * pairs, the narrow phase queries each LSNIF object, and a ray's hit
 * information is updated with the nearest hit).
 *
 *  d_rays       [n_rays] world-space rays.
 *  d_pair_ray   [n_pairs] ray index of each pair; d_pair_inst the instance index.
 *  d_inst       [n_inst] instances (object ids must name built objects).
 *  d_out        [n_rays] per-ray result: the pair with the smallest t wins, ties
 *               going to the lowest instance index; normal in world space.
 *
 * All device pointers; asynchronous on `stream`.  Pairs are grouped by object
 * and ordered for coherence on the device; every object that the pairs name
 * must share one kernel class (feature type, MLP type, F, width) with the
 * other objects of the context, else LSNIF_E_INVALID.  A pair whose ray or
 * instance index is out of range, or whose instance names no built object,
 * contributes nothing.  Rays with no hit get the miss record. */
lsnif_status lsnif_query_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                               const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                               const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out,
                               void *stream);

/* Broad phase (Sec. 4, the step that lists which instances a ray may hit).
 * Pair (r, i) is listed when ray r, mapped into instance i's object space as
 * the pair query maps it, meets the object's voxel grid on [max(ta, tmin), tb]
 * with positive length (the slab test the pair query's narrow phase starts
 * with) and that segment starts no later than tmax (a hit's t lies in
 * [ta, tb] and must not exceed tmax), so every pair that can hit is listed.
 * Pairs come sorted by ray, then instance index; instances naming no built
 * object give none.
 *
 *  d_rays / d_inst  as for lsnif_query_pairs (device pointers).
 *  d_pair_ray, d_pair_inst  device buffers of `cap` entries each.
 *  n_pairs          host: receives the number of pairs.
 *
 * The pairs are counted on `stream`, which the call then synchronises once to
 * read the count; the writing pass is enqueued after it and returns without
 * waiting.  If the count exceeds cap, nothing is written and LSNIF_E_NOMEM is
 * returned with *n_pairs set.  n_rays x n_inst must be below 2^32 (else
 * LSNIF_E_INVALID).  Uses a workspace of the context: 4 bytes per ray, and
 * with at most 256 instances 4 more per ray and 32 instances, where the
 * counting pass keeps the instances each ray meets so that the writing pass
 * does not test them again. */
lsnif_status lsnif_broad_phase(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                               const lsnif_instance *d_inst, uint32_t n_inst, uint32_t *d_pair_ray,
                               uint32_t *d_pair_inst, uint32_t cap, uint32_t *n_pairs, void *stream);

/* World rays against instances: the broad phase above into the context's
 * workspace, then lsnif_query_pairs over its pairs; d_out[r] is ray r's
 * nearest hit (the same answer as lsnif_query_pairs given every pair that can
 * hit).  Synchronises `stream` once, after counting the pairs; the rest is
 * asynchronous.  Not for graph capture (the pair count is read on the host). */
lsnif_status lsnif_query_scene(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                               const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out, void *stream);

/* The consumer side of a wavefront path tracer (the paper renders with one,
 * Sec. 7): every ray i with a hit spawns one diffuse bounce ray, compacted in
 * the order of i, for the next lsnif_query_scene.  New origin x + eps n, with
 * x = o + t d evaluated per axis as o + (t d) and n the hit normal, negated
 * if it faces along d (the paper offsets new rays by a small epsilon along
 * the normal); direction (lx tx + ly bx) + lz n, cosine-distributed about n
 * (Malley's method: r = sqrt(u1), phi = 2 pi u2, lx = r cos phi,
 * ly = r sin phi, lz = sqrt(max(0, 1 - u1))) in the orthonormal basis of Duff
 * et al. 2017 (s = copysign(1, nz), a = -1 / (s + nz), b = nx ny a,
 * tx = (1 + s nx nx a, s b, -s nx), bx = (b, s + ny ny a, -ny)); tmin 0,
 * tmax +inf.  u1 = (h1 >> 8) 2^-24 and u2 = (h2 >> 8) 2^-24 with
 * h1 = pcg(i ^ pcg(seed ^ pcg(bounce))) and h2 = pcg(h1), pcg the PCG hash
 * of Jarzynski and Olano 2020.  d_parent[j] = the index of new ray j's
 * parent.  Counts on `stream`, synchronises it once to read the count into
 * *n_next, then writes asynchronously; LSNIF_E_NOMEM (nothing written) when
 * the count exceeds cap. */
lsnif_status lsnif_bounce(lsnif_ctx *ctx, const lsnif_ray *d_rays, const lsnif_hit *d_hits, uint32_t n, uint32_t seed,
                          uint32_t bounce, float eps, lsnif_ray *d_next, uint32_t *d_parent, uint32_t cap,
                          uint32_t *n_next, void *stream);

/* ------------------------------------------------------------------ tuning
 *
 * Launch parameters of an object that change speed but never a result (a
 * ray's answer does not depend on which rays share its tile or in what order
 * rays run, nor on whether a table entry is read from HBM or from LDS):
 *  sort_bits      single-object queries of at least 8192 rays are first sorted
 *                 by direction octant and by the cell of the voxel grid where
 *                 the ray's segment starts, 2^sort_bits cells per axis
 *                 (0 = no sort, 1..6), or at 7 by the cell alone (128 cells
 *                 per axis, no octant); rays that meet the grid close together
 *                 then share 256-ray tiles (the work decomposition of Sec. 4:
 *                 dispatch sorted rays rather than scattered ones).
 *  pair_bits      the same grouping, 2^pair_bits cells per axis (1..5), or at 6
 *                 by the cell alone (64 cells per axis, no octant), for the
 *                 object's pairs in pair queries, within the object's tiles.
 *  hot_lds_bytes  LDS per workgroup for the object's coarsest levels (0..40960):
 *                 those levels, all of whose used entries fit, are copied into
 *                 LDS by every workgroup and gathered from there.
 *  walk_chunks    tile ranges (1..16) of a direct or captured query: the voxel
 *                 walk of each range runs on a side stream of the context
 *                 (default priority) ahead of the query kernel, which starts on
 *                 range i as soon as its walk is done, so walk and query kernel
 *                 share the GPU.  1 (the default) walks the whole batch first.
 *                 Ranges hold at least 256 tiles; the serving loop always walks
 *                 whole requests.
 *  persistent     0 or 1: with 1, width-64 objects with a matrix-core MLP
 *                 run the query kernel as a persistent grid (as many
 *                 workgroups as the GPU holds at once) whose workgroups on
 *                 each XCD take tiles from that XCD's own contiguous eighth of
 *                 the coherence order, then from the tails of the others, so
 *                 each XCD's L2 serves one region of rays (or one object's
 *                 pairs) at a time; 0 launches one workgroup per tile, dealt to
 *                 the XCDs in runs of 8.  Width-128 and FP32-MLP objects always
 *                 take one workgroup per tile.
 * lsnif_autotune times each candidate (sort_bits 0, 4, 5, 6, 7 x hot_lds_bytes 0,
 * 20480, 40960, then walk_chunks 1, 2, 4, 8, then persistent 0 and 1, each for
 * the best so far) on the
 * caller's batch, a warm-up and three timed queries each on a private stream,
 * keeps the fastest for the object and returns it.  lsnif_autotune_pairs does
 * the same for a pair query (pair_bits 2, 3, 4, 5, 6 x hot_lds_bytes, then
 * walk_chunks, then persistent), applying one choice to every object of the context.  Both
 * overwrite d_out, synchronise the device and, like lsnif_set_tuning, make the
 * context's captured graphs stale.
 */
typedef struct {
    int32_t sort_bits;
    int32_t pair_bits;
    int32_t hot_lds_bytes;
    int32_t walk_chunks;
    int32_t persistent;
} lsnif_tuning;

lsnif_status lsnif_get_tuning(lsnif_ctx *ctx, uint32_t object_id, lsnif_tuning *tuning);
lsnif_status lsnif_set_tuning(lsnif_ctx *ctx, uint32_t object_id, const lsnif_tuning *tuning);
lsnif_status lsnif_autotune(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                            lsnif_hit *d_out, lsnif_tuning *best);
lsnif_status lsnif_autotune_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                                  const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                                  const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out,
                                  lsnif_tuning *best);

/* ------------------------------------------------------------------ graphs
 *
 * A query captured once into a HIP graph and replayed with one launch.  A
 * replay reruns the whole query (coherence sort or pair grouping, the query
 * kernel, the nearest-hit payload) on the buffers named at capture, so the
 * caller refills those buffers between replays; results equal the direct
 * call's on the same inputs.  A graph owns its workspace (allocated at
 * capture, freed by lsnif_graph_destroy) and reads the context's objects
 * through pointers taken at capture: after any lsnif_build or lsnif_release
 * on the context, lsnif_graph_launch returns LSNIF_E_INVALID.  Destroy every
 * graph before its context.  The capture runs on a private stream; the
 * context's kernel timing is not recorded inside graphs.
 *
 *  lsnif_graph_query  captures lsnif_query(ctx, object_id, d_rays, n, d_out).
 *  lsnif_graph_pairs  captures lsnif_query_pairs with the same arguments.
 *  lsnif_graph_launch enqueues one replay on `stream` (asynchronous).
 */
typedef struct lsnif_graph lsnif_graph;
lsnif_status lsnif_graph_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                               lsnif_hit *d_out, lsnif_graph **out);
lsnif_status lsnif_graph_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                               const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                               const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out,
                               lsnif_graph **out);
lsnif_status lsnif_graph_launch(lsnif_graph *graph, void *stream);
void lsnif_graph_destroy(lsnif_graph *graph);

/* ------------------------------------------------------------------ serving
 *
 * Continuous batching of queries that arrive over time (requests of many
 * sizes, single-object or instanced pairs).  A host thread admits waiting
 * requests in arrival order as soon as a slot and workspace within the HBM
 * budget are free, spreads admitted requests over several HIP streams so
 * their kernels overlap on the device, and frees each request's slot and
 * workspace when its work completes.  Small requests waiting together are
 * merged: the request at the head of the queue and the ones right behind it
 * with the same target (the same object_id, or pairs over the same d_inst and
 * n_inst), each of at most merge_rays rays, up to merge_max requests and
 * 8,388,608 rays in all, are admitted as one launch that takes one slot: their
 * rays and pairs are staged into one batch in the launch's workspace, one
 * query answers it, and each request's answers are copied to its own d_out;
 * they complete together.  Results are those of the direct calls: a request's
 * answer does not depend on what else is in flight or merged with it.
 *
 * The serve calls are thread-safe.  The caller owns every buffer a request
 * names and keeps it alive until the request is done; buffers are device
 * pointers.  Objects must not be built or released while requests are
 * admitted. */
typedef struct {
    uint32_t max_inflight;  /* requests admitted at once; 0 = 8 */
    uint64_t hbm_budget;    /* bytes of query workspace admitted requests may hold; 0 = 4 GiB */
    uint32_t n_streams;     /* HIP streams (default priority) requests are spread over; 0 = 4 */
    uint32_t max_queue;     /* waiting requests beyond which submit returns LSNIF_E_BUSY; 0 = 65536 */
    uint64_t dry_run_ns_per_ray; /* > 0: touch no device; a request "completes" this many ns per
                                    ray after admission and writes nothing (tests of the
                                    admission logic on hosts without a GPU; merged launches
                                    take the time of all their rays) */
    uint32_t merge_rays;    /* largest request (rays) that may be merged; 0 = 262144 */
    uint32_t merge_max;     /* requests per merged launch, 1..32 (1: no merging); 0 = 32 */
} lsnif_serve_cfg;

enum { LSNIF_REQ_SINGLE = 0, LSNIF_REQ_PAIRS = 1 };

typedef struct {
    int32_t kind;                    /* LSNIF_REQ_SINGLE (object_id, rays) or LSNIF_REQ_PAIRS */
    uint32_t object_id;              /* single-object request: the object */
    const lsnif_ray *d_rays;         /* [n_rays] */
    uint32_t n_rays;
    const uint32_t *d_pair_ray;      /* pair request: [n_pairs] ray and instance indices (may be
                                        NULL when n_pairs is 0) */
    const uint32_t *d_pair_inst;
    uint32_t n_pairs;
    const lsnif_instance *d_inst;    /* [n_inst] */
    uint32_t n_inst;
    lsnif_hit *d_out;                /* [n_rays] */
    int64_t timeout_ns;              /* > 0: dropped with LSNIF_E_TIMEOUT if not admitted in time */
} lsnif_request;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, cancelled, timed_out, failed;
    uint64_t queued, inflight;       /* at the time of the call */
    uint64_t rays_completed;
    uint64_t ws_bytes_peak;          /* most workspace held at once */
    double p50_ms, p99_ms, mean_ms, max_ms;   /* submit -> completion, completed requests */
    double elapsed_s;                /* since lsnif_serve_start */
    uint64_t launches;               /* admitted launches (a merged launch answers several requests) */
} lsnif_serve_stats;

/* Request states reported by lsnif_serve_poll (negative values are the final
 * lsnif_status of a request that did not complete). */
enum { LSNIF_REQ_QUEUED = 0, LSNIF_REQ_RUNNING = 1, LSNIF_REQ_DONE = 2 };

lsnif_status lsnif_serve_start(lsnif_ctx *ctx, const lsnif_serve_cfg *cfg);
/* LSNIF_E_NOMEM: the request's workspace can never fit the budget;
 * LSNIF_E_BUSY: the queue is full; LSNIF_E_INVALID / E_NOTFOUND: bad request. */
lsnif_status lsnif_serve_submit(lsnif_ctx *ctx, const lsnif_request *req, uint64_t *ticket);
lsnif_status lsnif_serve_poll(lsnif_ctx *ctx, uint64_t ticket, int32_t *state);
/* Waits until the request is finished: returns its final status (LSNIF_OK when
 * it completed), or LSNIF_E_TIMEOUT if timeout_ns (>= 0) passes first. */
lsnif_status lsnif_serve_wait(lsnif_ctx *ctx, uint64_t ticket, int64_t timeout_ns);
/* Cancels a waiting request (LSNIF_E_BUSY once admitted). */
lsnif_status lsnif_serve_cancel(lsnif_ctx *ctx, uint64_t ticket);
lsnif_status lsnif_serve_stats_get(lsnif_ctx *ctx, lsnif_serve_stats *stats);
/* Waits for admitted requests, cancels waiting ones, stops the loop. */
lsnif_status lsnif_serve_stop(lsnif_ctx *ctx);

/* ------------------------------------------------------------------ training
 * Joint optimisation of an object's hash-grid tables and MLP weights with
 * Adam (Sec. 5.2) under the per-signal activations and losses of Sec. 5.3.
 *
 * A trainer works on an object of the context built with FP32 features and an
 * FP32 MLP, in place: the object's device tables and weights ARE the trained
 * parameters, so the object answers lsnif_query with the current parameters
 * between steps (a query and a step in flight at once race).  The trainer
 * adds, on the device, first and second moments of every parameter, the
 * weight gradients, up to 8 copies of the table gradient (as many as fit in
 * 1 GiB, at least one; the scatter spreads its atomics over them) and a
 * per-step workspace that grows with the batch (about 4 (in_dim + n_hidden
 * width + 2 outputs) + 4 H/2 + 1 bytes per ray, plus the weight-gradient
 * partial sums, a few tens of MB).
 *
 * Loss of one training batch of n rays: (1/n) sum over the rays of
 *   softplus(z0) - y.hit z0                                  occlusion: sigmoid + binary cross-entropy
 *   + y.hit * ( |sigmoid(z1) - tau|                          local hit distance: sigmoid + mean absolute error
 *             + 1 - <zn, y.n> / max(|zn|, 1e-8)              normal: identity + cosine similarity
 *             + mean_c (a_c - y.albedo_c)^2 / (a'_c + 0.01)^2   albedo (objects with the head):
 *                                                            a = sigmoid(z_a), a' = a held constant
 *                                                            (relative L2 of Lehtinen et al. 2018)
 *             + logsumexp(zm) - zm[y.material] )             material: softmax + categorical cross-entropy
 * where z are the object's raw network outputs for the ray (zn = z2..z4,
 * z_a the albedo outputs, zm the material logits), tau = (y.t - ta) /
 * (tb - ta) clamped to [0, 1] over the ray's AABB interval [ta, tb], and a
 * ray with no listed voxel adds nothing (its network input is zero and a query
 * calls it a miss without running the network).  The non-occlusion terms are
 * zero when the reference says miss, as the paper prescribes.  |x| at 0 and
 * the activation at 0 take derivative 0; the leaky slope applies below 0.
 *
 * Adam (Kingma and Ba 2015), per parameter, step t = 1, 2, ...:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * over every table entry and weight (dense), moments starting at 0.  The
 * paper's setting is lr 0.01 with batches of 2^18 rays. */
typedef struct lsnif_trainer lsnif_trainer;

/* A trainer's gradients, moments and workspace are shared by its calls: steps
 * on one trainer must be ordered (one stream, or synchronised between
 * streams).  Calls take the context's lock while they enqueue;
 * lsnif_trainer_destroy must not overlap another call on the same trainer. */

/* Reference signals of one training ray (from ray casting the true geometry). */
typedef struct {
    uint32_t hit;        /* 1: the ray hits the object, at parameter t of the ray */
    float t;
    float n[3];          /* unit shading normal at the hit */
    float albedo[3];     /* read when the object has an albedo head */
    int32_t material;    /* 0 .. n_mat - 1 */
} lsnif_train_target;    /* 36 bytes */

typedef struct {
    float lr, beta1, beta2, eps;
} lsnif_adam_cfg;

/* Creates a trainer for object_id (FP32 features and MLP, else
 * LSNIF_E_INVALID); cfg NULL means lr 0.01, b1 0.9, b2 0.999, eps 1e-8.  The
 * object must outlive the trainer. */
lsnif_status lsnif_trainer_create(lsnif_ctx *ctx, uint32_t object_id, const lsnif_adam_cfg *cfg, lsnif_trainer **out);
/* Waits for the device and frees the trainer's buffers; the object keeps its
 * trained parameters. */
void lsnif_trainer_destroy(lsnif_trainer *tr);
/* Forward pass, loss and backward pass of one batch (device buffers, n >= 1,
 * at most 2^24; rays 16-byte and targets 4-byte aligned): the gradients of the
 * batch loss replace the trainer's gradients and the loss goes to d_loss[0]
 * (device float; NULL skips it).  Targets must be finite where hit = 1.
 * Asynchronous on `stream`; the trainer's workspace grows to the batch
 * (LSNIF_E_NOMEM if it cannot). */
lsnif_status lsnif_train_grads(lsnif_trainer *tr, const lsnif_ray *d_rays, const lsnif_train_target *d_gt,
                               uint32_t n, float *d_loss, void *stream);
/* One Adam step with the trainer's current gradients.  Asynchronous. */
lsnif_status lsnif_train_apply(lsnif_trainer *tr, void *stream);
/* lsnif_train_grads then lsnif_train_apply: one training step. */
lsnif_status lsnif_train_step(lsnif_trainer *tr, const lsnif_ray *d_rays, const lsnif_train_target *d_gt,
                              uint32_t n, float *d_loss, void *stream);
/* Host copies of the parameters and gradients (synchronises the device; any
 * pointer may be NULL): tables as [L][2^log2_T][F], weights per layer
 * row-major [out][in] as in lsnif_object_desc; *steps = Adam steps taken. */
lsnif_status lsnif_trainer_read(lsnif_trainer *tr, float *tables, float *const *W, float *grad_tables,
                                float *const *grad_W, uint64_t *steps);
/* Training kernel time.  While the trainer's context has kernel timing on
 * (lsnif_profile_enable), every lsnif_train_grads / lsnif_train_step records
 * HIP events on its stream around the forward layer products, around the
 * backward layer products (weight and input gradients, with the partial-product
 * sums), and around the scatter of the encoding's gradient onto the tables.
 * This call waits for those events and returns, summed over the steps since
 * the last read, the layer products' milliseconds (forward + backward) and the
 * scatter's, and the number of steps (any pointer may be NULL). */
lsnif_status lsnif_train_profile_read(lsnif_trainer *tr, double *products_ms, double *scatter_ms,
                                      uint32_t *steps);

/* Kernel timing.  While enabled, every query on the context records HIP
 * events on its stream before the coherence sort (pair queries: the pair
 * preparation), before the voxel-walk kernel, before the query kernel and
 * after it.  lsnif_profile_read waits for the recorded queries, returns the
 * summed milliseconds of the three phases and the number of queries since the
 * last read, and forgets them.  Any output pointer may be NULL.  When the walk
 * runs ahead in ranges (walk_chunks > 1), the walk phase ends once the query
 * kernel may start on the first range and the query phase holds the rest. */
lsnif_status lsnif_profile_enable(lsnif_ctx *ctx, int32_t on);
lsnif_status lsnif_profile_read(lsnif_ctx *ctx, double *sort_ms, double *walk_ms, double *kernel_ms,
                                uint64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* LSNIF_H */
