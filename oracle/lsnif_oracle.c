/*
 * LSNIF query oracle: a plain, slow CPU definition of what one LSNIF query
 * computes, written from the paper (Fujieda, Kao, Harada, "LSNIF:
 * Locally-Subdivided Neural Intersection Function", 2025).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with
 * the GPU library and must never serve a product query.
 *
 * Precision: the slab test, the voxel walk, the boundary points and the
 * grid-vertex indices are float32 (every operation written out, no fused
 * multiply-add: build with -ffp-contract=off); interpolation, the MLP and the
 * decode are float64 from the float32 master tables and weights.
 *
 * Passages followed, per step:
 *   - ray / AABB slab and voxel walk: Sec. 3.1 (voxels hit by the ray found
 *     with a DDA, then ray-box intersection points on their boundaries) and
 *     Sec. 4 (narrow phase).
 *   - boundary points: Sec. 3.1 and 3.2 (all inputs lie on voxel boundaries).
 *   - cap H and zero fill: Sec. 5.1.
 *   - sparse multiresolution hash-grid encoding, concatenation: Sec. 3.2.
 *   - MLP without biases, hidden activations: Sec. 3.3, 5.1.
 *   - output heads, 0.5 threshold, local hit distance over the ray-AABB
 *     interval: Sec. 5.1, 5.3.
 *   - per-ray hit update from the nearest LSNIF hit: Sec. 4.
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes): two points per occupied voxel, entry then exit, in walk
 * order; only voxels overlapping [max(t_aabb_in, tmin), t_aabb_out] with
 * positive length; the first H/2 such voxels; the hash of Mueller et al.
 * 2022 (Eq. 4) with direct indexing when a level's (R+1)^3 vertices fit in
 * the table; level vertices 0..R spanning the voxel-grid box; a hit iff the
 * occlusion logit is > 0 and the hit distance is <= tmax; material = lowest
 * index among the maximal logits; normal = normalised linear head; when an
 * object asks for it, a grazing voxel (float32 overlap at most
 * 2^-16 max(1, |entry|)) is listed by its float64 slab interval instead.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_RELU 0
#define OR_LEAKY 1

typedef struct {
    float bmin[3], bmax[3];
    int32_t V;
    const uint32_t *occ;       /* V^3 bits, bit x + V*(y + V*z), LSB first */
    int32_t L, F, log2_T;
    const int32_t *R;          /* L level resolutions */
    const float *tables;       /* [L][T][F] */
    int32_t H;
    int32_t n_layers;          /* weight matrices, hidden + 1 */
    const int32_t *dims;       /* n_layers + 1 widths, dims[0] = H*L*F */
    const float *const *W;     /* row-major [out][in], no biases */
    int32_t act;
    float leaky_slope;
    int32_t n_mat, has_albedo;
    int32_t grazing_recheck;   /* 1: grazing voxels of the walk are re-decided in float64 */
} oracle_object;

/* Per-ray walk result. */
typedef struct {
    int32_t valid;             /* passes the validity rules */
    int32_t candidate;         /* ta < tb */
    float ta, tb;
    float o[3], d[3];          /* voxel-space origin and direction */
    int32_t nvox;
    int32_t ijk[64][3];
    float tin[64], tout[64];
    int32_t in_axis[64], out_axis[64];
} walk_t;

static float fmin2(float a, float b) { return a < b ? a : b; }
static float fmax2(float a, float b) { return a > b ? a : b; }

/* Plane function of one axis: the ray parameter where the line crosses the
 * voxel-space plane x_a = k. */
static float plane_t(float k, float o, float inv) { return (k - o) * inv; }

static int occupied(const oracle_object *ob, int x, int y, int z)
{
    int64_t V = ob->V;
    int64_t bit = (int64_t)x + V * ((int64_t)y + V * (int64_t)z);
    return (ob->occ[bit >> 5] >> (bit & 31)) & 1u;
}

/* Validity: no NaN anywhere, no infinity in origin or direction, a non-zero
 * direction, tmin <= tmax.  An invalid ray is reported as a miss. */
static int ray_valid(const float *r)
{
    for (int i = 0; i < 8; ++i)
        if (isnan(r[i])) return 0;
    for (int i = 0; i < 6; ++i)
        if (isinf(r[i])) return 0;
    if (r[3] == 0.0f && r[4] == 0.0f && r[5] == 0.0f) return 0;
    if (r[6] > r[7]) return 0;
    return 1;
}

/* Entry and exit parameter of cell k on one moving axis. */
static float cell_entry(int k, float o, float inv, float d)
{
    return d > 0.0f ? plane_t((float)k, o, inv) : plane_t((float)(k + 1), o, inv);
}
static float cell_exit(int k, float o, float inv, float d)
{
    return d > 0.0f ? plane_t((float)(k + 1), o, inv) : plane_t((float)k, o, inv);
}

/*
 * Optional float64 re-decision of a voxel the float32 walk finds grazing: its
 * overlap with [ta, tb] is no longer than 2^-16 max(1, |entry|), or the whole
 * segment [ta, tb] is that short.  The slab intervals of the voxel and of the
 * grid are recomputed in float64 from the same float32 voxel-space origin and
 * direction, over the axes the float32 walk treats as moving, and the voxel is
 * kept iff the float64 overlap has positive length.  Only the decision to list
 * a voxel the walk visits changes; its t values stay the float32 ones.
 */
static int grazing(float tin, float tout, float ta, float tb)
{
    const float lo = fmax2(tin, ta), hi = fmin2(tout, tb);
    const float q = 0x1p-16f;
    return hi - lo <= q * fmax2(1.0f, fabsf(tin)) || tb - ta <= q * fmax2(1.0f, fabsf(ta));
}

static int keep_f64(const walk_t *w, const int moving[3], const int c[3], int V, float tmin)
{
    double t0 = -INFINITY, t1 = INFINITY, tin = -INFINITY, tout = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (!moving[a]) continue;
        const double o = w->o[a], d = w->d[a];
        const double g0 = (0.0 - o) / d, g1 = ((double)V - o) / d;
        const double e0 = ((double)c[a] - o) / d, e1 = ((double)(c[a] + 1) - o) / d;
        t0 = fmax(t0, fmin(g0, g1));
        t1 = fmin(t1, fmax(g0, g1));
        tin = fmax(tin, fmin(e0, e1));
        tout = fmin(tout, fmax(e0, e1));
    }
    const double ta = fmax(t0, (double)tmin), tb = t1;
    return fmin(tout, tb) > fmax(tin, ta);
}

/*
 * Ray-AABB slab test, then the voxel walk over the occupancy grid
 * (Amanatides-Woo style DDA).  Every decision compares values of the same
 * per-axis plane function, so the emitted list equals the list obtained by
 * slab-testing every voxel on its own.
 */
/* Validity rules and the ray/AABB slab test in voxel space: fills valid, o, d,
 * ta, tb and candidate (ta < tb), and each axis' reciprocal and moving flag. */
static void segment(const oracle_object *ob, const float *ray, walk_t *w, float inv[3], int moving[3])
{
    memset(w, 0, sizeof(*w));
    moving[0] = moving[1] = moving[2] = 0;
    inv[0] = inv[1] = inv[2] = 0.0f;
    if (!ray_valid(ray)) return;
    w->valid = 1;
    const int V = ob->V;
    for (int a = 0; a < 3; ++a) {
        float s = (float)V / (ob->bmax[a] - ob->bmin[a]);
        w->o[a] = (ray[a] - ob->bmin[a]) * s;
        w->d[a] = ray[3 + a] * s;
        moving[a] = 0;
        inv[a] = 0.0f;
        if (w->d[a] != 0.0f) {
            float iv = 1.0f / w->d[a];
            if (isfinite(iv)) { moving[a] = 1; inv[a] = iv; }
        }
    }
    /* slab */
    float t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (moving[a]) {
            float lo = plane_t(0.0f, w->o[a], inv[a]);
            float hi = plane_t((float)V, w->o[a], inv[a]);
            t0 = fmax2(t0, fmin2(lo, hi));
            t1 = fmin2(t1, fmax2(lo, hi));
        } else if (!(w->o[a] >= 0.0f && w->o[a] <= (float)V)) {
            return;
        }
    }
    if (!moving[0] && !moving[1] && !moving[2]) return;
    w->ta = fmax2(t0, ray[6]);
    w->tb = t1;
    w->candidate = w->ta < w->tb;
}

static void walk(const oracle_object *ob, const float *ray, walk_t *w)
{
    float inv[3];
    int moving[3];
    segment(ob, ray, w, inv, moving);
    if (!w->candidate) return;
    const int V = ob->V;
    const float ta = w->ta, tb = w->tb;

    /* start cell: on a moving axis the unique cell whose [entry, exit)
     * contains ta (found by scanning every cell: slow and plain); on a still
     * axis the half-open cell of the origin, V mapping to V-1 */
    int c[3];
    for (int a = 0; a < 3; ++a) {
        if (moving[a]) {
            c[a] = -1;
            for (int k = 0; k < V; ++k) {
                float en = cell_entry(k, w->o[a], inv[a], w->d[a]);
                float ex = cell_exit(k, w->o[a], inv[a], w->d[a]);
                if (en <= ta && ta < ex) { c[a] = k; break; }
            }
            if (c[a] < 0) { w->candidate = 0; return; }   /* unreachable */
        } else {
            int k = (int)floorf(w->o[a]);
            c[a] = k > V - 1 ? V - 1 : k;
        }
    }
    const int cap = ob->H / 2;
    for (;;) {
        float tin = -INFINITY, tout = INFINITY;
        int ia = -1, oa = -1;
        for (int a = 0; a < 3; ++a) {
            if (!moving[a]) continue;
            float en = cell_entry(c[a], w->o[a], inv[a], w->d[a]);
            float ex = cell_exit(c[a], w->o[a], inv[a], w->d[a]);
            if (ia < 0 || en > tin) { tin = en; ia = a; }
            if (oa < 0 || ex < tout) { tout = ex; oa = a; }
        }
        int keep = fmin2(tout, tb) > fmax2(tin, ta);
        if (ob->grazing_recheck && grazing(tin, tout, ta, tb)) keep = keep_f64(w, moving, c, V, ray[6]);
        if (occupied(ob, c[0], c[1], c[2]) && keep) {
            int j = w->nvox++;
            for (int a = 0; a < 3; ++a) w->ijk[j][a] = c[a];
            w->tin[j] = tin;
            w->tout[j] = tout;
            w->in_axis[j] = ia;
            w->out_axis[j] = oa;
            if (w->nvox == cap) break;
        }
        if (tout >= tb) break;
        c[oa] += w->d[oa] > 0.0f ? 1 : -1;
        if (c[oa] < 0 || c[oa] >= V) break;
    }
}

/* Boundary point of voxel j: point 2j is where the line enters the voxel,
 * point 2j+1 where it leaves.  On the crossing axis the coordinate is the
 * integer face plane itself; other coordinates are evaluated on the line and
 * clamped into the voxel. */
static void boundary_point(const walk_t *w, int h, float p[3])
{
    int j = h >> 1, is_exit = h & 1;
    float t = is_exit ? w->tout[j] : w->tin[j];
    int face = is_exit ? w->out_axis[j] : w->in_axis[j];
    for (int b = 0; b < 3; ++b) {
        float lo = (float)w->ijk[j][b], hi = (float)(w->ijk[j][b] + 1);
        if (b == face) {
            int upper = (w->d[b] > 0.0f) == (is_exit != 0);
            p[b] = upper ? hi : lo;
        } else {
            float v = w->o[b] + t * w->d[b];
            p[b] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
}

/* Grid vertex of level l covering p (voxel space): cell origin i, fractional
 * weights w, and the table slots of the 8 cell corners, corner bit b of the
 * slot number = offset on axis b. */
static void level_corners(const oracle_object *ob, int l, const float p[3],
                          uint32_t slot[8], float wt[3])
{
    const int32_t R = ob->R[l];
    const uint64_t T = (uint64_t)1 << ob->log2_T;
    const float scale = (float)R / (float)ob->V;
    uint32_t i[3];
    for (int b = 0; b < 3; ++b) {
        float x = p[b] * scale;
        if (x < 0.0f) x = 0.0f;
        if (x > (float)R) x = (float)R;
        int k = (int)floorf(x);
        if (k > R - 1) k = R - 1;
        i[b] = (uint32_t)k;
        wt[b] = x - (float)k;
    }
    const uint64_t side = (uint64_t)R + 1;
    const int dense = side * side * side <= T;
    for (int cidx = 0; cidx < 8; ++cidx) {
        uint32_t vx = i[0] + (cidx & 1), vy = i[1] + ((cidx >> 1) & 1), vz = i[2] + ((cidx >> 2) & 1);
        if (dense) {
            slot[cidx] = (uint32_t)(vx + side * (vy + side * vz));
        } else {
            /* Mueller et al. 2022, Eq. 4: xor of coordinate times prime, mod T */
            uint32_t hsh = (vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u);
            slot[cidx] = (uint32_t)(hsh & (uint32_t)(T - 1));
        }
    }
}

/* Trilinear interpolation of the F features of level l at one point
 * (float64; zero-weight corners included). */
static void interpolate(const oracle_object *ob, int l, const uint32_t slot[8], const float wt[3],
                        double *feat)
{
    const size_t T = (size_t)1 << ob->log2_T;
    const float *tab = ob->tables + (size_t)l * T * ob->F;
    for (int f = 0; f < ob->F; ++f) feat[f] = 0.0;
    for (int cidx = 0; cidx < 8; ++cidx) {
        double wx = (cidx & 1) ? (double)wt[0] : 1.0 - (double)wt[0];
        double wy = ((cidx >> 1) & 1) ? (double)wt[1] : 1.0 - (double)wt[1];
        double wz = ((cidx >> 2) & 1) ? (double)wt[2] : 1.0 - (double)wt[2];
        double wgt = (wx * wy) * wz;
        for (int f = 0; f < ob->F; ++f)
            feat[f] += wgt * (double)tab[(size_t)slot[cidx] * ob->F + f];
    }
}

/* Fully connected layers without biases; activation after every hidden layer. */
static void mlp(const oracle_object *ob, const double *in, double *out, double *buf_a, double *buf_b)
{
    const double *x = in;
    for (int k = 0; k < ob->n_layers; ++k) {
        const int ni = ob->dims[k], no = ob->dims[k + 1];
        double *y = (k == ob->n_layers - 1) ? out : ((k & 1) ? buf_b : buf_a);
        const float *Wk = ob->W[k];
        for (int j = 0; j < no; ++j) {
            double s = 0.0;
            for (int i = 0; i < ni; ++i) s += (double)Wk[(size_t)j * ni + i] * x[i];
            if (k < ob->n_layers - 1) {
                if (ob->act == OR_LEAKY) s = s > 0.0 ? s : (double)ob->leaky_slope * s;
                else s = s > 0.0 ? s : 0.0;
            }
            y[j] = s;
        }
        x = y;
    }
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

typedef struct {
    int32_t *count;            /* [n] boundary points (2 per voxel), -1 invalid ray */
    float *tatb;               /* [n][2] */
    int32_t *vox_ijk;          /* [n][H/2][3] */
    float *vox_t;              /* [n][H/2][2] tin, tout */
    int8_t *vox_axis;          /* [n][H/2][2] entry axis, exit axis */
    float *points;             /* [n][H][3] */
    uint32_t *slots;           /* [n][H][L][8] */
    float *weights;            /* [n][H][L][3] */
    double *enc;               /* [n][H*L*F] */
    double *out;               /* [n][out_dim] raw network outputs */
    uint32_t *hit;             /* [n] */
    float *t;                  /* [n] */
    float *nrm;                /* [n][3] */
    int32_t *material;         /* [n] */
    float *albedo;             /* [n][3] */
} oracle_outputs;

static void query_one(const oracle_object *ob, const float *ray, int64_t r, const oracle_outputs *o,
                      walk_t *w, double *enc, double *out, double *ba, double *bb)
{
    const int H = ob->H, L = ob->L, F = ob->F;
    const int in_dim = H * L * F, out_dim = ob->dims[ob->n_layers];
    walk(ob, ray, w);
    const int count = 2 * w->nvox;
    if (o->count) o->count[r] = w->valid ? count : -1;
    if (o->tatb) { o->tatb[2 * r] = w->ta; o->tatb[2 * r + 1] = w->tb; }
    if (o->vox_ijk || o->vox_t || o->vox_axis) {
        for (int j = 0; j < H / 2; ++j) {
            int in = j < w->nvox;
            for (int a = 0; a < 3; ++a)
                if (o->vox_ijk) o->vox_ijk[(r * (H / 2) + j) * 3 + a] = in ? w->ijk[j][a] : -1;
            if (o->vox_t) {
                o->vox_t[(r * (H / 2) + j) * 2] = in ? w->tin[j] : 0.0f;
                o->vox_t[(r * (H / 2) + j) * 2 + 1] = in ? w->tout[j] : 0.0f;
            }
            if (o->vox_axis) {
                o->vox_axis[(r * (H / 2) + j) * 2] = (int8_t)(in ? w->in_axis[j] : -1);
                o->vox_axis[(r * (H / 2) + j) * 2 + 1] = (int8_t)(in ? w->out_axis[j] : -1);
            }
        }
    }
    /* encoding: points beyond the count stay zero */
    for (int i = 0; i < in_dim; ++i) enc[i] = 0.0;
    for (int h = 0; h < H; ++h) {
        float p[3] = {0.0f, 0.0f, 0.0f};
        if (h < count) boundary_point(w, h, p);
        if (o->points)
            for (int b = 0; b < 3; ++b) o->points[(r * H + h) * 3 + b] = h < count ? p[b] : 0.0f;
        for (int l = 0; l < L; ++l) {
            uint32_t slot[8] = {0};
            float wt[3] = {0.0f, 0.0f, 0.0f};
            if (h < count) {
                level_corners(ob, l, p, slot, wt);
                interpolate(ob, l, slot, wt, enc + ((size_t)h * L + l) * F);
            }
            if (o->slots)
                for (int cc = 0; cc < 8; ++cc) o->slots[((r * H + h) * L + l) * 8 + cc] = slot[cc];
            if (o->weights)
                for (int b = 0; b < 3; ++b) o->weights[((r * H + h) * L + l) * 3 + b] = wt[b];
        }
    }
    if (o->enc) memcpy(o->enc + r * in_dim, enc, sizeof(double) * in_dim);
    /* a ray with no occupied voxel is a miss and the network is not run */
    int hit = 0;
    double t_hit = INFINITY;
    double n[3] = {0.0, 0.0, 0.0}, alb[3] = {0.0, 0.0, 0.0};
    int mat = -1;
    for (int k = 0; k < out_dim; ++k) out[k] = 0.0;
    if (count > 0) {
        mlp(ob, enc, out, ba, bb);
        t_hit = (double)w->ta + sigmoid(out[1]) * ((double)w->tb - (double)w->ta);
        hit = out[0] > 0.0 && t_hit <= (double)ray[7];
    }
    if (o->out) memcpy(o->out + r * out_dim, out, sizeof(double) * out_dim);
    if (hit) {
        double nn = sqrt(out[2] * out[2] + out[3] * out[3] + out[4] * out[4]);
        for (int b = 0; b < 3; ++b) n[b] = nn > 0.0 ? out[2 + b] / nn : 0.0;
        int m0 = 5 + 3 * ob->has_albedo;
        mat = 0;
        for (int k = 1; k < ob->n_mat; ++k)
            if (out[m0 + k] > out[m0 + mat]) mat = k;
        if (ob->has_albedo)
            for (int b = 0; b < 3; ++b) alb[b] = sigmoid(out[5 + b]);
    } else {
        t_hit = INFINITY;
    }
    if (o->hit) o->hit[r] = (uint32_t)hit;
    if (o->t) o->t[r] = (float)t_hit;
    if (o->nrm) for (int b = 0; b < 3; ++b) o->nrm[r * 3 + b] = (float)n[b];
    if (o->material) o->material[r] = mat;
    if (o->albedo) for (int b = 0; b < 3; ++b) o->albedo[r * 3 + b] = (float)alb[b];
}

/* Threads the parallel loops use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Query n rays against one object; any NULL output array is skipped. */
int oracle_query(const oracle_object *ob, const float *rays, int64_t n, const oracle_outputs *o)
{
    if (ob->H > 128 || (ob->H & 1)) return -1;
    const int in_dim = ob->H * ob->L * ob->F;
    int maxw = 0;
    for (int k = 0; k <= ob->n_layers; ++k) if (ob->dims[k] > maxw) maxw = ob->dims[k];
    if (ob->dims[0] != in_dim) return -1;
    int err = 0;
#pragma omp parallel
    {
        walk_t *w = (walk_t *)malloc(sizeof(walk_t));
        double *enc = (double *)malloc(sizeof(double) * in_dim);
        double *out = (double *)malloc(sizeof(double) * maxw);
        double *ba = (double *)malloc(sizeof(double) * maxw);
        double *bb = (double *)malloc(sizeof(double) * maxw);
        if (!w || !enc || !out || !ba || !bb) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t r = 0; r < n; ++r) query_one(ob, rays + 8 * r, r, o, w, enc, out, ba, bb);
        }
        free(w); free(enc); free(out); free(ba); free(bb);
    }
    return err;
}

/* Instanced query over (ray, instance) pairs with the nearest hit per ray.
 * Each instance holds an object index and a row-major 3x4 world-to-object
 * matrix A|b; rays are mapped with x_obj = A x + b, d_obj = A d (not
 * renormalised, so t is shared by both spaces).  Per ray the smallest t wins,
 * ties going to the lowest instance index; the winner's normal goes back to
 * world space as normalize(A^T n). */
typedef struct {
    int32_t object;
    float m[12];
} oracle_instance;

/* World ray rw mapped into an instance's object space: x_obj = A x + b, d_obj = A d, each
 * row evaluated as ((m0 x + m1 y) + m2 z) + m3; an invalid world ray stays invalid. */
static void to_object(const oracle_instance *I, const float *rw, float ro[8])
{
    for (int a = 0; a < 3; ++a) {
        const float *m = I->m + 4 * a;
        ro[a] = ((m[0] * rw[0] + m[1] * rw[1]) + m[2] * rw[2]) + m[3];
        ro[3 + a] = (m[0] * rw[3] + m[1] * rw[4]) + m[2] * rw[5];
    }
    ro[6] = rw[6];
    ro[7] = rw[7];
    if (!ray_valid(rw)) ro[0] = NAN;
}

int oracle_query_pairs(const oracle_object *objs, const oracle_instance *inst, int32_t n_inst,
                       const float *rays, int64_t n_rays, const uint32_t *pair_ray,
                       const uint32_t *pair_inst, int64_t n_pairs,
                       uint32_t *hit, float *t, float *nrm, int32_t *material, int32_t *winner)
{
    (void)n_inst;
    const size_t np = (size_t)(n_pairs > 0 ? n_pairs : 1);
    uint32_t *ph = (uint32_t *)malloc(sizeof(uint32_t) * np);
    float *pt = (float *)malloc(sizeof(float) * np);
    float *pn = (float *)malloc(sizeof(float) * 3 * np);
    int32_t *pm = (int32_t *)malloc(sizeof(int32_t) * np);
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rays > 0 ? n_rays : 1));
    int err = (!ph || !pt || !pn || !pm || !best) ? -2 : 0;
    if (!err) {
#pragma omp parallel
        {
            int maxw = 0;
            for (int32_t i = 0; i < n_inst; ++i) {
                const oracle_object *ob = &objs[inst[i].object];
                for (int k = 0; k <= ob->n_layers; ++k) if (ob->dims[k] > maxw) maxw = ob->dims[k];
            }
            walk_t *w = (walk_t *)malloc(sizeof(walk_t));
            double *enc = (double *)malloc(sizeof(double) * maxw);
            double *out = (double *)malloc(sizeof(double) * maxw);
            double *ba = (double *)malloc(sizeof(double) * maxw);
            double *bb = (double *)malloc(sizeof(double) * maxw);
            oracle_outputs o;
            memset(&o, 0, sizeof(o));
            o.hit = ph; o.t = pt; o.nrm = pn; o.material = pm;
            if (!w || !enc || !out || !ba || !bb) {
#pragma omp atomic write
                err = -2;
            } else {
#pragma omp for schedule(dynamic, 64)
                for (int64_t p = 0; p < n_pairs; ++p) {
                    const oracle_instance *I = &inst[pair_inst[p]];
                    float ro[8];
                    to_object(I, rays + 8 * (int64_t)pair_ray[p], ro);
                    query_one(&objs[I->object], ro, p, &o, w, enc, out, ba, bb);
                }
            }
            free(w); free(enc); free(out); free(ba); free(bb);
        }
    }
    if (!err) {
        for (int64_t r = 0; r < n_rays; ++r) {
            hit[r] = 0; t[r] = INFINITY; material[r] = -1; best[r] = -1;
            nrm[3 * r] = nrm[3 * r + 1] = nrm[3 * r + 2] = 0.0f;
        }
        for (int64_t p = 0; p < n_pairs; ++p) {
            if (!ph[p]) continue;
            uint32_t r = pair_ray[p];
            int32_t ii = (int32_t)pair_inst[p];
            if (hit[r] && !(pt[p] < t[r] || (pt[p] == t[r] && ii < best[r]))) continue;
            hit[r] = 1;
            t[r] = pt[p];
            material[r] = pm[p];
            best[r] = ii;
            const float *m = inst[ii].m;
            double wn[3];
            for (int b = 0; b < 3; ++b)
                wn[b] = (double)m[b] * pn[3 * p] + (double)m[4 + b] * pn[3 * p + 1] + (double)m[8 + b] * pn[3 * p + 2];
            double nn = sqrt(wn[0] * wn[0] + wn[1] * wn[1] + wn[2] * wn[2]);
            for (int b = 0; b < 3; ++b) nrm[3 * r + b] = nn > 0.0 ? (float)(wn[b] / nn) : 0.0f;
        }
        if (winner) for (int64_t r = 0; r < n_rays; ++r) winner[r] = best[r];
    }
    free(ph); free(pt); free(pn); free(pm); free(best);
    return err;
}

/* Broad phase (Sec. 4, the step that finds which instances a ray may hit):
 * pair (r, i) exists when ray r, mapped into instance i's object space as
 * above, meets the object's voxel grid on [max(ta, tmin), tb] with positive
 * length (the narrow phase's slab test makes it a candidate) and that
 * segment starts no later than tmax; no other pair can hit, since a hit's t
 * lies in [ta, tb] and must not exceed tmax.  counts[r] receives ray r's
 * number of pairs.  Pairs are listed by ray, then instance; at most cap are
 * written.  Returns the total. */
int64_t oracle_broad_phase(const oracle_object *objs, const oracle_instance *inst, int32_t n_inst,
                           const float *rays, int64_t n_rays, uint32_t *counts, uint32_t *pair_ray,
                           uint32_t *pair_inst, int64_t cap)
{
#pragma omp parallel
    {
        walk_t *w = (walk_t *)malloc(sizeof(walk_t));
        float inv[3], ro[8];
        int moving[3];
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < n_rays; ++r) {
            uint32_t c = 0;
            for (int32_t i = 0; w && i < n_inst; ++i) {
                to_object(&inst[i], rays + 8 * r, ro);
                segment(&objs[inst[i].object], ro, w, inv, moving);
                c += w->candidate && w->ta <= ro[7] ? 1u : 0u;
            }
            counts[r] = c;
        }
        free(w);
    }
    int64_t total = 0;
    for (int64_t r = 0; r < n_rays; ++r) total += counts[r];
    if (total > cap) return total;
    int64_t off = 0;
    walk_t *w = (walk_t *)malloc(sizeof(walk_t));
    if (!w) return -2;
    for (int64_t r = 0; r < n_rays; ++r) {
        if (!counts[r]) continue;
        float inv[3], ro[8];
        int moving[3];
        for (int32_t i = 0; i < n_inst; ++i) {
            to_object(&inst[i], rays + 8 * r, ro);
            segment(&objs[inst[i].object], ro, w, inv, moving);
            if (w->candidate && w->ta <= ro[7]) {
                pair_ray[off] = (uint32_t)r;
                pair_inst[off] = (uint32_t)i;
                ++off;
            }
        }
    }
    free(w);
    return total;
}

/* PCG hash (Jarzynski and Olano 2020, "Hash Functions for GPU Rendering"). */
static uint32_t pcg_hash(uint32_t v)
{
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

/* Diffuse bounce rays of a wavefront path tracer (the paper renders with one,
 * Sec. 7).  For every ray i with a hit, in order of i: the hit point
 * x = o + t d, the hit normal turned to face the incoming ray, the new origin
 * x + eps n, and a direction cosine-distributed about n by Malley's method
 * (a uniform point of the unit disk, r = sqrt(u1), phi = 2 pi u2, lifted to the
 * hemisphere) expressed in the orthonormal basis of Duff et al. 2017; the
 * uniforms come from the PCG hash of (seed, bounce, i).  Writes the new rays
 * (tmin 0, tmax +inf) and their parents; returns their number. */
int64_t oracle_bounce(const float *rays, const uint32_t *hit, const float *t, const float *nrm, int64_t n,
                      uint32_t seed, uint32_t bounce, float eps, float *next, uint32_t *parent)
{
    const uint32_t k = pcg_hash(seed ^ pcg_hash(bounce));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!hit[i]) continue;
        const float *r = rays + 8 * i;
        float nv[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        if ((nv[0] * r[3] + nv[1] * r[4]) + nv[2] * r[5] > 0.0f)
            for (int a = 0; a < 3; ++a) nv[a] = -nv[a];
        float *q = next + 8 * m;
        for (int a = 0; a < 3; ++a) q[a] = (r[a] + t[i] * r[3 + a]) + eps * nv[a];
        const uint32_t h1 = pcg_hash((uint32_t)i ^ k), h2 = pcg_hash(h1);
        const float u1 = (float)(h1 >> 8) * 5.9604644775390625e-8f, u2 = (float)(h2 >> 8) * 5.9604644775390625e-8f;
        const float rr = sqrtf(u1), phi = 6.2831855f * u2;
        const float lx = rr * cosf(phi), ly = rr * sinf(phi), lz = sqrtf(fmaxf(0.0f, 1.0f - u1));
        const float s = copysignf(1.0f, nv[2]);
        const float a = -1.0f / (s + nv[2]);
        const float b = nv[0] * nv[1] * a;
        const float tx[3] = {1.0f + s * nv[0] * nv[0] * a, s * b, -s * nv[0]};
        const float bx[3] = {b, s + nv[1] * nv[1] * a, -nv[1]};
        for (int c = 0; c < 3; ++c) q[3 + c] = (lx * tx[c] + ly * bx[c]) + lz * nv[c];
        q[6] = 0.0f;
        q[7] = INFINITY;
        parent[m] = (uint32_t)i;
        ++m;
    }
    return m;
}
