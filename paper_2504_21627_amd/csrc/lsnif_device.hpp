// Device-side steps of an LSNIF query: ray setup, AABB slab test, the voxel
// walk, boundary points and grid-vertex slots (paper Sec. 3.1, 3.2).
//
// Every float32 operation here is written out in the order it is evaluated
// and compiled without contraction into fused multiply-adds, so that the
// voxel list, the points and the table slots are a deterministic function of
// the ray: the same ray gives the same list in every kernel of the library.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsnif {

constexpr int kMaxLevels = 32;
constexpr int kMaxList = 32;          // H/2 <= 32
constexpr int kCoarseLdsWords = 2048; // brick bits staged in LDS when the grid has <= 65536 bricks
constexpr uint32_t kHotLdsBudget = 40 << 10;  // LDS bytes per block for hot levels (two blocks per CU still fit)
constexpr uint32_t kTablePad = 16;     // spare bytes after an object's tables (a paired gather may read one entry past the slot it needs)
constexpr uint32_t kPrimeY = 2654435761u;   // spatial hash of Mueller et al. 2022, Eq. 4
constexpr uint32_t kPrimeZ = 805459861u;

// Object geometry and grid description shared by every query kernel.
//
// Occupancy is held as 4x4x4 bricks: `fine` has one 64-bit mask per brick
// (bit (x&3) + 4 (y&3) + 16 (z&3)), brick (x>>2) + NB ((y>>2) + NB (z>>2)),
// and `coarse` one bit per brick telling whether its mask is non-zero.
//
// A level's table slot of vertex v is (vx + my vy + mz vz) & dmask when the
// level is indexed directly (my = R+1, mz = (R+1)^2, dmask = ~0, hmask = 0)
// and (vx ^ my vy ^ mz vz) & hmask when it is hashed (my, mz = the primes,
// dmask = 0, hmask = T-1); the kernels combine both forms without branching.
struct Geom {
    float bmin[3];
    float s[3];               // voxels per object-space unit, (float)V / (bmax - bmin)
    int32_t V;
    int32_t NB;               // bricks per axis, ceil(V / 4)
    const uint64_t *fine;
    const uint32_t *coarse;
    int32_t coarse_words;     // uint32 words of `coarse`
    int32_t L, F, log2_T, H;
    uint32_t dense_mask;      // bit l: level l indexed directly ((R+1)^3 <= T)
    uint32_t aligned_mask;    // bit l: R % V == 0, the crossing-axis weight is 0 or 1
    uint32_t recheck;         // 1: grazing voxels of the walk are re-decided in float64
    uint32_t sort_bits;       // coherence sort of single-object batches: 2^bits cells per axis (0 = no sort, <= 6)
    uint32_t pair_bits;       // grouping of pairs within an object: 2^bits cells per axis (<= 5)
    uint32_t hot_mask;        // bit l: level l is copied into LDS for the launch (hot level)
    uint32_t hot_bytes;       // LDS bytes of the hot levels
    uint32_t hot_off[kMaxLevels], hot_len[kMaxLevels];   // LDS byte offset, bytes copied (multiples of 16)
    int32_t R[kMaxLevels];
    float lsc[kMaxLevels];    // (float)R / (float)V
    uint32_t my[kMaxLevels], mz[kMaxLevels], dmask[kMaxLevels], hmask[kMaxLevels];
};

// A ray in voxel space with its slab interval.
struct VRay {
    float o[3], d[3], inv[3];
    uint32_t mov;             // bit a: axis a moves (d != 0 with a finite reciprocal)
    float ta, tb, tmax, tmin;
    bool valid, cand;
};

__device__ __forceinline__ float fmin2(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float fmax2(float a, float b) { return a > b ? a : b; }

// Parameter where the line crosses the voxel-space plane x_a = k.
__device__ __forceinline__ float plane_t(float k, float o, float inv) { return (k - o) * inv; }

__device__ __forceinline__ bool bad(float x) { return !(x == x); }
__device__ __forceinline__ bool inf_or_nan(float x) { return !(__builtin_fabsf(x) <= 3.402823466e38f); }

// Validity, voxel-space transform and slab test against [0, V]^3.
__device__ __forceinline__ void setup_ray(const Geom &g, float4 r0, float4 r1, VRay &w)
{
    const float in[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    w.valid = false;
    w.cand = false;
    w.mov = 0;
    w.ta = 0.0f;
    w.tb = 0.0f;
    w.tmax = in[7];
    w.tmin = in[6];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) ok = ok && !inf_or_nan(in[i]);
    ok = ok && !bad(in[6]) && !bad(in[7]);
    ok = ok && !(in[3] == 0.0f && in[4] == 0.0f && in[5] == 0.0f);
    ok = ok && !(in[6] > in[7]);
    if (!ok) return;
    w.valid = true;
    const float V = (float)g.V;
    float t0 = -__builtin_inff(), t1 = __builtin_inff();
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w.o[a] = (in[a] - g.bmin[a]) * g.s[a];
        w.d[a] = in[3 + a] * g.s[a];
        w.inv[a] = 0.0f;
        if (w.d[a] != 0.0f) {
            float iv = 1.0f / w.d[a];
            if (__builtin_fabsf(iv) <= 3.402823466e38f) {
                w.mov |= 1u << a;
                w.inv[a] = iv;
            }
        }
        if (w.mov & (1u << a)) {
            float lo = plane_t(0.0f, w.o[a], w.inv[a]);
            float hi = plane_t(V, w.o[a], w.inv[a]);
            t0 = fmax2(t0, fmin2(lo, hi));
            t1 = fmin2(t1, fmax2(lo, hi));
        } else {
            inside = inside && (w.o[a] >= 0.0f && w.o[a] <= V);
        }
    }
    if (!inside || w.mov == 0) return;
    w.ta = fmax2(t0, in[6]);
    w.tb = t1;
    w.cand = w.ta < w.tb;
}

// Entry and exit parameter of cell k along one moving axis.
__device__ __forceinline__ void cell_span(const VRay &w, int a, int k, float &en, float &ex)
{
    float lo = plane_t((float)k, w.o[a], w.inv[a]);
    float hi = plane_t((float)(k + 1), w.o[a], w.inv[a]);
    if (w.d[a] > 0.0f) { en = lo; ex = hi; } else { en = hi; ex = lo; }
}

// Entry/exit of a cell: the latest axis entry and the earliest axis exit over
// moving axes, each tie going to the lowest axis.
__device__ __forceinline__ void cell_interval(const VRay &w, const int c[3], float &tin, float &tout,
                                              int &ia, int &oa)
{
    tin = -__builtin_inff();
    tout = __builtin_inff();
    ia = -1;
    oa = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (w.mov & (1u << a)) {
            float en, ex;
            cell_span(w, a, c[a], en, ex);
            if (ia < 0 || en > tin) { tin = en; ia = a; }
            if (oa < 0 || ex < tout) { tout = ex; oa = a; }
        }
    }
}

__device__ __forceinline__ uint32_t pack_ijk(const int c[3])
{
    return (uint32_t)c[0] | ((uint32_t)c[1] << 10) | ((uint32_t)c[2] << 20);
}
__device__ __forceinline__ void unpack_ijk(uint32_t v, int c[3])
{
    c[0] = (int)(v & 1023u);
    c[1] = (int)((v >> 10) & 1023u);
    c[2] = (int)(v >> 20);
}

__device__ __forceinline__ uint32_t brick_of(const Geom &g, const int c[3])
{
    const uint32_t NB = (uint32_t)g.NB;
    return ((uint32_t)c[0] >> 2) + NB * (((uint32_t)c[1] >> 2) + NB * ((uint32_t)c[2] >> 2));
}

__device__ __forceinline__ uint32_t bit_in_brick(const int c[3])
{
    return ((uint32_t)c[0] & 3u) + 4u * ((uint32_t)c[1] & 3u) + 16u * ((uint32_t)c[2] & 3u);
}

// Start cell of the walk: on a moving axis the cell whose [entry, exit)
// holds ta (a floor guess corrected by at most a few steps), on a still axis
// the half-open cell of the origin with V mapped to V - 1.
__device__ __forceinline__ int start_cell(const Geom &g, const VRay &w, int a)
{
    const int V = g.V;
    if (!(w.mov & (1u << a))) {
        int k = (int)__builtin_floorf(w.o[a]);
        return k > V - 1 ? V - 1 : k;
    }
    float x = w.o[a] + w.ta * w.d[a];
    x = x < 0.0f ? 0.0f : (x > (float)(V - 1) ? (float)(V - 1) : x);
    int k = (int)__builtin_floorf(x);
    const int fwd = w.d[a] > 0.0f ? 1 : -1;
    for (int it = 0; it < V; ++it) {
        float en, ex;
        cell_span(w, a, k, en, ex);
        int nk;
        if (en > w.ta) nk = k - fwd;
        else if (ex <= w.ta) nk = k + fwd;
        else break;
        if (nk < 0 || nk >= V) break;
        k = nk;
    }
    return k;
}

// Optional float64 re-decision of a voxel the float32 walk finds grazing: its
// overlap with [ta, tb] is no longer than 2^-16 max(1, |entry|), or all of
// [ta, tb] is that short.  The slab intervals of the voxel and of the grid are
// recomputed in float64 (IEEE division) from the same float32 voxel-space
// origin and direction, over the axes the float32 walk moves along, and the
// voxel is kept iff the float64 overlap has positive length.  Only whether a
// visited voxel is listed changes; its t values stay float32.
__device__ __forceinline__ bool grazing(float tin, float tout, float ta, float tb)
{
    const float lo = fmax2(tin, ta), hi = fmin2(tout, tb);
    const float q = 0x1p-16f;
    return hi - lo <= q * fmax2(1.0f, __builtin_fabsf(tin)) || tb - ta <= q * fmax2(1.0f, __builtin_fabsf(ta));
}

__device__ __forceinline__ bool keep_f64(const VRay &w, const int c[3], int V)
{
    double t0 = -__builtin_inf(), t1 = __builtin_inf(), tin = -__builtin_inf(), tout = __builtin_inf();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!(w.mov & (1u << a))) continue;
        const double o = w.o[a], d = w.d[a];
        const double g0 = (0.0 - o) / d, g1 = ((double)V - o) / d;
        const double e0 = ((double)c[a] - o) / d, e1 = ((double)(c[a] + 1) - o) / d;
        t0 = __builtin_fmax(t0, __builtin_fmin(g0, g1));
        t1 = __builtin_fmin(t1, __builtin_fmax(g0, g1));
        tin = __builtin_fmax(tin, __builtin_fmin(e0, e1));
        tout = __builtin_fmin(tout, __builtin_fmax(e0, e1));
    }
    const double ta = __builtin_fmax(t0, (double)w.tmin), tb = t1;
    return __builtin_fmin(tout, tb) > __builtin_fmax(tin, ta);
}

// The voxel walk.  Emits, in order along the ray, the packed coordinates of
// the first `cap` occupied voxels whose [entry, exit] overlaps [ta, tb] with
// positive length; list[j * stride] receives voxel j.  Steps the axis of the
// earliest exit, the lowest axis on ties.  Occupancy is read a brick at a
// time: the coarse bit (from `coarse`, LDS or global) and, for a non-empty
// brick, its 64-bit mask, loaded once on entering the brick.  An empty brick
// is crossed in one step that lands on the cell the cell-by-cell walk reaches
// next; every decision still compares values of the same plane functions.
template <bool RECHECK>
__device__ __forceinline__ int walk_voxels(const Geom &g, const VRay &w, const uint32_t *coarse,
                                           uint32_t *list, uint32_t stride, int cap)
{
    if (!w.cand) return 0;
    int c[3], st[3], pk[3];
    float en[3], ex[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c[a] = start_cell(g, w, a);
        const bool up = w.d[a] > 0.0f;
        st[a] = up ? 1 : -1;   // cell step along the ray
        pk[a] = up ? 1 : 0;    // exit plane of cell k: k + pk
        if (w.mov & (1u << a)) {
            cell_span(w, a, c[a], en[a], ex[a]);
        } else {
            en[a] = -__builtin_inff();
            ex[a] = __builtin_inff();
        }
    }
    int n = 0;
    const int V = g.V;
    uint32_t cur = 0xffffffffu;
    uint64_t mask = 0;
    for (int it = 0; it < 3 * V; ++it) {
        const uint32_t b = brick_of(g, c);
        if (b != cur) {
            cur = b;
            mask = ((coarse[b >> 5] >> (b & 31u)) & 1u) ? g.fine[b] : 0ull;
        }
        if (mask == 0ull) {
            // An empty brick lists nothing: go straight to the cell where the cell-by-cell
            // walk would leave it.  That walk merges the axes' plane crossings in order of
            // t, ties to the lowest axis, so it leaves along the axis whose brick-boundary
            // plane comes first in that order, after every other axis has crossed exactly
            // its in-brick planes that come before it.
            float T = __builtin_inff();
            int as = -1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (w.mov & (1u << a)) {
                    const int lo = c[a] & ~3, hi = lo + 4 < V ? lo + 4 : V;
                    const float ta = plane_t((float)(w.d[a] > 0.0f ? hi : lo), w.o[a], w.inv[a]);
                    if (as < 0 || ta < T) { T = ta; as = a; }
                }
            }
            if (T >= w.tb) break;   // the segment ends inside the brick
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (!(w.mov & (1u << a))) continue;
                const bool up = w.d[a] > 0.0f;
                if (a == as) {
                    const int lo = c[a] & ~3;
                    c[a] = up ? lo + 4 : lo - 1;
                    out = c[a] < 0 || c[a] >= V;
                } else {
                    for (int s = 0; s < 3; ++s) {
                        const int nk = up ? c[a] + 1 : c[a] - 1;
                        if ((nk & ~3) != (c[a] & ~3)) break;
                        const float t = plane_t((float)(up ? c[a] + 1 : c[a]), w.o[a], w.inv[a]);
                        if (t < T || (t == T && a < as)) c[a] = nk;
                        else break;
                    }
                }
            }
            if (out) break;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (w.mov & (1u << a)) cell_span(w, a, c[a], en[a], ex[a]);
            continue;
        }
        // A still axis has en = -inf and ex = +inf, so it never decides the interval; the
        // exit axis is the lowest one whose exit equals the earliest (the axis order of ties).
        const float tin = __builtin_fmaxf(__builtin_fmaxf(en[0], en[1]), en[2]);
        const float tout = __builtin_fminf(__builtin_fminf(ex[0], ex[1]), ex[2]);
        const int oa = ex[0] == tout ? 0 : (ex[1] == tout ? 1 : 2);
        bool keep = fmin2(tout, w.tb) > fmax2(tin, w.ta);
        if constexpr (RECHECK)
            if (g.recheck && grazing(tin, tout, w.ta, w.tb)) keep = keep_f64(w, c, V);
        if (keep && ((mask >> bit_in_brick(c)) & 1ull)) {
            list[(size_t)n * stride] = pack_ijk(c);
            if (++n == cap) break;
        }
        if (tout >= w.tb) break;
        // step along the exit axis, as selects rather than a branch per axis
        const bool s0 = oa == 0, s1 = oa == 1;
        const bool s2 = !s0 && !s1;
        c[0] += s0 ? st[0] : 0;
        c[1] += s1 ? st[1] : 0;
        c[2] += s2 ? st[2] : 0;
        const int cn = s0 ? c[0] : (s1 ? c[1] : c[2]);
        const int kp = cn + (s0 ? pk[0] : (s1 ? pk[1] : pk[2]));
        const float xn = plane_t((float)kp, s0 ? w.o[0] : (s1 ? w.o[1] : w.o[2]),
                                 s0 ? w.inv[0] : (s1 ? w.inv[1] : w.inv[2]));
        en[0] = s0 ? ex[0] : en[0];
        en[1] = s1 ? ex[1] : en[1];
        en[2] = s2 ? ex[2] : en[2];
        ex[0] = s0 ? xn : ex[0];
        ex[1] = s1 ? xn : ex[1];
        ex[2] = s2 ? xn : ex[2];
        if (cn < 0 || cn >= V) break;
    }
    return n;
}

// Boundary point h of a listed voxel: even h = where the line enters the
// voxel, odd h = where it leaves.  The crossing axis takes the face plane
// itself; other axes are evaluated on the line and clamped into the voxel.
// Also returns the crossing axis.
__device__ __forceinline__ int boundary_point(const VRay &w, uint32_t packed, bool is_exit, float p[3])
{
    int c[3];
    unpack_ijk(packed, c);
    float tin, tout;
    int ia, oa;
    cell_interval(w, c, tin, tout, ia, oa);
    const float t = is_exit ? tout : tin;
    const int face = is_exit ? oa : ia;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float lo = (float)c[b], hi = (float)(c[b] + 1);
        if (b == face) {
            const bool upper = (w.d[b] > 0.0f) == is_exit;
            p[b] = upper ? hi : lo;
        } else {
            float v = w.o[b] + t * w.d[b];
            p[b] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
    return face;
}

// Cell of level l holding p: base vertex i and fractional weights wt.
__device__ __forceinline__ void level_cell(const Geom &g, int l, const float p[3], uint32_t i[3], float wt[3])
{
    const int R = g.R[l];
    const float Rf = (float)R;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        float x = p[b] * g.lsc[l];
        x = x < 0.0f ? 0.0f : (x > Rf ? Rf : x);
        int k = (int)__builtin_floorf(x);
        k = k > R - 1 ? R - 1 : k;
        i[b] = (uint32_t)k;
        wt[b] = x - (float)k;
    }
}

// Table slot of vertex v on level l.
__device__ __forceinline__ uint32_t vertex_slot(const Geom &g, int l, uint32_t vx, uint32_t vy, uint32_t vz)
{
    const uint32_t y = vy * g.my[l], z = vz * g.mz[l];
    return ((vx + y + z) & g.dmask[l]) | ((vx ^ y ^ z) & g.hmask[l]);
}

}  // namespace lsnif
