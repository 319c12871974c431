// Query kernels for gfx950.
//
//  k_query_f32   one ray per lane; fused walk, encoding, float32 MLP on the
//                vector ALU (weights are wave-uniform scalar operands), decode.
//  k_query_mma   one ray per lane, 64 rays per wave; the same walk and
//                encoding, then every MLP layer on the matrix cores
//                (v_mfma_f32_32x32x16_{f16,bf16}, float32 accumulation).
//  k_debug       one ray per lane; writes every intermediate of the walk and
//                the grid lookups for bit-exact checks.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "lsnif_device.hpp"
#include "lsnif_launch.hpp"
#include "../../include/lsnif.h"

namespace lsnif {

constexpr int kBlock = 256;
constexpr int kMaxOut = 16;

// MLP description for the kernels.
struct Mlp {
    const void *W;            // packed weights (layout depends on the kernel)
    int32_t off[8];           // element offset of each layer in W
    int32_t n_hidden;
    int32_t out_dim;
    int32_t act;              // LSNIF_RELU / LSNIF_LEAKY_RELU
    float slope;
    int32_t n_mat, has_albedo;
    int32_t kb_point;         // matrix-core path: K blocks (16 wide) per boundary point
    int32_t fp;               // matrix-core path: features per level after padding
    int32_t woff[8];          // matrix-core path: dword offset of each layer's fragments
    float qs[8];              // FP8: 1 / activation scale of each layer's input (1 otherwise)
    float dq[8];              // FP8: weight scale x activation scale of each layer (1 otherwise)
};

struct Dbg {
    int32_t *count;
    float *tatb;
    float *out;
    float *enc;
    float *act_amax;          // float32 path: largest |input| of each layer, for FP8 scales
};

// Result of one (ray, instance) pair, kept until the nearest hit is known.
struct PairRes {
    float t;                  // +inf on a miss
    float n[3];               // object-space normal
    int32_t material;
};

// A built object as the pair kernels see it (device object table, indexed by id).
struct ObjDev {
    Geom g;
    Mlp m;
    const void *tables;
    int32_t live;
    int32_t kb_point;
};

struct PairArgs {
    const uint32_t *pair_ray;
    const uint32_t *pair_inst;
    const lsnif_instance *inst;
    const ObjDev *objs;
    const int32_t *tile_obj;      // object id of each 256-slot tile, -1 for none
    const uint32_t *slot_pair;    // pair index of each sorted slot, 0xffffffff for padding
    unsigned long long *minkey;   // per ray: (ordered t << 32) | instance of the nearest hit
    PairRes *res;                 // per pair
};

struct QueryArgs {
    Geom g;
    Mlp m;
    const void *tables;       // [L][T][F] in the feature type
    const float4 *rays;
    lsnif_hit *hits;
    uint32_t n;               // rays (single object) or sorted pair slots (pairs)
    const uint32_t *order;    // processing order of the rays (coherence sort), or NULL
    uint32_t *lists;          // voxel lists by slot: entry j of slot i at lists[j n + i]
    uint8_t *nvox;            // listed voxels of each slot
    uint32_t tile0;           // first tile of the launch (a launch may cover a range of the tiles)
    uint32_t n_tiles;         // tiles of the launch (persistent kernels: the range they share out)
    unsigned long long *queue;   // persistent kernels: 8 tile-queue counters, zero at launch
    uint32_t persistent;      // run the query kernel as a persistent grid (width-64 matrix-core kernels)
    uint32_t width;           // hidden width of the launch's objects (64 or 128), picks the kernel
    Dbg dbg;
    PairArgs pr;
    uint32_t hot_lds;         // dynamic LDS bytes after the voxel lists for hot levels
};

// Order-preserving map of a float to 32 unsigned bits.
__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Instance transform x_obj = A x + b (row-major 3x4), evaluated in the order
// ((m0 x + m1 y) + m2 z) + m3; directions are not renormalised, so t is
// shared by both spaces.  An invalid world ray stays invalid.
__device__ __forceinline__ void to_object_space(const lsnif_instance &I, float4 &r0, float4 &r1)
{
    const float in[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) ok = ok && (__builtin_fabsf(in[i]) <= 3.402823466e38f);
    ok = ok && (in[6] == in[6]) && (in[7] == in[7]);
    ok = ok && !(in[3] == 0.0f && in[4] == 0.0f && in[5] == 0.0f) && !(in[6] > in[7]);
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *m = I.world_to_object + 4 * a;
        o[a] = ((m[0] * in[0] + m[1] * in[1]) + m[2] * in[2]) + m[3];
        d[a] = (m[0] * in[3] + m[1] * in[4]) + m[2] * in[5];
    }
    r0 = make_float4(ok ? o[0] : __builtin_nanf(""), o[1], o[2], d[0]);
    r1 = make_float4(d[1], d[2], in[6], in[7]);
}

template <typename TF> __device__ __forceinline__ float to_f32(TF v);
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<__bf16>(__bf16 v) { return (float)v; }

template <typename TF> __device__ __forceinline__ float lo16(uint32_t x)
{
    uint16_t u = (uint16_t)(x & 0xffffu);
    TF v;
    __builtin_memcpy(&v, &u, 2);
    return to_f32<TF>(v);
}
template <typename TF> __device__ __forceinline__ float hi16(uint32_t x)
{
    uint16_t u = (uint16_t)(x >> 16);
    TF v;
    __builtin_memcpy(&v, &u, 2);
    return to_f32<TF>(v);
}

// Raw bytes of one table entry (F features of type TF) at byte offset `off`.
template <typename TF, int F> struct Entry {
    static constexpr int W = (F * (int)sizeof(TF) + 3) / 4;   // dwords
    uint32_t d[W];
    __device__ __forceinline__ void load(const char *base, uint32_t off)
    {
        if constexpr (F * sizeof(TF) == 4) {
            d[0] = *reinterpret_cast<const uint32_t *>(base + off);
        } else if constexpr (F * sizeof(TF) == 8) {
            uint2 x = *reinterpret_cast<const uint2 *>(base + off);
            d[0] = x.x;
            d[1] = x.y;
        } else if constexpr (F * sizeof(TF) == 16) {
            uint4 x = *reinterpret_cast<const uint4 *>(base + off);
            d[0] = x.x; d[1] = x.y; d[2] = x.z; d[3] = x.w;
        } else {
            const TF *p = reinterpret_cast<const TF *>(base + off);
            uint16_t u[2 * W] = {};
            float f32[W] = {};
            for (int f = 0; f < F; ++f) {
                if constexpr (sizeof(TF) == 2) __builtin_memcpy(&u[f], &p[f], 2);
                else f32[f] = to_f32<TF>(p[f]);
            }
            for (int k = 0; k < W; ++k) {
                if constexpr (sizeof(TF) == 2) d[k] = (uint32_t)u[2 * k] | ((uint32_t)u[2 * k + 1] << 16);
                else d[k] = __float_as_uint(f32[k]);
            }
        }
    }
    // An opaque use of the loaded dwords: nothing that reads them can be
    // moved above this point, so a batch of gathers is issued in full first.
    __device__ __forceinline__ void pin()
    {
#pragma unroll
        for (int k = 0; k < W; ++k) asm volatile("" : "+v"(d[k]));
    }
    __device__ __forceinline__ float get(int f) const
    {
        if constexpr (sizeof(TF) == 4) return __uint_as_float(d[f]);
        else return (f & 1) ? hi16<TF>(d[f >> 1]) : lo16<TF>(d[f >> 1]);
    }
};

// Cell of point p on level l and the weights inside it, as level_cell, with the
// clamps as min/max (the debug path keeps level_cell itself).
__device__ __forceinline__ void level_cell_mm(const Geom &g, int l, const float p[3], uint32_t i[3], float wt[3])
{
    const float Rf = (float)g.R[l], sc = g.lsc[l];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float x = __builtin_amdgcn_fmed3f(p[b] * sc, 0.0f, Rf);   // clamp to [0, R]
        const float k = __builtin_fminf(__builtin_floorf(x), Rf - 1.0f);
        i[b] = (uint32_t)k;
        wt[b] = x - k;
    }
}

// Interpolated features of NL consecutive levels l0 .. l0 + NL - 1 at the
// boundary point p (voxel units) whose crossing axis is `face`; levels at or
// beyond L give zeros.  All slots are formed first and all gathers issued
// before any is consumed.  On a level aligned with the voxel faces the
// crossing-axis weight is exactly 0 or 1, and the 4 zero-weight corners do
// not touch their own entries (the LDS variant re-reads the 4 face corners,
// the other reads the level's first entry).
template <typename TF, int F, int NL, bool HOT>
__device__ __forceinline__ void encode_levels(const Geom &g, const TF *__restrict__ tab, const uint32_t *hot, int l0,
                                              const float p[3], int face, float out[NL][F])
{
    const char *base[NL];
    bool in_lds[NL];
    uint32_t hoff[NL];
    uint32_t off[NL][8];
    float wx[NL][2], wy[NL][2], wz[NL][2];
    constexpr uint32_t esz = F * sizeof(TF);
#pragma unroll
    for (int lv = 0; lv < NL; ++lv) {
        const int l = l0 + lv < g.L ? l0 + lv : g.L - 1;
        uint32_t i[3];
        float wt[3];
        if constexpr (HOT) {
            // the LDS variant keeps the branch-free form: with the wave-uniform branches
            // below, the compiler merges the LDS and HBM gathers into flat loads
            level_cell(g, l, p, i, wt);
            const uint32_t my = g.my[l], mz = g.mz[l];
            uint32_t t[3][2] = {{i[0], i[0] + 1u}, {i[1] * my, i[1] * my + my}, {i[2] * mz, i[2] * mz + mz}};
            const bool al = (g.aligned_mask >> l) & 1u;
            const float wf = face == 0 ? wt[0] : (face == 1 ? wt[1] : wt[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const bool col = al && a == face;
                const uint32_t sel = wf != 0.0f ? t[a][1] : t[a][0];
                t[a][0] = col ? sel : t[a][0];
                t[a][1] = col ? sel : t[a][1];
            }
            const uint32_t dm = g.dmask[l], hm = g.hmask[l];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint32_t x = t[0][c & 1], y = t[1][(c >> 1) & 1], z = t[2][c >> 2];
                off[lv][c] = (((x + y + z) & dm) | ((x ^ y ^ z) & hm)) * esz;
            }
        } else {
            level_cell_mm(g, l, p, i, wt);
            // With a power-of-two entry size the byte offset is formed directly: scaling
            // x, y my and z mz by esz commutes with the sum and, as a shift, with the xor
            // and the mask.
            constexpr uint32_t sh = esz == 4 ? 2u : (esz == 8 ? 3u : (esz == 16 ? 4u : 0u));
            constexpr bool scaled = sh != 0u;
            const uint32_t my = g.my[l] << sh, mz = g.mz[l] << sh;
            const uint32_t x0 = i[0] << sh;
            uint32_t t[3][2] = {{x0, x0 + (1u << sh)}, {i[1] * my, i[1] * my + my}, {i[2] * mz, i[2] * mz + mz}};
            // vertex slot: x + y + z on a directly indexed level, (x ^ y ^ z) & (T - 1) on a
            // hashed one (y, z already times their multipliers); the level kind is wave-uniform
            constexpr uint32_t m = scaled ? 1u : esz;
            if ((g.dense_mask >> l) & 1u) {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    off[lv][c] = (t[0][c & 1] + t[1][(c >> 1) & 1] + t[2][c >> 2]) * m;
            } else {
                const uint32_t hm = g.hmask[l] << sh;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t yz = t[1][q & 1] ^ t[2][q >> 1];
                    off[lv][2 * q] = ((t[0][0] ^ yz) & hm) * m;
                    off[lv][2 * q + 1] = ((t[0][1] ^ yz) & hm) * m;
                }
            }
            if ((g.aligned_mask >> l) & 1u) {
                // On a face-aligned level the crossing axis' weight is exactly 0 or 1, so the 4
                // corners on the other side weigh 0.  They read the level's first entry: one
                // line for every lane, where their own slots would cost the addresser a line
                // per lane.  Weight 0 times a finite entry adds nothing (the sum is never -0).
                const float wf = face == 0 ? wt[0] : (face == 1 ? wt[1] : wt[2]);
                const uint32_t fb = 1u << face, keep = wf != 0.0f ? fb : 0u;
#pragma unroll
                for (int c = 0; c < 8; ++c) off[lv][c] = ((uint32_t)c & fb) == keep ? off[lv][c] : 0u;
            }
        }
        wx[lv][0] = 1.0f - wt[0]; wx[lv][1] = wt[0];
        wy[lv][0] = 1.0f - wt[1]; wy[lv][1] = wt[1];
        wz[lv][0] = 1.0f - wt[2]; wz[lv][1] = wt[2];
        in_lds[lv] = HOT && ((g.hot_mask >> l) & 1u);
        hoff[lv] = HOT ? g.hot_off[l] : 0u;
        base[lv] = reinterpret_cast<const char *>(tab + ((size_t)l << g.log2_T) * F);
    }
    Entry<TF, F> e[NL][8];
    typedef uint32_t u32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
#pragma unroll
    for (int lv = 0; lv < NL; ++lv) {
        const int l = l0 + lv < g.L ? l0 + lv : g.L - 1;
        const bool pairx = !HOT && F * sizeof(TF) == 4 && ((g.dense_mask & ~g.aligned_mask) >> l) & 1u;
        if (pairx) {
            // directly indexed level: the two x-vertices of an edge are adjacent entries
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const u32x2a4 v = *reinterpret_cast<const u32x2a4 *>(base[lv] + off[lv][2 * q]);
                e[lv][2 * q].d[0] = v.x;
                e[lv][2 * q + 1].d[0] = v.y;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                // a hot level is read from its LDS copy (the pointer stays in the LDS address space)
                if (HOT && in_lds[lv]) e[lv][c].load(reinterpret_cast<const char *>(hot) + hoff[lv], off[lv][c]);
                else e[lv][c].load(base[lv], off[lv][c]);
            }
        }
    }
    // keep every gather of the batch in flight before the first is consumed
    asm volatile("" ::: "memory");
#pragma unroll
    for (int lv = 0; lv < NL; ++lv)
#pragma unroll
        for (int c = 0; c < 8; ++c) e[lv][c].pin();
#pragma unroll
    for (int lv = 0; lv < NL; ++lv) {
#pragma unroll
        for (int f = 0; f < F; ++f) out[lv][f] = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float wyz = wy[lv][q & 1] * wz[lv][q >> 1];
#pragma unroll
            for (int xb = 0; xb < 2; ++xb) {
                const float w = wx[lv][xb] * wyz;
#pragma unroll
                for (int f = 0; f < F; ++f) out[lv][f] = __builtin_fmaf(w, e[lv][2 * q + xb].get(f), out[lv][f]);
            }
        }
        if (l0 + lv >= g.L) {
#pragma unroll
            for (int f = 0; f < F; ++f) out[lv][f] = 0.0f;
        }
    }
}

// Tables with 4- or 8-byte entries may keep their coarsest levels in LDS.
template <typename TF, int F> constexpr bool hot_entries()
{
    return F * sizeof(TF) == 4 || F * sizeof(TF) == 8;
}

// Copy the object's hot levels (the coarsest, all of whose used slots fit the
// LDS budget) into LDS; every ray of the block reads them.  Visible after the
// block's next barrier.
template <typename TF, int F>
__device__ __forceinline__ void stage_hot_levels(const Geom &g, const TF *__restrict__ tab, uint32_t *hot)
{
    if constexpr (hot_entries<TF, F>()) {
        for (int l = 0; l < g.L; ++l) {
            if (!((g.hot_mask >> l) & 1u)) continue;
            const uint4 *src = reinterpret_cast<const uint4 *>(tab + ((size_t)l << g.log2_T) * F);
            uint4 *dst = reinterpret_cast<uint4 *>(hot) + (g.hot_off[l] >> 4);
            for (uint32_t i = threadIdx.x; i < (g.hot_len[l] >> 4); i += kBlock) dst[i] = src[i];
        }
    }
}

__device__ __forceinline__ float act_f(float x, int act, float slope)
{
    return x > 0.0f ? x : (act == LSNIF_LEAKY_RELU ? x * slope : 0.0f);
}

// Largest non-negative value of the wave folded into *dst (float bits of
// non-negative numbers order like unsigned integers).
__device__ __forceinline__ void fold_max(float *dst, float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax2(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63u) == 0) atomicMax(reinterpret_cast<unsigned int *>(dst), __float_as_uint(v));
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        int u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

// Output heads (Sec. 5.1, 5.3): occlusion logit > 0 is a hit, the hit
// distance is the sigmoid of its logit over [ta, tb], the normal is the
// normalised linear head, the material the arg-max logit.
template <bool PAIRS>
__device__ __forceinline__ void decode_store(const QueryArgs &A, const Mlp &mm, uint32_t r, uint32_t pair,
                                             const VRay &w, int count, const float *o)
{
    lsnif_hit h;
    h.hit = 0;
    h.t = __builtin_inff();
    h.n[0] = h.n[1] = h.n[2] = 0.0f;
    h.material = -1;
    if (count > 0) {
        const float sig = 1.0f / (1.0f + expf(-o[1]));
        const float th = w.ta + sig * (w.tb - w.ta);
        if (o[0] > 0.0f && th <= w.tmax) {
            h.hit = 1;
            h.t = th;
            const float nn = o[2] * o[2] + o[3] * o[3] + o[4] * o[4];
            if (nn > 0.0f) {
                const float inv = 1.0f / __builtin_sqrtf(nn);
                h.n[0] = o[2] * inv;
                h.n[1] = o[3] * inv;
                h.n[2] = o[4] * inv;
            }
            // argmax over the material logits o[m0 .. m0 + n_mat), ties to the lowest index;
            // written over the static slots of o so that o stays in registers
            const int m0 = 5 + 3 * mm.has_albedo;
            int best = 0;
            float bv = 0.0f;
#pragma unroll
            for (int k = 5; k < kMaxOut; ++k) {
                const int mk = k - m0;
                if (mk >= 0 && mk < mm.n_mat && (mk == 0 || o[k] > bv)) {
                    bv = o[k];
                    best = mk;
                }
            }
            h.material = best;
        }
    }
    if constexpr (!PAIRS) {
        A.hits[r] = h;
    } else {
        PairRes pr;
        pr.t = h.t;
        pr.n[0] = h.n[0];
        pr.n[1] = h.n[1];
        pr.n[2] = h.n[2];
        pr.material = h.material;
        A.pr.res[pair] = pr;
        if (h.hit) {
            const unsigned long long key =
                ((unsigned long long)ordered_bits(h.t) << 32) | (unsigned long long)A.pr.pair_inst[pair];
            atomicMin(&A.pr.minkey[r], key);
        }
    }
}

// ------------------------------------------------------------- shared prologue
//
// The walk kernel lists the voxels of slot blockIdx-tile * kBlock + threadIdx.x
// into the workspace; the query kernels then load each slot's list into LDS
// and order the block's rays by voxel count (most first), so that each wave
// encodes rays with similar numbers of boundary points.  After the prologue,
// lane `tid` works on ray `src` of the block; its voxel list is at
// s_list[j * kBlock + src] and its walk state has been reloaded from LDS.
constexpr int kState = 15;          // words of walk state per ray kept in LDS

struct Shared {
    float state[kState * kBlock];
    uint32_t hist[kMaxList + 2];
    uint16_t perm[kBlock];
};

struct Lane {
    VRay w;
    int nvox;
    uint32_t src;     // ray index within the block
    uint32_t r;       // global ray index
    uint32_t pair;    // pair index (pair queries)
    bool live;
};

// Tile of rays (or pairs) this block works on.  The dispatcher deals
// workgroups to the 8 XCDs in turn (block b runs on XCD b mod 8), each XCD with
// an L2 of its own, and tiles follow the coherence order of the rays.  Runs of
// C consecutive tiles go to one XCD, so the rays an XCD has in flight lie in
// fewer regions of the object and share more of its L2; short runs keep the
// work of the XCDs even where the cost per tile drifts along the order.  Any
// grid size maps one to one (the last partial round keeps b itself).  A launch
// covers tiles tile0 .. tile0 + gridDim.x - 1.
__device__ __forceinline__ uint32_t block_tile(uint32_t tile0)
{
    constexpr uint32_t C = 8;
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    const uint32_t full = nb / (8u * C) * (8u * C);
    if (b >= full) return tile0 + b;
    const uint32_t x = b & 7u, k = b >> 3;
    return tile0 + ((k / C) * 8u + x) * C + k % C;
}

// Persistent query kernels: a grid of as many blocks as fit on the chip at once,
// each taking tiles until none are left.  The launch's n_tiles tiles are cut
// into 8 contiguous ranges of the coherence order, range x for the blocks that
// run on XCD x (blockIdx mod 8: the dispatcher's round robin), so each XCD's
// L2 serves one stretch of rays (or of one object's pairs) at a time.  A
// block takes the next tile from the head of its own range; once that range
// is empty it takes tiles from the tails of the other ranges.  Each range's
// counter packs the head claims (low 32 bits) and the tail claims (high 32
// bits) into one 64-bit word, so one atomic add both claims and sees the
// other side: a head claim h is valid iff h + s < len, a tail claim iff
// len - 1 - s >= h, for the (h, s) it read.  Every tile is claimed exactly
// once, every claim fails once the range is used up, and each block leaves
// when all eight ranges are: the grid always drains.
constexpr uint32_t kNoTile = 0xffffffffu;

__device__ __forceinline__ uint32_t queue_take(const QueryArgs &A, uint32_t x)
{
    for (uint32_t q = 0; q < 8u; ++q) {
        const uint32_t v = (x + q) & 7u;
        const uint32_t lo = (uint32_t)((uint64_t)A.n_tiles * v / 8u);
        const uint32_t len = (uint32_t)((uint64_t)A.n_tiles * (v + 1u) / 8u) - lo;
        unsigned long long *c = A.queue + v;
        const unsigned long long seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint64_t)(uint32_t)seen + (seen >> 32) >= len) continue;   // used up (the atomic decides)
        const unsigned long long old = atomicAdd(c, q == 0 ? 1ull : (1ull << 32));
        const uint32_t h = (uint32_t)old, s = (uint32_t)(old >> 32);
        if ((uint64_t)h + s < len) return A.tile0 + lo + (q == 0 ? h : len - 1u - s);
    }
    return kNoTile;
}

// The block's next tile (kNoTile: none left), the same value for every thread.
// The trailing barrier also ends the block's use of LDS for the previous tile.
__device__ __forceinline__ uint32_t next_tile(const QueryArgs &A, uint32_t &s_tile)
{
    __syncthreads();
    if (threadIdx.x == 0) s_tile = queue_take(A, blockIdx.x & 7u);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(s_tile);
}

template <bool PAIRS>
__device__ __forceinline__ void slot_ray(const QueryArgs &A, const Geom &g, uint32_t slot, uint32_t &r,
                                         uint32_t &pair, bool &live, VRay &w)
{
    r = 0u;
    pair = 0xffffffffu;
    if constexpr (PAIRS) {
        pair = slot < A.n ? A.pr.slot_pair[slot] : 0xffffffffu;
        live = pair != 0xffffffffu;
        if (live) r = A.pr.pair_ray[pair];
    } else {
        live = slot < A.n;
        if (live) r = A.order ? A.order[slot] : slot;
    }
    w.valid = w.cand = false;
    w.ta = w.tb = w.tmax = w.tmin = 0.0f;
    w.mov = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) w.o[a] = w.d[a] = w.inv[a] = 0.0f;
    if (live) {
        float4 ra = A.rays[2 * r], rb = A.rays[2 * r + 1];
        if constexpr (PAIRS) to_object_space(A.pr.inst[A.pr.pair_inst[pair]], ra, rb);
        setup_ray(g, ra, rb, w);
    }
}

// The voxel walk of every slot, in a kernel of its own: it needs few registers,
// so many waves per SIMD hide the latency of its dependent brick-mask loads,
// which the query kernels (two waves per SIMD) could not.
template <bool PAIRS, bool RECHECK>
__device__ __forceinline__ void walk_body(const QueryArgs &A, const Geom &g, uint32_t *coarse)
{
    const uint32_t tid = threadIdx.x;
    const bool lds_coarse = g.coarse_words <= kCoarseLdsWords;
    if (lds_coarse)
        for (int i = tid; i < g.coarse_words; i += kBlock) coarse[i] = g.coarse[i];
    __syncthreads();
    const uint32_t slot = block_tile(A.tile0) * kBlock + tid;
    uint32_t r, pair;
    bool live;
    VRay w;
    slot_ray<PAIRS>(A, g, slot, r, pair, live, w);
    int nvox = 0;
    if (live) {
        uint32_t *list = A.lists + slot;
        nvox = lds_coarse ? walk_voxels<RECHECK>(g, w, coarse, list, A.n, g.H >> 1)
                          : walk_voxels<RECHECK>(g, w, g.coarse, list, A.n, g.H >> 1);
    }
    if (slot < A.n) A.nvox[slot] = (uint8_t)nvox;
}

template <bool PAIRS>
__device__ __forceinline__ void walk_and_sort(const QueryArgs &A, const Geom &g, Shared &S, uint32_t *s_list,
                                              Lane &L, uint32_t tile)
{
    const uint32_t tid = threadIdx.x;
    const int cap = g.H >> 1;
    if (tid <= (uint32_t)cap) S.hist[tid] = 0;
    __syncthreads();
    const uint32_t slot0 = tile * kBlock + tid;
    uint32_t r0, pair0;
    bool live0;
    VRay w;
    slot_ray<PAIRS>(A, g, slot0, r0, pair0, live0, w);
    // the slot's voxel list into LDS, eight loads in flight at a time
    const int nvox = live0 ? (int)A.nvox[slot0] : 0;
    const int nmax = __builtin_amdgcn_readfirstlane(wave_max(nvox));
    for (int j0 = 0; j0 < nmax; j0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (j0 + q < nvox) v[q] = A.lists[(size_t)(j0 + q) * A.n + slot0];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (j0 + q < nvox) s_list[(j0 + q) * kBlock + tid] = v[q];
    }
    float *st = S.state;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st[(0 + a) * kBlock + tid] = w.o[a];
        st[(3 + a) * kBlock + tid] = w.d[a];
        st[(6 + a) * kBlock + tid] = w.inv[a];
    }
    st[9 * kBlock + tid] = w.ta;
    st[10 * kBlock + tid] = w.tb;
    st[11 * kBlock + tid] = w.tmax;
    st[12 * kBlock + tid] = __uint_as_float(w.mov | (w.valid ? 8u : 0u) | (w.cand ? 16u : 0u) | ((uint32_t)nvox << 8));
    st[13 * kBlock + tid] = __uint_as_float(r0);
    st[14 * kBlock + tid] = __uint_as_float(live0 ? pair0 : 0xffffffffu);
    const uint32_t pos = atomicAdd(&S.hist[cap - nvox], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int b = 0; b <= cap; ++b) {
            const uint32_t c = S.hist[b];
            S.hist[b] = acc;
            acc += c;
        }
    }
    __syncthreads();
    S.perm[S.hist[cap - nvox] + pos] = (uint16_t)tid;
    __syncthreads();
    const uint32_t src = S.perm[tid];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        L.w.o[a] = st[(0 + a) * kBlock + src];
        L.w.d[a] = st[(3 + a) * kBlock + src];
        L.w.inv[a] = st[(6 + a) * kBlock + src];
    }
    L.w.ta = st[9 * kBlock + src];
    L.w.tb = st[10 * kBlock + src];
    L.w.tmax = st[11 * kBlock + src];
    const uint32_t pk = __float_as_uint(st[12 * kBlock + src]);
    L.w.mov = pk & 7u;
    L.w.valid = (pk & 8u) != 0;
    L.w.cand = (pk & 16u) != 0;
    L.nvox = (int)(pk >> 8);
    L.src = src;
    L.r = __float_as_uint(st[13 * kBlock + src]);
    L.pair = __float_as_uint(st[14 * kBlock + src]);
    L.live = PAIRS ? L.pair != 0xffffffffu : tile * kBlock + src < A.n;
}

// ---------------------------------------------------------------- float32 path
//
// Weights: layer k transposed to [in][out_pad] float32 (out_pad = WIDTH for
// hidden layers, kMaxOut for the head) so the outputs fed by one input are
// contiguous and every lane reads the same address.
// Object of this block's tile: one value for the whole block, read through the
// scalar path so that everything derived from it (tables, weights) stays uniform.
__device__ __forceinline__ int tile_object(const PairArgs &P, uint32_t tile)
{
    typedef const __attribute__((address_space(4))) int32_t cint;
    return __builtin_amdgcn_readfirstlane(((cint *)P.tile_obj)[tile]);
}
// The object table, read through the constant address space in the device pass (the
// host pass only type-checks kernel bodies and has no such address space).
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) ObjDev cObjDev;
#else
typedef const ObjDev cObjDev;
#endif

// A float in the constant address space (read-only during a launch; scalar loads).
typedef const __attribute__((address_space(4))) float cfloat;

template <typename TF, int F, int WIDTH, bool PAIRS, bool HOT>
__device__ __forceinline__ void query_f32_body(const QueryArgs &A, const Geom &g, const Mlp &mm,
                                               const TF *__restrict__ tab, uint32_t *s_list, Shared &S,
                                               uint32_t tile)
{
    constexpr int NL = 4;
    Lane ln;
    uint32_t *hot = s_list + (A.g.H >> 1) * kBlock;   // after the voxel lists (sized for the launch)
    if constexpr (HOT) stage_hot_levels<TF, F>(g, tab, hot);
    walk_and_sort<PAIRS>(A, g, S, s_list, ln, tile);
    const uint32_t src = ln.src, r = ln.r;
    const bool live = ln.live;
    const VRay &w = ln.w;
    const int count = 2 * ln.nvox;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(count));
    // The weights are read-only for the whole launch and every lane of a wave reads the same
    // one: through the constant address space the loads are scalar and the FMAs take them
    // from scalar registers.
    const cfloat *Wf = (const cfloat *)(mm.W);
    const int LF = g.L * F;

    float acc[WIDTH];
#pragma unroll
    for (int j = 0; j < WIDTH; ++j) acc[j] = 0.0f;
    float amax = 0.0f;        // largest |input| of the current layer (calibration)
    for (int h = 0; h < wmax; ++h) {
        if (h < count) {
            float p[3];
            const int face = boundary_point(w, s_list[(h >> 1) * kBlock + src], h & 1, p);
            for (int l0 = 0; l0 < g.L; l0 += NL) {
                float e[NL][F];
                encode_levels<TF, F, NL, HOT>(g, tab, hot, l0, p, face, e);
#pragma unroll
                for (int lv = 0; lv < NL; ++lv) {
                    const int l = l0 + lv;
                    if (l < g.L) {
#pragma unroll
                        for (int f = 0; f < F; ++f) amax = fmax2(amax, __builtin_fabsf(e[lv][f]));
                        if (A.dbg.enc) {
#pragma unroll
                            for (int f = 0; f < F; ++f)
                                A.dbg.enc[(size_t)r * g.H * LF + h * LF + l * F + f] = e[lv][f];
                        }
                        const cfloat *Wk = Wf + mm.off[0] + (size_t)(h * LF + l * F) * WIDTH;
#pragma unroll
                        for (int f = 0; f < F; ++f)
#pragma unroll
                            for (int j = 0; j < WIDTH; ++j) acc[j] = __builtin_fmaf(Wk[f * WIDTH + j], e[lv][f], acc[j]);
                    }
                }
            }
        }
    }
    float o[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k) o[k] = 0.0f;
    if (A.dbg.act_amax) fold_max(A.dbg.act_amax + 0, amax);
    if (wmax > 0) {
        for (int k = 1; k < mm.n_hidden; ++k) {
            float nxt[WIDTH];
#pragma unroll
            for (int j = 0; j < WIDTH; ++j) nxt[j] = 0.0f;
            const cfloat *Wk = Wf + mm.off[k];
            amax = 0.0f;
#pragma unroll
            for (int i = 0; i < WIDTH; ++i) {
                const float x = act_f(acc[i], mm.act, mm.slope);
                amax = fmax2(amax, __builtin_fabsf(x));
#pragma unroll
                for (int j = 0; j < WIDTH; ++j) nxt[j] = __builtin_fmaf(Wk[i * WIDTH + j], x, nxt[j]);
            }
#pragma unroll
            for (int j = 0; j < WIDTH; ++j) acc[j] = nxt[j];
            if (A.dbg.act_amax) fold_max(A.dbg.act_amax + k, amax);
        }
        const cfloat *Wo = Wf + mm.off[mm.n_hidden];
        amax = 0.0f;
#pragma unroll
        for (int i = 0; i < WIDTH; ++i) {
            const float x = act_f(acc[i], mm.act, mm.slope);
            amax = fmax2(amax, __builtin_fabsf(x));
#pragma unroll
            for (int j = 0; j < kMaxOut; ++j) o[j] = __builtin_fmaf(Wo[i * kMaxOut + j], x, o[j]);
        }
        if (A.dbg.act_amax) fold_max(A.dbg.act_amax + mm.n_hidden, amax);
    }
    if (!live) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out) {
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k)
            if (k < mm.out_dim) A.dbg.out[(size_t)r * mm.out_dim + k] = count > 0 ? o[k] : 0.0f;
    }
    decode_store<PAIRS>(A, mm, r, ln.pair, w, count, o);
}

template <typename TF, int F, int WIDTH, bool PAIRS, bool HOT>
__device__ __forceinline__ void query_f32_tile(const QueryArgs &A, uint32_t *s_list, Shared &S, uint32_t tile)
{
    if constexpr (PAIRS) {
        const int o = tile_object(A.pr, tile);
        if (o < 0) return;
        const cObjDev &O = ((const cObjDev *)A.pr.objs)[o];
        query_f32_body<TF, F, WIDTH, true, HOT>(A, O.g, O.m, (const TF *)O.tables, s_list, S, tile);
    } else {
        query_f32_body<TF, F, WIDTH, false, HOT>(A, A.g, A.m, reinterpret_cast<const TF *>(A.tables), s_list, S,
                                                 tile);
    }
}

template <typename TF, int F, int WIDTH, bool PAIRS, bool HOT>
__global__ __launch_bounds__(kBlock) void k_query_f32(QueryArgs A)
{
    extern __shared__ uint32_t s_list[];
    __shared__ Shared S;
    query_f32_tile<TF, F, WIDTH, PAIRS, HOT>(A, s_list, S, block_tile(A.tile0));
}


// ------------------------------------------------------------ matrix-core path
//
// Layer k computes D = W_k * X with the weights as the A operand (M = output
// units, 32 per block) and the activations as the B operand (N = rays, 32 per
// block, two blocks per wave), v_mfma_f32_32x32x16.  Operand layout per lane
// l (i = l % 32, half q = l / 32): A holds W[i][8q .. 8q+7] of the K block,
// B holds X[8q .. 8q+7][i], and the 16 accumulators hold
// D[8(r/4) + 4q + r%4][i], r = 0..15.
//
// Layer 1 input: lane l encodes its own ray; per 16-wide K block it holds the
// ray's features k0..7 and k8..15, and one permlane32 swap turns these into
// the B operands of ray blocks 0-31 and 32-63.  Hidden layers take the
// accumulators as they lie: K slot 8q + e of 16-block s of output block m
// stands for unit 32m + 16s + (e < 4 ? 4q + e : 8 + 4q + e - 4); the host
// packs the weights of later layers in that order.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));
typedef float f16_t __attribute__((ext_vector_type(16)));

// MLP types of the matrix-core path.  Every fragment holds 8 values per
// lane (DW dwords); FP8 values are OCP e4m3 with a per-layer scale.
struct fp8e4m3 {};
typedef long f8x8_t;

template <typename TM> struct MmaT;
template <> struct MmaT<_Float16> {
    typedef h8_t vec;
    static constexpr int DW = 4;
    static constexpr bool scaled = false;
    static __device__ __forceinline__ f16_t mma(vec a, vec b, f16_t c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MmaT<__bf16> {
    typedef b8_t vec;
    static constexpr int DW = 4;
    static constexpr bool scaled = false;
    static __device__ __forceinline__ f16_t mma(vec a, vec b, f16_t c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct MmaT<fp8e4m3> {
    typedef f8x8_t vec;
    static constexpr int DW = 2;
    static constexpr bool scaled = true;
    static __device__ __forceinline__ f16_t mma(vec a, vec b, f16_t c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
    }
};

// Two 16-bit TM values in one dword.
template <typename TM> __device__ __forceinline__ uint32_t pack2(float a, float b)
{
    TM x = (TM)a, y = (TM)b;
    uint16_t u, v;
    __builtin_memcpy(&u, &x, 2);
    __builtin_memcpy(&v, &y, 2);
    return (uint32_t)u | ((uint32_t)v << 16);
}

// Eight values, times `scale`, rounded to TM and packed into DW dwords.
template <typename TM>
__device__ __forceinline__ void pack8(const float *v, float scale, uint32_t *d)
{
    if constexpr (MmaT<TM>::scaled) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float y = v[e] * scale;
            x[e] = y < -448.0f ? -448.0f : (y > 448.0f ? 448.0f : y);   // saturate to the e4m3 range
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(x[4 * q], x[4 * q + 1], 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(x[4 * q + 2], x[4 * q + 3], w, true);
            d[q] = (uint32_t)w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = pack2<TM>(v[2 * q], v[2 * q + 1]);
    }
}

// Value e (0..7) of a packed fragment, widened to float (not rescaled).
template <typename TM> __device__ __forceinline__ float unpack8(const uint32_t *d, int e)
{
    if constexpr (MmaT<TM>::scaled) {
        const uint32_t w = d[e >> 2];
        switch (e & 3) {
        case 0: return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
        case 1: return __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
        case 2: return __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
        default: return __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
        }
    } else {
        const uint16_t u = (uint16_t)((e & 1) ? (d[e >> 1] >> 16) : (d[e >> 1] & 0xffffu));
        TM v;
        __builtin_memcpy(&v, &u, 2);
        return (float)v;
    }
}

template <typename V8, int DW> __device__ __forceinline__ V8 as_vec(const uint32_t *d)
{
    V8 v;
    __builtin_memcpy(&v, d, 4 * DW);
    return v;
}

// One weight fragment (DW dwords of this lane).
template <int DW> __device__ __forceinline__ void load_frag(const uint32_t *p, uint32_t *d)
{
    if constexpr (DW == 4) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        d[0] = x.x; d[1] = x.y; d[2] = x.z; d[3] = x.w;
    } else {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        d[0] = x.x; d[1] = x.y;
    }
}

// Exchange the upper half-wave of x with the lower half-wave of y.
__device__ __forceinline__ void swap32(uint32_t &x, uint32_t &y)
{
    auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
}

template <typename TF, typename TM, int F, int WIDTH, int KBM, bool PAIRS, bool HOT>
__device__ __forceinline__ void query_mma_body(const QueryArgs &A, const Geom &g, const Mlp &mm,
                                               const TF *__restrict__ tab, uint32_t *s_list, Shared &S,
                                               uint32_t tile)
{
    typedef typename MmaT<TM>::vec vec_t;
    constexpr int DW = MmaT<TM>::DW;
    constexpr int FP = F == 3 ? 4 : F;        // features per level, padded to divide 16
    constexpr int MB = WIDTH / 32;            // output blocks of a hidden layer
    constexpr int LPB = 16 / FP;              // levels per K block
    constexpr int NL = (F * sizeof(TF) <= 4 && LPB >= 8) ? 8 : (LPB < 4 ? LPB : 4);   // levels per gather batch
    Lane ln;
    uint32_t *hot = s_list + (A.g.H >> 1) * kBlock;   // after the voxel lists (sized for the launch)
    if constexpr (HOT) stage_hot_levels<TF, F>(g, tab, hot);
    walk_and_sort<PAIRS>(A, g, S, s_list, ln, tile);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t src = ln.src, r = ln.r;
    const bool live = ln.live;
    const VRay &w = ln.w;
    const int count = 2 * ln.nvox;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(count));
    const uint32_t *__restrict__ Wv = reinterpret_cast<const uint32_t *>(mm.W);
    const int KB = mm.kb_point;

    f16_t acc[MB][2];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[m][nb][e] = 0.0f;

    // The entry point of a voxel equals the exit point of the voxel before it
    // when the two share a face (about 30 % of points on c2); such a point
    // reuses the previous point's features, so its lane issues no gathers.
    uint32_t plo[KBM][DW], phi[KBM][DW];
#pragma unroll
    for (int kb = 0; kb < KBM; ++kb)
#pragma unroll
        for (int q = 0; q < DW; ++q) plo[kb][q] = phi[kb][q] = 0u;
    uint32_t pp[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    int pface = -1;
    for (int h = 0; h < wmax; ++h) {
        float p[3] = {0.0f, 0.0f, 0.0f};
        int face = 0;
        const bool has = h < count;
        if (has) face = boundary_point(w, s_list[(h >> 1) * kBlock + src], h & 1, p);
        const bool dup = has && (h & 1) == 0 && face == pface && __float_as_uint(p[0]) == pp[0] &&
                         __float_as_uint(p[1]) == pp[1] && __float_as_uint(p[2]) == pp[2];
        const bool fresh = has && !dup;
#pragma unroll
        for (int kb = 0; kb < KBM; ++kb) {
            if (kb >= KB) break;
            // this K block's layer-1 weight fragments, requested ahead of the gathers so that
            // their latency overlaps the gathers' rather than following them
            uint32_t wd[MB][DW];
            const uint32_t *Wk = Wv + mm.woff[0] + ((size_t)((h * KB + kb) * MB) * 64 + lane) * DW;
#pragma unroll
            for (int m = 0; m < MB; ++m) load_frag<DW>(Wk + (size_t)m * 64 * DW, wd[m]);
            uint32_t lo[DW], hi[DW];
            if (fresh) {
                float e[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) e[q] = 0.0f;
#pragma unroll
                for (int c0 = 0; c0 < LPB; c0 += NL) {
                    float v[NL][F];
                    encode_levels<TF, F, NL, HOT>(g, tab, hot, kb * LPB + c0, p, face, v);
#pragma unroll
                    for (int lv = 0; lv < NL; ++lv)
#pragma unroll
                        for (int f = 0; f < F; ++f) e[(c0 + lv) * FP + f] = v[lv][f];
                }
                pack8<TM>(e, mm.qs[0], lo);
                pack8<TM>(e + 8, mm.qs[0], hi);
            } else {
#pragma unroll
                for (int q = 0; q < DW; ++q) {
                    lo[q] = dup ? plo[kb][q] : 0u;
                    hi[q] = dup ? phi[kb][q] : 0u;
                }
            }
#pragma unroll
            for (int q = 0; q < DW; ++q) {
                plo[kb][q] = lo[q];
                phi[kb][q] = hi[q];
            }
            if (A.dbg.enc && live && has) {
                // K slot k holds feature k % FP of level k / FP; the buffer is [H][L][F]
                const int LF = g.L * F;
                for (int q = 0; q < 16; ++q) {
                    const int k = kb * 16 + q, l = k / FP, f = k % FP;
                    if (l < g.L && f < F) {
                        const float v = q < 8 ? unpack8<TM>(lo, q) : unpack8<TM>(hi, q - 8);
                        A.dbg.enc[(size_t)r * g.H * LF + h * LF + l * F + f] = MmaT<TM>::scaled ? v / mm.qs[0] : v;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < DW; ++q) swap32(lo[q], hi[q]);
            const vec_t b0 = as_vec<vec_t, DW>(lo), b1 = as_vec<vec_t, DW>(hi);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const vec_t a = as_vec<vec_t, DW>(wd[m]);
                acc[m][0] = MmaT<TM>::mma(a, b0, acc[m][0]);
                acc[m][1] = MmaT<TM>::mma(a, b1, acc[m][1]);
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) pp[b] = __float_as_uint(p[b]);
        pface = has ? face : -1;
    }

    // hidden layers 2..n_hidden, then the head
    float o[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k) o[k] = 0.0f;
    if (wmax > 0) {
        for (int k = 1; k <= mm.n_hidden; ++k) {
            const bool head = k == mm.n_hidden;
            // activations -> B operands: 16-block s of output block m holds the
            // outputs lying in accumulator registers 8s .. 8s+7
            const float dqi = mm.dq[k - 1], qsi = mm.qs[k];
            const int MO = head ? 1 : MB;
            const uint32_t *Wk = Wv + mm.woff[k] + (size_t)lane * DW;
            // width 64: the whole layer's weight fragments requested before the activations are
            // converted, so that their latency overlaps that work
            constexpr int PF = MB == 2 ? MB : 1;   // output blocks prefetched
            uint32_t wpf[PF][MB][2][DW];
#pragma unroll
            for (int mo = 0; mo < PF; ++mo)
                if (mo < MO)
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int s = 0; s < 2; ++s)
                            load_frag<DW>(Wk + (size_t)((mo * MB + m) * 2 + s) * 64 * DW, wpf[mo][m][s]);
            asm volatile("" ::: "memory");   // keep the requests ahead of the conversion
            uint32_t xb[MB][2][2][DW];
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        float v[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const float y = MmaT<TM>::scaled ? acc[m][nb][8 * s + e] * dqi : acc[m][nb][8 * s + e];
                            v[e] = act_f(y, mm.act, mm.slope);
                        }
                        pack8<TM>(v, qsi, xb[m][nb][s]);
                    }
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[m][nb][e] = 0.0f;
#pragma unroll
            for (int mo = 0; mo < MB; ++mo) {
                if (mo < MO) {
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            uint32_t wd[DW];
                            if (mo < PF) {
#pragma unroll
                                for (int q = 0; q < DW; ++q) wd[q] = wpf[mo < PF ? mo : 0][m][s][q];
                            } else {
                                load_frag<DW>(Wk + (size_t)((mo * MB + m) * 2 + s) * 64 * DW, wd);
                            }
                            const vec_t a = as_vec<vec_t, DW>(wd);
                            acc[mo][0] = MmaT<TM>::mma(a, as_vec<vec_t, DW>(xb[m][0][s]), acc[mo][0]);
                            acc[mo][1] = MmaT<TM>::mma(a, as_vec<vec_t, DW>(xb[m][1][s]), acc[mo][1]);
                        }
                }
            }
        }
        // bring each ray's outputs to its own lane: rows 8q + r in x, 8q + 4 + r in y
        uint32_t x[8], y[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            x[e] = __float_as_uint(acc[0][0][e]);
            y[e] = __float_as_uint(acc[0][1][e]);
            swap32(x[e], y[e]);
        }
        const float dqo = MmaT<TM>::scaled ? mm.dq[mm.n_hidden] : 1.0f;
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                o[8 * q + rr] = __uint_as_float(x[4 * q + rr]) * dqo;
                o[8 * q + 4 + rr] = __uint_as_float(y[4 * q + rr]) * dqo;
            }
    }
    if (!live) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out) {
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k)
            if (k < mm.out_dim) A.dbg.out[(size_t)r * mm.out_dim + k] = count > 0 ? o[k] : 0.0f;
    }
    decode_store<PAIRS>(A, mm, r, ln.pair, w, count, o);
}

template <typename TF, typename TM, int F, int WIDTH, int KBM, bool PAIRS, bool HOT>
__device__ __forceinline__ void query_mma_tile(const QueryArgs &A, uint32_t *s_list, Shared &S, uint32_t tile)
{
    if constexpr (PAIRS) {
        const int o = tile_object(A.pr, tile);
        if (o < 0) return;
        const cObjDev &O = ((const cObjDev *)A.pr.objs)[o];
        query_mma_body<TF, TM, F, WIDTH, KBM, true, HOT>(A, O.g, O.m, (const TF *)O.tables, s_list, S, tile);
    } else {
        query_mma_body<TF, TM, F, WIDTH, KBM, false, HOT>(A, A.g, A.m, reinterpret_cast<const TF *>(A.tables), s_list,
                                                          S, tile);
    }
}

template <typename TF, typename TM, int F, int WIDTH, int KBM, bool PAIRS, bool HOT>
__global__ __launch_bounds__(kBlock) void k_query_mma(QueryArgs A)
{
    extern __shared__ uint32_t s_list[];
    __shared__ Shared S;
    query_mma_tile<TF, TM, F, WIDTH, KBM, PAIRS, HOT>(A, s_list, S, block_tile(A.tile0));
}

template <typename TF, typename TM, int F, int WIDTH, int KBM, bool PAIRS, bool HOT>
__global__ __launch_bounds__(kBlock) void k_query_mma_persist(QueryArgs A)
{
    extern __shared__ uint32_t s_list[];
    __shared__ Shared S;
    __shared__ uint32_t s_tile;
    for (;;) {
        const uint32_t tile = next_tile(A, s_tile);
        if (tile == kNoTile) break;
        query_mma_tile<TF, TM, F, WIDTH, KBM, PAIRS, HOT>(A, s_list, S, tile);
    }
}

// ------------------------------------------------------------- small batches
//
// One wave per ray, for batches too small to fill the chip with one ray per
// lane (FP32 features and MLP, width 64, at most 16 levels): a point's
// 8-corner gathers of up to 8 levels are spread over the lanes (lane 8q + c:
// corner c of level 8 round + q), a butterfly sum over each level's 8 lanes
// interpolates, and lane j then owns output j of every layer, taking the
// layer's inputs one at a time from the lanes that hold them.  Cells, slots,
// corner weights and every sum's order are those of the ray-per-lane FP32
// kernel, so a ray's answer and debug outputs are the same bits whichever of
// the two kernels its batch runs on.  The walk kernel's lists are read from
// the workspace.
constexpr int kLatWaves = 4;     // rays (one wave each) per workgroup
constexpr int kLatMaxLF = 48;    // features per point: at most 16 levels of at most 3

template <typename TF, int F>
__device__ __forceinline__ void lat_level(const Geom &g, const TF *__restrict__ tab, int l, uint32_t c,
                                          const float p[3], float v[F])
{
    const bool in = l < g.L;
    const int lc = in ? l : g.L - 1;
    uint32_t i[3];
    float wt[3];
    level_cell_mm(g, lc, p, i, wt);
    const uint32_t x = i[0] + (c & 1u), y = (i[1] + ((c >> 1) & 1u)) * g.my[lc], z = (i[2] + (c >> 2)) * g.mz[lc];
    const uint32_t s = ((x + y + z) & g.dmask[lc]) | ((x ^ y ^ z) & g.hmask[lc]);
    const float wx = (c & 1u) ? wt[0] : 1.0f - wt[0];
    const float wy = ((c >> 1) & 1u) ? wt[1] : 1.0f - wt[1];
    const float wz = (c >> 2) ? wt[2] : 1.0f - wt[2];
    const float wc = wx * (wy * wz);
    Entry<TF, F> en;
    en.load(reinterpret_cast<const char *>(tab + ((size_t)lc << g.log2_T) * F), s * (uint32_t)(F * sizeof(TF)));
    // every lane of the level sums the 8 corners in corner order, as one fused
    // multiply-add chain on the raw entries: the ray-per-lane kernel's sum, bit for bit
    const int g0 = (int)((threadIdx.x & 63u) & ~7u);
#pragma unroll
    for (int f = 0; f < F; ++f) v[f] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float wk = __shfl(wc, g0 + k, 64);
        Entry<TF, F> ek;
#pragma unroll
        for (int d = 0; d < Entry<TF, F>::W; ++d) ek.d[d] = (uint32_t)__shfl((int)en.d[d], g0 + k, 64);
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] = __builtin_fmaf(wk, ek.get(f), v[f]);
    }
    if (!in) {
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] = 0.0f;
    }
}

// The lane's corner of lat_level without the sum: corner c of level l (levels at
// or beyond L read level L - 1), its weight and its entry.
template <typename TF, int F>
__device__ __forceinline__ void lat_corner(const Geom &g, const TF *__restrict__ tab, int l, uint32_t c,
                                           const float p[3], float &wc, Entry<TF, F> &en)
{
    const int lc = l < g.L ? l : g.L - 1;
    uint32_t i[3];
    float wt[3];
    level_cell_mm(g, lc, p, i, wt);
    const uint32_t x = i[0] + (c & 1u), y = (i[1] + ((c >> 1) & 1u)) * g.my[lc], z = (i[2] + (c >> 2)) * g.mz[lc];
    const uint32_t s = ((x + y + z) & g.dmask[lc]) | ((x ^ y ^ z) & g.hmask[lc]);
    const float wx = (c & 1u) ? wt[0] : 1.0f - wt[0];
    const float wy = ((c >> 1) & 1u) ? wt[1] : 1.0f - wt[1];
    const float wz = (c >> 2) ? wt[2] : 1.0f - wt[2];
    wc = wx * (wy * wz);
    en.load(reinterpret_cast<const char *>(tab + ((size_t)lc << g.log2_T) * F), s * (uint32_t)(F * sizeof(TF)));
}

template <int F>
__global__ __launch_bounds__(64 * kLatWaves) void k_query_lat(QueryArgs A)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t slot = A.tile0 * kBlock + blockIdx.x * kLatWaves + (threadIdx.x >> 6);
    if (slot >= A.n) return;   // the whole wave
    const Geom &g = A.g;
    const Mlp &mm = A.m;
    const float *__restrict__ tab = reinterpret_cast<const float *>(A.tables);
    const float *__restrict__ W = reinterpret_cast<const float *>(mm.W);
    uint32_t r, pair;
    bool live;
    VRay w;
    slot_ray<false>(A, g, slot, r, pair, live, w);
    const int count = __builtin_amdgcn_readfirstlane(live ? 2 * (int)A.nvox[slot] : 0);
    const int LF = g.L * F;
    const uint32_t q = lane >> 3, c = lane & 7u;
    float acc = 0.0f;
    float fv[2][F];   // this lane's level features (rounds 0 and 1), kept for a repeated point
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) fv[k][f] = 0.0f;
    uint32_t pp[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    int pface = -1;
    float amax = 0.0f;   // largest |input| of the current layer (calibration)
    for (int h = 0; h < count; ++h) {
        // this point's layer-1 weights (output `lane` of each input), requested ahead of the gathers
        float wk[kLatMaxLF];
        const float *W1 = W + mm.off[0] + (size_t)h * LF * 64 + lane;
#pragma unroll
        for (int k = 0; k < kLatMaxLF; ++k) wk[k] = W1[(size_t)(k < LF ? k : 0) * 64];   // k >= LF: unused
        float p[3];
        const int face = boundary_point(w, A.lists[(size_t)(h >> 1) * A.n + slot], h & 1, p);
        const bool dup = (h & 1) == 0 && face == pface && __float_as_uint(p[0]) == pp[0] &&
                         __float_as_uint(p[1]) == pp[1] && __float_as_uint(p[2]) == pp[2];
        if (!dup) {
            lat_level<float, F>(g, tab, (int)q, c, p, fv[0]);
            if (g.L > 8) lat_level<float, F>(g, tab, 8 + (int)q, c, p, fv[1]);
        }
        if (A.dbg.act_amax) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int f = 0; f < F; ++f) amax = fmax2(amax, __builtin_fabsf(fv[k][f]));
        }
        if (A.dbg.enc && live && c == 0u) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int l = 8 * k + (int)q;
                if (l < g.L)
#pragma unroll
                    for (int f = 0; f < F; ++f) A.dbg.enc[((size_t)r * g.H + h) * LF + l * F + f] = fv[k][f];
            }
        }
        // input k = l F + f lives in lane 8 (l mod 8), round l / 8
#pragma unroll
        for (int k = 0; k < kLatMaxLF; ++k) {
            if (k < LF) {
                const int l = k / F, f = k % F;
                const float x = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, fv[l >> 3][f]), 8 * (l & 7)));
                acc = __builtin_fmaf(wk[k], x, acc);
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) pp[b] = __float_as_uint(p[b]);
        pface = face;
    }
    // hidden layers, then the head (lanes below kMaxOut)
    float o = 0.0f;
    if (A.dbg.act_amax) fold_max(A.dbg.act_amax + 0, amax);
    if (count > 0) {
        for (int k = 1; k <= mm.n_hidden; ++k) {
            const bool head = k == mm.n_hidden;
            const float x = act_f(acc, mm.act, mm.slope);
            if (A.dbg.act_amax) fold_max(A.dbg.act_amax + k, __builtin_fabsf(x));
            const float *Wk = W + mm.off[k] + (head ? (lane < (uint32_t)kMaxOut ? lane : 0u) : lane);
            const int stride = head ? kMaxOut : 64;
            float nxt = 0.0f;
#pragma unroll 16
            for (int i = 0; i < 64; ++i) {
                const float xi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), i));
                nxt = __builtin_fmaf(Wk[(size_t)i * stride], xi, nxt);
            }
            if (head) o = lane < (uint32_t)kMaxOut ? nxt : 0.0f;
            else acc = nxt;
        }
    }
    float oo[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k)
        oo[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, o), k));
    if (!live || lane != 0u) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out) {
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k)
            if (k < mm.out_dim) A.dbg.out[(size_t)r * mm.out_dim + k] = count > 0 ? oo[k] : 0.0f;
    }
    decode_store<false>(A, mm, r, pair, w, count, oo);
}

// The matrix-core form of the one-wave-per-ray kernel (two features per level,
// width 64, at most two K blocks per point).  The wave's lanes interpolate the
// ray's point as above; every lane then packs the point's 16 K slots of a K
// block, and the B operand puts slots 0..7 in lanes 0..31 and 8..15 in lanes
// 32..63, so each of the 32 columns is this ray.  A column of a matrix-core
// product does not depend on the other columns, so every column, and the
// answer, has the bits the ray gets in k_query_mma.
template <typename TF, typename TM, int KBM>
__global__ __launch_bounds__(64 * kLatWaves) void k_query_mma_lat(QueryArgs A)
{
    typedef typename MmaT<TM>::vec vec_t;
    constexpr int F = 2, MB = 2, DW = MmaT<TM>::DW;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t slot = A.tile0 * kBlock + blockIdx.x * kLatWaves + (threadIdx.x >> 6);
    if (slot >= A.n) return;   // the whole wave
    const Geom &g = A.g;
    const Mlp &mm = A.m;
    const TF *__restrict__ tab = reinterpret_cast<const TF *>(A.tables);
    const uint32_t *__restrict__ Wv = reinterpret_cast<const uint32_t *>(mm.W);
    uint32_t r, pair;
    bool live;
    VRay w;
    slot_ray<false>(A, g, slot, r, pair, live, w);
    const int count = __builtin_amdgcn_readfirstlane(live ? 2 * (int)A.nvox[slot] : 0);
    const int KB = mm.kb_point;
    const uint32_t q = lane >> 3, c = lane & 7u;
    f16_t acc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[m][e] = 0.0f;
    uint32_t prev[KBM][DW];
#pragma unroll
    for (int kb = 0; kb < KBM; ++kb)
#pragma unroll
        for (int d = 0; d < DW; ++d) prev[kb][d] = 0u;
    uint32_t pp[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    int pface = -1;
    for (int h = 0; h < count; ++h) {
        // the point's layer-1 weight fragments, requested ahead of the gathers
        uint32_t wd[KBM][MB][DW];
#pragma unroll
        for (int kb = 0; kb < KBM; ++kb)
#pragma unroll
            for (int m = 0; m < MB; ++m)
                load_frag<DW>(Wv + mm.woff[0] + ((size_t)(((h * KB + (kb < KB ? kb : 0)) * MB + m) * 64) + lane) * DW,
                              wd[kb][m]);
        float p[3];
        const int face = boundary_point(w, A.lists[(size_t)(h >> 1) * A.n + slot], h & 1, p);
        const bool dup = (h & 1) == 0 && face == pface && __float_as_uint(p[0]) == pp[0] &&
                         __float_as_uint(p[1]) == pp[1] && __float_as_uint(p[2]) == pp[2];
        // this lane's corner: c of level 8 kb + q, for the two K blocks
        float wcr[2] = {0.0f, 0.0f};
        Entry<TF, F> enr[2];
        if (!dup) {
            lat_corner<TF, F>(g, tab, (int)q, c, p, wcr[0], enr[0]);
            if (g.L > 8) lat_corner<TF, F>(g, tab, 8 + (int)q, c, p, wcr[1], enr[1]);
        }
        const uint32_t hf = lane >> 5;
#pragma unroll
        for (int kb = 0; kb < KBM; ++kb) {
            if (kb >= KB) break;
            uint32_t bk[DW];
            if (!dup) {
                // Lanes 0..31 form the B operand's K slots 0..7 (levels 8 kb .. 8 kb + 3), lanes
                // 32..63 slots 8..15 (levels 8 kb + 4 .. 8 kb + 7): each lane sums those 4 levels'
                // corners itself, in corner order, and packs them, as a lane of k_query_mma
                // does for its own ray (the same expressions, so the same roundings).
                float e[8];
#pragma unroll
                for (int li = 0; li < 4; ++li) {
                    const int j = 4 * (int)hf + li;   // level 8 kb + j: corners in lanes 8 j ..
                    float v[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) v[f] = 0.0f;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const float wk = __shfl(wcr[kb], 8 * j + k, 64);
                        Entry<TF, F> ek;
#pragma unroll
                        for (int d = 0; d < Entry<TF, F>::W; ++d)
                            ek.d[d] = (uint32_t)__shfl((int)enr[kb].d[d], 8 * j + k, 64);
#pragma unroll
                        for (int f = 0; f < F; ++f) v[f] = __builtin_fmaf(wk, ek.get(f), v[f]);
                    }
                    if (8 * kb + j >= g.L) {
#pragma unroll
                        for (int f = 0; f < F; ++f) v[f] = 0.0f;
                    }
#pragma unroll
                    for (int f = 0; f < F; ++f) e[2 * li + f] = v[f];
                }
                pack8<TM>(e, mm.qs[0], bk);
            } else {
#pragma unroll
                for (int d = 0; d < DW; ++d) bk[d] = prev[kb][d];
            }
            if (A.dbg.enc && live && (lane & 31u) == 0u) {
                // lane 0 writes K slots 0..7, lane 32 slots 8..15 (a repeated point: the previous one's)
                const int LF = g.L * F;
                for (int k = 0; k < 8; ++k) {
                    const int l = kb * 8 + 4 * (int)hf + k / 2, f = k % 2;
                    if (l < g.L) {
                        const float v = unpack8<TM>(bk, k);
                        A.dbg.enc[(size_t)r * g.H * LF + h * LF + l * F + f] = MmaT<TM>::scaled ? v / mm.qs[0] : v;
                    }
                }
            }
#pragma unroll
            for (int d = 0; d < DW; ++d) prev[kb][d] = bk[d];
            const vec_t b0 = as_vec<vec_t, DW>(bk);
#pragma unroll
            for (int m = 0; m < MB; ++m) acc[m] = MmaT<TM>::mma(as_vec<vec_t, DW>(wd[kb][m]), b0, acc[m]);
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) pp[b] = __float_as_uint(p[b]);
        pface = face;
    }
    // hidden layers 2..n_hidden, then the head, as k_query_mma with one column block
    float o[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k) o[k] = 0.0f;
    if (count > 0) {
        for (int k = 1; k <= mm.n_hidden; ++k) {
            const bool head = k == mm.n_hidden;
            const float dqi = mm.dq[k - 1], qsi = mm.qs[k];
            uint32_t xb[MB][2][DW];
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    float v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float y = MmaT<TM>::scaled ? acc[m][8 * s2 + e] * dqi : acc[m][8 * s2 + e];
                        v[e] = act_f(y, mm.act, mm.slope);
                    }
                    pack8<TM>(v, qsi, xb[m][s2]);
                }
            const int MO = head ? 1 : MB;
            const uint32_t *Wk = Wv + mm.woff[k] + (size_t)lane * DW;
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[m][e] = 0.0f;
#pragma unroll
            for (int mo = 0; mo < MB; ++mo) {
                if (mo < MO) {
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2) {
                            uint32_t wd2[DW];
                            load_frag<DW>(Wk + (size_t)((mo * MB + m) * 2 + s2) * 64 * DW, wd2);
                            acc[mo] = MmaT<TM>::mma(as_vec<vec_t, DW>(wd2), as_vec<vec_t, DW>(xb[m][s2]), acc[mo]);
                        }
                }
            }
        }
        // rows 8q + r of the head lie in lanes 0..31, rows 8q + 4 + r in lanes 32..63
        uint32_t x[8], y[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            x[e] = __float_as_uint(acc[0][e]);
            y[e] = x[e];
            swap32(x[e], y[e]);
        }
        const float dqo = MmaT<TM>::scaled ? mm.dq[mm.n_hidden] : 1.0f;
#pragma unroll
        for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                o[8 * q2 + rr] = __uint_as_float(x[4 * q2 + rr]) * dqo;
                o[8 * q2 + 4 + rr] = __uint_as_float(y[4 * q2 + rr]) * dqo;
            }
    }
    if (!live || lane != 0u) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out) {
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k)
            if (k < mm.out_dim) A.dbg.out[(size_t)r * mm.out_dim + k] = count > 0 ? o[k] : 0.0f;
    }
    decode_store<false>(A, mm, r, pair, w, count, o);
}

// ------------------------------------------------------------- gather ceiling
//
// The query kernel's gathers alone, for measurement: the same prologue (voxel
// lists from the walk, count sort), the same boundary points, repeated-point
// reuse and encode_levels batches, but each ray's interpolated features are
// summed into sums[r] instead of feeding the MLP.  Without the accumulators
// it runs at the occupancy its gathers and address arithmetic allow, so its
// time bounds what the query kernel's gathers can take.
template <typename TF, int F>
__device__ __forceinline__ void gather_only_body(const QueryArgs &A, float *sums, uint32_t *s_list, Shared &S)
{
    constexpr int FP = F == 3 ? 4 : F;
    constexpr int LPB = 16 / FP;
    constexpr int NL = (F * sizeof(TF) <= 4 && LPB >= 8) ? 8 : (LPB < 4 ? LPB : 4);
    const Geom &g = A.g;
    const TF *__restrict__ tab = reinterpret_cast<const TF *>(A.tables);
    Lane ln;
    walk_and_sort<false>(A, g, S, s_list, ln, block_tile(A.tile0));
    const int count = 2 * ln.nvox;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(count));
    float total = 0.0f, prev = 0.0f;
    uint32_t pp[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    int pface = -1;
    for (int h = 0; h < wmax; ++h) {
        float p[3] = {0.0f, 0.0f, 0.0f};
        int face = 0;
        const bool has = h < count;
        if (has) face = boundary_point(ln.w, s_list[(h >> 1) * kBlock + ln.src], h & 1, p);
        const bool dup = has && (h & 1) == 0 && face == pface && __float_as_uint(p[0]) == pp[0] &&
                         __float_as_uint(p[1]) == pp[1] && __float_as_uint(p[2]) == pp[2];
        float here = 0.0f;
        if (has && !dup) {
            for (int l0 = 0; l0 < g.L; l0 += NL) {
                float v[NL][F];
                encode_levels<TF, F, NL, false>(g, tab, nullptr, l0, p, face, v);
#pragma unroll
                for (int lv = 0; lv < NL; ++lv)
#pragma unroll
                    for (int f = 0; f < F; ++f) here += v[lv][f];
            }
        } else if (dup) {
            here = prev;
        }
        total += here;
        prev = here;
#pragma unroll
        for (int b = 0; b < 3; ++b) pp[b] = __float_as_uint(p[b]);
        pface = has ? face : -1;
    }
    if (ln.live) sums[ln.r] = total;
}

template <typename TF, int F>
__global__ __launch_bounds__(kBlock) void k_gather_only(QueryArgs A, float *sums)
{
    extern __shared__ uint32_t s_list[];
    __shared__ Shared S;
    gather_only_body<TF, F>(A, sums, s_list, S);
}

// ------------------------------------------------------------------ broad phase
struct BroadArgs {
    const float4 *rays;
    uint32_t n_rays;
    const lsnif_instance *inst;
    uint32_t n_inst;
    const ObjDev *objs;       // object table by id
    uint32_t n_objs;
    uint32_t *offsets;        // [n_rays + 1]: pairs per ray, then their exclusive scan
    uint32_t *pair_ray, *pair_inst;
    // With mask_words > 0 the counting pass also records which instances each ray
    // meets (bit i % 32 of word i / 32, word-major: masks[(i / 32) n_rays + r]) and
    // the writing pass lists the pairs from those bits instead of testing again.
    uint32_t *masks;
    uint32_t mask_words;
};
constexpr uint32_t kBroadMaskWords = 8;   // instance masks for launches of at most 256 instances

// ------------------------------------------------------------ merged serving
// One member of a merged serving launch: its own buffers and where its rays and
// pairs start in the staged arrays.
struct MergeMember {
    const float4 *rays;           // [2 n_rays] (a ray is two float4)
    lsnif_hit *out;               // [n_rays]
    const uint32_t *pair_ray, *pair_inst;   // [n_pairs] (pair requests)
    uint32_t ray0, pair0, n_rays, n_pairs;
};
constexpr uint32_t kMergeMax = 32;   // members of one merged launch (the kernel argument holds them)
struct MergeArgs {
    MergeMember m[kMergeMax];
    uint32_t n_members, n_rays, n_pairs;
    float4 *rays;                 // staged rays [2 n_rays]
    uint32_t *pair_ray, *pair_inst;   // staged pairs [n_pairs]
    lsnif_hit *out;               // staged answers [n_rays]
};
static_assert(sizeof(MergeArgs) <= 4096, "merged-launch arguments must fit a kernel's argument space");

// ------------------------------------------------------------------ bounce rays
struct BounceArgs {
    const float4 *rays;       // the rays just answered (world space)
    const lsnif_hit *hits;    // their nearest hits
    uint32_t n;
    uint32_t seed, bounce;
    float eps;                // offset of the new origin along the facing normal
    uint32_t *offsets;        // [n + 1]: 1 per hit, then their exclusive scan
    float4 *next;             // new rays, compacted in the order of their parents
    uint32_t *parent;         // index of each new ray's parent
};

// PCG hash (Jarzynski and Olano 2020, "Hash Functions for GPU Rendering"): a
// 32-bit counter-based generator, one permuted congruential step of the input.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v)
{
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// ------------------------------------------------------------------ voxel walk
// RECHECK: some object of the launch asks for the float64 re-decision of grazing voxels.
template <bool PAIRS, bool RECHECK>
__global__ __launch_bounds__(kBlock) void k_walk(QueryArgs A)
{
    __shared__ uint32_t coarse[kCoarseLdsWords];
    if constexpr (PAIRS) {
        const int o = tile_object(A.pr, block_tile(A.tile0));
        if (o < 0) return;   // the query kernel skips such a tile too
        const cObjDev &O = ((const cObjDev *)A.pr.objs)[o];
        walk_body<true, RECHECK>(A, O.g, coarse);
    } else {
        walk_body<false, RECHECK>(A, A.g, coarse);
    }
}

// ------------------------------------------------------------------ debug path
struct DebugArgs {
    Geom g;
    const float4 *rays;
    uint32_t n;
    lsnif_debug_bufs b;
};

}  // namespace lsnif
