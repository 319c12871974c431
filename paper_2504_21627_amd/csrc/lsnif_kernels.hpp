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
};

struct Dbg {
    int32_t *count;
    float *tatb;
    float *out;
    float *enc;
};

struct QueryArgs {
    Geom g;
    Mlp m;
    const void *tables;       // [L][T][F] in the feature type
    const float4 *rays;
    lsnif_hit *hits;
    uint32_t n;
    Dbg dbg;
};

template <typename TF> __device__ __forceinline__ float to_f32(TF v);
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<__bf16>(__bf16 v) { return (float)v; }

// F features of table slot `slot`.
template <typename TF, int F>
__device__ __forceinline__ void load_entry(const TF *__restrict__ base, uint32_t slot, float v[F])
{
    const TF *p = base + (size_t)slot * F;
    if constexpr (F == 2 && sizeof(TF) == 4) {
        float2 x = *reinterpret_cast<const float2 *>(p);
        v[0] = x.x;
        v[1] = x.y;
    } else if constexpr (F == 2 && sizeof(TF) == 2) {
        uint32_t x = *reinterpret_cast<const uint32_t *>(p);
        TF lo, hi;
        uint16_t l16 = (uint16_t)(x & 0xffffu), h16 = (uint16_t)(x >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        v[0] = to_f32<TF>(lo);
        v[1] = to_f32<TF>(hi);
    } else if constexpr (F == 4 && sizeof(TF) == 4) {
        float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] = to_f32<TF>(p[f]);
    }
}

// Interpolated F features of level l at boundary point p (voxel units)
// whose crossing axis is `face`.  Levels aligned with the voxel faces read
// only the 4 corners of the face (the other 4 carry weight exactly 0).
template <typename TF, int F>
__device__ __forceinline__ void encode_level(const Geom &g, const TF *__restrict__ tab, int l,
                                             const float p[3], int face, float out[F])
{
    uint32_t i[3];
    float wt[3];
    level_cell(g, l, p, i, wt);
    const TF *base = tab + ((size_t)l << g.log2_T) * F;
    const bool dense = (g.dense_mask >> l) & 1u;
    const uint32_t side = (uint32_t)g.R[l] + 1u;
    // per-axis vertex terms of the slot: slot = combine(tx, ty, tz)
    uint32_t tx0 = i[0], tx1 = i[0] + 1u;
    uint32_t ty0, ty1, tz0, tz1;
    if (dense) {
        ty0 = side * i[1]; ty1 = ty0 + side;
        tz0 = side * side * i[2]; tz1 = tz0 + side * side;
    } else {
        ty0 = i[1] * kPrimeY; ty1 = ty0 + kPrimeY;
        tz0 = i[2] * kPrimeZ; tz1 = tz0 + kPrimeZ;
    }
    const uint32_t mask = (1u << g.log2_T) - 1u;
#pragma unroll
    for (int f = 0; f < F; ++f) out[f] = 0.0f;
    if ((g.aligned_mask >> l) & 1u) {
        // put the crossing axis last: u, v = the two other axes in order
        const uint32_t tf[3][2] = {{tx0, tx1}, {ty0, ty1}, {tz0, tz1}};
        const int ua = face == 0 ? 1 : 0, va = face == 2 ? 1 : 2;
        const uint32_t u0 = ua == 0 ? tf[0][0] : tf[1][0], u1 = ua == 0 ? tf[0][1] : tf[1][1];
        const uint32_t v0 = va == 1 ? tf[1][0] : tf[2][0], v1 = va == 1 ? tf[1][1] : tf[2][1];
        const float wu = ua == 0 ? wt[0] : wt[1];
        const float wv = va == 1 ? wt[1] : wt[2];
        const float wf = face == 0 ? wt[0] : (face == 1 ? wt[1] : wt[2]);
        const uint32_t fsel = wf != 0.0f ? 1u : 0u;
        const uint32_t ff = face == 0 ? (fsel ? tx1 : tx0) : (face == 1 ? (fsel ? ty1 : ty0) : (fsel ? tz1 : tz0));
        uint32_t s[4];
        s[0] = dense ? u0 + v0 + ff : ((u0 ^ v0 ^ ff) & mask);
        s[1] = dense ? u1 + v0 + ff : ((u1 ^ v0 ^ ff) & mask);
        s[2] = dense ? u0 + v1 + ff : ((u0 ^ v1 ^ ff) & mask);
        s[3] = dense ? u1 + v1 + ff : ((u1 ^ v1 ^ ff) & mask);
        float e[4][F];
#pragma unroll
        for (int c = 0; c < 4; ++c) load_entry<TF, F>(base, s[c], e[c]);
        const float w[4] = {(1.0f - wu) * (1.0f - wv), wu * (1.0f - wv), (1.0f - wu) * wv, wu * wv};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int f = 0; f < F; ++f) out[f] = __builtin_fmaf(w[c], e[c][f], out[f]);
    } else {
        uint32_t s[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t a = (c & 1) ? tx1 : tx0, b = (c & 2) ? ty1 : ty0, d = (c & 4) ? tz1 : tz0;
            s[c] = dense ? a + b + d : ((a ^ b ^ d) & mask);
        }
        float e[8][F];
#pragma unroll
        for (int c = 0; c < 8; ++c) load_entry<TF, F>(base, s[c], e[c]);
        const float wx[2] = {1.0f - wt[0], wt[0]}, wy[2] = {1.0f - wt[1], wt[1]}, wz[2] = {1.0f - wt[2], wt[2]};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float w = (wx[c & 1] * wy[(c >> 1) & 1]) * wz[(c >> 2) & 1];
#pragma unroll
            for (int f = 0; f < F; ++f) out[f] = __builtin_fmaf(w, e[c][f], out[f]);
        }
    }
}

__device__ __forceinline__ float act_f(float x, int act, float slope)
{
    return x > 0.0f ? x : (act == LSNIF_LEAKY_RELU ? x * slope : 0.0f);
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
__device__ __forceinline__ void decode_store(const QueryArgs &A, uint32_t r, const VRay &w, int count,
                                             const float *o)
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
            const int m0 = 5 + 3 * A.m.has_albedo;
            int best = 0;
            float bv = o[m0];
            for (int k = 1; k < A.m.n_mat; ++k)
                if (o[m0 + k] > bv) { bv = o[m0 + k]; best = k; }
            h.material = best;
        }
    }
    A.hits[r] = h;
}

// ---------------------------------------------------------------- float32 path
//
// Weights: layer k transposed to [in][out_pad] float32 (out_pad = WIDTH for
// hidden layers, kMaxOut for the head) so the outputs fed by one input are
// contiguous and every lane reads the same address.
template <typename TF, int F, int WIDTH>
__global__ __launch_bounds__(kBlock) void k_query_f32(QueryArgs A)
{
    __shared__ uint32_t s_list[kMaxList * kBlock];
    const uint32_t tid = threadIdx.x;
    const uint32_t r = blockIdx.x * kBlock + tid;
    const bool live = r < A.n;
    const Geom &g = A.g;
    VRay w;
    w.valid = w.cand = false;
    w.ta = w.tb = 0.0f;
    w.tmax = 0.0f;
    w.mov = 0;
    if (live) setup_ray(g, A.rays[2 * r], A.rays[2 * r + 1], w);
    const int nvox = live ? walk_voxels(g, w, s_list + tid, kBlock, g.H >> 1) : 0;
    const int count = 2 * nvox;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(count));
    const float *__restrict__ Wf = reinterpret_cast<const float *>(A.m.W);
    const TF *__restrict__ tab = reinterpret_cast<const TF *>(A.tables);
    const int LF = g.L * F;

    float acc[WIDTH];
#pragma unroll
    for (int j = 0; j < WIDTH; ++j) acc[j] = 0.0f;
    for (int h = 0; h < wmax; ++h) {
        if (h < count) {
            float p[3];
            const int face = boundary_point(w, s_list[(h >> 1) * kBlock + tid], h & 1, p);
            for (int l = 0; l < g.L; ++l) {
                float e[F];
                encode_level<TF, F>(g, tab, l, p, face, e);
                if (A.dbg.enc) {
#pragma unroll
                    for (int f = 0; f < F; ++f) A.dbg.enc[(size_t)r * g.H * LF + h * LF + l * F + f] = e[f];
                }
                const float *Wk = Wf + A.m.off[0] + (size_t)(h * LF + l * F) * WIDTH;
#pragma unroll
                for (int f = 0; f < F; ++f)
#pragma unroll
                    for (int j = 0; j < WIDTH; ++j) acc[j] = __builtin_fmaf(Wk[f * WIDTH + j], e[f], acc[j]);
            }
        }
    }
    float o[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k) o[k] = 0.0f;
    if (wmax > 0) {
        for (int k = 1; k < A.m.n_hidden; ++k) {
            float nxt[WIDTH];
#pragma unroll
            for (int j = 0; j < WIDTH; ++j) nxt[j] = 0.0f;
            const float *Wk = Wf + A.m.off[k];
#pragma unroll
            for (int i = 0; i < WIDTH; ++i) {
                const float x = act_f(acc[i], A.m.act, A.m.slope);
#pragma unroll
                for (int j = 0; j < WIDTH; ++j) nxt[j] = __builtin_fmaf(Wk[i * WIDTH + j], x, nxt[j]);
            }
#pragma unroll
            for (int j = 0; j < WIDTH; ++j) acc[j] = nxt[j];
        }
        const float *Wo = Wf + A.m.off[A.m.n_hidden];
#pragma unroll
        for (int i = 0; i < WIDTH; ++i) {
            const float x = act_f(acc[i], A.m.act, A.m.slope);
#pragma unroll
            for (int j = 0; j < kMaxOut; ++j) o[j] = __builtin_fmaf(Wo[i * kMaxOut + j], x, o[j]);
        }
    }
    if (!live) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out)
        for (int k = 0; k < A.m.out_dim; ++k) A.dbg.out[(size_t)r * A.m.out_dim + k] = count > 0 ? o[k] : 0.0f;
    decode_store(A, r, w, count, o);
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

template <typename TM> struct MmaT;
template <> struct MmaT<_Float16> {
    typedef h8_t vec;
    static __device__ __forceinline__ f16_t mma(vec a, vec b, f16_t c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MmaT<__bf16> {
    typedef b8_t vec;
    static __device__ __forceinline__ f16_t mma(vec a, vec b, f16_t c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// Two TM values in one dword.
template <typename TM> __device__ __forceinline__ uint32_t pack2(float a, float b)
{
    TM x = (TM)a, y = (TM)b;
    uint16_t u, v;
    __builtin_memcpy(&u, &x, 2);
    __builtin_memcpy(&v, &y, 2);
    return (uint32_t)u | ((uint32_t)v << 16);
}
template <typename TM> __device__ __forceinline__ float unpack_lo(uint32_t x)
{
    uint16_t u = (uint16_t)(x & 0xffffu);
    TM v;
    __builtin_memcpy(&v, &u, 2);
    return (float)v;
}
template <typename TM> __device__ __forceinline__ float unpack_hi(uint32_t x)
{
    uint16_t u = (uint16_t)(x >> 16);
    TM v;
    __builtin_memcpy(&v, &u, 2);
    return (float)v;
}

template <typename V8> __device__ __forceinline__ V8 as_vec(const uint32_t d[4])
{
    V8 v;
    __builtin_memcpy(&v, d, 16);
    return v;
}

// Exchange the upper half-wave of x with the lower half-wave of y.
__device__ __forceinline__ void swap32(uint32_t &x, uint32_t &y)
{
    auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
}

template <typename TF, typename TM, int F, int WIDTH>
__global__ __launch_bounds__(kBlock) void k_query_mma(QueryArgs A)
{
    typedef typename MmaT<TM>::vec vec_t;
    constexpr int FP = F == 3 ? 4 : F;        // features per level, padded to divide 16
    constexpr int MB = WIDTH / 32;            // output blocks of a hidden layer
    constexpr int LPB = 16 / FP;              // levels per K block
    __shared__ uint32_t s_list[kMaxList * kBlock];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t r = blockIdx.x * kBlock + tid;
    const bool live = r < A.n;
    const Geom &g = A.g;
    VRay w;
    w.valid = w.cand = false;
    w.ta = w.tb = 0.0f;
    w.tmax = 0.0f;
    w.mov = 0;
    if (live) setup_ray(g, A.rays[2 * r], A.rays[2 * r + 1], w);
    const int nvox = live ? walk_voxels(g, w, s_list + tid, kBlock, g.H >> 1) : 0;
    const int count = 2 * nvox;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(count));
    const TF *__restrict__ tab = reinterpret_cast<const TF *>(A.tables);
    const uint4 *__restrict__ Wv = reinterpret_cast<const uint4 *>(A.m.W);
    const int KB = A.m.kb_point;

    f16_t acc[MB][2];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[m][nb][e] = 0.0f;

    for (int h = 0; h < wmax; ++h) {
        float p[3] = {0.0f, 0.0f, 0.0f};
        int face = 0;
        const bool has = h < count;
        if (has) face = boundary_point(w, s_list[(h >> 1) * kBlock + tid], h & 1, p);
        for (int kb = 0; kb < KB; ++kb) {
            float e[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) e[q] = 0.0f;
            if (has) {
#pragma unroll
                for (int lv = 0; lv < LPB; ++lv) {
                    const int l = kb * LPB + lv;
                    if (l < g.L) {
                        float v[F];
                        encode_level<TF, F>(g, tab, l, p, face, v);
#pragma unroll
                        for (int f = 0; f < F; ++f) e[lv * FP + f] = v[f];
                    }
                }
            }
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lo[q] = pack2<TM>(e[2 * q], e[2 * q + 1]);
                hi[q] = pack2<TM>(e[8 + 2 * q], e[8 + 2 * q + 1]);
            }
            if (A.dbg.enc && live && has) {
                const int LFp = g.L * FP;
                for (int q = 0; q < 16; ++q) {
                    const int k = kb * 16 + q;
                    if (k < LFp) {
                        uint32_t word = q < 8 ? lo[q >> 1] : hi[(q - 8) >> 1];
                        A.dbg.enc[(size_t)r * g.H * LFp + h * LFp + k] =
                            (q & 1) ? unpack_hi<TM>(word) : unpack_lo<TM>(word);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) swap32(lo[q], hi[q]);
            const vec_t b0 = as_vec<vec_t>(lo), b1 = as_vec<vec_t>(hi);
            const uint4 *Wk = Wv + A.m.off[0] / 8 + (size_t)((h * KB + kb) * MB) * 64 + lane;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const uint4 wa = Wk[m * 64];
                const uint32_t wd[4] = {wa.x, wa.y, wa.z, wa.w};
                const vec_t a = as_vec<vec_t>(wd);
                acc[m][0] = MmaT<TM>::mma(a, b0, acc[m][0]);
                acc[m][1] = MmaT<TM>::mma(a, b1, acc[m][1]);
            }
        }
    }

    // hidden layers 2..n_hidden, then the head
    float o[kMaxOut];
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k) o[k] = 0.0f;
    if (wmax > 0) {
        for (int k = 1; k <= A.m.n_hidden; ++k) {
            const bool head = k == A.m.n_hidden;
            // activations -> B operands: 16-block s of output block m
            uint32_t xb[MB][2][2][4];
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int s = 0; s < 2; ++s)
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int r0 = 8 * s + 2 * q;
                            xb[m][nb][s][q] = pack2<TM>(act_f(acc[m][nb][r0], A.m.act, A.m.slope),
                                                        act_f(acc[m][nb][r0 + 1], A.m.act, A.m.slope));
                            xb[m][nb][s][2 + q] = pack2<TM>(act_f(acc[m][nb][r0 + 4], A.m.act, A.m.slope),
                                                            act_f(acc[m][nb][r0 + 5], A.m.act, A.m.slope));
                        }
            const int MO = head ? 1 : MB;
            const uint4 *Wk = Wv + A.m.off[k] / 8 + lane;
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
                            const uint4 wa = Wk[(size_t)((mo * MB + m) * 2 + s) * 64];
                            const uint32_t wd[4] = {wa.x, wa.y, wa.z, wa.w};
                            const vec_t a = as_vec<vec_t>(wd);
                            acc[mo][0] = MmaT<TM>::mma(a, as_vec<vec_t>(xb[m][0][s]), acc[mo][0]);
                            acc[mo][1] = MmaT<TM>::mma(a, as_vec<vec_t>(xb[m][1][s]), acc[mo][1]);
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
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                o[8 * q + rr] = __uint_as_float(x[4 * q + rr]);
                o[8 * q + 4 + rr] = __uint_as_float(y[4 * q + rr]);
            }
    }
    if (!live) return;
    if (A.dbg.count) A.dbg.count[r] = w.valid ? count : -1;
    if (A.dbg.tatb) {
        A.dbg.tatb[2 * r] = w.ta;
        A.dbg.tatb[2 * r + 1] = w.tb;
    }
    if (A.dbg.out)
        for (int k = 0; k < A.m.out_dim; ++k) A.dbg.out[(size_t)r * A.m.out_dim + k] = count > 0 ? o[k] : 0.0f;
    decode_store(A, r, w, count, o);
}

// ------------------------------------------------------------------ debug path
struct DebugArgs {
    Geom g;
    const float4 *rays;
    uint32_t n;
    lsnif_debug_bufs b;
};

}  // namespace lsnif
