// Host runtime of the LSNIF query library: contexts, the HBM-resident object
// registry, descriptor validation, precision conversion and weight packing,
// and the query entry points of lsnif.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lsnif_internal.hpp"

using namespace lsnif;

namespace lsnif {

thread_local std::string g_err;

lsnif_status fail(lsnif_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace lsnif

namespace {

size_t dtype_size(int t) { return t == LSNIF_FP32 ? 4 : (t == LSNIF_FP8_E4M3 ? 1 : 2); }

uint16_t f32_to_f16(float x)
{
    _Float16 h = (_Float16)x;   // round to nearest even
    uint16_t u;
    memcpy(&u, &h, 2);
    return u;
}

uint16_t f32_to_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                             // round to nearest even
    return (uint16_t)(u >> 16);
}

// OCP FP8 E4M3 (bias 7, no infinities, largest finite 448), round to nearest
// even, saturating at +-448.
uint8_t f32_to_e4m3(float x)
{
    if (x != x) return 0x7f;
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    double a = std::fabs((double)x);
    if (a >= 448.0) return sign | 0x7e;
    if (a < std::ldexp(1.0, -6)) {                       // subnormal: multiples of 2^-9
        const double q = std::nearbyint(a * 512.0);      // ties to even (default rounding mode)
        return sign | (uint8_t)q;                        // q == 8 is the smallest normal, 0x08
    }
    int e;
    const double m = std::frexp(a, &e);                  // a = m 2^e, m in [0.5, 1)
    double q = std::nearbyint((m * 2.0 - 1.0) * 8.0);    // 3 mantissa bits
    int E = e - 1;
    if (q == 8.0) { q = 0.0; ++E; }
    if (E > 8 || (E == 8 && q > 6.0)) return sign | 0x7e;
    return sign | (uint8_t)(((E + 7) << 3) | (int)q);
}

void store_elem(void *dst, size_t i, float v, int dtype)
{
    if (dtype == LSNIF_FP32) static_cast<float *>(dst)[i] = v;
    else if (dtype == LSNIF_FP16) static_cast<uint16_t *>(dst)[i] = f32_to_f16(v);
    else if (dtype == LSNIF_BF16) static_cast<uint16_t *>(dst)[i] = f32_to_bf16(v);
    else static_cast<uint8_t *>(dst)[i] = f32_to_e4m3(v);
}

int out_dim_of(const lsnif_object_desc *d) { return 5 + 3 * (d->has_albedo ? 1 : 0) + d->n_mat; }

lsnif_status validate(const lsnif_object_desc *d)
{
    if (!d) return fail(LSNIF_E_INVALID, "descriptor is NULL");
    if (d->V < 1 || d->V > 1024 || (d->V & (d->V - 1)))
        return fail(LSNIF_E_INVALID, "V = %d must be a power of two in [1, 1024]", d->V);
    for (int a = 0; a < 3; ++a)
        if (!(d->aabb_max[a] > d->aabb_min[a]) || !std::isfinite(d->aabb_min[a]) || !std::isfinite(d->aabb_max[a]))
            return fail(LSNIF_E_INVALID, "empty or non-finite AABB on axis %d", a);
    if (!d->occupancy) return fail(LSNIF_E_INVALID, "occupancy is NULL");
    if (d->L < 1 || d->L > kMaxLevels) return fail(LSNIF_E_INVALID, "L = %d not in [1, %d]", d->L, kMaxLevels);
    if (d->F < 1 || d->F > 4) return fail(LSNIF_E_INVALID, "F = %d not in [1, 4]", d->F);
    if (d->log2_T < 1 || d->log2_T > 30) return fail(LSNIF_E_INVALID, "log2_T = %d not in [1, 30]", d->log2_T);
    if (!d->R || !d->tables) return fail(LSNIF_E_INVALID, "R or tables is NULL");
    for (int l = 0; l < d->L; ++l)
        if (d->R[l] < 1 || d->R[l] > (1 << 20)) return fail(LSNIF_E_INVALID, "R[%d] = %d out of range", l, d->R[l]);
    if (d->H < 2 || d->H > 2 * kMaxList || (d->H & 1))
        return fail(LSNIF_E_INVALID, "H = %d must be even in [2, %d]", d->H, 2 * kMaxList);
    if (d->n_hidden < 1 || d->n_hidden > 6) return fail(LSNIF_E_INVALID, "n_hidden = %d not in [1, 6]", d->n_hidden);
    if (d->width < 1) return fail(LSNIF_E_INVALID, "width = %d", d->width);
    if (d->act != LSNIF_RELU && d->act != LSNIF_LEAKY_RELU) return fail(LSNIF_E_INVALID, "unknown activation %d", d->act);
    if (d->n_mat < 1) return fail(LSNIF_E_INVALID, "n_mat = %d", d->n_mat);
    if (out_dim_of(d) > kMaxOut) return fail(LSNIF_E_INVALID, "%d outputs exceed %d", out_dim_of(d), kMaxOut);
    if (!d->W) return fail(LSNIF_E_INVALID, "W is NULL");
    for (int k = 0; k <= d->n_hidden; ++k)
        if (!d->W[k]) return fail(LSNIF_E_INVALID, "W[%d] is NULL", k);
    if (d->feat_dtype < LSNIF_FP32 || d->feat_dtype > LSNIF_BF16)
        return fail(LSNIF_E_INVALID, "feat_dtype %d unsupported", d->feat_dtype);
    if (d->mlp_dtype < LSNIF_FP32 || d->mlp_dtype > LSNIF_FP8_E4M3)
        return fail(LSNIF_E_INVALID, "mlp_dtype %d unknown", d->mlp_dtype);
    return LSNIF_OK;
}

// Kernel support beyond what the ABI allows in general.
lsnif_status supported(const lsnif_object_desc *d)
{
    if (d->F != 2 && d->F != 3) return fail(LSNIF_E_INVALID, "kernels support F = 2 or 3 (got %d)", d->F);
    if (d->width != 64 && d->width != 128)
        return fail(LSNIF_E_INVALID, "kernels support width 64 or 128 (got %d)", d->width);
    if (d->width == 128 && d->mlp_dtype != LSNIF_FP32) {
        // the matrix-core kernels of width 128 hold at most 2 K blocks (32 inputs) per point
        const int fp = d->F == 3 ? 4 : d->F;
        if (d->L * fp > 32)
            return fail(LSNIF_E_INVALID, "width 128 on matrix cores needs L x %d <= 32 inputs per point (L = %d)",
                        fp, d->L);
    }
    // the gathers address a level with 32-bit byte offsets
    const uint64_t level_bytes = ((uint64_t)1 << d->log2_T) * d->F * dtype_size(d->feat_dtype);
    if (level_bytes > ((uint64_t)1 << 32))
        return fail(LSNIF_E_INVALID, "a level of 2^%d entries x %d features is %llu bytes; kernels address at most 4 GiB",
                    d->log2_T, d->F, (unsigned long long)level_bytes);
    if (d->mlp_dtype == LSNIF_FP8_E4M3) {
        if (!d->fp8_act_scale) return fail(LSNIF_E_INVALID, "an FP8 MLP needs fp8_act_scale");
        for (int k = 0; k <= d->n_hidden; ++k)
            if (!(d->fp8_act_scale[k] > 0.0f) || !std::isfinite(d->fp8_act_scale[k]))
                return fail(LSNIF_E_INVALID, "fp8_act_scale[%d] must be positive and finite", k);
    }
    return LSNIF_OK;
}

uint64_t algorithmic_bytes(const lsnif_object_desc *d)
{
    const uint64_t V = (uint64_t)d->V;
    const uint64_t vox = (V * V * V + 7) / 8;
    const uint64_t tab = (uint64_t)d->L * ((uint64_t)1 << d->log2_T) * d->F * dtype_size(d->feat_dtype);
    const uint64_t in = (uint64_t)d->H * d->L * d->F;
    const uint64_t w = in * d->width + (uint64_t)(d->n_hidden - 1) * d->width * d->width +
                       (uint64_t)d->width * out_dim_of(d);
    return vox + tab + w * dtype_size(d->mlp_dtype);
}

// float32 path: each layer transposed to [in][out_pad].
std::vector<float> pack_f32(const lsnif_object_desc *d, int32_t off[8])
{
    const int Wd = d->width, in0 = d->H * d->L * d->F, od = out_dim_of(d);
    std::vector<float> w;
    off[0] = 0;
    w.resize((size_t)in0 * Wd);
    for (int j = 0; j < Wd; ++j)
        for (int i = 0; i < in0; ++i) w[(size_t)i * Wd + j] = d->W[0][(size_t)j * in0 + i];
    for (int k = 1; k < d->n_hidden; ++k) {
        off[k] = (int32_t)w.size();
        w.resize(w.size() + (size_t)Wd * Wd);
        float *dst = w.data() + off[k];
        for (int j = 0; j < Wd; ++j)
            for (int i = 0; i < Wd; ++i) dst[(size_t)i * Wd + j] = d->W[k][(size_t)j * Wd + i];
    }
    off[d->n_hidden] = (int32_t)w.size();
    w.resize(w.size() + (size_t)Wd * kMaxOut, 0.0f);
    float *dst = w.data() + off[d->n_hidden];
    for (int j = 0; j < od; ++j)
        for (int i = 0; i < Wd; ++i) dst[(size_t)i * kMaxOut + j] = d->W[d->n_hidden][(size_t)j * Wd + i];
    return w;
}

// Matrix-core path: A-operand fragments of v_mfma_f32_32x32x16 (8 values per
// lane, lane l holding row l % 32 and K slots 8 (l / 32) .. +7).
//  layer 1: fragment ((h * KB + kb) * MB + m) for point h, 16-wide K block kb
//           of the point's features padded to FP per level, output block m;
//  later layers: fragment ((mo * MB + m) * 2 + s), K slot 8q + e standing for
//           input unit 32m + 16s + (e < 4 ? 4q + e : 8 + 4q + e - 4) -- the
//           order in which the previous layer's accumulators lie.
std::vector<float> pack_mma(const lsnif_object_desc *d, int32_t off[8], int &KB)
{
    const int Wd = d->width, MB = Wd / 32, L = d->L, F = d->F, H = d->H, od = out_dim_of(d);
    const int FP = F == 3 ? 4 : F;
    const int in0 = H * L * F;
    KB = (L * FP + 15) / 16;
    std::vector<float> w;
    off[0] = 0;
    w.assign((size_t)H * KB * MB * 64 * 8, 0.0f);
    for (int h = 0; h < H; ++h)
        for (int kb = 0; kb < KB; ++kb)
            for (int m = 0; m < MB; ++m)
                for (int lane = 0; lane < 64; ++lane)
                    for (int e = 0; e < 8; ++e) {
                        const int k = 16 * kb + 8 * (lane / 32) + e;
                        const int lvl = k / FP, f = k % FP, out = 32 * m + lane % 32;
                        if (lvl >= L || f >= F) continue;
                        const int in = h * L * F + lvl * F + f;
                        w[((((size_t)h * KB + kb) * MB + m) * 64 + lane) * 8 + e] = d->W[0][(size_t)out * in0 + in];
                    }
    for (int k = 1; k <= d->n_hidden; ++k) {
        const bool head = k == d->n_hidden;
        const int MO = head ? 1 : MB, rows = head ? od : Wd;
        off[k] = (int32_t)w.size();
        w.resize(w.size() + (size_t)MO * MB * 2 * 64 * 8, 0.0f);
        float *dst = w.data() + off[k];
        for (int mo = 0; mo < MO; ++mo)
            for (int m = 0; m < MB; ++m)
                for (int s = 0; s < 2; ++s)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int e = 0; e < 8; ++e) {
                            const int q = lane / 32, out = 32 * mo + lane % 32;
                            const int in = 32 * m + 16 * s + (e < 4 ? 4 * q + e : 8 + 4 * q + (e - 4));
                            if (out >= rows) continue;
                            dst[((((size_t)mo * MB + m) * 2 + s) * 64 + lane) * 8 + e] = d->W[k][(size_t)out * Wd + in];
                        }
    }
    return w;
}

}  // namespace

extern "C" {

int32_t lsnif_version(void) { return 100; }

const char *lsnif_last_error(void) { return g_err.c_str(); }

lsnif_status lsnif_create(const lsnif_ctx_desc *desc, lsnif_ctx **out)
{
    if (!out) return fail(LSNIF_E_INVALID, "out is NULL");
    *out = nullptr;
    const int dev = desc ? desc->device : 0;
    if (dev != -1) {
        int n = 0;
        HIP_TRY(hipGetDeviceCount(&n));
        if (dev < 0 || dev >= n) return fail(LSNIF_E_INVALID, "device %d not in [0, %d)", dev, n);
    }
    if (dev >= 0) {
        const lsnif_status st = noalloc_init(dev);
        if (st) return st;
    }
    lsnif_ctx *c = new (std::nothrow) lsnif_ctx();
    if (!c) return fail(LSNIF_E_NOMEM, "host allocation failed");
    c->device = dev;
    c->budget = desc ? desc->hbm_budget : 0;
    c->arch = device_arch(dev);
    if (desc && desc->autotune_cache && desc->autotune_cache[0]) {
        c->cache_path = desc->autotune_cache;
        if (const lsnif_status st = cache_load(c)) {
            delete c;
            return st;
        }
    }
    *out = c;
    return LSNIF_OK;
}

void lsnif_destroy(lsnif_ctx *ctx)
{
    if (!ctx) return;
    destroy_server(ctx);
    if (ctx->device < 0) {
        delete ctx;
        return;
    }
    DeviceGuard g(ctx->device);
    for (auto &kv : ctx->objects) {
        (void)hipFree(kv.second.d_occ);
        (void)hipFree(kv.second.d_tab);
        (void)hipFree(kv.second.d_w);
    }
    (void)hipFree(ctx->ws);
    (void)hipFree(ctx->d_table);
    (void)hipFree(ctx->pws);
    (void)hipFree(ctx->bws);
    (void)hipFree(ctx->sws);
    for (auto &v : ctx->pending)
        for (hipEvent_t e : v)
            if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->order_events) (void)hipEventDestroy(e);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

lsnif_status lsnif_desc_bytes(const lsnif_object_desc *desc, uint64_t *bytes)
{
    if (!bytes) return fail(LSNIF_E_INVALID, "bytes is NULL");
    lsnif_status st = validate(desc);
    if (st) return st;
    *bytes = algorithmic_bytes(desc);
    return LSNIF_OK;
}

lsnif_status lsnif_build(lsnif_ctx *ctx, const lsnif_object_desc *d, uint32_t *object_id)
{
    if (!ctx || !object_id) return fail(LSNIF_E_INVALID, "ctx or object_id is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    lsnif_status st = validate(d);
    if (st) return st;
    if ((st = supported(d))) return st;
    DeviceGuard guard(ctx->device);
    Object ob;
    ob.feat_dtype = d->feat_dtype;
    ob.mlp_dtype = d->mlp_dtype;
    ob.F = d->F;
    ob.width = d->width;
    Geom &g = ob.geom;
    for (int a = 0; a < 3; ++a) {
        g.bmin[a] = d->aabb_min[a];
        g.s[a] = (float)d->V / (d->aabb_max[a] - d->aabb_min[a]);
    }
    g.V = d->V;
    g.L = d->L;
    g.F = d->F;
    g.log2_T = d->log2_T;
    g.H = d->H;
    g.recheck = d->grazing_recheck ? 1u : 0u;
    g.sort_bits = 5;
    g.pair_bits = d->V >= 64 ? 4 : 3;
    const uint64_t T = (uint64_t)1 << d->log2_T;
    for (int l = 0; l < d->L; ++l) {
        g.R[l] = d->R[l];
        g.lsc[l] = (float)d->R[l] / (float)d->V;
        const uint64_t side = (uint64_t)d->R[l] + 1;
        if (side * side * side <= T) {
            g.dense_mask |= 1u << l;
            g.my[l] = (uint32_t)side;
            g.mz[l] = (uint32_t)(side * side);
            g.dmask[l] = 0xffffffffu;
            g.hmask[l] = 0u;
        } else {
            g.my[l] = kPrimeY;
            g.mz[l] = kPrimeZ;
            g.dmask[l] = 0u;
            g.hmask[l] = (uint32_t)(T - 1);
        }
        if (d->R[l] % d->V == 0) g.aligned_mask |= 1u << l;
    }
    ob.esz = (uint32_t)(d->F * dtype_size(d->feat_dtype));
    ob.hot_budget = 0;   // hot levels are off until a tuning asks for them
    plan_hot_levels(g, ob.esz, ob.hot_budget);
    // an autotune cache entry for this architecture, shape and precision replaces the defaults
    auto cached = ctx->cache.find(cache_key(ctx, ob));
    if (cached != ctx->cache.end()) {
        g.sort_bits = (uint32_t)cached->second.sort_bits;
        g.pair_bits = (uint32_t)cached->second.pair_bits;
        ob.hot_budget = (uint32_t)cached->second.hot_lds_bytes;
        ob.walk_chunks = (uint32_t)cached->second.walk_chunks;
        ob.persistent = (uint32_t)cached->second.persistent;
        plan_hot_levels(g, ob.esz, ob.hot_budget);
    }
    // occupancy as 4x4x4 bricks: one 64-bit mask per brick, then one bit per brick
    const int V = d->V, NB = (V + 3) / 4;
    const size_t nbricks = (size_t)NB * NB * NB;
    const size_t coarse_words = (nbricks + 31) / 32;
    std::vector<uint64_t> occ_dev(nbricks + (coarse_words + 1) / 2, 0ull);
    uint32_t *coarse = reinterpret_cast<uint32_t *>(occ_dev.data() + nbricks);
    for (int z = 0; z < V; ++z)
        for (int y = 0; y < V; ++y)
            for (int x = 0; x < V; ++x) {
                const uint64_t bit = (uint64_t)x + (uint64_t)V * ((uint64_t)y + (uint64_t)V * (uint64_t)z);
                if (!((d->occupancy[bit >> 5] >> (bit & 31)) & 1u)) continue;
                const size_t b = (size_t)(x >> 2) + (size_t)NB * ((size_t)(y >> 2) + (size_t)NB * (size_t)(z >> 2));
                occ_dev[b] |= 1ull << ((x & 3) + 4 * (y & 3) + 16 * (z & 3));
                coarse[b >> 5] |= 1u << (b & 31);
            }
    g.NB = NB;
    g.coarse_words = (int32_t)coarse_words;
    const size_t occ_bytes = occ_dev.size() * sizeof(uint64_t);
    // host-side conversions
    const size_t n_tab = (size_t)d->L * T * d->F;
    std::vector<uint8_t> tab(n_tab * dtype_size(d->feat_dtype));
    for (size_t i = 0; i < n_tab; ++i) store_elem(tab.data(), i, d->tables[i], d->feat_dtype);
    std::vector<float> wf;
    int KB = 0;
    if (d->mlp_dtype == LSNIF_FP32) wf = pack_f32(d, ob.mlp.off);
    else wf = pack_mma(d, ob.mlp.off, KB);
    const int wdt = d->mlp_dtype == LSNIF_FP32 ? LSNIF_FP32 : d->mlp_dtype;
    for (int k = 0; k < 8; ++k) {
        ob.mlp.qs[k] = 1.0f;
        ob.mlp.dq[k] = 1.0f;
    }
    if (wdt == LSNIF_FP8_E4M3) {
        // per-layer weight scale amax|W| / 448; the stored values are W / scale
        for (int k = 0; k <= d->n_hidden; ++k) {
            const size_t b = (size_t)ob.mlp.off[k], e = k < d->n_hidden ? (size_t)ob.mlp.off[k + 1] : wf.size();
            float amax = 0.0f;
            for (size_t i = b; i < e; ++i) amax = std::max(amax, std::fabs(wf[i]));
            const float sw = amax > 0.0f ? amax / 448.0f : 1.0f;
            for (size_t i = b; i < e; ++i) wf[i] /= sw;
            ob.mlp.qs[k] = 1.0f / d->fp8_act_scale[k];
            ob.mlp.dq[k] = sw * d->fp8_act_scale[k];
        }
    }
    std::vector<uint8_t> wbytes(wf.size() * dtype_size(wdt));
    for (size_t i = 0; i < wf.size(); ++i) store_elem(wbytes.data(), i, wf[i], wdt);
    if (wdt != LSNIF_FP32)
        for (int k = 0; k <= d->n_hidden; ++k) ob.mlp.woff[k] = (int32_t)((size_t)ob.mlp.off[k] * dtype_size(wdt) / 4);
    ob.bytes = occ_bytes + tab.size() + wbytes.size();
    if (ctx->budget && ctx->used + ob.bytes > ctx->budget)
        return fail(LSNIF_E_NOMEM, "object needs %llu bytes, %llu of %llu in use", (unsigned long long)ob.bytes,
                    (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
    auto cleanup = [&]() {
        (void)hipFree(ob.d_occ);
        (void)hipFree(ob.d_tab);
        (void)hipFree(ob.d_w);
    };
    tab.resize(tab.size() + kTablePad, 0);   // not counted in the footprint
    if (hipMalloc(&ob.d_occ, occ_bytes) != hipSuccess || hipMalloc(&ob.d_tab, tab.size()) != hipSuccess ||
        hipMalloc(&ob.d_w, wbytes.size()) != hipSuccess) {
        cleanup();
        return fail(LSNIF_E_NOMEM, "device allocation of %llu bytes failed", (unsigned long long)ob.bytes);
    }
    if (hipMemcpy(ob.d_occ, occ_dev.data(), occ_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ob.d_tab, tab.data(), tab.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ob.d_w, wbytes.data(), wbytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return fail(LSNIF_E_DEVICE, "copy to device failed");
    }
    g.fine = static_cast<const uint64_t *>(ob.d_occ);
    g.coarse = reinterpret_cast<const uint32_t *>(g.fine + nbricks);
    Mlp &m = ob.mlp;
    m.W = ob.d_w;
    m.n_hidden = d->n_hidden;
    m.out_dim = out_dim_of(d);
    m.act = d->act;
    m.slope = d->leaky_slope;
    m.n_mat = d->n_mat;
    m.has_albedo = d->has_albedo ? 1 : 0;
    m.kb_point = KB;
    m.fp = d->F == 3 ? 4 : d->F;
    const uint32_t id = ctx->next_id++;
    ctx->objects[id] = ob;
    ctx->used += ob.bytes;
    ctx->table_dirty = true;
    ++ctx->generation;
    *object_id = id;
    return LSNIF_OK;
}

lsnif_status lsnif_release(lsnif_ctx *ctx, uint32_t object_id)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();   // queries in flight may still read the object
    (void)hipFree(it->second.d_occ);
    (void)hipFree(it->second.d_tab);
    (void)hipFree(it->second.d_w);
    ctx->used -= it->second.bytes;
    ctx->objects.erase(it);
    ctx->table_dirty = true;
    ++ctx->generation;
    return LSNIF_OK;
}

lsnif_status lsnif_object_bytes(lsnif_ctx *ctx, uint32_t object_id, uint64_t *bytes)
{
    if (!ctx || !bytes) return fail(LSNIF_E_INVALID, "ctx or bytes is NULL");
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    *bytes = it->second.bytes;
    return LSNIF_OK;
}

lsnif_status lsnif_profile_enable(lsnif_ctx *ctx, int32_t on)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->profiling = on != 0;
    return LSNIF_OK;
}

lsnif_status lsnif_profile_read(lsnif_ctx *ctx, double *sort_ms, double *walk_ms, double *kernel_ms,
                                uint64_t *launches)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    double so = 0.0, wk = 0.0, kq = 0.0;
    const uint64_t k = ctx->pending.size();
    lsnif_status st = LSNIF_OK;
    for (auto &v : ctx->pending) {
        float a = 0.0f, b = 0.0f, c = 0.0f;
        if (st == LSNIF_OK &&
            (hipEventSynchronize(v[3]) != hipSuccess || hipEventElapsedTime(&a, v[0], v[1]) != hipSuccess ||
             hipEventElapsedTime(&b, v[1], v[2]) != hipSuccess || hipEventElapsedTime(&c, v[2], v[3]) != hipSuccess))
            st = fail(LSNIF_E_DEVICE, "reading query events failed");
        so += a;
        wk += b;
        kq += c;
        for (hipEvent_t e : v) ctx->spare.push_back(e);
    }
    ctx->pending.clear();
    if (sort_ms) *sort_ms = so;
    if (walk_ms) *walk_ms = wk;
    if (kernel_ms) *kernel_ms = kq;
    if (launches) *launches = k;
    return st;
}



static lsnif_status run_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                              lsnif_hit *d_out, const lsnif_debug_bufs *dbg, void *stream)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    const Object *ob = nullptr;
    lsnif_status st = check_query(ctx, object_id, d_rays, n, d_out, ob);
    if (st || n == 0) return st;
    DeviceGuard guard(ctx->device);
    if ((st = grow_workspace(ctx->ws, ctx->ws_bytes, query_ws_bytes(n, ob->geom.sort_bits, ob->geom.H >> 1)))) return st;
    return enqueue_query(ctx, *ob, d_rays, n, d_out, dbg, static_cast<hipStream_t>(stream), ctx->ws);
}

lsnif_status lsnif_query_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays, const uint32_t *d_pair_ray,
                               const uint32_t *d_pair_inst, uint32_t n_pairs, const lsnif_instance *d_inst,
                               uint32_t n_inst, lsnif_hit *d_out, void *stream)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (n_rays == 0) return LSNIF_OK;
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    DeviceGuard guard(ctx->device);
    PairsSetup ps;
    lsnif_status st = pairs_setup(ctx, ps);
    if (st) return st;
    if ((st = grow_workspace(ctx->pws, ctx->pws_bytes, pairs_ws_bytes(n_rays, n_pairs, ps.n_objs, ps.maxH >> 1, ps.pair_bits))))
        return st;
    return enqueue_pairs(ctx, ps, d_rays, n_rays, d_pair_ray, d_pair_inst, n_pairs, d_inst, n_inst, d_out,
                         static_cast<hipStream_t>(stream), ctx->pws);
}

lsnif_status lsnif_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                         lsnif_hit *d_out, void *stream)
{
    return run_query(ctx, object_id, d_rays, n, d_out, nullptr, stream);
}

lsnif_status lsnif_query_debug(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                               lsnif_hit *d_out, const lsnif_debug_bufs *dbg, void *stream)
{
    if (!dbg) return fail(LSNIF_E_INVALID, "dbg is NULL");
    return run_query(ctx, object_id, d_rays, n, d_out, dbg, stream);
}

lsnif_status lsnif_gather_ceiling(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                                  float *d_sums, void *stream)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    const Object *ob = nullptr;
    lsnif_status st = check_query(ctx, object_id, d_rays, n, reinterpret_cast<lsnif_hit *>(d_sums), ob);
    if (st || n == 0) return st;
    DeviceGuard guard(ctx->device);
    if ((st = grow_workspace(ctx->ws, ctx->ws_bytes, query_ws_bytes(n, ob->geom.sort_bits, ob->geom.H >> 1)))) return st;
    return enqueue_query(ctx, *ob, d_rays, n, nullptr, nullptr, static_cast<hipStream_t>(stream), ctx->ws, 1, d_sums);
}

}  // extern "C"

// ------------------------------------------------------------------ enqueue
namespace lsnif {

lsnif_status grow_workspace(void *&buf, size_t &have, size_t need)
{
    if (need <= have) return LSNIF_OK;
    (void)hipFree(buf);   // waits for work that may still use the old buffer
    buf = nullptr;
    have = 0;
    if (hipMalloc(&buf, need) != hipSuccess)
        return fail(LSNIF_E_NOMEM, "workspace of %llu bytes", (unsigned long long)need);
    have = need;
    return LSNIF_OK;
}

// Hot levels: the coarsest levels, in order, while all their used slots (plus
// the spare entry a paired gather may read) fit `budget` bytes of LDS and two
// blocks still fit a CU (static LDS + voxel lists + hot levels within half of
// its 160 KiB); 4- and 8-byte entries only.
void plan_hot_levels(Geom &g, uint32_t esz, uint32_t budget)
{
    g.hot_mask = 0;
    g.hot_bytes = 0;
    for (int l = 0; l < kMaxLevels; ++l) g.hot_off[l] = g.hot_len[l] = 0;
    if (esz != 4 && esz != 8) return;
    const int64_t lds_left = (int64_t)(80 << 10) - (int64_t)sizeof(Shared) - (int64_t)(g.H / 2) * kBlock * 4;
    const uint32_t cap = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(std::min(budget, kHotLdsBudget), lds_left));
    const uint64_t T = (uint64_t)1 << g.log2_T;
    uint32_t off = 0;
    for (int l = 0; l < g.L; ++l) {
        const uint64_t side = (uint64_t)g.R[l] + 1;
        const uint64_t used = (g.dense_mask >> l) & 1u ? side * side * side : T;
        const uint64_t len = ((used + 1) * esz + 15) / 16 * 16;
        if (off + len > cap) break;
        g.hot_mask |= 1u << l;
        g.hot_off[l] = off;
        g.hot_len[l] = (uint32_t)len;
        off += (uint32_t)len;
    }
    g.hot_bytes = off;
}

lsnif_status check_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                         lsnif_hit *d_out, const Object *&ob)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    ob = &it->second;
    if (n == 0) return LSNIF_OK;
    if (!d_rays || !d_out) return fail(LSNIF_E_INVALID, "rays or output is NULL");
    if (reinterpret_cast<uintptr_t>(d_rays) % 16 || reinterpret_cast<uintptr_t>(d_out) % 4)
        return fail(LSNIF_E_INVALID, "rays must be 16-byte and hits 4-byte aligned");
    return LSNIF_OK;
}

static hipEvent_t take_event(lsnif_ctx *ctx)
{
    if (!ctx->spare.empty()) {
        hipEvent_t e = ctx->spare.back();
        ctx->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Coherence-sort arrays (keys and ray indices twice, digit counters, scan partials), when
// the batch is sorted.
static size_t sort_ws_bytes(uint32_t n, uint32_t sort_bits)
{
    if (n < kSortMin || sort_bits == 0) return 0;
    return al256(radix_ws_words(n) * sizeof(uint32_t));
}

// Voxel counts (one byte) and voxel lists (cap entries) of n_slots slots.
static size_t list_ws_bytes(size_t n_slots, uint32_t cap)
{
    return al256(n_slots) + al256(n_slots * cap * sizeof(uint32_t));
}

// The persistent query kernel's 8 tile-queue counters: one 256-byte granule after the lists.
constexpr size_t kQueueBytes = 256;

size_t query_ws_bytes(uint32_t n, uint32_t sort_bits, uint32_t cap)
{
    return sort_ws_bytes(n, sort_bits) + list_ws_bytes(n, cap) + kQueueBytes;
}

size_t pairs_ws_bytes(uint32_t n_rays, uint32_t n_pairs, uint32_t n_objs, uint32_t cap, uint32_t pair_bits)
{
    (void)pair_bits;   // the radix passes' workspace does not depend on the grouping
    const size_t n_slots = (size_t)(n_pairs + kBlock - 1) / kBlock * kBlock + (size_t)kBlock * n_objs;
    return al256((size_t)n_rays * 8) + al256((size_t)n_pairs * sizeof(PairRes)) + al256((size_t)n_pairs * 4) +
           al256(n_slots * 4) + al256(n_slots / kBlock * 4) + 4 * al256((size_t)n_pairs * 4) +
           al256(radix_hist_words(n_pairs) * 4) + al256((size_t)(n_objs + 1) * 4) + al256((size_t)n_objs * 4) +
           list_ws_bytes(n_slots, cap) + kQueueBytes;
}

// The walk kernel, then the query kernel, over `ntiles` tiles.  With k > 1 tile
// ranges the walk of every range runs on the context's side stream, in order,
// and the query kernel of range i waits only for the walk of range i, so the
// walk of the later ranges (vector-ALU bound) shares the GPU with the query
// kernel (gather bound).  `ev_mid`, when timing, is recorded once the query
// kernel may start.
template <typename Query>
static lsnif_status walk_then_query(lsnif_ctx *ctx, QueryArgs A, bool pairs, bool recheck, uint32_t ntiles,
                                    uint32_t chunks, hipStream_t s, hipEvent_t ev_mid, Query &&query)
{
    const uint32_t k = std::max(1u, std::min(chunks, ntiles / kMinChunkTiles));
    if (k == 1) {
        A.tile0 = 0;
        HIP_TRY(launch_walk(A, pairs, recheck, ntiles, s));
        if (ev_mid) HIP_TRY(hipEventRecord(ev_mid, s));
        HIP_TRY(query(A, ntiles));
        return LSNIF_OK;
    }
    if (!ctx->side && hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess) {
        ctx->side = nullptr;
        return fail(LSNIF_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    while (ctx->order_events.size() < k + 1) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(LSNIF_E_DEVICE, "hipEventCreateWithFlags failed");
        ctx->order_events.push_back(e);
    }
    hipEvent_t *ev = ctx->order_events.data();
    auto first = [&](uint32_t i) { return (uint32_t)((uint64_t)ntiles * i / k); };
    HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(hipStreamWaitEvent(ctx->side, ev[0], 0));
    for (uint32_t i = 0; i < k; ++i) {
        A.tile0 = first(i);
        HIP_TRY(launch_walk(A, pairs, recheck, first(i + 1) - first(i), ctx->side));
        HIP_TRY(hipEventRecord(ev[i + 1], ctx->side));
    }
    for (uint32_t i = 0; i < k; ++i) {
        HIP_TRY(hipStreamWaitEvent(s, ev[i + 1], 0));
        if (i == 0 && ev_mid) HIP_TRY(hipEventRecord(ev_mid, s));
        A.tile0 = first(i);
        HIP_TRY(query(A, first(i + 1) - first(i)));
    }
    return LSNIF_OK;
}

lsnif_status enqueue_query(lsnif_ctx *ctx, const Object &ob, const lsnif_ray *d_rays, uint32_t n, lsnif_hit *d_out,
                           const lsnif_debug_bufs *dbg, hipStream_t s, void *ws, int chunks, float *gather_sums,
                           bool timed)
{
    QueryArgs A{};
    A.g = ob.geom;
    A.hot_lds = ob.geom.hot_bytes;
    A.width = (uint32_t)ob.width;
    A.m = ob.mlp;
    A.tables = ob.d_tab;
    A.rays = reinterpret_cast<const float4 *>(d_rays);
    A.hits = d_out;
    A.n = n;
    if (dbg) {
        if (dbg->act_amax && ob.mlp_dtype != LSNIF_FP32)
            return fail(LSNIF_E_INVALID, "act_amax is reported by objects with an FP32 MLP");
        DebugArgs D{};
        D.g = ob.geom;
        D.rays = A.rays;
        D.n = n;
        D.b = *dbg;
        D.b.count = nullptr;
        D.b.tatb = nullptr;
        D.b.enc = nullptr;
        D.b.out = nullptr;
        HIP_TRY(launch_debug(D, s));
        A.dbg.count = dbg->count;
        A.dbg.tatb = dbg->tatb;
        A.dbg.out = dbg->out;
        A.dbg.enc = dbg->enc;
        A.dbg.act_amax = dbg->act_amax;
    }
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (ctx->profiling && timed) {
        for (auto &e : ev)
            if (!(e = take_event(ctx))) return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    const size_t sort_bytes = sort_ws_bytes(n, ob.geom.sort_bits);
    if (sort_bytes) {
        uint32_t *order = nullptr;
        HIP_TRY(launch_coherence_sort(ob.geom, A.rays, n, static_cast<uint32_t *>(ws), &order, s));
        A.order = order;
    }
    if (ev[1]) HIP_TRY(hipEventRecord(ev[1], s));
    const uint32_t grid = (n + kBlock - 1) / kBlock;
    char *wl = static_cast<char *>(ws) + sort_bytes;
    A.nvox = reinterpret_cast<uint8_t *>(wl);
    A.lists = reinterpret_cast<uint32_t *>(wl + al256(n));
    A.queue = reinterpret_cast<unsigned long long *>(wl + list_ws_bytes(n, ob.geom.H >> 1));
    A.persistent = ob.persistent && !dbg && !gather_sums ? 1u : 0u;
    const int kbm = ob.mlp.kb_point;
    // Batches too small to fill the chip with one ray per lane run one wave per ray (width 64,
    // at most 16 levels; FP32 MLP with FP32 features and F <= 3, or a matrix-core MLP with
    // F = 2), whichever debug buffers are asked for: the answers are the same bits.
    const bool small = !gather_sums && n <= kSmallBatchRays && ob.width == 64 && ob.geom.L <= 16 &&
                       (ob.mlp_dtype == LSNIF_FP32 ? ob.feat_dtype == LSNIF_FP32 && ob.F <= 3
                                                   : ob.F == 2 && ob.mlp.kb_point <= 2);
    auto query = [&](const QueryArgs &a, uint32_t g) -> hipError_t {
        if (gather_sums) return launch_gather_only(a, ob.feat_dtype, ob.F, gather_sums, g, s);
        if (small) {
            if (ob.mlp_dtype == LSNIF_FP32) return launch_lat(a, ob.F, g, s);
            if (ob.mlp_dtype == LSNIF_FP16) return launch_mma_small_f16(a, ob.feat_dtype, kbm, g, s);
            if (ob.mlp_dtype == LSNIF_BF16) return launch_mma_small_bf16(a, ob.feat_dtype, kbm, g, s);
            return launch_mma_small_fp8(a, ob.feat_dtype, kbm, g, s);
        }
        if (ob.mlp_dtype == LSNIF_FP32) return launch_f32(a, ob.feat_dtype, ob.F, false, g, s);
        if (ob.mlp_dtype == LSNIF_FP16) return launch_mma_f16(a, ob.feat_dtype, ob.F, kbm, false, g, s);
        if (ob.mlp_dtype == LSNIF_BF16) return launch_mma_bf16(a, ob.feat_dtype, ob.F, kbm, false, g, s);
        return launch_mma_fp8(a, ob.feat_dtype, ob.F, kbm, false, g, s);
    };
    const uint32_t k = dbg ? 1u : (chunks > 0 ? (uint32_t)chunks : ob.walk_chunks);
    lsnif_status st = walk_then_query(ctx, A, false, ob.geom.recheck != 0, grid, k, s, ev[2], query);
    if (st) return st;
    if (ev[3]) {
        HIP_TRY(hipEventRecord(ev[3], s));
        ctx->pending.push_back({ev[0], ev[1], ev[2], ev[3]});
    }
    return LSNIF_OK;
}

lsnif_status upload_table(lsnif_ctx *ctx, uint32_t &n_objs)
{
    n_objs = ctx->objects.empty() ? 1u : ctx->objects.rbegin()->first + 1u;
    if (!ctx->table_dirty && ctx->d_table) return LSNIF_OK;
    std::vector<ObjDev> t(n_objs);
    memset(t.data(), 0, t.size() * sizeof(ObjDev));
    for (auto &kv : ctx->objects) {
        ObjDev &d = t[kv.first];
        d.g = kv.second.geom;
        d.m = kv.second.mlp;
        d.tables = kv.second.d_tab;
        d.live = 1;
        d.kb_point = kv.second.mlp.kb_point;
    }
    const size_t bytes = t.size() * sizeof(ObjDev);
    // earlier queries may still read the old table
    HIP_TRY(hipDeviceSynchronize());
    if (bytes > ctx->table_cap) {
        (void)hipFree(ctx->d_table);
        ctx->d_table = nullptr;
        ctx->table_cap = 0;
        if (hipMalloc(&ctx->d_table, bytes) != hipSuccess) return fail(LSNIF_E_NOMEM, "object table");
        ctx->table_cap = bytes;
    }
    HIP_TRY(hipMemcpy(ctx->d_table, t.data(), bytes, hipMemcpyHostToDevice));
    ctx->table_dirty = false;
    return LSNIF_OK;
}

lsnif_status pairs_setup(lsnif_ctx *ctx, PairsSetup &ps)
{
    if (ctx->objects.empty()) return fail(LSNIF_E_NOTFOUND, "no objects built");
    ps.first = &ctx->objects.begin()->second;
    ps.kbm = 1;
    ps.maxH = 2;
    ps.hot_max = 0;
    ps.recheck = false;
    ps.walk_chunks = 1;
    ps.pair_bits = 1;
    for (auto &kv : ctx->objects) {
        if (!same_class(kv.second, *ps.first))
            return fail(LSNIF_E_INVALID, "pair queries need every object of the context in one kernel class "
                                         "(feature type, MLP type, F, width)");
        ps.kbm = std::max(ps.kbm, kv.second.mlp.kb_point);
        ps.maxH = std::max(ps.maxH, kv.second.geom.H);
        ps.hot_max = std::max(ps.hot_max, kv.second.geom.hot_bytes);
        ps.recheck = ps.recheck || kv.second.geom.recheck;
        ps.walk_chunks = std::max(ps.walk_chunks, kv.second.walk_chunks);
        ps.pair_bits = std::max(ps.pair_bits, kv.second.geom.pair_bits);
        ps.persistent = std::max(ps.persistent, kv.second.persistent);
    }
    lsnif_status st = upload_table(ctx, ps.n_objs);
    if (st) return st;
    if ((uint64_t)ps.n_objs * pair_bins(ps.pair_bits) >= 0xffffffffull)   // 32-bit pair keys; n_objs bins: dropped
        return fail(LSNIF_E_INVALID, "object ids up to %u need pair_bits below %u", ps.n_objs - 1, ps.pair_bits);
    return LSNIF_OK;
}

lsnif_status enqueue_pairs(lsnif_ctx *ctx, const PairsSetup &ps, const lsnif_ray *d_rays, uint32_t n_rays,
                           const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                           const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out, hipStream_t s, void *ws,
                           int chunks)
{
    if (!d_rays || !d_out || (n_pairs && (!d_pair_ray || !d_pair_inst || !d_inst)))
        return fail(LSNIF_E_INVALID, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(d_rays) % 16 || reinterpret_cast<uintptr_t>(d_out) % 4)
        return fail(LSNIF_E_INVALID, "rays must be 16-byte and hits 4-byte aligned");
    const Object &first = *ps.first;
    const uint32_t n_objs = ps.n_objs;
    const uint32_t n_slots = (n_pairs + kBlock - 1) / kBlock * kBlock + kBlock * n_objs;
    const uint32_t n_tiles = n_slots / kBlock;
    char *w = static_cast<char *>(ws);
    PairPlan P{};
    P.rays = reinterpret_cast<const float4 *>(d_rays);
    P.n_rays = n_rays;
    P.pair_ray = d_pair_ray;
    P.pair_inst = d_pair_inst;
    P.n_pairs = n_pairs;
    P.inst = d_inst;
    P.n_inst = n_inst;
    P.objs = static_cast<const ObjDev *>(ctx->d_table);
    P.n_objs = n_objs;
    P.out = d_out;
    P.minkey = reinterpret_cast<unsigned long long *>(w);
    w += al256((size_t)n_rays * 8);
    P.res = reinterpret_cast<PairRes *>(w);
    w += al256((size_t)n_pairs * sizeof(PairRes));
    P.keys = reinterpret_cast<uint32_t *>(w);
    w += al256((size_t)n_pairs * 4);
    P.slot_pair = reinterpret_cast<uint32_t *>(w);
    w += al256((size_t)n_slots * 4);
    P.tile_obj = reinterpret_cast<int32_t *>(w);
    w += al256((size_t)n_tiles * 4);
    for (int q = 0; q < 2; ++q) {
        P.rk[q] = reinterpret_cast<uint32_t *>(w);
        w += al256((size_t)n_pairs * 4);
        P.rv[q] = reinterpret_cast<uint32_t *>(w);
        w += al256((size_t)n_pairs * 4);
    }
    P.hist = reinterpret_cast<uint32_t *>(w);
    w += al256(radix_hist_words(n_pairs) * 4);
    P.bits = ps.pair_bits;
    P.bins = pair_bins(ps.pair_bits);
    P.obj_start = reinterpret_cast<uint32_t *>(w);
    w += al256((size_t)(n_objs + 1) * 4);
    P.obj_off = reinterpret_cast<uint32_t *>(w);
    w += al256((size_t)n_objs * 4);
    uint8_t *nvox = reinterpret_cast<uint8_t *>(w);
    uint32_t *lists = reinterpret_cast<uint32_t *>(w + al256(n_slots));
    P.n_slots = n_slots;
    P.n_tiles = n_tiles;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (ctx->profiling) {
        for (auto &e : ev)
            if (!(e = take_event(ctx))) return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    HIP_TRY(launch_pairs_prepare(P, s));
    if (ev[1]) HIP_TRY(hipEventRecord(ev[1], s));
    if (n_pairs) {
        QueryArgs A{};
        A.g.H = ps.maxH;
        A.hot_lds = ps.hot_max;   // every object's hot levels fit
        A.width = (uint32_t)first.width;   // one kernel class: every object has this width
        A.rays = P.rays;
        A.n = n_slots;
        A.pr.pair_ray = d_pair_ray;
        A.pr.pair_inst = d_pair_inst;
        A.pr.inst = d_inst;
        A.pr.objs = P.objs;
        A.pr.tile_obj = P.tile_obj;
        A.pr.slot_pair = P.slot_pair;
        A.pr.minkey = P.minkey;
        A.pr.res = P.res;
        A.nvox = nvox;
        A.lists = lists;
        A.queue = reinterpret_cast<unsigned long long *>(w + list_ws_bytes(n_slots, (uint32_t)ps.maxH >> 1));
        A.persistent = ps.persistent;
        const int kbm = ps.kbm;
        const uint32_t k = chunks > 0 ? (uint32_t)chunks : ps.walk_chunks;
        lsnif_status st = walk_then_query(ctx, A, true, ps.recheck, n_tiles, k, s, ev[2],
                                          [&](const QueryArgs &a, uint32_t g) -> hipError_t {
            if (first.mlp_dtype == LSNIF_FP32) return launch_f32(a, first.feat_dtype, first.F, true, g, s);
            if (first.mlp_dtype == LSNIF_FP16) return launch_mma_f16(a, first.feat_dtype, first.F, kbm, true, g, s);
            if (first.mlp_dtype == LSNIF_BF16) return launch_mma_bf16(a, first.feat_dtype, first.F, kbm, true, g, s);
            return launch_mma_fp8(a, first.feat_dtype, first.F, kbm, true, g, s);
        });
        if (st) return st;
    }
    if (ev[3]) {
        if (!n_pairs) HIP_TRY(hipEventRecord(ev[2], s));
        HIP_TRY(hipEventRecord(ev[3], s));
        ctx->pending.push_back({ev[0], ev[1], ev[2], ev[3]});
    }
    HIP_TRY(launch_pairs_payload(P, s));
    return LSNIF_OK;
}

}  // namespace lsnif
