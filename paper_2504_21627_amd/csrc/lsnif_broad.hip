// Broad phase on the device, and the scene query that chains it to the pair
// query: world rays and instances in, the nearest hit per ray out (Sec. 4).
#include <hip/hip_runtime.h>

#include <cmath>

#include "lsnif_internal.hpp"
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

using namespace lsnif;

namespace {

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

lsnif_status check_broad(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays, const lsnif_instance *d_inst,
                         uint32_t n_inst)
{
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    if (n_rays && !d_rays) return fail(LSNIF_E_INVALID, "rays is NULL");
    if (n_inst && !d_inst) return fail(LSNIF_E_INVALID, "instances is NULL");
    if (reinterpret_cast<uintptr_t>(d_rays) % 16) return fail(LSNIF_E_INVALID, "rays must be 16-byte aligned");
    if ((uint64_t)n_rays * n_inst > 0xffffffffull)
        return fail(LSNIF_E_INVALID, "n_rays x n_inst = %llu must stay below 2^32",
                    (unsigned long long)n_rays * n_inst);
    if (ctx->objects.empty()) return fail(LSNIF_E_NOTFOUND, "no objects built");
    return LSNIF_OK;
}

// Count the pairs of every ray, scan the counts, and read the total back: the one point
// where the host waits for the stream.
lsnif_status count_pairs(lsnif_ctx *ctx, uint32_t n_objs, const lsnif_ray *d_rays, uint32_t n_rays,
                         const lsnif_instance *d_inst, uint32_t n_inst, hipStream_t s, BroadArgs &B,
                         uint32_t &total)
{
    const size_t n1 = (size_t)n_rays + 1, parts = (n1 + 1023) / 1024;
    const uint32_t words = (n_inst + 31) / 32;
    const uint32_t mask_words = words <= kBroadMaskWords ? words : 0u;
    lsnif_status st = grow_workspace(ctx->bws, ctx->bws_bytes,
                                     al256(n1 * 4) + al256(parts * 4) + al256((size_t)mask_words * n_rays * 4));
    if (st) return st;
    B = BroadArgs{};
    B.rays = reinterpret_cast<const float4 *>(d_rays);
    B.n_rays = n_rays;
    B.inst = d_inst;
    B.n_inst = n_inst;
    B.objs = static_cast<const ObjDev *>(ctx->d_table);
    B.n_objs = n_objs;
    B.offsets = static_cast<uint32_t *>(ctx->bws);
    uint32_t *part = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->bws) + al256(n1 * 4));
    B.mask_words = mask_words;
    B.masks = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->bws) + al256(n1 * 4) + al256(parts * 4));
    HIP_TRY(launch_broad_count(B, s));
    HIP_TRY(launch_exclusive_scan(B.offsets, (uint32_t)n1, part, s));
    HIP_TRY(hipMemcpyAsync(&total, B.offsets + n_rays, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LSNIF_OK;
}

}  // namespace

extern "C" {

lsnif_status lsnif_broad_phase(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays, const lsnif_instance *d_inst,
                               uint32_t n_inst, uint32_t *d_pair_ray, uint32_t *d_pair_inst, uint32_t cap,
                               uint32_t *n_pairs, void *stream)
{
    if (!ctx || !n_pairs) return fail(LSNIF_E_INVALID, "ctx or n_pairs is NULL");
    *n_pairs = 0;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    lsnif_status st = check_broad(ctx, d_rays, n_rays, d_inst, n_inst);
    if (st) return st;
    if (cap && (!d_pair_ray || !d_pair_inst)) return fail(LSNIF_E_INVALID, "pair buffers are NULL");
    DeviceGuard guard(ctx->device);
    uint32_t n_objs = 0;
    if ((st = upload_table(ctx, n_objs))) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    BroadArgs B;
    uint32_t total = 0;
    if ((st = count_pairs(ctx, n_objs, d_rays, n_rays, d_inst, n_inst, s, B, total))) return st;
    *n_pairs = total;
    if (total > cap) return fail(LSNIF_E_NOMEM, "%u pairs do not fit a buffer of %u", total, cap);
    B.pair_ray = d_pair_ray;
    B.pair_inst = d_pair_inst;
    HIP_TRY(launch_broad_write(B, s));
    return LSNIF_OK;
}

lsnif_status lsnif_query_scene(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays, const lsnif_instance *d_inst,
                               uint32_t n_inst, lsnif_hit *d_out, void *stream)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (n_rays == 0) return LSNIF_OK;
    lsnif_status st = check_broad(ctx, d_rays, n_rays, d_inst, n_inst);
    if (st) return st;
    if (!d_out) return fail(LSNIF_E_INVALID, "output is NULL");
    DeviceGuard guard(ctx->device);
    PairsSetup ps;
    if ((st = pairs_setup(ctx, ps))) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    BroadArgs B;
    uint32_t total = 0;
    if ((st = count_pairs(ctx, ps.n_objs, d_rays, n_rays, d_inst, n_inst, s, B, total))) return st;
    if ((st = grow_workspace(ctx->sws, ctx->sws_bytes, 2 * al256((size_t)total * 4)))) return st;
    B.pair_ray = static_cast<uint32_t *>(ctx->sws);
    B.pair_inst = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->sws) + al256((size_t)total * 4));
    HIP_TRY(launch_broad_write(B, s));
    if ((st = grow_workspace(ctx->pws, ctx->pws_bytes, pairs_ws_bytes(n_rays, total, ps.n_objs, ps.maxH >> 1, ps.pair_bits))))
        return st;
    return enqueue_pairs(ctx, ps, d_rays, n_rays, B.pair_ray, B.pair_inst, total, d_inst, n_inst, d_out, s, ctx->pws);
}

lsnif_status lsnif_bounce(lsnif_ctx *ctx, const lsnif_ray *d_rays, const lsnif_hit *d_hits, uint32_t n, uint32_t seed,
                          uint32_t bounce, float eps, lsnif_ray *d_next, uint32_t *d_parent, uint32_t cap,
                          uint32_t *n_next, void *stream)
{
    if (!ctx || !n_next) return fail(LSNIF_E_INVALID, "ctx or n_next is NULL");
    *n_next = 0;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    if (n && (!d_rays || !d_hits)) return fail(LSNIF_E_INVALID, "rays or hits is NULL");
    if (cap && (!d_next || !d_parent)) return fail(LSNIF_E_INVALID, "output buffers are NULL");
    if (reinterpret_cast<uintptr_t>(d_rays) % 16 || reinterpret_cast<uintptr_t>(d_next) % 16)
        return fail(LSNIF_E_INVALID, "rays must be 16-byte aligned");
    if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(LSNIF_E_INVALID, "eps must be finite and >= 0");
    DeviceGuard guard(ctx->device);
    const size_t n1 = (size_t)n + 1, parts = (n1 + 1023) / 1024;
    lsnif_status st = grow_workspace(ctx->bws, ctx->bws_bytes, al256(n1 * 4) + al256(parts * 4));
    if (st) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    BounceArgs B{};
    B.rays = reinterpret_cast<const float4 *>(d_rays);
    B.hits = d_hits;
    B.n = n;
    B.seed = seed;
    B.bounce = bounce;
    B.eps = eps;
    B.offsets = static_cast<uint32_t *>(ctx->bws);
    B.next = reinterpret_cast<float4 *>(d_next);
    B.parent = d_parent;
    uint32_t *part = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->bws) + al256(n1 * 4));
    HIP_TRY(launch_bounce_mark(B, s));
    HIP_TRY(launch_exclusive_scan(B.offsets, (uint32_t)n1, part, s));
    uint32_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, B.offsets + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_next = total;
    if (total > cap) return fail(LSNIF_E_NOMEM, "%u bounce rays do not fit a buffer of %u", total, cap);
    HIP_TRY(launch_bounce_write(B, s));
    return LSNIF_OK;
}

}  // extern "C"
