// Per-object launch parameters and the autotuner that picks them by timing.
// With an autotune cache (lsnif_cache.hip) each winner is also written to the
// cache file, under the key of every object it applies to.
//
// Every candidate runs the real query on the caller's batch (one warm-up, then
// three timed queries between HIP events on a private stream), so the choice
// reflects the batch's own coherence, the object's table sizes and the LDS
// left for hot levels.  None of the parameters changes a result.

#include <hip/hip_runtime.h>

#include <vector>

#include "lsnif_internal.hpp"

using namespace lsnif;

namespace lsnif {

lsnif_status check_tuning(const lsnif_tuning *t)
{
    if (!t) return fail(LSNIF_E_INVALID, "tuning is NULL");
    if (t->sort_bits < 0 || t->sort_bits > 7) return fail(LSNIF_E_INVALID, "sort_bits must be 0..7");
    if (t->pair_bits < 1 || t->pair_bits > 6) return fail(LSNIF_E_INVALID, "pair_bits must be 1..6");
    if (t->hot_lds_bytes < 0 || t->hot_lds_bytes > (int32_t)kHotLdsBudget)
        return fail(LSNIF_E_INVALID, "hot_lds_bytes must be 0..%u", kHotLdsBudget);
    if (t->walk_chunks < 1 || t->walk_chunks > 16) return fail(LSNIF_E_INVALID, "walk_chunks must be 1..16");
    if (t->persistent != 0 && t->persistent != 1) return fail(LSNIF_E_INVALID, "persistent must be 0 or 1");
    return LSNIF_OK;
}

void apply_tuning(lsnif_ctx *ctx, Object &ob, const lsnif_tuning &t)
{
    ob.geom.sort_bits = (uint32_t)t.sort_bits;
    ob.geom.pair_bits = (uint32_t)t.pair_bits;
    ob.hot_budget = (uint32_t)t.hot_lds_bytes;
    ob.walk_chunks = (uint32_t)t.walk_chunks;
    ob.persistent = (uint32_t)t.persistent;
    plan_hot_levels(ob.geom, ob.esz, ob.hot_budget);
    ctx->table_dirty = true;
    ++ctx->generation;
}

lsnif_tuning object_tuning(const Object &ob)
{
    return lsnif_tuning{(int32_t)ob.geom.sort_bits, (int32_t)ob.geom.pair_bits, (int32_t)ob.hot_budget,
                        (int32_t)ob.walk_chunks, (int32_t)ob.persistent};
}

}  // namespace lsnif

namespace {

constexpr int kTimedReps = 3;

void apply(lsnif_ctx *ctx, Object &ob, const lsnif_tuning &t) { apply_tuning(ctx, ob, t); }
lsnif_tuning current(const Object &ob) { return object_tuning(ob); }

// Milliseconds per call of `enqueue(stream)`, averaged over kTimedReps after a warm-up.
template <typename Enqueue> lsnif_status time_ms(Enqueue &&enqueue, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float &ms)
{
    lsnif_status st = enqueue(s);
    if (st) return st;
    HIP_TRY(hipEventRecord(e0, s));
    for (int i = 0; i < kTimedReps; ++i)
        if ((st = enqueue(s))) return st;
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    ms /= kTimedReps;
    return LSNIF_OK;
}

// Runs `fn(stream, e0, e1)` with a private stream and two events, releasing them after.
template <typename Fn> lsnif_status with_stream(Fn &&fn)
{
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return fail(LSNIF_E_DEVICE, "hipStreamCreateWithFlags failed");
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipStreamDestroy(s);
        return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
    }
    const lsnif_status st = fn(s, e0, e1);
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return st;
}

const int32_t kHotCandidates[] = {0, 20 << 10, 40 << 10};
const int32_t kChunkCandidates[] = {1, 2, 4, 8};

}  // namespace

extern "C" {

lsnif_status lsnif_get_tuning(lsnif_ctx *ctx, uint32_t object_id, lsnif_tuning *tuning)
{
    if (!ctx || !tuning) return fail(LSNIF_E_INVALID, "ctx or tuning is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    *tuning = current(it->second);
    return LSNIF_OK;
}

lsnif_status lsnif_set_tuning(lsnif_ctx *ctx, uint32_t object_id, const lsnif_tuning *tuning)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    lsnif_status st = check_tuning(tuning);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    if (ctx->device >= 0) {
        DeviceGuard guard(ctx->device);
        HIP_TRY(hipDeviceSynchronize());   // queries in flight read the old parameters by value
    }
    apply(ctx, it->second, *tuning);
    return LSNIF_OK;
}

lsnif_status lsnif_autotune(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                            lsnif_hit *d_out, lsnif_tuning *best)
{
    if (!ctx || !best) return fail(LSNIF_E_INVALID, "ctx or best is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    const Object *cob = nullptr;
    lsnif_status st = check_query(ctx, object_id, d_rays, n, d_out, cob);
    if (st) return st;
    if (n == 0) return fail(LSNIF_E_INVALID, "nothing to time (n = 0)");
    Object &ob = ctx->objects[object_id];
    DeviceGuard guard(ctx->device);
    if ((st = grow_workspace(ctx->ws, ctx->ws_bytes, query_ws_bytes(n, 7, ob.geom.H >> 1)))) return st;   // the most bins
    HIP_TRY(hipDeviceSynchronize());
    const lsnif_tuning start = current(ob);
    lsnif_tuning win = start;
    float win_ms = -1.0f;
    st = with_stream([&](hipStream_t s, hipEvent_t e0, hipEvent_t e1) -> lsnif_status {
        auto run = [&](const lsnif_tuning &t) -> lsnif_status {
            apply(ctx, ob, t);
            float ms = 0.0f;
            lsnif_status e = time_ms(
                [&](hipStream_t q) { return enqueue_query(ctx, ob, d_rays, n, d_out, nullptr, q, ctx->ws); }, s, e0,
                e1, ms);
            if (e) return e;
            if (win_ms < 0.0f || ms < win_ms) {
                win_ms = ms;
                win = t;
            }
            return LSNIF_OK;
        };
        for (int sb : {0, 4, 5, 6, 7})
            for (int32_t hot : kHotCandidates)
                if (lsnif_status e = run(lsnif_tuning{sb, start.pair_bits, hot, start.walk_chunks, start.persistent}))
                    return e;
        const lsnif_tuning best = win;
        for (int32_t ch : kChunkCandidates)
            if (ch != best.walk_chunks)
                if (lsnif_status e = run(lsnif_tuning{best.sort_bits, best.pair_bits, best.hot_lds_bytes, ch,
                                                      best.persistent}))
                    return e;
        lsnif_tuning flip = win;
        flip.persistent = 1 - flip.persistent;
        return run(flip);
    });
    apply(ctx, ob, st ? start : win);
    if (st) return st;
    *best = win;
    if (ctx->cache_path.empty()) return LSNIF_OK;
    ctx->cache[cache_key(ctx, ob)] = win;
    return cache_save(ctx);
}

lsnif_status lsnif_autotune_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays,
                                  const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                                  const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out,
                                  lsnif_tuning *best)
{
    if (!ctx || !best) return fail(LSNIF_E_INVALID, "ctx or best is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    if (n_rays == 0 || n_pairs == 0) return fail(LSNIF_E_INVALID, "nothing to time");
    if (ctx->objects.empty()) return fail(LSNIF_E_NOTFOUND, "no objects built");
    DeviceGuard guard(ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    std::vector<std::pair<uint32_t, lsnif_tuning>> start;
    for (auto &kv : ctx->objects) start.push_back({kv.first, current(kv.second)});
    auto apply_all = [&](const lsnif_tuning &t) {
        for (auto &kv : ctx->objects)
            apply(ctx, kv.second,
                  lsnif_tuning{(int32_t)kv.second.geom.sort_bits, t.pair_bits, t.hot_lds_bytes, t.walk_chunks,
                               t.persistent});
    };
    lsnif_tuning win{};
    float win_ms = -1.0f;
    const uint32_t start_chunks = ctx->objects.begin()->second.walk_chunks;
    const int32_t start_persist = (int32_t)ctx->objects.begin()->second.persistent;
    lsnif_status st = with_stream([&](hipStream_t s, hipEvent_t e0, hipEvent_t e1) -> lsnif_status {
        auto run = [&](const lsnif_tuning &t) -> lsnif_status {
            apply_all(t);
            PairsSetup ps;
            lsnif_status e = pairs_setup(ctx, ps);   // uploads the changed object table
            if (e) return e;
            if ((e = grow_workspace(ctx->pws, ctx->pws_bytes,
                                    pairs_ws_bytes(n_rays, n_pairs, ps.n_objs, ps.maxH >> 1, ps.pair_bits))))
                return e;
            float ms = 0.0f;
            e = time_ms(
                [&](hipStream_t q) {
                    return enqueue_pairs(ctx, ps, d_rays, n_rays, d_pair_ray, d_pair_inst, n_pairs, d_inst, n_inst,
                                         d_out, q, ctx->pws);
                },
                s, e0, e1, ms);
            if (e) return e;
            if (win_ms < 0.0f || ms < win_ms) {
                win_ms = ms;
                win = t;
            }
            return LSNIF_OK;
        };
        for (int pb : {2, 3, 4, 5, 6})
            for (int32_t hot : kHotCandidates)
                if (lsnif_status e = run(lsnif_tuning{0, pb, hot, (int32_t)start_chunks, start_persist})) return e;
        const lsnif_tuning best = win;
        for (int32_t ch : kChunkCandidates)
            if (ch != best.walk_chunks)
                if (lsnif_status e = run(lsnif_tuning{0, best.pair_bits, best.hot_lds_bytes, ch, best.persistent}))
                    return e;
        lsnif_tuning flip = win;
        flip.persistent = 1 - flip.persistent;
        return run(flip);
    });
    if (st) {
        for (auto &p : start) apply(ctx, ctx->objects[p.first], p.second);
        return st;
    }
    apply_all(win);
    *best = current(ctx->objects.begin()->second);
    if (ctx->cache_path.empty()) return LSNIF_OK;
    for (auto &kv : ctx->objects) ctx->cache[cache_key(ctx, kv.second)] = current(kv.second);
    return cache_save(ctx);
}

}  // extern "C"
