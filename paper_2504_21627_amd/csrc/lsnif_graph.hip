// Queries captured into HIP graphs: one capture, many one-launch replays.
//
// A capture records exactly the work the direct call enqueues (the fill
// kernels that clear counters are kernels, not memset nodes) on a private
// stream, with the graph's own workspace, so replays never share scratch
// memory with direct calls or with each other's graphs.

#include <hip/hip_runtime.h>

#include <new>

#include "lsnif_internal.hpp"

using namespace lsnif;

struct lsnif_graph {
    lsnif_ctx *ctx = nullptr;
    uint64_t generation = 0;
    int device = 0;
    void *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <typename Enqueue>
lsnif_status capture(lsnif_ctx *ctx, size_t ws_bytes, Enqueue &&enqueue, lsnif_graph **out)
{
    lsnif_graph *gr = new (std::nothrow) lsnif_graph;
    if (!gr) return fail(LSNIF_E_NOMEM, "graph");
    gr->ctx = ctx;
    gr->generation = ctx->generation;
    gr->device = ctx->device;
    auto drop = [&](lsnif_status st) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        (void)hipFree(gr->ws);
        delete gr;
        return st;
    };
    if (ws_bytes && hipMalloc(&gr->ws, ws_bytes) != hipSuccess)
        return drop(fail(LSNIF_E_NOMEM, "graph workspace of %llu bytes", (unsigned long long)ws_bytes));
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return drop(fail(LSNIF_E_DEVICE, "hipStreamCreateWithFlags failed"));
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return drop(fail(LSNIF_E_DEVICE, "hipStreamBeginCapture failed"));
    }
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    lsnif_status st = enqueue(s, gr->ws);
    ctx->profiling = prof;
    const hipError_t ec = hipStreamEndCapture(s, &gr->graph);
    (void)hipStreamDestroy(s);
    if (st) return drop(st);
    if (ec != hipSuccess || !gr->graph) return drop(fail(LSNIF_E_DEVICE, "hipStreamEndCapture failed"));
    if (hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess)
        return drop(fail(LSNIF_E_DEVICE, "hipGraphInstantiate failed"));
    *out = gr;
    return LSNIF_OK;
}

}  // namespace

extern "C" {

lsnif_status lsnif_graph_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                               lsnif_hit *d_out, lsnif_graph **out)
{
    if (!ctx || !out) return fail(LSNIF_E_INVALID, "ctx or out is NULL");
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    const Object *ob = nullptr;
    lsnif_status st = check_query(ctx, object_id, d_rays, n, d_out, ob);
    if (st) return st;
    if (n == 0) return fail(LSNIF_E_INVALID, "nothing to capture (n = 0)");
    DeviceGuard guard(ctx->device);
    return capture(
        ctx, query_ws_bytes(n, ob->geom.sort_bits, ob->geom.H >> 1),
        [&](hipStream_t s, void *ws) { return enqueue_query(ctx, *ob, d_rays, n, d_out, nullptr, s, ws); }, out);
}

lsnif_status lsnif_graph_pairs(lsnif_ctx *ctx, const lsnif_ray *d_rays, uint32_t n_rays, const uint32_t *d_pair_ray,
                               const uint32_t *d_pair_inst, uint32_t n_pairs, const lsnif_instance *d_inst,
                               uint32_t n_inst, lsnif_hit *d_out, lsnif_graph **out)
{
    if (!ctx || !out) return fail(LSNIF_E_INVALID, "ctx or out is NULL");
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    if (n_rays == 0) return fail(LSNIF_E_INVALID, "nothing to capture (n_rays = 0)");
    DeviceGuard guard(ctx->device);
    PairsSetup ps;
    lsnif_status st = pairs_setup(ctx, ps);
    if (st) return st;
    return capture(
        ctx, pairs_ws_bytes(n_rays, n_pairs, ps.n_objs, ps.maxH >> 1, ps.pair_bits),
        [&](hipStream_t s, void *ws) {
            return enqueue_pairs(ctx, ps, d_rays, n_rays, d_pair_ray, d_pair_inst, n_pairs, d_inst, n_inst, d_out,
                                 s, ws);
        },
        out);
}

lsnif_status lsnif_graph_launch(lsnif_graph *gr, void *stream)
{
    if (!gr) return fail(LSNIF_E_INVALID, "graph is NULL");
    if (gr->generation != gr->ctx->generation)
        return fail(LSNIF_E_INVALID, "objects were built or released since the graph was captured");
    DeviceGuard guard(gr->device);
    HIP_TRY(hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream)));
    return LSNIF_OK;
}

void lsnif_graph_destroy(lsnif_graph *gr)
{
    if (!gr) return;
    DeviceGuard guard(gr->device);
    (void)hipDeviceSynchronize();   // replays still running keep the graph and its workspace
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    (void)hipFree(gr->ws);
    delete gr;
}

}  // extern "C"
