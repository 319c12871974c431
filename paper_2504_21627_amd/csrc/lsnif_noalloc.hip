// Allocation-free single-object query: lsnif_query's kernels with their
// workspace (coherence-sort keys, order and bins; voxel counts and lists) in a
// fixed device array instead of the context's grown-on-demand buffer.
//
// The array is a file-scope __device__ object, so every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  In host
// code the array's name is only a stand-in for that object: the device address
// comes from hipGetSymbolAddress, taken once per device, with the device
// current, when a context is created on it (lsnif_create), and that address is
// what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lsnif_internal.hpp"

namespace lsnif {

namespace {

static __device__ __align__(256) unsigned char scratch[LSNIF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

lsnif_status noalloc_init(int device)
{
    if (device < 0) return LSNIF_OK;
    if (device >= kMaxDevices) return fail(LSNIF_E_INVALID, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return LSNIF_OK;
    DeviceGuard guard(device);
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(LSNIF_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                    hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return LSNIF_OK;
}

}  // namespace lsnif

using namespace lsnif;

extern "C" {

lsnif_status lsnif_query_noalloc(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n,
                                 lsnif_hit *d_out, void *stream)
{
    if (!ctx) return fail(LSNIF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    const Object *ob = nullptr;
    lsnif_status st = check_query(ctx, object_id, d_rays, n, d_out, ob);
    if (st || n == 0) return st;
    const size_t need = query_ws_bytes(n, ob->geom.sort_bits, ob->geom.H >> 1);
    if (need > (size_t)LSNIF_NOALLOC_SCRATCH_BYTES)
        return fail(LSNIF_E_INVALID,
                    "%u rays need %llu bytes of workspace; the allocation-free query holds %llu "
                    "(at most about %u rays of this object)",
                    n, (unsigned long long)need, (unsigned long long)LSNIF_NOALLOC_SCRATCH_BYTES,
                    (unsigned)((unsigned long long)n * LSNIF_NOALLOC_SCRATCH_BYTES / need));
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        ws = ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
    }
    if (!ws) return fail(LSNIF_E_DEVICE, "no scratch address for device %d", ctx->device);
    DeviceGuard guard(ctx->device);
    // one tile range (no side stream), no timing events: nothing here creates or allocates
    return enqueue_query(ctx, *ob, d_rays, n, d_out, nullptr, static_cast<hipStream_t>(stream), ws, 1, nullptr,
                         false);
}

}  // extern "C"
