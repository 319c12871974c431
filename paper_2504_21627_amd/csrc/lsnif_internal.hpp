// Internals shared by the host units of the library: the context, the object
// record, error reporting and the enqueue functions behind the query calls.
#pragma once
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"
#include "lsnif_pairs.hpp"
#include "../../include/lsnif.h"

namespace lsnif {

// Records a message for lsnif_last_error() (per thread) and returns `st`.
lsnif_status fail(lsnif_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::lsnif::fail(LSNIF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Default tile ranges of a query whose walk runs ahead of the query kernel (1:
// the walk of the whole batch first), and the fewest tiles a range may hold.
constexpr uint32_t kWalkChunks = 1;
constexpr uint32_t kMinChunkTiles = 256;

struct Object {
    Geom geom{};
    Mlp mlp{};
    void *d_occ = nullptr, *d_tab = nullptr, *d_w = nullptr;   // d_occ: brick masks, then brick bits
    int feat_dtype = 0, mlp_dtype = 0, F = 0, width = 0;
    uint32_t esz = 0;             // bytes of one table entry on the device
    uint32_t hot_budget = kHotLdsBudget;   // LDS budget the hot levels were planned for
    uint32_t walk_chunks = kWalkChunks;    // tile ranges of a query whose walk runs ahead
    uint32_t persistent = 0;               // query kernel as a persistent grid (width 64)
    uint64_t bytes = 0;
};

// Objects that one query kernel can serve together.
inline bool same_class(const Object &a, const Object &b)
{
    return a.feat_dtype == b.feat_dtype && a.mlp_dtype == b.mlp_dtype && a.F == b.F && a.width == b.width;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

class Server;
void destroy_server(lsnif_ctx *ctx);   // stops a running serving loop

// Batches below this size are processed in the order given (no coherence sort).
constexpr uint32_t kSortMin = 8192;
// FP32 batches of at most this many rays run one wave per ray (k_query_lat).
constexpr uint32_t kSmallBatchRays = 8192;

// Workspace bytes of one query of n rays, and of one pair query; cap is the
// longest voxel list (H / 2, the largest over the objects for pairs).
size_t query_ws_bytes(uint32_t n, uint32_t sort_bits, uint32_t cap);
size_t pairs_ws_bytes(uint32_t n_rays, uint32_t n_pairs, uint32_t n_objs, uint32_t cap, uint32_t pair_bits);

}  // namespace lsnif

struct lsnif_ctx {
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    uint32_t next_id = 1;
    std::map<uint32_t, lsnif::Object> objects;
    // query workspaces of the direct calls (coherence sort; pair work lists), grown on demand
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *pws = nullptr;
    size_t pws_bytes = 0;
    // broad phase: per-ray counts and their scan; the pairs of lsnif_query_scene
    void *bws = nullptr;
    size_t bws_bytes = 0;
    void *sws = nullptr;
    size_t sws_bytes = 0;
    // device copy of the object table for pair queries, indexed by object id
    void *d_table = nullptr;
    size_t table_cap = 0;
    bool table_dirty = true;
    // bumped by every build and release: graphs captured before are stale
    uint64_t generation = 0;
    // kernel timing: per query, events before the sort, before and after the query kernel
    bool profiling = false;
    std::vector<std::vector<hipEvent_t>> pending;
    std::vector<hipEvent_t> spare;
    // walk of the next tile range while the query kernel works on the current one: a side
    // stream (default priority) and the events that order the two
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> order_events;
    // serving loop, when started; `mu` orders the direct calls against it
    lsnif::Server *server = nullptr;
    std::recursive_mutex mu;
    // autotune cache: the device's architecture name, the file's path (empty: none) and
    // its entries, read at creation and rewritten by every autotune call
    std::string arch;
    std::string cache_path;
    std::map<std::string, lsnif_tuning> cache;
};

namespace lsnif {

// Class of the objects a pair query can reach, uploaded object table included.
struct PairsSetup {
    const Object *first = nullptr;
    int kbm = 1, maxH = 2;
    uint32_t hot_max = 0;   // largest hot-level LDS footprint of the objects
    bool recheck = false;   // some object re-decides grazing voxels in float64
    uint32_t walk_chunks = 1;   // largest walk_chunks of the objects
    uint32_t pair_bits = 1;     // finest pair grouping of the objects
    uint32_t persistent = 0;    // some object asks for the persistent query kernel
    uint32_t n_objs = 0;
};
lsnif_status pairs_setup(lsnif_ctx *ctx, PairsSetup &ps);
// Upload the object table (by object id) if objects changed; n_objs = largest id + 1.
lsnif_status upload_table(lsnif_ctx *ctx, uint32_t &n_objs);
// Grow a device workspace to `need` bytes (frees the old one, which waits for its users).
lsnif_status grow_workspace(void *&buf, size_t &have, size_t need);
// Choose an object's hot levels for an LDS budget (bytes).
void plan_hot_levels(Geom &g, uint32_t esz, uint32_t budget);
// Object `object_id` of ctx and the checks every single-object query makes.
lsnif_status check_query(lsnif_ctx *ctx, uint32_t object_id, const lsnif_ray *d_rays, uint32_t n, lsnif_hit *d_out,
                         const Object *&ob);

// Enqueue one query on `s`.  `ws` must hold query_ws_bytes(n) (pairs_ws_bytes for
// pairs) bytes and stay untouched until the stream has run the query.
// `chunks`: tile ranges whose walk runs ahead of the query kernel on the side stream
// (<= 0: the object's tuning; 1: the walk of the whole batch first).
lsnif_status enqueue_query(lsnif_ctx *ctx, const Object &ob, const lsnif_ray *d_rays, uint32_t n, lsnif_hit *d_out,
                           const lsnif_debug_bufs *dbg, hipStream_t s, void *ws, int chunks = 0,
                           float *gather_sums = nullptr, bool timed = true);
// Launch parameters: range checks, and setting them on an object (re-plans its hot levels).
lsnif_status check_tuning(const lsnif_tuning *t);
void apply_tuning(lsnif_ctx *ctx, Object &ob, const lsnif_tuning &t);
lsnif_tuning object_tuning(const Object &ob);
// Autotune cache (lsnif_cache.hip): architecture name of a device ("host" for -1), an
// object's cache key, reading the file into ctx->cache and writing ctx->cache back.
std::string device_arch(int device);
std::string cache_key(const lsnif_ctx *ctx, const Object &ob);
lsnif_status cache_load(lsnif_ctx *ctx);
lsnif_status cache_save(lsnif_ctx *ctx);
// Device address of the allocation-free query's scratch array on `device`, taken once
// per device (with that device current) at context creation.
lsnif_status noalloc_init(int device);
lsnif_status enqueue_pairs(lsnif_ctx *ctx, const PairsSetup &ps, const lsnif_ray *d_rays, uint32_t n_rays,
                           const uint32_t *d_pair_ray, const uint32_t *d_pair_inst, uint32_t n_pairs,
                           const lsnif_instance *d_inst, uint32_t n_inst, lsnif_hit *d_out, hipStream_t s, void *ws,
                           int chunks = 0);

}  // namespace lsnif
