// Training: one step = the voxel walk, the encoding, the forward layer
// products, the losses, the backward layer products, the scatter of the
// encoding's gradient onto the tables, and Adam over every parameter.
//
// The parameters are the FP32 object's own device buffers: the tables
// [L][T][F] and the weights in the FP32 query kernel's layout, each layer
// stored as [in][ld] (ld = width for hidden layers, kMaxOut for the head, the
// columns past the outputs zero).  Gradients and moments use the same layout,
// so the head's spare columns get zero gradient and never move.
//
// The table gradient is accumulated with float atomics into several copies
// (one per XCD when memory allows; contention on the entries many rays reach
// is what bounds the scatter), summed into the first copy at the end.  Weight
// gradients go through per-chunk partial products and a sum, no atomics.
//
// Activations of the backward pass overwrite the forward ones layer by layer:
// a layer's input is read for its weight gradient, then replaced by the
// gradient with respect to it (the derivative epilogue reads each element
// before the same thread writes it), and the encoding buffer finally holds
// d loss / d encoding for the scatter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <new>
#include <vector>

#include "lsnif_internal.hpp"
#include "lsnif_launch.hpp"
#include "lsnif_train.hpp"

using namespace lsnif;

struct lsnif_trainer {
    lsnif_ctx *ctx = nullptr;
    uint32_t id = 0;
    const void *d_tab = nullptr;   // the object's buffers when the trainer was made
    lsnif_adam_cfg cfg{};
    uint64_t steps = 0;
    size_t n_tab = 0, n_w = 0;     // floats of tables and packed weights
    uint32_t copies = 1;           // copies of the table gradient
    float *grad = nullptr;         // [copies x n_tab] table gradient copies, then [n_w] weight gradients
    float *m = nullptr, *v = nullptr;   // [n_tab + n_w]
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // with the context's profiling on: per step, events around the forward layer products,
    // the backward layer products (with their partial sums) and the table-gradient scatter
    std::vector<std::array<hipEvent_t, 6>> prof;
    std::vector<hipEvent_t> spare;
};

namespace {

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

size_t weight_floats(const Object &ob)
{
    return (size_t)ob.mlp.off[ob.mlp.n_hidden] + (size_t)ob.width * kMaxOut;
}

hipEvent_t take_event(lsnif_trainer *tr)
{
    if (!tr->spare.empty()) {
        hipEvent_t e = tr->spare.back();
        tr->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

lsnif_status find(lsnif_trainer *tr, Object *&ob)
{
    auto it = tr->ctx->objects.find(tr->id);
    if (it == tr->ctx->objects.end() || it->second.d_tab != tr->d_tab)
        return fail(LSNIF_E_NOTFOUND, "the trainer's object %u was released", tr->id);
    ob = &it->second;
    return LSNIF_OK;
}

// Workspace of a batch of n rays.
struct StepWs {
    uint32_t *lists;
    uint8_t *nvox;
    float *x0;        // [n][in_dim]
    float *act[8];    // act[k] = [n][width], k = 1 .. n_hidden
    float *z, *dz;    // [n][out_dim]
    float *part;      // partial weight-gradient products
    float *loss_part; // per-block loss sums
};

constexpr uint32_t kCopyBudget = 1u << 30;   // bytes for the table-gradient copies

// K chunk of a weight-gradient product: enough blocks to fill the chip.
uint32_t wgrad_chunk(uint32_t M, uint32_t N, uint32_t n)
{
    const uint32_t tiles = ((M + kGM - 1) / kGM) * ((N + kGN - 1) / kGN);
    const uint32_t want = tiles >= 2048 ? 1 : 2048 / tiles;
    uint32_t c = (n + want - 1) / want;
    c = (c + kGK - 1) / kGK * kGK;
    return c < 256 ? 256 : c;
}

// Floats of the largest partial-product set of the weight gradients, plus the
// scratch of their two-pass sum.
size_t part_floats(const Object &ob, uint32_t n)
{
    const uint32_t in0 = (uint32_t)(ob.geom.H * ob.geom.L * ob.geom.F), Wd = (uint32_t)ob.width;
    size_t best = 0;
    for (int k = 0; k <= ob.mlp.n_hidden; ++k) {
        const uint32_t M = k == 0 ? in0 : Wd, N = k == ob.mlp.n_hidden ? (uint32_t)ob.mlp.out_dim : Wd;
        const size_t z = (n + wgrad_chunk(M, N, n) - 1) / wgrad_chunk(M, N, n);
        best = std::max(best, (z + kSumGroups) * M * N);
    }
    return best;
}

size_t step_ws_bytes(const Object &ob, uint32_t n)
{
    const size_t in = (size_t)ob.geom.H * ob.geom.L * ob.geom.F, od = (size_t)ob.mlp.out_dim;
    return al256((size_t)n * (ob.geom.H / 2) * 4) + al256(n) + al256((size_t)n * in * 4) +
           (size_t)ob.mlp.n_hidden * al256((size_t)n * ob.width * 4) + 2 * al256((size_t)n * od * 4) +
           al256(part_floats(ob, n) * 4) + al256((size_t)(n + kBlock - 1) / kBlock * 4);
}

StepWs carve(const Object &ob, uint32_t n, void *ws)
{
    const size_t in = (size_t)ob.geom.H * ob.geom.L * ob.geom.F, od = (size_t)ob.mlp.out_dim;
    char *w = static_cast<char *>(ws);
    StepWs S{};
    S.lists = reinterpret_cast<uint32_t *>(w);
    w += al256((size_t)n * (ob.geom.H / 2) * 4);
    S.nvox = reinterpret_cast<uint8_t *>(w);
    w += al256(n);
    S.x0 = reinterpret_cast<float *>(w);
    w += al256((size_t)n * in * 4);
    for (int k = 1; k <= ob.mlp.n_hidden; ++k) {
        S.act[k] = reinterpret_cast<float *>(w);
        w += al256((size_t)n * ob.width * 4);
    }
    S.z = reinterpret_cast<float *>(w);
    w += al256((size_t)n * od * 4);
    S.dz = reinterpret_cast<float *>(w);
    w += al256((size_t)n * od * 4);
    S.part = reinterpret_cast<float *>(w);
    w += al256(part_floats(ob, n) * 4);
    S.loss_part = reinterpret_cast<float *>(w);
    return S;
}

lsnif_status grads(lsnif_trainer *tr, const Object &ob, const lsnif_ray *d_rays, const lsnif_train_target *d_gt,
                   uint32_t n, float *d_loss, hipStream_t s)
{
    const Mlp &mlp = ob.mlp;
    const uint32_t nh = (uint32_t)mlp.n_hidden, Wd = (uint32_t)ob.width, od = (uint32_t)mlp.out_dim;
    const uint32_t in0 = (uint32_t)(ob.geom.H * ob.geom.L * ob.geom.F);
    lsnif_status st = grow_workspace(tr->ws, tr->ws_bytes, step_ws_bytes(ob, n));
    if (st) return st;
    const StepWs S = carve(ob, n, tr->ws);
    std::array<hipEvent_t, 6> ev{};
    if (tr->ctx->profiling) {
        for (auto &e : ev)
            if (!(e = take_event(tr))) return fail(LSNIF_E_DEVICE, "hipEventCreate failed");
    }
    auto mark = [&](int i) -> hipError_t { return ev[i] ? hipEventRecord(ev[i], s) : hipSuccess; };
    float *tab = static_cast<float *>(ob.d_tab);
    float *W = static_cast<float *>(const_cast<void *>(ob.d_w));
    float *gtab = tr->grad, *gW = tr->grad + tr->copies * tr->n_tab;
    HIP_TRY(launch_train_fill(gtab, tr->copies * tr->n_tab, gW, tr->n_w, s));
    // voxel lists: the query path's walk, rays in their given order
    QueryArgs A{};
    A.g = ob.geom;
    A.rays = reinterpret_cast<const float4 *>(d_rays);
    A.n = n;
    A.lists = S.lists;
    A.nvox = S.nvox;
    HIP_TRY(launch_walk(A, false, ob.geom.recheck != 0, (n + kBlock - 1) / kBlock, s));
    TrainEncArgs E{};
    E.g = ob.geom;
    E.rays = A.rays;
    E.n = n;
    E.lists = S.lists;
    E.nvox = S.nvox;
    E.tab = tab;
    E.gtab = gtab;
    E.replicas = tr->copies;
    E.n_tab = tr->n_tab;
    E.x = S.x0;
    HIP_TRY(launch_train_encode(E, false, s));
    const float slope = mlp.act == LSNIF_LEAKY_RELU ? mlp.slope : 0.0f;
    auto layer_in = [&](uint32_t k) { return k == 0 ? S.x0 : S.act[k]; };
    auto in_dim = [&](uint32_t k) { return k == 0 ? in0 : Wd; };
    auto out_dim = [&](uint32_t k) { return k == nh ? od : Wd; };
    auto ld = [&](uint32_t k) { return k == nh ? (uint32_t)kMaxOut : Wd; };
    // forward: layer k maps its input to act[k + 1] (or the raw outputs z)
    HIP_TRY(mark(0));
    for (uint32_t k = 0; k <= nh; ++k) {
        GemmArgs G{};
        G.A = layer_in(k);
        G.sai = in_dim(k);
        G.sak = 1;
        G.B = W + mlp.off[k];
        G.sbk = ld(k);
        G.sbj = 1;
        G.C = k == nh ? S.z : S.act[k + 1];
        G.ldc = out_dim(k);
        G.M = n;
        G.N = out_dim(k);
        G.K = in_dim(k);
        G.kchunk = G.K;
        G.slope = slope;
        HIP_TRY(launch_train_gemm(G, k == nh ? kEpiStore : kEpiAct, s));
    }
    HIP_TRY(mark(1));
    TrainLossArgs Lo{};
    Lo.g = ob.geom;
    Lo.rays = A.rays;
    Lo.gt = d_gt;
    Lo.n = n;
    Lo.nvox = S.nvox;
    Lo.z = S.z;
    Lo.dz = S.dz;
    Lo.ldz = od;
    Lo.out_dim = od;
    Lo.n_mat = (uint32_t)mlp.n_mat;
    Lo.has_albedo = (uint32_t)mlp.has_albedo;
    Lo.loss_part = S.loss_part;
    HIP_TRY(launch_train_loss(Lo, s));
    // backward: g holds d loss / d (output of layer k)
    const float *g = S.dz;
    HIP_TRY(mark(2));
    for (int k = (int)nh; k >= 0; --k) {
        const uint32_t ku = (uint32_t)k;
        GemmArgs Gw{};   // weight gradient: input^T x g over the batch
        Gw.A = layer_in(ku);
        Gw.sai = 1;
        Gw.sak = in_dim(ku);
        Gw.B = g;
        Gw.sbk = out_dim(ku);
        Gw.sbj = 1;
        Gw.C = S.part;
        Gw.ldc = out_dim(ku);
        Gw.M = in_dim(ku);
        Gw.N = out_dim(ku);
        Gw.K = n;
        Gw.kchunk = wgrad_chunk(Gw.M, Gw.N, n);
        HIP_TRY(launch_train_gemm(Gw, kEpiPartial, s));
        const uint32_t nz = (n + Gw.kchunk - 1) / Gw.kchunk;
        HIP_TRY(launch_sum_partials(S.part, nz, Gw.M, Gw.N, S.part + (size_t)nz * Gw.M * Gw.N, gW + mlp.off[ku],
                                    ld(ku), s));
        GemmArgs Gd{};   // input gradient: g x W^T, times the activation's derivative below the head's input
        Gd.A = g;
        Gd.sai = out_dim(ku);
        Gd.sak = 1;
        Gd.B = W + mlp.off[ku];
        Gd.sbk = 1;
        Gd.sbj = ld(ku);
        float *dst = layer_in(ku);
        Gd.C = dst;
        Gd.ldc = in_dim(ku);
        Gd.aux = dst;
        Gd.M = n;
        Gd.N = in_dim(ku);
        Gd.K = out_dim(ku);
        Gd.kchunk = Gd.K;
        Gd.slope = slope;
        HIP_TRY(launch_train_gemm(Gd, k > 0 ? kEpiActGrad : kEpiStore, s));
        g = dst;
    }
    HIP_TRY(mark(3));
    HIP_TRY(mark(4));
    HIP_TRY(launch_train_encode(E, true, s));   // E.x = x0, now d loss / d encoding
    HIP_TRY(mark(5));
    if (ev[0]) tr->prof.push_back(ev);
    HIP_TRY(launch_sum_copies(gtab, tr->n_tab, tr->copies, s));
    if (d_loss) HIP_TRY(launch_train_loss_final(S.loss_part, n, d_loss, s));
    return LSNIF_OK;
}

lsnif_status apply(lsnif_trainer *tr, const Object &ob, hipStream_t s)
{
    const uint64_t t = tr->steps + 1;
    AdamArgs A{};
    A.lr = tr->cfg.lr;
    A.b1 = tr->cfg.beta1;
    A.b2 = tr->cfg.beta2;
    A.eps = tr->cfg.eps;
    A.c1 = (float)(1.0 / (1.0 - std::pow((double)tr->cfg.beta1, (double)t)));
    A.c2 = (float)(1.0 / (1.0 - std::pow((double)tr->cfg.beta2, (double)t)));
    A.p = static_cast<float *>(ob.d_tab);
    A.g = tr->grad;
    A.m = tr->m;
    A.v = tr->v;
    A.count = tr->n_tab;
    HIP_TRY(launch_adam(A, s));
    A.p = static_cast<float *>(const_cast<void *>(ob.d_w));
    A.g = tr->grad + tr->copies * tr->n_tab;
    A.m = tr->m + tr->n_tab;
    A.v = tr->v + tr->n_tab;
    A.count = tr->n_w;
    HIP_TRY(launch_adam(A, s));
    tr->steps = t;
    return LSNIF_OK;
}

lsnif_status check_batch(const lsnif_ray *d_rays, const lsnif_train_target *d_gt, uint32_t n)
{
    if (n == 0) return fail(LSNIF_E_INVALID, "empty batch");
    if (n > (1u << 24)) return fail(LSNIF_E_INVALID, "batch of %u rays exceeds 2^24", n);
    if (!d_rays || !d_gt) return fail(LSNIF_E_INVALID, "rays or targets are NULL");
    if (reinterpret_cast<uintptr_t>(d_rays) % 16 || reinterpret_cast<uintptr_t>(d_gt) % 4)
        return fail(LSNIF_E_INVALID, "rays must be 16-byte and targets 4-byte aligned");
    return LSNIF_OK;
}

}  // namespace

extern "C" {

lsnif_status lsnif_trainer_create(lsnif_ctx *ctx, uint32_t object_id, const lsnif_adam_cfg *cfg, lsnif_trainer **out)
{
    if (!ctx || !out) return fail(LSNIF_E_INVALID, "ctx or out is NULL");
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->device < 0) return fail(LSNIF_E_DEVICE, "host-only context");
    auto it = ctx->objects.find(object_id);
    if (it == ctx->objects.end()) return fail(LSNIF_E_NOTFOUND, "no object %u", object_id);
    const Object &ob = it->second;
    if (ob.feat_dtype != LSNIF_FP32 || ob.mlp_dtype != LSNIF_FP32)
        return fail(LSNIF_E_INVALID, "training needs an object with FP32 features and an FP32 MLP");
    lsnif_adam_cfg c = cfg ? *cfg : lsnif_adam_cfg{0.01f, 0.9f, 0.999f, 1e-8f};
    if (!(c.lr > 0.0f) || !(c.beta1 >= 0.0f && c.beta1 < 1.0f) || !(c.beta2 >= 0.0f && c.beta2 < 1.0f) ||
        !(c.eps > 0.0f) || !std::isfinite(c.lr) || !std::isfinite(c.eps))
        return fail(LSNIF_E_INVALID, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
    DeviceGuard guard(ctx->device);
    lsnif_trainer *tr = new (std::nothrow) lsnif_trainer;
    if (!tr) return fail(LSNIF_E_NOMEM, "trainer");
    tr->ctx = ctx;
    tr->id = object_id;
    tr->d_tab = ob.d_tab;
    tr->cfg = c;
    tr->n_tab = (size_t)ob.geom.L * ((size_t)1 << ob.geom.log2_T) * ob.geom.F;
    tr->n_w = weight_floats(ob);
    tr->copies = (uint32_t)std::max<size_t>(1, std::min<size_t>(8, kCopyBudget / (tr->n_tab * sizeof(float))));
    const size_t bytes = (tr->n_tab + tr->n_w) * sizeof(float);
    const size_t gbytes = (tr->copies * tr->n_tab + tr->n_w) * sizeof(float);
    if (hipMalloc(&tr->grad, gbytes) != hipSuccess || hipMalloc(&tr->m, bytes) != hipSuccess ||
        hipMalloc(&tr->v, bytes) != hipSuccess) {
        (void)hipFree(tr->grad);
        (void)hipFree(tr->m);
        (void)hipFree(tr->v);
        delete tr;
        return fail(LSNIF_E_NOMEM, "trainer buffers of 3 x %llu bytes", (unsigned long long)bytes);
    }
    if (hipMemset(tr->grad, 0, gbytes) != hipSuccess || hipMemset(tr->m, 0, bytes) != hipSuccess ||
        hipMemset(tr->v, 0, bytes) != hipSuccess) {
        lsnif_trainer_destroy(tr);
        return fail(LSNIF_E_DEVICE, "clearing the trainer buffers failed");
    }
    *out = tr;
    return LSNIF_OK;
}

void lsnif_trainer_destroy(lsnif_trainer *tr)
{
    if (!tr) return;
    DeviceGuard guard(tr->ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(tr->grad);
    (void)hipFree(tr->m);
    (void)hipFree(tr->v);
    (void)hipFree(tr->ws);
    for (auto &v : tr->prof)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    for (hipEvent_t e : tr->spare) (void)hipEventDestroy(e);
    delete tr;
}

lsnif_status lsnif_train_grads(lsnif_trainer *tr, const lsnif_ray *d_rays, const lsnif_train_target *d_gt,
                               uint32_t n, float *d_loss, void *stream)
{
    if (!tr) return fail(LSNIF_E_INVALID, "trainer is NULL");
    lsnif_status st = check_batch(d_rays, d_gt, n);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(tr->ctx->mu);
    Object *ob = nullptr;
    if ((st = find(tr, ob))) return st;
    DeviceGuard guard(tr->ctx->device);
    return grads(tr, *ob, d_rays, d_gt, n, d_loss, static_cast<hipStream_t>(stream));
}

lsnif_status lsnif_train_apply(lsnif_trainer *tr, void *stream)
{
    if (!tr) return fail(LSNIF_E_INVALID, "trainer is NULL");
    std::lock_guard<std::recursive_mutex> lk(tr->ctx->mu);
    Object *ob = nullptr;
    lsnif_status st = find(tr, ob);
    if (st) return st;
    DeviceGuard guard(tr->ctx->device);
    return apply(tr, *ob, static_cast<hipStream_t>(stream));
}

lsnif_status lsnif_train_step(lsnif_trainer *tr, const lsnif_ray *d_rays, const lsnif_train_target *d_gt, uint32_t n,
                              float *d_loss, void *stream)
{
    if (!tr) return fail(LSNIF_E_INVALID, "trainer is NULL");
    lsnif_status st = check_batch(d_rays, d_gt, n);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(tr->ctx->mu);
    Object *ob = nullptr;
    if ((st = find(tr, ob))) return st;
    DeviceGuard guard(tr->ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = grads(tr, *ob, d_rays, d_gt, n, d_loss, s))) return st;
    return apply(tr, *ob, s);
}

lsnif_status lsnif_train_profile_read(lsnif_trainer *tr, double *products_ms, double *scatter_ms, uint32_t *steps)
{
    if (!tr) return fail(LSNIF_E_INVALID, "trainer is NULL");
    std::lock_guard<std::recursive_mutex> lk(tr->ctx->mu);
    DeviceGuard guard(tr->ctx->device);
    double prod = 0.0, scat = 0.0;
    lsnif_status st = LSNIF_OK;
    for (auto &v : tr->prof) {
        float a = 0.0f, b = 0.0f, c = 0.0f;
        if (!st && (hipEventSynchronize(v[5]) != hipSuccess || hipEventElapsedTime(&a, v[0], v[1]) != hipSuccess ||
                    hipEventElapsedTime(&b, v[2], v[3]) != hipSuccess ||
                    hipEventElapsedTime(&c, v[4], v[5]) != hipSuccess))
            st = fail(LSNIF_E_DEVICE, "reading the training step's events failed");
        prod += (double)a + (double)b;
        scat += c;
        for (hipEvent_t e : v) tr->spare.push_back(e);
    }
    if (steps) *steps = (uint32_t)tr->prof.size();
    tr->prof.clear();
    if (products_ms) *products_ms = prod;
    if (scatter_ms) *scatter_ms = scat;
    return st;
}

lsnif_status lsnif_trainer_read(lsnif_trainer *tr, float *tables, float *const *W, float *grad_tables,
                                float *const *grad_W, uint64_t *steps)
{
    if (!tr) return fail(LSNIF_E_INVALID, "trainer is NULL");
    std::lock_guard<std::recursive_mutex> lk(tr->ctx->mu);
    Object *ob = nullptr;
    lsnif_status st = find(tr, ob);
    if (st) return st;
    DeviceGuard guard(tr->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    if (tables) HIP_TRY(hipMemcpy(tables, ob->d_tab, tr->n_tab * 4, hipMemcpyDeviceToHost));
    if (grad_tables) HIP_TRY(hipMemcpy(grad_tables, tr->grad, tr->n_tab * 4, hipMemcpyDeviceToHost));
    const Mlp &mlp = ob->mlp;
    const int nh = mlp.n_hidden, Wd = ob->width, in0 = ob->geom.H * ob->geom.L * ob->geom.F;
    std::vector<float> packed(tr->n_w);
    for (int which = 0; which < 2; ++which) {
        float *const *dst = which ? grad_W : W;
        if (!dst) continue;
        const void *src = which ? static_cast<const void *>(tr->grad + tr->copies * tr->n_tab) : ob->d_w;
        HIP_TRY(hipMemcpy(packed.data(), src, tr->n_w * 4, hipMemcpyDeviceToHost));
        for (int k = 0; k <= nh; ++k) {
            if (!dst[k]) continue;
            const int ni = k == 0 ? in0 : Wd, no = k == nh ? mlp.out_dim : Wd, ldk = k == nh ? kMaxOut : Wd;
            const float *p = packed.data() + mlp.off[k];
            for (int j = 0; j < no; ++j)
                for (int i = 0; i < ni; ++i) dst[k][(size_t)j * ni + i] = p[(size_t)i * ldk + j];
        }
    }
    if (steps) *steps = tr->steps;
    return LSNIF_OK;
}

}  // extern "C"
