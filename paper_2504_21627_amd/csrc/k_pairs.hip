// Instanced pair queries: the work list and the nearest-hit update.
//
// Before the query kernel, the (ray, instance) pairs are grouped by object
// and, within an object, by direction octant and the cell (2^b per axis,
// b <= 4 chosen per object) of the segment start in that object's voxel grid (a counting sort with wave-aggregated
// atomics).  Each object's run is padded to whole 256-slot tiles, so every
// workgroup of the query kernel serves one object with one set of weights.
// Pairs whose ray misses the object's box, or that name a ray, instance or
// object that does not exist, are dropped here.
//
// The query kernel stores each pair's result and folds its hit into a 64-bit
// key per ray, (order-preserving bits of t) << 32 | instance, with atomicMin;
// afterwards the pair whose key equals the ray's minimum writes the payload,
// with the normal taken back to world space.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"
#include "lsnif_pairs.hpp"

namespace lsnif {

__global__ __launch_bounds__(kBlock) void k_pairs_init(PairPlan P)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= P.n_rays) return;
    P.minkey[r] = ~0ull;
    lsnif_hit h;
    h.hit = 0;
    h.t = __builtin_inff();
    h.n[0] = h.n[1] = h.n[2] = 0.0f;
    h.material = -1;
    P.out[r] = h;
}

__global__ __launch_bounds__(kBlock) void k_pairs_fill(PairPlan P)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < P.n_objs * kPairBins) P.hist[i] = 0u;
    if (i < P.n_slots) P.slot_pair[i] = 0xffffffffu;
    if (i < P.n_tiles) P.tile_obj[i] = -1;
}

__device__ __forceinline__ uint32_t spread4(uint32_t x)
{
    x &= 15u;
    return (x & 1u) | ((x & 2u) << 2) | ((x & 4u) << 4) | ((x & 8u) << 6);
}

__global__ __launch_bounds__(kBlock) void k_pairs_keys(PairPlan P)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    uint32_t bin = 0xffffffffu;
    if (p < P.n_pairs) {
        const uint32_t r = P.pair_ray[p], i = P.pair_inst[p];
        if (r < P.n_rays && i < P.n_inst) {
            const uint32_t o = P.inst[i].object_id;
            if (o < P.n_objs && P.objs[o].live) {
                const Geom &g = P.objs[o].g;
                float4 ra = P.rays[2 * r], rb = P.rays[2 * r + 1];
                to_object_space(P.inst[i], ra, rb);
                VRay w;
                setup_ray(g, ra, rb, w);
                if (w.cand) {
                    uint32_t c[3];
                    const float cells = (float)(1u << g.pair_bits);
                    const float sc = cells / (float)g.V;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        float x = (w.o[a] + w.ta * w.d[a]) * sc;
                        x = x < 0.0f ? 0.0f : (x > cells - 1.0f ? cells - 1.0f : x);
                        c[a] = (uint32_t)x;
                    }
                    const uint32_t oct = (w.d[0] < 0.0f ? 1u : 0u) | (w.d[1] < 0.0f ? 2u : 0u) |
                                         (w.d[2] < 0.0f ? 4u : 0u);
                    bin = o * kPairBins + ((oct << 12) | spread4(c[0]) | (spread4(c[1]) << 1) | (spread4(c[2]) << 2));
                }
            }
        }
        P.keys[p] = bin;
    }
    (void)wave_aggregated_add(P.hist, bin, bin != 0xffffffffu);
}

// Block o: exclusive scan of object o's kPairBins counters in place; total to obj_total[o].
__global__ __launch_bounds__(kBlock) void k_pairs_scan_obj(PairPlan P)
{
    __shared__ uint32_t tmp[kBlock];
    constexpr uint32_t per = kPairBins / kBlock;
    uint32_t *h = P.hist + (size_t)blockIdx.x * kPairBins;
    const uint32_t t = threadIdx.x;
    uint32_t v[per], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < per; ++q) {
        v[q] = h[t * per + q];
        sum += v[q];
    }
    tmp[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kBlock; off <<= 1) {
        const uint32_t u = t >= off ? tmp[t - off] : 0u;
        __syncthreads();
        tmp[t] += u;
        __syncthreads();
    }
    uint32_t run = tmp[t] - sum;
    if (t == kBlock - 1) P.obj_total[blockIdx.x] = tmp[t];
#pragma unroll
    for (uint32_t q = 0; q < per; ++q) {
        h[t * per + q] = run;
        run += v[q];
    }
}

// One block: object runs padded to whole tiles, their offsets, and each tile's object.
__global__ __launch_bounds__(kBlock) void k_pairs_offsets(PairPlan P)
{
    __shared__ uint32_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (uint32_t o = 0; o < P.n_objs; ++o) {
        const uint32_t padded = (P.obj_total[o] + kBlock - 1) / kBlock * kBlock;
        const uint32_t b = base;
        if (threadIdx.x == 0) P.obj_off[o] = b;
        for (uint32_t t = threadIdx.x; t < padded / kBlock; t += kBlock) P.tile_obj[b / kBlock + t] = (int32_t)o;
        __syncthreads();
        if (threadIdx.x == 0) base = b + padded;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_pairs_scatter(PairPlan P)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t bin = p < P.n_pairs ? P.keys[p] : 0xffffffffu;
    const bool live = bin != 0xffffffffu;
    const uint32_t within = wave_aggregated_add(P.hist, bin, live);
    if (live) P.slot_pair[P.obj_off[bin / kPairBins] + within] = p;
}

__global__ __launch_bounds__(kBlock) void k_pairs_payload(PairPlan P)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= P.n_pairs || P.keys[p] == 0xffffffffu) return;
    const PairRes res = P.res[p];
    if (!(res.t <= 3.402823466e38f)) return;
    const uint32_t r = P.pair_ray[p], i = P.pair_inst[p];
    const unsigned long long key = ((unsigned long long)ordered_bits(res.t) << 32) | (unsigned long long)i;
    if (key != P.minkey[r]) return;
    const float *m = P.inst[i].world_to_object;
    double wn[3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
        wn[b] = (double)m[b] * res.n[0] + (double)m[4 + b] * res.n[1] + (double)m[8 + b] * res.n[2];
    const double nn = sqrt(wn[0] * wn[0] + wn[1] * wn[1] + wn[2] * wn[2]);
    lsnif_hit h;
    h.hit = 1;
    h.t = res.t;
#pragma unroll
    for (int b = 0; b < 3; ++b) h.n[b] = nn > 0.0 ? (float)(wn[b] / nn) : 0.0f;
    h.material = res.material;
    P.out[r] = h;
}

hipError_t launch_pairs_prepare(const PairPlan &P, hipStream_t s)
{
    const uint32_t nfill = P.n_objs * kPairBins > P.n_slots ? P.n_objs * kPairBins : P.n_slots;
    hipLaunchKernelGGL(k_pairs_init, dim3((P.n_rays + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_fill, dim3((nfill + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    if (P.n_pairs == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_pairs_keys, dim3((P.n_pairs + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_scan_obj, dim3(P.n_objs), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_offsets, dim3(1), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_scatter, dim3((P.n_pairs + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_pairs_payload(const PairPlan &P, hipStream_t s)
{
    if (P.n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_payload, dim3((P.n_pairs + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

}  // namespace lsnif
