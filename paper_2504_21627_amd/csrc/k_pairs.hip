// Instanced pair queries: the work list and the nearest-hit update.
//
// Before the query kernel, the (ray, instance) pairs are grouped by object
// and, within an object, by direction octant and the cell (2^b per axis,
// b <= 5 chosen per object) of the segment start in that object's voxel grid
// (a counting sort with wave-aggregated atomics).  Each object's run is padded to whole 256-slot tiles, so every
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
    if (i < P.n_objs * P.bins) P.hist[i] = 0u;
    if (i < P.n_slots) P.slot_pair[i] = 0xffffffffu;
    if (i < P.n_tiles) P.tile_obj[i] = -1;
}

// The low 6 bits of x spread to every third bit (one axis of a Morton code).
__device__ __forceinline__ uint32_t spread6(uint32_t x)
{
    x &= 63u;
    return (x & 1u) | ((x & 2u) << 2) | ((x & 4u) << 4) | ((x & 8u) << 6) | ((x & 16u) << 8) |
           ((x & 32u) << 10);
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
                    const uint32_t cell = spread6(c[0]) | (spread6(c[1]) << 1) | (spread6(c[2]) << 2);
                    // the octant above the object's own cell bits, none at 64 cells per axis
                    bin = o * P.bins + (g.pair_bits >= 6u ? cell : (oct << (3u * g.pair_bits)) | cell);
                }
            }
        }
        P.keys[p] = bin;
    }
    (void)wave_aggregated_add(P.hist, bin, bin != 0xffffffffu);
}

// Block o: exclusive scan of object o's P.bins counters in place, total to
// obj_total[o].  The counters go in chunks of kScanChunk (each thread 8
// consecutive, two 16-byte loads): per-thread sums, a wave scan with lane
// shuffles, the four wave totals through LDS, and a carry between chunks.
constexpr uint32_t kScanPer = 8, kScanChunk = kScanPer * kBlock;

__global__ __launch_bounds__(kBlock) void k_pairs_scan_obj(PairPlan P)
{
    __shared__ uint32_t wsum[kBlock / 64];
    uint32_t *h = P.hist + (size_t)blockIdx.x * P.bins;
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < P.bins; base += kScanChunk) {
        uint4 *p = reinterpret_cast<uint4 *>(h + base + t * kScanPer);
        const uint4 a = p[0], b = p[1];
        const uint32_t v[kScanPer] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint32_t s = 0;
#pragma unroll
        for (uint32_t q = 0; q < kScanPer; ++q) s += v[q];
        uint32_t inc = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o) inc += u;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        uint32_t run = carry + inc - s, chunk = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBlock / 64; ++k) {
            const uint32_t x = wsum[k];
            run += k < wv ? x : 0u;
            chunk += x;
        }
        __syncthreads();   // wsum is rewritten by the next chunk
        uint32_t out[kScanPer];
#pragma unroll
        for (uint32_t q = 0; q < kScanPer; ++q) {
            out[q] = run;
            run += v[q];
        }
        p[0] = make_uint4(out[0], out[1], out[2], out[3]);
        p[1] = make_uint4(out[4], out[5], out[6], out[7]);
        carry += chunk;
    }
    if (t == 0) P.obj_total[blockIdx.x] = carry;
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
    if (live) P.slot_pair[P.obj_off[bin / P.bins] + within] = p;
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
    // World normal: the object normal through the transpose of the 3x3 block of
    // world_to_object (the inverse transpose of object_to_world), renormalised.
    // float32 throughout; a few ulp of the unit normal, far inside the normal bar.
    const float *m = P.inst[i].world_to_object;
    float wn[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) wn[b] = fmaf(m[8 + b], res.n[2], fmaf(m[4 + b], res.n[1], m[b] * res.n[0]));
    const float nn2 = fmaf(wn[2], wn[2], fmaf(wn[1], wn[1], wn[0] * wn[0]));
    const float inv = nn2 > 0.0f ? 1.0f / sqrtf(nn2) : 0.0f;
    lsnif_hit h;
    h.hit = 1;
    h.t = res.t;
#pragma unroll
    for (int b = 0; b < 3; ++b) h.n[b] = wn[b] * inv;
    h.material = res.material;
    P.out[r] = h;
}

hipError_t launch_pairs_prepare(const PairPlan &P, hipStream_t s)
{
    const uint32_t nfill = P.n_objs * P.bins > P.n_slots ? P.n_objs * P.bins : P.n_slots;
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
