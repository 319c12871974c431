// Instanced pair queries: the work list and the nearest-hit update.
//
// Before the query kernel, the (ray, instance) pairs are grouped by object
// and, within an object, by direction octant and the cell (2^b per axis,
// b <= 5 chosen per object) of the segment start in that object's voxel grid,
// or at b = 6 by the cell alone (64 per axis): a key per pair, object-major,
// put in order by the radix passes of the coherence sort (stable, so pairs
// of one key keep their given order).  The sorted keys give each object's
// first position; each object's run is then padded to whole 256-slot tiles,
// so every workgroup of the query kernel serves one object with one set of
// weights.
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

// Block b: the keys of pairs [kRadixTile b, kRadixTile (b + 1)) -- object o's keys are
// o bins + (octant, cell) bin; a dropped pair's is n_objs bins, after every object --
// and the count of each value of their lowest digit, to hist[digit nblk + b].
__global__ __launch_bounds__(kBlock) void k_pairs_keys(PairPlan P, uint32_t nblk)
{
    __shared__ uint32_t cnt[256];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    cnt[t] = 0u;
    __syncthreads();
    for (uint32_t j = 0; j < kRadixTile / kBlock; ++j) {
        const uint32_t p = b * kRadixTile + j * kBlock + t;
        if (p >= P.n_pairs) continue;
        uint32_t bin = P.n_objs * P.bins;
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
        atomicAdd(&cnt[bin & 255u], 1u);
    }
    __syncthreads();
    P.hist[(size_t)t * nblk + b] = cnt[t];
}

// Sorted position i (of n): where the objects between its predecessor's and its own
// start; the last position also closes the objects after its own.  sk: sorted keys.
__global__ __launch_bounds__(kBlock) void k_pairs_bounds(PairPlan P, const uint32_t *sk)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= P.n_pairs) return;
    const uint32_t sh = (uint32_t)__builtin_ctz(P.bins);
    const uint32_t o = min(sk[i] >> sh, P.n_objs);
    const uint32_t from = i ? min(sk[i - 1] >> sh, P.n_objs) + 1u : 0u;
    for (uint32_t q = from; q <= o; ++q) P.obj_start[q] = i;
    if (i + 1 == P.n_pairs)
        for (uint32_t q = o + 1; q <= P.n_objs; ++q) P.obj_start[q] = P.n_pairs;
}

// One block: object runs padded to whole tiles, their offsets, and each tile's object.
__global__ __launch_bounds__(kBlock) void k_pairs_offsets(PairPlan P)
{
    __shared__ uint32_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (uint32_t o = 0; o < P.n_objs; ++o) {
        const uint32_t total = P.obj_start[o + 1] - P.obj_start[o];
        const uint32_t padded = (total + kBlock - 1) / kBlock * kBlock;
        const uint32_t b = base;
        if (threadIdx.x == 0) P.obj_off[o] = b;
        for (uint32_t t = threadIdx.x; t < padded / kBlock; t += kBlock) P.tile_obj[b / kBlock + t] = (int32_t)o;
        __syncthreads();
        if (threadIdx.x == 0) base = b + padded;
        __syncthreads();
    }
}

// Sorted position i: its pair into its object's next slot.  sk, sv: sorted keys and pairs.
__global__ __launch_bounds__(kBlock) void k_pairs_place(PairPlan P, const uint32_t *sk, const uint32_t *sv)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= P.obj_start[P.n_objs]) return;   // the dropped pairs sort last
    const uint32_t o = sk[i] >> (uint32_t)__builtin_ctz(P.bins);
    const uint32_t slot = P.obj_off[o] + (i - P.obj_start[o]);
    if (slot < P.n_slots) P.slot_pair[slot] = sv[i];
}

__global__ __launch_bounds__(kBlock) void k_pairs_payload(PairPlan P)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= P.n_pairs || P.keys[p] >= P.n_objs * P.bins) return;   // dropped
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
    hipLaunchKernelGGL(k_pairs_init, dim3((P.n_rays + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_fill, dim3((P.n_slots + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    if (P.n_pairs == 0) return hipGetLastError();
    const uint32_t nblk = (P.n_pairs + kRadixTile - 1) / kRadixTile, grid = (P.n_pairs + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_pairs_keys, dim3(nblk), dim3(kBlock), 0, s, P, nblk);
    // passes enough for the dropped pairs' key, n_objs bins
    const uint32_t top = P.n_objs * P.bins, passes = (32u - (uint32_t)__builtin_clz(top | 1u) + 7u) / 8u;
    const uint32_t *sk = P.keys, *sv = nullptr;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t *dk = P.rk[p & 1u], *dv = P.rv[p & 1u];
        const hipError_t e = launch_radix_pass(sk, sv, dk, dv, P.n_pairs, P.hist, 8u * p, p == 0, s);
        if (e != hipSuccess) return e;
        sk = dk;
        sv = dv;
    }
    hipLaunchKernelGGL(k_pairs_bounds, dim3(grid), dim3(kBlock), 0, s, P, sk);
    hipLaunchKernelGGL(k_pairs_offsets, dim3(1), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_pairs_place, dim3(grid), dim3(kBlock), 0, s, P, sk, sv);
    return hipGetLastError();
}

hipError_t launch_pairs_payload(const PairPlan &P, hipStream_t s)
{
    if (P.n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_payload, dim3((P.n_pairs + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

}  // namespace lsnif
