// Coherence order of a ray batch: a one-pass counting sort of the rays by a
// coarse key -- direction octant, then the Morton code of the cell (2^b per
// axis, b <= 6 chosen per object) of the voxel grid where the ray's segment
// [ta, tb] starts; at b = 7 (128^3 cells) the cell alone, without the
// octant.  Rays that meet the
// grid close together and head the same way then share waves, so their
// walks and their hash-grid gathers touch the same cache lines.  Order within
// a key is whatever the atomics give; every ray's result is independent of
// the order the rays are processed in.
#include <map>
#include <mutex>
#include <tuple>

#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

// Bits 0..6 of x spread to bits 0, 3, 6, ..., 18 (one axis of a 3-D Morton code).
__device__ __forceinline__ uint32_t spread7(uint32_t x)
{
    x &= 127u;
    x = (x | (x << 8)) & 0x0000f00fu;
    x = (x | (x << 4)) & 0x000c30c3u;
    x = (x | (x << 2)) & 0x00249249u;
    return x;
}


__device__ __forceinline__ uint32_t coherence_key(const Geom &g, float4 r0, float4 r1)
{
    VRay w;
    setup_ray(g, r0, r1, w);
    if (!w.cand) return sort_bins(g.sort_bits) - 1;
    uint32_t cell[3];
    const float cells = (float)(1u << g.sort_bits);
    const float sc = cells / (float)g.V;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float x = (w.o[a] + w.ta * w.d[a]) * sc;
        x = x < 0.0f ? 0.0f : (x > cells - 1.0f ? cells - 1.0f : x);
        cell[a] = (uint32_t)x;
    }
    const uint32_t morton = spread7(cell[0]) | (spread7(cell[1]) << 1) | (spread7(cell[2]) << 2);
    if (g.sort_bits >= 7u) return morton;
    const uint32_t oct = (w.d[0] < 0.0f ? 1u : 0u) | (w.d[1] < 0.0f ? 2u : 0u) | (w.d[2] < 0.0f ? 4u : 0u);
    return (oct << (3u * g.sort_bits)) | morton;
}

__global__ __launch_bounds__(kBlock) void k_fill(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_sort_keys(Geom g, const float4 *rays, uint32_t n, uint32_t *keys,
                                                      uint32_t *hist)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < n;
    uint32_t k = 0;
    if (live) {
        k = coherence_key(g, rays[2 * i], rays[2 * i + 1]);
        keys[i] = k;
    }
    (void)wave_aggregated_add(hist, k, live);
}

// Exclusive scan of the kSortBins counters in two passes: block b first sums
// counters [1024 b, 1024 b + 1024), then rescans them with the sum of the
// blocks before it as the carry-in.
constexpr uint32_t kScanChunk = 1024;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t &total)
{
    // 256 threads: inclusive scan in LDS (Hillis-Steele), then exclusive value
    const uint32_t t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < kBlock; off <<= 1) {
        const uint32_t u = t >= off ? tmp[t - off] : 0u;
        __syncthreads();
        tmp[t] += u;
        __syncthreads();
    }
    total = tmp[kBlock - 1];
    const uint32_t incl = tmp[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_partial(const uint32_t *hist, uint32_t nbins, uint32_t *part)
{
    __shared__ uint32_t tmp[kBlock];
    const uint32_t b0 = blockIdx.x * kScanChunk;
    uint32_t v = 0;
#pragma unroll
    for (uint32_t q = 0; q < kScanChunk / kBlock; ++q) {
        const uint32_t i = b0 + q * kBlock + threadIdx.x;
        if (i < nbins) v += hist[i];
    }
    uint32_t total;
    (void)block_exclusive_scan(v, tmp, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_final(uint32_t *hist, uint32_t nbins, const uint32_t *part)
{
    __shared__ uint32_t tmp[kBlock];
    const uint32_t t = threadIdx.x;
    // carry-in: sum of the partial sums of the blocks before this one
    uint32_t c = 0;
    for (uint32_t j = t; j < blockIdx.x; j += kBlock) c += part[j];
    uint32_t carry;
    (void)block_exclusive_scan(c, tmp, carry);
    // each thread scans 4 consecutive counters
    const uint32_t i0 = blockIdx.x * kScanChunk + 4 * t;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = i0 + q < nbins ? hist[i0 + q] : 0u;
        sum += v[q];
    }
    uint32_t total;
    uint32_t run = carry + block_exclusive_scan(sum, tmp, total);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (i0 + q < nbins) hist[i0 + q] = run;
        run += v[q];
    }
}

// kScatterPer rays per thread (rays blockIdx kBlock kScatterPer + j kBlock +
// threadIdx), their counter atomics all in flight before the first position is
// used (c2: 109 -> 78 us).
constexpr uint32_t kScatterPer = 4;

__global__ __launch_bounds__(kBlock) void k_sort_scatter(const uint32_t *keys, uint32_t n, uint32_t *cursor,
                                                         uint32_t *order)
{
    const uint32_t i0 = blockIdx.x * kBlock * kScatterPer + threadIdx.x;
    AggAdd a[kScatterPer];
#pragma unroll
    for (uint32_t j = 0; j < kScatterPer; ++j) {
        const uint32_t i = i0 + j * kBlock;
        const bool live = i < n;
        a[j] = wave_aggregated_issue(cursor, live ? keys[i] : 0u, live);
    }
#pragma unroll
    for (uint32_t j = 0; j < kScatterPer; ++j) {
        const uint32_t i = i0 + j * kBlock;
        const uint32_t pos = wave_aggregated_rank(a[j]);
        if (i < n) order[pos] = i;
    }
}

hipError_t launch_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *part, hipStream_t s)
{
    const uint32_t nblocks = (n + kScanChunk - 1) / kScanChunk;
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_scan_partial, dim3(nblocks), dim3(kBlock), 0, s, v, n, part);
    hipLaunchKernelGGL(k_scan_final, dim3(nblocks), dim3(kBlock), 0, s, v, n, part);
    return hipGetLastError();
}

__global__ void k_clear_queue(unsigned long long *q)
{
    if (threadIdx.x < 8) q[threadIdx.x] = 0ull;
}

hipError_t launch_clear_queue(unsigned long long *q, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_queue, dim3(1), dim3(64), 0, s, q);
    return hipGetLastError();
}

uint32_t persistent_blocks(const void *kernel, size_t lds, uint32_t tiles)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, uint32_t> known;
    int dev = 0;
    (void)hipGetDevice(&dev);
    uint32_t nb = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find({dev, kernel, lds});
        if (it != known.end()) nb = it->second;
    }
    if (!nb) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess) per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 8;
        nb = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 8);
        nb = nb < 8 ? 8 : nb / 8 * 8;
        std::lock_guard<std::mutex> lk(mu);
        known[{dev, kernel, lds}] = nb;
    }
    const uint32_t want = (tiles + 7u) / 8u * 8u;
    return want < nb ? (want ? want : 8u) : nb;
}

hipError_t launch_coherence_sort(const Geom &g, const float4 *rays, uint32_t n, uint32_t *keys, uint32_t *hist,
                                 uint32_t *order, hipStream_t s)
{
    // the workspace holds this resolution's bins, then one partial sum per 1024 bins
    const uint32_t nbins = sort_bins(g.sort_bits), nblocks = sort_scan_blocks(g.sort_bits);
    const dim3 gb((nbins + kBlock - 1) / kBlock), gr((n + kBlock - 1) / kBlock);
    const dim3 gj((n + kBlock * kScatterPer - 1) / (kBlock * kScatterPer));
    uint32_t *part = hist + nbins;
    hipLaunchKernelGGL(k_fill, gb, dim3(kBlock), 0, s, hist, nbins, 0u);
    hipLaunchKernelGGL(k_sort_keys, gr, dim3(kBlock), 0, s, g, rays, n, keys, hist);
    hipLaunchKernelGGL(k_scan_partial, dim3(nblocks), dim3(kBlock), 0, s, hist, nbins, part);
    hipLaunchKernelGGL(k_scan_final, dim3(nblocks), dim3(kBlock), 0, s, hist, nbins, part);
    hipLaunchKernelGGL(k_sort_scatter, gj, dim3(kBlock), 0, s, keys, n, hist, order);
    return hipGetLastError();
}

}  // namespace lsnif
