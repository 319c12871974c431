// Coherence order of a ray batch: the rays sorted by a coarse key --
// direction octant, then the Morton code of the cell (2^b per axis, b <= 6
// chosen per object) of the voxel grid where the ray's segment [ta, tb]
// starts; at b = 7 (128^3 cells) the cell alone, without the octant.  Rays
// that meet the grid close together and head the same way then share waves,
// so their walks and their hash-grid gathers touch the same cache lines.
//
// The sort is a least-significant-digit radix sort with 8-bit digits (three
// passes for the largest keys).  Each pass counts the digit per block of
// kRadixTile consecutive rays of its input (the first pass while forming the
// keys) in LDS, scans the counters digit-major, which gives every (digit,
// block) its output range, then ranks each block's rays stably (a wave
// matches equal digits with one ballot per digit bit and keeps running counts
// per digit in LDS) and writes them there.  No global atomics: a counting
// sort's histogram and scatter take one device-wide atomic per ray, and those
// atomics, not the bytes moved, set its pace.
// Every ray's result is independent of the order the rays are processed in.
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

constexpr uint32_t kRadixPer = kRadixTile / kBlock;   // items per thread in a block of the passes
constexpr uint32_t kRadixMaxPasses = 3;                 // coherence keys of at most 24 bits

// Block b: the coherence keys of rays [kRadixTile b, kRadixTile (b + 1)), and the
// count of each value of their lowest digit, to hist[digit nblk + b].
__global__ __launch_bounds__(kBlock) void k_radix_keys(Geom g, const float4 *rays, uint32_t n, uint32_t *keys,
                                                       uint32_t *hist, uint32_t nblk)
{
    __shared__ uint32_t cnt[256];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    cnt[t] = 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kRadixPer; ++j) {
        const uint32_t i = b * kRadixTile + j * kBlock + t;
        if (i < n) {
            const uint32_t k = coherence_key(g, rays[2 * i], rays[2 * i + 1]);
            keys[i] = k;
            atomicAdd(&cnt[k & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)t * nblk + b] = cnt[t];
}

// Block b: the count of each value of the digit at `shift` among keys
// [kRadixTile b, kRadixTile (b + 1)), to hist[digit nblk + b].
__global__ __launch_bounds__(kBlock) void k_radix_count(const uint32_t *sk, uint32_t n, uint32_t *hist,
                                                        uint32_t nblk, uint32_t shift)
{
    __shared__ uint32_t cnt[256];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    cnt[t] = 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kRadixPer; ++j) {
        const uint32_t i = b * kRadixTile + j * kBlock + t;
        if (i < n) atomicAdd(&cnt[(sk[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)t * nblk + b] = cnt[t];
}

// One pass: block b moves rays [kRadixTile b, kRadixTile (b + 1)) of (sk, sv) to
// their places in (dk, dv) by the digit at `shift`, keeping their order within a
// digit.  off: the exclusive scan of this pass's counters (digit-major), less
// `base`.  sv NULL: the indices are the positions;
// dk NULL: the keys are not needed after this pass.  Wave w takes rays
// 512 w .. 512 w + 511 of the block, 64 at a time, so (wave, step, lane) is
// the rays' order.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t *sk, const uint32_t *sv, uint32_t *dk,
                                                          uint32_t *dv, uint32_t n, const uint32_t *off,
                                                          uint32_t nblk, uint32_t shift, uint32_t base)
{
    __shared__ uint32_t run[kBlock / 64][256];   // per wave: rays of each digit so far, then the wave's start
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6, b = blockIdx.x;
    for (uint32_t i = t; i < (kBlock / 64) * 256u; i += kBlock) (&run[0][0])[i] = 0u;
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64u - lane)) : 0ull;
    uint32_t key[kRadixPer], val[kRadixPer], pos[kRadixPer];
#pragma unroll
    for (uint32_t j = 0; j < kRadixPer; ++j) {
        const uint32_t i = b * kRadixTile + w * (kRadixTile / 4u) + j * 64u + lane;
        const bool live = i < n;
        key[j] = live ? sk[i] : 0u;
        val[j] = live ? (sv ? sv[i] : i) : 0u;
        const uint32_t d = (key[j] >> shift) & 255u;
        // lanes holding this lane's digit: one ballot per digit bit
        uint64_t same = __ballot(live);
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
            const uint64_t ones = __ballot((d >> q) & 1u);
            same &= ((d >> q) & 1u) ? ones : ~ones;
        }
        const uint32_t before = run[w][d];
        pos[j] = before + (uint32_t)__builtin_popcountll(same & below);
        if (live && (same & below) == 0ull) run[w][d] = before + (uint32_t)__builtin_popcountll(same);
    }
    __syncthreads();
    {   // thread t = digit t: the start of each wave's rays of that digit
        uint32_t at = off[(size_t)t * nblk + b] - base;
#pragma unroll
        for (uint32_t q = 0; q < kBlock / 64; ++q) {
            const uint32_t c = run[q][t];
            run[q][t] = at;
            at += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kRadixPer; ++j) {
        const uint32_t i = b * kRadixTile + w * (kRadixTile / 4u) + j * 64u + lane;
        const uint32_t dst = run[w][(key[j] >> shift) & 255u] + pos[j];
        if (i < n && dst < n) {
            if (dk) dk[dst] = key[j];
            dv[dst] = val[j];
        }
    }
}

// Exclusive scan of n counters in two passes: block b first sums counters
// [1024 b, 1024 b + 1024), then rescans them with the sum of the blocks before
// it as the carry-in.
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

hipError_t launch_radix_pass(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv, uint32_t n,
                             uint32_t *hist, uint32_t shift, bool counted, hipStream_t s)
{
    static_assert(kRadixTile == 4u * 512u && kBlock == 256u, "a block of the passes is 4 waves of 8 x 64 items");
    const uint32_t nblk = (n + kRadixTile - 1) / kRadixTile, counters = 256u * nblk;
    if (!nblk) return hipSuccess;
    if (!counted) hipLaunchKernelGGL(k_radix_count, dim3(nblk), dim3(kBlock), 0, s, sk, n, hist, nblk, shift);
    const hipError_t e = launch_exclusive_scan(hist, counters, hist + counters, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kBlock), 0, s, sk, sv, dk, dv, n, hist, nblk, shift, 0u);
    return hipGetLastError();
}

hipError_t launch_coherence_sort(const Geom &g, const float4 *rays, uint32_t n, uint32_t *ws, uint32_t **order,
                                 hipStream_t s)
{
    const uint32_t passes = radix_passes(g.sort_bits), nblk = (n + kRadixTile - 1) / kRadixTile;
    if (passes > kRadixMaxPasses) return hipErrorInvalidValue;
    uint32_t *k0 = ws, *v0 = k0 + n, *k1 = v0 + n, *v1 = k1 + n, *hist = v1 + n;
    hipLaunchKernelGGL(k_radix_keys, dim3(nblk), dim3(kBlock), 0, s, g, rays, n, k0, hist, nblk);
    const uint32_t *sk = k0, *sv = nullptr;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t *dk = (p & 1u) ? k0 : k1, *dv = (p & 1u) ? v0 : v1;
        const hipError_t e = launch_radix_pass(sk, sv, p + 1 < passes ? dk : nullptr, dv, n, hist, 8u * p, p == 0, s);
        if (e != hipSuccess) return e;
        sk = dk;
        sv = dv;
    }
    *order = const_cast<uint32_t *>(sv);
    return hipGetLastError();
}

}  // namespace lsnif
