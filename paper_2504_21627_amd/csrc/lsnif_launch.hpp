// Kernel launchers shared between the host runtime and the kernel units.
#pragma once
#include <hip/hip_runtime.h>

namespace lsnif {
// Keys of a coherence sort with 2^bits cells per axis: 8 octants x cells^3 (bits <= 6) or
// cells^3 alone (bits 7), then one for misses.
__host__ __device__ inline uint32_t sort_bins(uint32_t bits)
{
    return bits >= 7u ? (1u << 21) + 1u : (8u << (3u * bits)) + 1u;
}
// The coherence keys are put in order by a least-significant-digit radix sort with 8-bit
// digits, each block of the passes taking kRadixTile consecutive rays: passes enough
// for the largest key (sort_bins(bits) - 1), and the 32-bit words of its workspace for n
// rays -- keys and ray indices twice (the passes alternate between the two copies), then
// a counter per (digit, block) of a pass and the partial sums of their scan.
constexpr uint32_t kRadixTile = 2048;
__host__ __device__ inline uint32_t radix_passes(uint32_t bits)
{
    const uint32_t top = sort_bins(bits) - 1u;
    const uint32_t used = 32u - (uint32_t)__builtin_clz(top | 1u);
    return (used + 7u) / 8u;
}
// Digit counters of a pass over n items, then the partial sums of their scan.
__host__ __device__ inline size_t radix_hist_words(uint32_t n)
{
    const size_t counters = (size_t)256u * ((n + kRadixTile - 1u) / kRadixTile);
    return counters + (counters + 1023u) / 1024u;
}
__host__ __device__ inline size_t radix_ws_words(uint32_t n) { return 4u * (size_t)n + radix_hist_words(n); }
struct Geom;
struct QueryArgs;
struct DebugArgs;
// Query kernels: `grid` blocks of 256 lanes; `pairs` selects the instanced-pair variant.
hipError_t launch_f32(const QueryArgs &A, int feat_dtype, int F, bool pairs, uint32_t grid, hipStream_t s);
// One wave per ray (FP32 features and MLP, width 64, F <= 3, at most 16 levels), for `grid`
// tiles' slots starting at tile A.tile0.
hipError_t launch_lat(const QueryArgs &A, int F, uint32_t grid, hipStream_t s);
// The same with the MLP on the matrix cores (two features per level, at most two K blocks).
hipError_t launch_mma_small_f16(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s);
hipError_t launch_mma_small_bf16(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s);
hipError_t launch_mma_small_fp8(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s);
hipError_t launch_mma_f16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                          hipStream_t s);
hipError_t launch_mma_bf16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                           hipStream_t s);
hipError_t launch_mma_fp8(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                          hipStream_t s);
// Voxel walk of every slot into A.lists / A.nvox, before the query kernel of the same `grid`;
// `recheck` when some object of the launch re-decides grazing voxels in float64.
hipError_t launch_walk(const QueryArgs &A, bool pairs, bool recheck, uint32_t grid, hipStream_t s);
hipError_t launch_debug(const DebugArgs &D, hipStream_t s);
// Gather ceiling: the query's gathers alone, each ray's feature sum into sums[r].
hipError_t launch_gather_only(const QueryArgs &A, int feat_dtype, int F, float *sums, uint32_t grid, hipStream_t s);
// Broad phase: pairs per ray into B.offsets (and 0 at offsets[n_rays]), then, after an
// exclusive scan of the n_rays + 1 counters, the pairs themselves.
struct BroadArgs;
hipError_t launch_broad_count(const BroadArgs &B, hipStream_t s);
hipError_t launch_broad_write(const BroadArgs &B, hipStream_t s);
// Bounce rays: 1 per hit into B.offsets (and 0 at offsets[n]); after their exclusive scan,
// the new rays and their parents.
struct BounceArgs;
hipError_t launch_bounce_mark(const BounceArgs &B, hipStream_t s);
hipError_t launch_bounce_write(const BounceArgs &B, hipStream_t s);
// Persistent query kernels: zero the 8 tile-queue counters at q (one 256-byte granule),
// and the grid for `kernel` with `lds` dynamic bytes: as many blocks as the chip holds at
// once (a multiple of 8, one per XCD in turn), at most the launch's tiles rounded up to 8.
hipError_t launch_clear_queue(unsigned long long *q, hipStream_t s);
uint32_t persistent_blocks(const void *kernel, size_t lds, uint32_t tiles);
// In-place exclusive scan of n counters; `part` holds (n + 1023) / 1024 partial sums.
hipError_t launch_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *part, hipStream_t s);
// Merged serving launches: stage the members' rays and re-indexed pairs, and copy the
// staged answers back to each member's output.
struct MergeArgs;
hipError_t launch_merge_pack(const MergeArgs &M, hipStream_t s);
hipError_t launch_merge_unpack(const MergeArgs &M, hipStream_t s);
struct PairPlan;
hipError_t launch_pairs_prepare(const PairPlan &P, hipStream_t s);
hipError_t launch_pairs_payload(const PairPlan &P, hipStream_t s);
// One pass of the radix sort (8-bit digit at `shift`, stable) over n items of (sk, sv)
// into (dk, dv): sv NULL means the values are the positions 0..n-1, dk NULL that the
// keys are not kept.  hist holds 256 counters per kRadixTile items and then the
// partial sums of their scan; counted: they already hold this pass's per-block counts.
hipError_t launch_radix_pass(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv, uint32_t n,
                             uint32_t *hist, uint32_t shift, bool counted, hipStream_t s);
// Sorts rays 0..n-1 by coherence key in `ws` (radix_ws_words(n) words);
// *order receives the sorted ray indices (inside ws).
hipError_t launch_coherence_sort(const Geom &g, const float4 *rays, uint32_t n, uint32_t *ws, uint32_t **order,
                                 hipStream_t s);
}  // namespace lsnif
