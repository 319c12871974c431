// Kernel launchers shared between the host runtime and the kernel units.
#pragma once
#include <hip/hip_runtime.h>

namespace lsnif {
constexpr uint32_t kSortBins = (1u << 18) + 1;   // 8 octants x 32^3 cells, plus one bin for rays that miss
constexpr uint32_t kSortScanBlocks = (kSortBins + 1023) / 1024;   // partial sums of the two-pass scan
struct Geom;
struct QueryArgs;
struct DebugArgs;
// Query kernels: `grid` blocks of 256 lanes; `pairs` selects the instanced-pair variant.
hipError_t launch_f32(const QueryArgs &A, int feat_dtype, int F, bool pairs, uint32_t grid, hipStream_t s);
hipError_t launch_mma_f16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                          hipStream_t s);
hipError_t launch_mma_bf16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                           hipStream_t s);
hipError_t launch_mma_fp8(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                          hipStream_t s);
hipError_t launch_debug(const DebugArgs &D, hipStream_t s);
struct PairPlan;
hipError_t launch_pairs_prepare(const PairPlan &P, hipStream_t s);
hipError_t launch_pairs_payload(const PairPlan &P, hipStream_t s);
hipError_t launch_coherence_sort(const Geom &g, const float4 *rays, uint32_t n, uint32_t *keys, uint32_t *hist,
                                 uint32_t *order, hipStream_t s);
}  // namespace lsnif
