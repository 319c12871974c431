// The matrix-core query kernel's launcher, templated on the MLP type; each
// k_mma_*.hip unit instantiates it for one type (so the three compile in
// parallel).  Width-64 objects can run the kernel as a persistent grid with
// per-XCD tile queues (QueryArgs::persistent); width 128, the paper's default,
// runs one block per tile.
#pragma once
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <typename K>
inline void launch_tiles(K kernel, K persistent, const QueryArgs &A, uint32_t grid, size_t lds, hipStream_t s)
{
    if (!A.persistent) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), lds, s, A);
        return;
    }
    QueryArgs P = A;
    P.n_tiles = grid;
    (void)launch_clear_queue(A.queue, s);
    hipLaunchKernelGGL(persistent, dim3(persistent_blocks(reinterpret_cast<const void *>(persistent), lds, grid)),
                       dim3(kBlock), lds, s, P);
}

template <typename TF, typename TM, int F, int KBM>
inline void mma_go(const QueryArgs &A, bool pairs, uint32_t grid, hipStream_t s)
{
    // voxel lists of H/2 entries per lane (for pairs, H is the largest over the objects)
    const size_t lists = (size_t)(A.g.H >> 1) * kBlock * sizeof(uint32_t);
    if constexpr (KBM <= 2) {
        if (A.width == 128) {   // the paper's default width: no hot-level variant (hot levels change no result)
            if (pairs) hipLaunchKernelGGL((k_query_mma<TF, TM, F, 128, KBM, true, false>), dim3(grid), dim3(kBlock), lists, s, A);
            else hipLaunchKernelGGL((k_query_mma<TF, TM, F, 128, KBM, false, false>), dim3(grid), dim3(kBlock), lists, s, A);
            return;
        }
    }
    const size_t lds = lists + A.hot_lds;
    // objects with hot levels take the variant that reads them from LDS
    if constexpr (hot_entries<TF, F>()) {
        if (A.hot_lds) {
            if (pairs) launch_tiles(k_query_mma<TF, TM, F, 64, KBM, true, true>, k_query_mma_persist<TF, TM, F, 64, KBM, true, true>, A, grid, lds, s);
            else launch_tiles(k_query_mma<TF, TM, F, 64, KBM, false, true>, k_query_mma_persist<TF, TM, F, 64, KBM, false, true>, A, grid, lds, s);
            return;
        }
    }
    if (pairs) launch_tiles(k_query_mma<TF, TM, F, 64, KBM, true, false>, k_query_mma_persist<TF, TM, F, 64, KBM, true, false>, A, grid, lds, s);
    else launch_tiles(k_query_mma<TF, TM, F, 64, KBM, false, false>, k_query_mma_persist<TF, TM, F, 64, KBM, false, false>, A, grid, lds, s);
}

template <typename TF, typename TM, int F>
inline void mma_by_kb(const QueryArgs &A, int kbm, bool pairs, uint32_t grid, hipStream_t s)
{
    if (kbm <= 1) mma_go<TF, TM, F, 1>(A, pairs, grid, s);
    else if (kbm <= 2) mma_go<TF, TM, F, 2>(A, pairs, grid, s);
    else mma_go<TF, TM, F, 8>(A, pairs, grid, s);
}

// One wave per ray (two features per level, width 64, at most two K blocks per point) over
// `grid` tiles' slots starting at tile A.tile0.
template <typename TF, typename TM>
inline void mma_small_go(const QueryArgs &A, int kbm, uint32_t grid, hipStream_t s)
{
    const dim3 blocks(grid * (kBlock / kLatWaves)), threads(64 * kLatWaves);
    if (kbm <= 1) hipLaunchKernelGGL((k_query_mma_lat<TF, TM, 1>), blocks, threads, 0, s, A);
    else hipLaunchKernelGGL((k_query_mma_lat<TF, TM, 2>), blocks, threads, 0, s, A);
}

template <typename TM>
inline hipError_t launch_mma_small(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) mma_small_go<float, TM>(A, kbm, grid, s);
    else if (feat_dtype == LSNIF_FP16) mma_small_go<_Float16, TM>(A, kbm, grid, s);
    else mma_small_go<__bf16, TM>(A, kbm, grid, s);
    return hipGetLastError();
}

template <typename TM>
inline hipError_t launch_mma(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid,
                             hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) {
        if (F == 2) mma_by_kb<float, TM, 2>(A, kbm, pairs, grid, s); else mma_by_kb<float, TM, 3>(A, kbm, pairs, grid, s);
    } else if (feat_dtype == LSNIF_FP16) {
        if (F == 2) mma_by_kb<_Float16, TM, 2>(A, kbm, pairs, grid, s); else mma_by_kb<_Float16, TM, 3>(A, kbm, pairs, grid, s);
    } else {
        if (F == 2) mma_by_kb<__bf16, TM, 2>(A, kbm, pairs, grid, s); else mma_by_kb<__bf16, TM, 3>(A, kbm, pairs, grid, s);
    }
    return hipGetLastError();
}

}  // namespace lsnif
