// Instantiations of the matrix-core query kernel with a BF16 MLP.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <typename TF, int F, int KBM>
static void go(const QueryArgs &A, bool pairs, uint32_t grid, hipStream_t s)
{
    // voxel lists of H/2 entries per lane (for pairs, H is the largest over the objects)
    const size_t lists = (size_t)(A.g.H >> 1) * kBlock * sizeof(uint32_t);
    if constexpr (KBM <= 2) {
        if (A.width == 128) {   // the paper's default width: no hot-level variant (hot levels change no result)
            if (pairs) hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 128, KBM, true, false>), dim3(grid), dim3(kBlock), lists, s, A);
            else hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 128, KBM, false, false>), dim3(grid), dim3(kBlock), lists, s, A);
            return;
        }
    }
    const size_t lds = lists + A.hot_lds;
    // objects with hot levels take the variant that reads them from LDS
    if constexpr (hot_entries<TF, F>()) {
        if (A.hot_lds) {
            if (pairs) hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 64, KBM, true, true>), dim3(grid), dim3(kBlock), lds, s, A);
            else hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 64, KBM, false, true>), dim3(grid), dim3(kBlock), lds, s, A);
            return;
        }
    }
    if (pairs) hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 64, KBM, true, false>), dim3(grid), dim3(kBlock), lds, s, A);
    else hipLaunchKernelGGL((k_query_mma<TF, __bf16, F, 64, KBM, false, false>), dim3(grid), dim3(kBlock), lds, s, A);
}

template <typename TF, int F>
static void by_kb(const QueryArgs &A, int kbm, bool pairs, uint32_t grid, hipStream_t s)
{
    if (kbm <= 1) go<TF, F, 1>(A, pairs, grid, s);
    else if (kbm <= 2) go<TF, F, 2>(A, pairs, grid, s);
    else go<TF, F, 8>(A, pairs, grid, s);
}

hipError_t launch_mma_bf16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid, hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) {
        if (F == 2) by_kb<float, 2>(A, kbm, pairs, grid, s); else by_kb<float, 3>(A, kbm, pairs, grid, s);
    } else if (feat_dtype == LSNIF_FP16) {
        if (F == 2) by_kb<_Float16, 2>(A, kbm, pairs, grid, s); else by_kb<_Float16, 3>(A, kbm, pairs, grid, s);
    } else {
        if (F == 2) by_kb<__bf16, 2>(A, kbm, pairs, grid, s); else by_kb<__bf16, 3>(A, kbm, pairs, grid, s);
    }
    return hipGetLastError();
}

}  // namespace lsnif
