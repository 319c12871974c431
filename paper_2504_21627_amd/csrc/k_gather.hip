// Instantiations of the gather-ceiling kernel (the query's gathers alone).
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <typename TF, int F>
static void go(const QueryArgs &A, float *sums, uint32_t grid, hipStream_t s)
{
    const size_t lds = (size_t)(A.g.H >> 1) * kBlock * sizeof(uint32_t);
    hipLaunchKernelGGL((k_gather_only<TF, F>), dim3(grid), dim3(kBlock), lds, s, A, sums);
}

hipError_t launch_gather_only(const QueryArgs &A, int feat_dtype, int F, float *sums, uint32_t grid, hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) {
        if (F == 2) go<float, 2>(A, sums, grid, s); else go<float, 3>(A, sums, grid, s);
    } else if (feat_dtype == LSNIF_FP16) {
        if (F == 2) go<_Float16, 2>(A, sums, grid, s); else go<_Float16, 3>(A, sums, grid, s);
    } else {
        if (F == 2) go<__bf16, 2>(A, sums, grid, s); else go<__bf16, 3>(A, sums, grid, s);
    }
    return hipGetLastError();
}

}  // namespace lsnif
