// Instantiations of the matrix-core (FP16 / BF16 MFMA) query kernel.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <typename TF, typename TM, int F>
static void go(const QueryArgs &A, hipStream_t s)
{
    const dim3 grid((A.n + kBlock - 1) / kBlock);
    const size_t lds = (size_t)(A.g.H >> 1) * kBlock * sizeof(uint32_t);
    hipLaunchKernelGGL((k_query_mma<TF, TM, F, 64>), grid, dim3(kBlock), lds, s, A);
}

template <typename TM>
static void by_feat(const QueryArgs &A, int feat_dtype, int F, hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) {
        if (F == 2) go<float, TM, 2>(A, s); else go<float, TM, 3>(A, s);
    } else if (feat_dtype == LSNIF_FP16) {
        if (F == 2) go<_Float16, TM, 2>(A, s); else go<_Float16, TM, 3>(A, s);
    } else {
        if (F == 2) go<__bf16, TM, 2>(A, s); else go<__bf16, TM, 3>(A, s);
    }
}

hipError_t launch_mma(const QueryArgs &A, int feat_dtype, int mlp_dtype, int F, hipStream_t s)
{
    if (mlp_dtype == LSNIF_FP16) by_feat<_Float16>(A, feat_dtype, F, s);
    else by_feat<__bf16>(A, feat_dtype, F, s);
    return hipGetLastError();
}

}  // namespace lsnif
