// Instantiations of the matrix-core query kernel with an FP8 (OCP e4m3) MLP.
#include "lsnif_query_launch.hpp"

namespace lsnif {

hipError_t launch_mma_fp8(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid, hipStream_t s)
{
    return launch_mma<fp8e4m3>(A, feat_dtype, F, kbm, pairs, grid, s);
}

hipError_t launch_mma_small_fp8(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s)
{
    return launch_mma_small<fp8e4m3>(A, feat_dtype, kbm, grid, s);
}

}  // namespace lsnif
