// Instantiations of the matrix-core query kernel with a BF16 MLP.
#include "lsnif_query_launch.hpp"

namespace lsnif {

hipError_t launch_mma_bf16(const QueryArgs &A, int feat_dtype, int F, int kbm, bool pairs, uint32_t grid, hipStream_t s)
{
    return launch_mma<__bf16>(A, feat_dtype, F, kbm, pairs, grid, s);
}

hipError_t launch_mma_small_bf16(const QueryArgs &A, int feat_dtype, int kbm, uint32_t grid, hipStream_t s)
{
    return launch_mma_small<__bf16>(A, feat_dtype, kbm, grid, s);
}

}  // namespace lsnif
