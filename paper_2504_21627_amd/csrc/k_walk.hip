// Instantiations of the voxel-walk kernel.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

hipError_t launch_walk(const QueryArgs &A, bool pairs, uint32_t grid, hipStream_t s)
{
    if (pairs) hipLaunchKernelGGL(k_walk<true>, dim3(grid), dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL(k_walk<false>, dim3(grid), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

}  // namespace lsnif
