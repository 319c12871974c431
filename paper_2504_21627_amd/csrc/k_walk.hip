// Instantiations of the voxel-walk kernel.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

hipError_t launch_walk(const QueryArgs &A, bool pairs, bool recheck, uint32_t grid, hipStream_t s)
{
    if (pairs) {
        if (recheck) hipLaunchKernelGGL((k_walk<true, true>), dim3(grid), dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_walk<true, false>), dim3(grid), dim3(kBlock), 0, s, A);
    } else {
        if (recheck) hipLaunchKernelGGL((k_walk<false, true>), dim3(grid), dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_walk<false, false>), dim3(grid), dim3(kBlock), 0, s, A);
    }
    return hipGetLastError();
}

}  // namespace lsnif
