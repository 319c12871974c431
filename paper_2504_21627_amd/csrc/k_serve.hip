// Merged serving launches: several small requests that arrive together are
// answered by one query over their concatenated rays (and pairs).  The pack
// kernel copies each member's rays into one staging array and its pairs with
// ray indices shifted by the member's first staged ray; the unpack kernel
// copies each member's answers back to its own output.  A pair naming a ray
// past its own request's rays is staged as naming no ray, so it is dropped
// exactly as the request's own direct call would drop it.  A ray's answer
// depends only on that ray and its own pairs, so every member gets the bits
// its direct call would.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

namespace {

// The member holding staged element i of the prefix offsets `first` (ascending, first[0] = 0).
__device__ __forceinline__ uint32_t member_of(const MergeArgs &M, uint32_t i, bool pairs)
{
    uint32_t lo = 0, hi = M.n_members;   // member lo holds i: first[lo] <= i < first[lo + 1]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t f = pairs ? M.m[mid].pair0 : M.m[mid].ray0;
        if (f <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_merge_pack(MergeArgs M)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < M.n_rays) {
        const MergeMember &m = M.m[member_of(M, i, false)];
        const uint32_t j = i - m.ray0;
        M.rays[2 * (size_t)i] = m.rays[2 * (size_t)j];
        M.rays[2 * (size_t)i + 1] = m.rays[2 * (size_t)j + 1];
    }
    if (i < M.n_pairs) {
        const MergeMember &m = M.m[member_of(M, i, true)];
        const uint32_t j = i - m.pair0;
        const uint32_t r = m.pair_ray[j];
        M.pair_ray[i] = r < m.n_rays ? m.ray0 + r : 0xffffffffu;
        M.pair_inst[i] = m.pair_inst[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_merge_unpack(MergeArgs M)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= M.n_rays) return;
    const MergeMember &m = M.m[member_of(M, i, false)];
    m.out[i - m.ray0] = M.out[i];
}

hipError_t launch_merge_pack(const MergeArgs &M, hipStream_t s)
{
    const uint32_t n = M.n_rays > M.n_pairs ? M.n_rays : M.n_pairs;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_pack, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M);
    return hipGetLastError();
}

hipError_t launch_merge_unpack(const MergeArgs &M, hipStream_t s)
{
    if (M.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_unpack, dim3((M.n_rays + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M);
    return hipGetLastError();
}

}  // namespace lsnif
