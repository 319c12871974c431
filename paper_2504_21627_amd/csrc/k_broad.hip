// Broad phase of instanced queries: which instances each ray may hit.
//
// Pair (r, i) exists when ray r, mapped into instance i's object space, meets
// the object's voxel grid on [max(ta, tmin), tb] with positive length and
// that segment starts no later than tmax: the same mapping and slab test the
// pair query's narrow phase starts with (to_object_space, setup_ray), and a
// hit's t lies in [ta, tb] and must not exceed tmax, so no pair that can hit
// is left out.
// One lane per ray walks every instance in order (the instance and its
// object's constants are wave-uniform, read through the scalar path); a
// counting pass, an exclusive scan of the counts and a writing pass list the
// pairs by ray, then instance.  For up to 256 instances the counting pass
// keeps each ray's hit instances as a bit mask, and the writing pass reads
// the masks rather than repeating the tests.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_broad(BroadArgs B)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    const bool live = r < B.n_rays;
    if (!WRITE && r == B.n_rays) B.offsets[r] = 0u;   // the exclusive scan leaves the total here
    float4 ra = make_float4(0.0f, 0.0f, 0.0f, 0.0f), rb = ra;
    if (live) {
        ra = B.rays[2 * r];
        rb = B.rays[2 * r + 1];
    }
    uint32_t n = 0, at = WRITE && live ? B.offsets[r] : 0u;
    if (WRITE && B.mask_words) {
        if (!live) return;
        for (uint32_t k = 0; k < B.mask_words; ++k) {
            uint32_t m = B.masks[(size_t)k * B.n_rays + r];
            while (m) {
                B.pair_ray[at] = r;
                B.pair_inst[at] = 32u * k + (uint32_t)__builtin_ctz(m);
                ++at;
                m &= m - 1u;
            }
        }
        return;
    }
    typedef const __attribute__((address_space(4))) lsnif_instance cinst;
    uint32_t bits = 0;
    for (uint32_t i = 0; i < B.n_inst; ++i) {
        const uint32_t o = ((cinst *)B.inst)[i].object_id;
        bool hit = false;
        if (o < B.n_objs && ((const cObjDev *)B.objs)[o].live) {   // else no such object: no pair
            const cObjDev &O = ((const cObjDev *)B.objs)[o];
            lsnif_instance I;
            I.object_id = o;
#pragma unroll
            for (int k = 0; k < 12; ++k) I.world_to_object[k] = ((cinst *)B.inst)[i].world_to_object[k];
            float4 a = ra, b = rb;
            to_object_space(I, a, b);
            VRay w;
            setup_ray(O.g, a, b, w);
            hit = live && w.cand && w.ta <= w.tmax;
        }
        if (hit) {
            if constexpr (WRITE) {
                B.pair_ray[at] = r;
                B.pair_inst[at] = i;
                ++at;
            } else {
                ++n;
                bits |= 1u << (i & 31u);
            }
        }
        if (!WRITE && B.mask_words && ((i & 31u) == 31u || i + 1 == B.n_inst)) {   // i is wave-uniform
            if (live) B.masks[(size_t)(i >> 5) * B.n_rays + r] = bits;
            bits = 0;
        }
    }
    if (!WRITE && live) B.offsets[r] = n;
}

hipError_t launch_broad_count(const BroadArgs &B, hipStream_t s)
{
    hipLaunchKernelGGL(k_broad<false>, dim3(B.n_rays / kBlock + 1), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_broad_write(const BroadArgs &B, hipStream_t s)
{
    if (B.n_rays) hipLaunchKernelGGL(k_broad<true>, dim3((B.n_rays + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

}  // namespace lsnif
