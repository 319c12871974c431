// The consumer side of a wavefront path tracer: every ray with a hit spawns one
// diffuse bounce ray, compacted in the order of its parent, ready to be the
// next request (Sec. 7's scenes are rendered this way, with the new origin
// offset by a small epsilon along the surface normal).
//
// New origin x + eps n with x = o + t d and n the hit normal turned to face the
// incoming ray; new direction cosine-distributed about n (Malley's method: a
// uniform point of the unit disk lifted to the hemisphere), in the
// orthonormal basis of Duff et al. 2017 ("Building an Orthonormal Basis,
// Revisited"); the two uniforms come from the PCG hash of (seed, bounce, ray).
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_bounce(BounceArgs B)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (!WRITE) {
        if (i < B.n) B.offsets[i] = B.hits[i].hit ? 1u : 0u;
        if (i == B.n) B.offsets[i] = 0u;   // the exclusive scan leaves the count here
        return;
    }
    if (i >= B.n || !B.hits[i].hit) return;
    const float4 r0 = B.rays[2 * i], r1 = B.rays[2 * i + 1];
    const lsnif_hit h = B.hits[i];
    const float o[3] = {r0.x, r0.y, r0.z}, d[3] = {r0.w, r1.x, r1.y};
    float nv[3] = {h.n[0], h.n[1], h.n[2]};
    if ((nv[0] * d[0] + nv[1] * d[1]) + nv[2] * d[2] > 0.0f)
        for (int a = 0; a < 3; ++a) nv[a] = -nv[a];
    float org[3];
    for (int a = 0; a < 3; ++a) org[a] = (o[a] + h.t * d[a]) + B.eps * nv[a];
    const uint32_t k = pcg_hash(B.seed ^ pcg_hash(B.bounce));
    const uint32_t h1 = pcg_hash(i ^ k), h2 = pcg_hash(h1);
    const float u1 = (float)(h1 >> 8) * 5.9604644775390625e-8f, u2 = (float)(h2 >> 8) * 5.9604644775390625e-8f;
    const float rr = __builtin_sqrtf(u1), phi = 6.2831855f * u2;
    const float lx = rr * __builtin_cosf(phi), ly = rr * __builtin_sinf(phi);
    const float lz = __builtin_sqrtf(__builtin_fmaxf(0.0f, 1.0f - u1));
    const float s = __builtin_copysignf(1.0f, nv[2]);
    const float a = -1.0f / (s + nv[2]);
    const float b = nv[0] * nv[1] * a;
    const float tx[3] = {1.0f + s * nv[0] * nv[0] * a, s * b, -s * nv[0]};
    const float bx[3] = {b, s + nv[1] * nv[1] * a, -nv[1]};
    float dir[3];
    for (int c = 0; c < 3; ++c) dir[c] = (lx * tx[c] + ly * bx[c]) + lz * nv[c];
    const uint32_t j = B.offsets[i];
    B.next[2 * j] = make_float4(org[0], org[1], org[2], dir[0]);
    B.next[2 * j + 1] = make_float4(dir[1], dir[2], 0.0f, __builtin_inff());
    B.parent[j] = i;
}

hipError_t launch_bounce_mark(const BounceArgs &B, hipStream_t s)
{
    hipLaunchKernelGGL(k_bounce<false>, dim3(B.n / kBlock + 1), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_bounce_write(const BounceArgs &B, hipStream_t s)
{
    if (B.n) hipLaunchKernelGGL(k_bounce<true>, dim3((B.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

}  // namespace lsnif
