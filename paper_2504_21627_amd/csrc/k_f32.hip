// Instantiations of the float32 vector-ALU query kernel and the debug kernel.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"

namespace lsnif {

// Writes every intermediate of the walk and the grid lookups of each ray.
__global__ __launch_bounds__(kBlock) void k_debug(DebugArgs D)
{
    __shared__ uint32_t s_list[kMaxList * kBlock];
    const uint32_t tid = threadIdx.x;
    const uint32_t r = blockIdx.x * kBlock + tid;
    if (r >= D.n) return;
    const Geom &g = D.g;
    VRay w;
    setup_ray(g, D.rays[2 * r], D.rays[2 * r + 1], w);
    const int H = g.H, L = g.L;
    const int nvox = walk_voxels<true>(g, w, g.coarse, s_list + tid, kBlock, H >> 1);
    const int count = 2 * nvox;
    if (D.b.count) D.b.count[r] = w.valid ? count : -1;
    if (D.b.tatb) {
        D.b.tatb[2 * r] = w.ta;
        D.b.tatb[2 * r + 1] = w.tb;
    }
    for (int j = 0; j < H / 2; ++j) {
        const bool in = j < nvox;
        int c[3] = {-1, -1, -1};
        float tin = 0.0f, tout = 0.0f;
        int ia = -1, oa = -1;
        if (in) {
            unpack_ijk(s_list[j * kBlock + tid], c);
            cell_interval(w, c, tin, tout, ia, oa);
        }
        if (D.b.vox_ijk)
            for (int a = 0; a < 3; ++a) D.b.vox_ijk[((size_t)r * (H / 2) + j) * 3 + a] = c[a];
        if (D.b.vox_t) {
            D.b.vox_t[((size_t)r * (H / 2) + j) * 2] = tin;
            D.b.vox_t[((size_t)r * (H / 2) + j) * 2 + 1] = tout;
        }
        if (D.b.vox_axis) {
            D.b.vox_axis[((size_t)r * (H / 2) + j) * 2] = (int8_t)ia;
            D.b.vox_axis[((size_t)r * (H / 2) + j) * 2 + 1] = (int8_t)oa;
        }
    }
    for (int h = 0; h < H; ++h) {
        float p[3] = {0.0f, 0.0f, 0.0f};
        if (h < count) boundary_point(w, s_list[(h >> 1) * kBlock + tid], h & 1, p);
        if (D.b.points)
            for (int b = 0; b < 3; ++b) D.b.points[((size_t)r * H + h) * 3 + b] = p[b];
        for (int l = 0; l < L; ++l) {
            uint32_t i[3] = {0, 0, 0};
            float wt[3] = {0.0f, 0.0f, 0.0f};
            if (h < count) level_cell(g, l, p, i, wt);
            const size_t base = ((size_t)r * H + h) * L + l;
            if (D.b.slots)
                for (int c = 0; c < 8; ++c)
                    D.b.slots[base * 8 + c] =
                        h < count ? vertex_slot(g, l, i[0] + (c & 1), i[1] + ((c >> 1) & 1), i[2] + ((c >> 2) & 1)) : 0u;
            if (D.b.weights)
                for (int b = 0; b < 3; ++b) D.b.weights[base * 3 + b] = wt[b];
        }
    }
}


template <typename TF, int F>
static void go(const QueryArgs &A, bool pairs, uint32_t grid, hipStream_t s)
{
    // voxel lists of H/2 entries per lane (for pairs, H is the largest over the objects)
    const size_t lists = (size_t)(A.g.H >> 1) * kBlock * sizeof(uint32_t);
    if (A.width == 128) {   // the paper's default width: no hot-level variant (hot levels change no result)
        if (pairs) hipLaunchKernelGGL((k_query_f32<TF, F, 128, true, false>), dim3(grid), dim3(kBlock), lists, s, A);
        else hipLaunchKernelGGL((k_query_f32<TF, F, 128, false, false>), dim3(grid), dim3(kBlock), lists, s, A);
        return;
    }
    const size_t lds = lists + A.hot_lds;
    // objects with hot levels take the variant that reads them from LDS
    if constexpr (hot_entries<TF, F>()) {
        if (A.hot_lds) {
            if (pairs) hipLaunchKernelGGL((k_query_f32<TF, F, 64, true, true>), dim3(grid), dim3(kBlock), lds, s, A);
            else hipLaunchKernelGGL((k_query_f32<TF, F, 64, false, true>), dim3(grid), dim3(kBlock), lds, s, A);
            return;
        }
    }
    if (pairs) hipLaunchKernelGGL((k_query_f32<TF, F, 64, true, false>), dim3(grid), dim3(kBlock), lds, s, A);
    else hipLaunchKernelGGL((k_query_f32<TF, F, 64, false, false>), dim3(grid), dim3(kBlock), lds, s, A);
}

hipError_t launch_lat(const QueryArgs &A, int F, uint32_t grid, hipStream_t s)
{
    const dim3 blocks(grid * (kBlock / kLatWaves));   // one wave per slot of the grid's tiles
    if (F == 2) hipLaunchKernelGGL(k_query_lat<2>, blocks, dim3(64 * kLatWaves), 0, s, A);
    else hipLaunchKernelGGL(k_query_lat<3>, blocks, dim3(64 * kLatWaves), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_f32(const QueryArgs &A, int feat_dtype, int F, bool pairs, uint32_t grid, hipStream_t s)
{
    if (feat_dtype == LSNIF_FP32) {
        if (F == 2) go<float, 2>(A, pairs, grid, s); else go<float, 3>(A, pairs, grid, s);
    } else if (feat_dtype == LSNIF_FP16) {
        if (F == 2) go<_Float16, 2>(A, pairs, grid, s); else go<_Float16, 3>(A, pairs, grid, s);
    } else {
        if (F == 2) go<__bf16, 2>(A, pairs, grid, s); else go<__bf16, 3>(A, pairs, grid, s);
    }
    return hipGetLastError();
}

hipError_t launch_debug(const DebugArgs &D, hipStream_t s)
{
    const dim3 grid((D.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_debug, grid, dim3(kBlock), 0, s, D);
    return hipGetLastError();
}

}  // namespace lsnif
