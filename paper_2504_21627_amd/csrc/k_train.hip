// Training step kernels: the encoding and its transpose, the layer products of
// the forward and backward passes, the per-signal losses and Adam.
//
// Everything is float32 (the FP32 object's own tables and weights are the
// parameters).  The voxel lists come from the query path's walk kernel, and
// the boundary points, cells and table slots from the same device functions,
// so a training ray sees exactly the encoding inputs a query sees.
#include "lsnif_kernels.hpp"
#include "lsnif_launch.hpp"
#include "lsnif_train.hpp"

namespace lsnif {

__global__ __launch_bounds__(kBlock) void k_train_fill(float *a, uint64_t na, float *b, uint64_t nb)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < na + nb; i += stride) {
        if (i < na) a[i] = 0.0f;
        else b[i - na] = 0.0f;
    }
}

// Forward: thread = (ray r, boundary point h): the point's L x F features,
// trilinear over the corners of its cell on every level, into
// x[r][(h L + l) F + f]; points past the ray's list get 0.  On a level aligned
// with the voxel faces the point's crossing-axis weight is exactly 0 or 1, so
// only the 4 corners on that side are visited (the others have weight 0; the
// sparse encoding of Sec. 3.2); other levels visit all 8.
//
// Backward: thread = (ray r, point h, feature f), so that the F features of a
// corner, adjacent in the table, go out from adjacent lanes of one atomic
// instruction.  d loss / d table entry += corner weight x dx for every corner
// of non-zero weight, with float atomics into one of several copies of the
// gradient (block b into copy b % copies: consecutive blocks go to different
// XCDs, so each copy's lines are contended by one XCD's blocks only); the
// copies are summed afterwards.  The order of the additions is not fixed.
// Where a ray leaves voxel j and enters voxel j + 1 at the same point (adjacent
// listed voxels: the same plane crossing, the same clamps), the exit point's
// threads add both points' gradients and the entry point's threads add
// nothing; each recomputes the other point, so both take the same decision.
template <bool BWD> __global__ __launch_bounds__(kBlock) void k_train_enc(TrainEncArgs A)
{
    const Geom &g = A.g;
    const uint32_t H = (uint32_t)g.H, L = (uint32_t)g.L, F = (uint32_t)g.F, LF = L * F;
    const uint32_t per = BWD ? F : 1u;   // threads per point
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t rh = idx / per;
    const uint32_t f0 = (uint32_t)(idx - rh * per);
    const uint64_t r = rh / H;
    const uint32_t h = (uint32_t)(rh - r * H);
    if (r >= A.n) return;
    float *x = A.x + (size_t)r * H * LF + (size_t)h * LF;
    const uint32_t nv = A.nvox[r];
    if (h >= 2u * nv) {
        if constexpr (!BWD)
            for (uint32_t q = 0; q < LF; ++q) x[q] = 0.0f;
        return;
    }
    VRay w;
    setup_ray(g, A.rays[2 * r], A.rays[2 * r + 1], w);
    const uint32_t packed = A.lists[(size_t)(h >> 1) * A.n + r];
    float p[3];
    const uint32_t face = (uint32_t)boundary_point(w, packed, (h & 1u) != 0u, p);
    bool merge_next = false;
    if constexpr (BWD) {
        auto same = [&](uint32_t j, bool is_exit) {
            float q[3];
            (void)boundary_point(w, A.lists[(size_t)j * A.n + r], is_exit, q);
            return q[0] == p[0] && q[1] == p[1] && q[2] == p[2];
        };
        if (!(h & 1u) && h >= 2u && same((h >> 1) - 1u, true)) return;   // added by the previous exit point
        merge_next = (h & 1u) && h + 1u < 2u * nv && same((h + 1u) >> 1, false);
    }
    const size_t T = (size_t)1 << g.log2_T;
    float *gcopy = nullptr;
    if constexpr (BWD) gcopy = A.gtab + (size_t)(blockIdx.x % A.replicas) * A.n_tab;
    for (uint32_t l = 0; l < L; ++l) {
        uint32_t i[3];
        float wt[3];
        level_cell(g, (int)l, p, i, wt);
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dx = 0.0f;
        if constexpr (BWD) {
            dx = x[l * F + f0];
            if (merge_next) dx += x[LF + l * F + f0];
            if (dx == 0.0f) continue;
        }
        const bool al = (g.aligned_mask >> l) & 1u;
        const uint32_t nc = al ? 4u : 8u, fb = wt[face] != 0.0f ? 1u : 0u;
        const uint32_t low = (1u << face) - 1u;
        for (uint32_t cc = 0; cc < nc; ++cc) {
            // aligned level: corner index cc with the crossing axis's bit (fb) inserted at bit `face`
            const uint32_t c = al ? ((cc & low) | (fb << face) | ((cc & ~low) << 1)) : cc;
            const uint32_t bx = c & 1u, by = (c >> 1) & 1u, bz = (c >> 2) & 1u;
            const float wx = bx ? wt[0] : 1.0f - wt[0];
            const float wy = by ? wt[1] : 1.0f - wt[1];
            const float wz = bz ? wt[2] : 1.0f - wt[2];
            const float wc = (wx * wy) * wz;
            const size_t e = ((size_t)l * T + vertex_slot(g, (int)l, i[0] + bx, i[1] + by, i[2] + bz)) * F;
            if constexpr (!BWD) {
                for (uint32_t f = 0; f < F; ++f) acc[f] = __builtin_fmaf(wc, A.tab[e + f], acc[f]);
            } else {
                if (wc != 0.0f) unsafeAtomicAdd(&gcopy[e + f0], wc * dx);
            }
        }
        if constexpr (!BWD)
            for (uint32_t f = 0; f < F; ++f) x[l * F + f] = acc[f];
    }
}

// Tiled float32 product on the matrix cores: 64 x BN outputs per 256-thread
// block (the launches use BN = 64: at 126 VGPRs it runs 4 waves per SIMD, and
// that beat BN = 128, which reads the row operand once but needs 212),
// K in slices of 32 staged through LDS, the next slice loaded into registers
// while the current one is multiplied.  Each wave computes a 32 x BN/2 block
// as BN/64 v_mfma_f32_32x32x2f32 accumulators (float32 operands and
// accumulation).
// Block x = row tile, y = column tile, z = K chunk.  Operand tiles are loaded
// along whichever index has unit stride, so plain and transposed operands
// both read contiguously.  Operand layout per lane l (i = l % 32, q = l / 32):
// A holds A[i][k0 + q], B holds B[k0 + q][i], and accumulator r holds
// D[8 (r / 4) + 4 q + r % 4][i].
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int EPI, uint32_t BN>
__global__ __launch_bounds__(kBlock) void k_train_gemm(GemmArgs G)
{
    constexpr uint32_t kLA = kGM * kGK / kBlock, kLB = BN * kGK / kBlock;   // loads per thread per slice
    constexpr uint32_t WB = BN / 64;                                       // 32 x 32 blocks per wave
    __shared__ float As[kGK][kGM + 4];
    __shared__ float Bs[kGK][BN + 4];
    const uint32_t tid = threadIdx.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * kGM;
    const uint32_t j0 = blockIdx.y * BN;
    const uint64_t kb = (uint64_t)blockIdx.z * G.kchunk;
    const uint64_t ke = kb + G.kchunk < G.K ? kb + G.kchunk : G.K;
    const bool a_k_unit = G.sak == 1, b_j_unit = G.sbj == 1;
    const uint32_t lane = tid & 63u, wv = tid >> 6, wi = wv & 1u, wj = wv >> 1, li = lane & 31u, lq = lane >> 5;
    // element e of a slice: A (i, k) and B (k, j) positions, chosen so that lanes read along the unit stride
    auto a_pos = [&](uint32_t e, uint32_t &ai, uint32_t &ak) {
        ai = a_k_unit ? e / kGK : e % kGM;
        ak = a_k_unit ? e % kGK : e / kGM;
    };
    auto b_pos = [&](uint32_t e, uint32_t &bk, uint32_t &bj) {
        bj = b_j_unit ? e % BN : e / kGK;
        bk = b_j_unit ? e / BN : e % kGK;
    };
    // each thread's elements keep their row / column across slices: a slice's operands are a
    // uniform base (the block's corner, advanced by whole slices) plus a fixed 32-bit offset per
    // element (small: within one 64 x 32 or 32 x BN tile), and a bit per element says whether
    // its row / column exists
    float ra[kLA], rb[kLB];
    uint32_t oa[kLA], ob[kLB], va = 0, vb = 0;
#pragma unroll
    for (uint32_t q = 0; q < kLA; ++q) {
        uint32_t ai, ak;
        a_pos(tid + q * kBlock, ai, ak);
        va |= (i0 + ai < G.M ? 1u : 0u) << q;
        oa[q] = (uint32_t)(ai * G.sai + ak * G.sak);
    }
#pragma unroll
    for (uint32_t q = 0; q < kLB; ++q) {
        uint32_t bk, bj;
        b_pos(tid + q * kBlock, bk, bj);
        vb |= (j0 + bj < G.N ? 1u : 0u) << q;
        ob[q] = (uint32_t)(bk * G.sbk + bj * G.sbj);
    }
    const float *A0 = G.A + i0 * G.sai + kb * G.sak, *B0 = G.B + kb * G.sbk + (uint64_t)j0 * G.sbj;
    const uint64_t step_a = (uint64_t)kGK * G.sak, step_b = (uint64_t)kGK * G.sbk;
    auto fetch = [&](uint64_t k0) {
        const uint64_t s = (k0 - kb) / kGK;
        const float *As0 = A0 + s * step_a, *Bs0 = B0 + s * step_b;
        if (k0 + kGK <= ke) {   // a whole slice: only the row / column bound
#pragma unroll
            for (uint32_t q = 0; q < kLA; ++q) ra[q] = (va >> q) & 1u ? As0[oa[q]] : 0.0f;
#pragma unroll
            for (uint32_t q = 0; q < kLB; ++q) rb[q] = (vb >> q) & 1u ? Bs0[ob[q]] : 0.0f;
        } else {
#pragma unroll
            for (uint32_t q = 0; q < kLA; ++q) {
                uint32_t ai, ak;
                a_pos(tid + q * kBlock, ai, ak);
                ra[q] = ((va >> q) & 1u) && k0 + ak < ke ? As0[oa[q]] : 0.0f;
            }
#pragma unroll
            for (uint32_t q = 0; q < kLB; ++q) {
                uint32_t bk, bj;
                b_pos(tid + q * kBlock, bk, bj);
                rb[q] = ((vb >> q) & 1u) && k0 + bk < ke ? Bs0[ob[q]] : 0.0f;
            }
        }
    };
    f32x16_t acc[WB];
#pragma unroll
    for (uint32_t h = 0; h < WB; ++h)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[h][r] = 0.0f;
    if (kb < ke) fetch(kb);
    for (uint64_t k0 = kb; k0 < ke; k0 += kGK) {
#pragma unroll
        for (uint32_t q = 0; q < kLA; ++q) {
            uint32_t ai, ak;
            a_pos(tid + q * kBlock, ai, ak);
            As[ak][ai] = ra[q];
        }
#pragma unroll
        for (uint32_t q = 0; q < kLB; ++q) {
            uint32_t bk, bj;
            b_pos(tid + q * kBlock, bk, bj);
            Bs[bk][bj] = rb[q];
        }
        __syncthreads();
        if (k0 + kGK < ke) fetch(k0 + kGK);   // in flight while this slice is multiplied
#pragma unroll
        for (uint32_t k = 0; k < kGK; k += 2) {
            const float a = As[k + lq][wi * 32 + li];
#pragma unroll
            for (uint32_t h = 0; h < WB; ++h)
                acc[h] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Bs[k + lq][wj * (BN / 2) + h * 32 + li], acc[h],
                                                              0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (uint32_t h = 0; h < WB; ++h) {
        const uint32_t gj = j0 + wj * (BN / 2) + h * 32 + li;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint64_t gi = i0 + wi * 32 + 8 * (r / 4) + 4 * lq + (r % 4);
            if (gi >= G.M || gj >= G.N) continue;
            float *dst = G.C + gi * G.ldc + gj;
            if constexpr (EPI == kEpiPartial) dst += (uint64_t)blockIdx.z * G.M * G.ldc;
            float v = acc[h][r];
            if constexpr (EPI == kEpiAct) v = v > 0.0f ? v : v * G.slope;
            if constexpr (EPI == kEpiActGrad) v = G.aux[gi * G.ldc + gj] > 0.0f ? v : v * G.slope;
            *dst = v;
        }
    }
}

// Sum of the K-chunk partials in two passes: pass 1, block (x, y) sums the
// chunks y, y + kSumGroups, ... of its 256 entries into part2[y]; pass 2 sums
// the kSumGroups rows into the layer's gradient.  Both read contiguously.
__global__ __launch_bounds__(kBlock) void k_sum_partials1(const float *part, uint32_t nz, uint32_t MN, float *part2)
{
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= MN) return;
    float s = 0.0f;
    for (uint32_t z = blockIdx.y; z < nz; z += kSumGroups) s += part[(size_t)z * MN + e];
    part2[(size_t)blockIdx.y * MN + e] = s;
}

__global__ __launch_bounds__(kBlock) void k_sum_partials2(const float *part2, uint32_t M, uint32_t N, float *dst,
                                                          uint32_t ld)
{
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= M * N) return;
    float s = 0.0f;
    for (uint32_t y = 0; y < kSumGroups; ++y) s += part2[(size_t)y * M * N + e];
    dst[(size_t)(e / N) * ld + e % N] = s;
}

__global__ __launch_bounds__(kBlock) void k_sum_copies(float *a, uint64_t n, uint32_t copies)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        float s = a[i];
        for (uint32_t r = 1; r < copies; ++r) s += a[(size_t)r * n + i];
        a[i] = s;
    }
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

// Thread = ray: its loss and d loss / d z.  The block's rays' losses are summed
// in float32 (waves, then the block) into loss_part[block]; k_train_loss_final
// adds the blocks' sums in a fixed order, so the batch loss is deterministic.
__global__ __launch_bounds__(kBlock) void k_train_loss(TrainLossArgs A)
{
    __shared__ float wsum[kBlock / 64];
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    float lsum = 0.0f;
    if (r < A.n) {
        const float *z = A.z + (size_t)r * A.ldz;
        float *dz = A.dz + (size_t)r * A.ldz;
        float d[kMaxOut];
#pragma unroll
        for (int k = 0; k < kMaxOut; ++k) d[k] = 0.0f;
        if (A.nvox[r] > 0) {
            VRay w;
            setup_ray(A.g, A.rays[2 * r], A.rays[2 * r + 1], w);
            const lsnif_train_target y = A.gt[r];
            const float inv_n = 1.0f / (float)A.n;
            const float yh = y.hit ? 1.0f : 0.0f;
            // occlusion: softplus(z0) - y z0, the stable form
            const float z0 = z[0];
            float l = (fmaxf(z0, 0.0f) + log1pf(expf(-fabsf(z0)))) - yh * z0;
            d[0] = sigmoidf(z0) - yh;
            if (y.hit) {
                // local hit distance
                float tau = (y.t - w.ta) / (w.tb - w.ta);
                tau = fminf(fmaxf(tau, 0.0f), 1.0f);
                const float s1 = sigmoidf(z[1]), e1 = s1 - tau;
                l += fabsf(e1);
                d[1] = (e1 > 0.0f ? 1.0f : (e1 < 0.0f ? -1.0f : 0.0f)) * (s1 * (1.0f - s1));
                // normal: 1 - cosine similarity
                const float nn = sqrtf((z[2] * z[2] + z[3] * z[3]) + z[4] * z[4]);
                const float dot = (z[2] * y.n[0] + z[3] * y.n[1]) + z[4] * y.n[2];
                const float den = fmaxf(nn, 1e-8f);
                const float cs = dot / den;
                l += 1.0f - cs;
                for (int b = 0; b < 3; ++b)
                    d[2 + b] = nn > 1e-8f ? -(y.n[b] / nn - cs * (z[2 + b] / nn) / nn) : -(y.n[b] / 1e-8f);
                uint32_t m0 = 5;
                if (A.has_albedo) {
                    for (int c = 0; c < 3; ++c) {
                        const float a = sigmoidf(z[5 + c]), e = a - y.albedo[c];
                        const float q = (a + 0.01f) * (a + 0.01f);
                        l += (e * e / q) / 3.0f;
                        d[5 + c] = ((2.0f * e / q) / 3.0f) * (a * (1.0f - a));
                    }
                    m0 = 8;
                }
                if (y.material >= 0 && (uint32_t)y.material < A.n_mat) {
                    float mx = z[m0];
                    for (uint32_t k = 1; k < A.n_mat; ++k) mx = fmaxf(mx, z[m0 + k]);
                    float sum = 0.0f;
                    for (uint32_t k = 0; k < A.n_mat; ++k) sum += expf(z[m0 + k] - mx);
                    l += (mx + logf(sum)) - z[m0 + y.material];
                    for (uint32_t k = 0; k < A.n_mat; ++k)
                        d[m0 + k] = expf(z[m0 + k] - mx) / sum - ((int32_t)k == y.material ? 1.0f : 0.0f);
                }
            }
            lsum = l;
#pragma unroll
            for (int k = 0; k < kMaxOut; ++k) d[k] *= inv_n;
        }
        for (uint32_t k = 0; k < A.out_dim; ++k) dz[k] = d[k];
    }
    for (int o = 32; o >= 1; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = 0.0f;
        for (uint32_t k = 0; k < kBlock / 64; ++k) b += wsum[k];
        A.loss_part[blockIdx.x] = b;
    }
}

// One block: the mean loss of the batch from the per-block sums.
__global__ __launch_bounds__(kBlock) void k_train_loss_final(const float *part, uint32_t nparts, uint32_t n,
                                                             float *loss)
{
    __shared__ float red[kBlock];
    float s = 0.0f;
    for (uint32_t i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)n;
}

__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs A)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < A.count; i += stride) {
        const float g = A.g[i];
        const float m = A.b1 * A.m[i] + (1.0f - A.b1) * g;
        const float v = A.b2 * A.v[i] + (1.0f - A.b2) * (g * g);
        A.m[i] = m;
        A.v[i] = v;
        A.p[i] = A.p[i] - A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
    }
}

static uint32_t stream_blocks(uint64_t count)
{
    const uint64_t b = (count + kBlock - 1) / kBlock;
    return (uint32_t)(b < 8192 ? (b ? b : 1) : 8192);
}

hipError_t launch_train_fill(float *a, uint64_t na, float *b, uint64_t nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_train_fill, dim3(stream_blocks(na + nb)), dim3(kBlock), 0, s, a, na, b, nb);
    return hipGetLastError();
}

hipError_t launch_train_encode(const TrainEncArgs &A, bool backward, hipStream_t s)
{
    const uint64_t threads = (uint64_t)A.n * (uint64_t)A.g.H * (backward ? (uint64_t)A.g.F : 1u);
    const dim3 grid((uint32_t)((threads + kBlock - 1) / kBlock));
    if (backward) hipLaunchKernelGGL(k_train_enc<true>, grid, dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL(k_train_enc<false>, grid, dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_train_gemm(const GemmArgs &G, int epi, hipStream_t s)
{
    const uint64_t chunks = (G.K + G.kchunk - 1) / G.kchunk;
    const uint32_t mt = (uint32_t)((G.M + kGM - 1) / kGM), z = (uint32_t)(chunks ? chunks : 1);
    const dim3 grid(mt, (G.N + kGN - 1) / kGN, z);
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_train_gemm<kEpiStore, kGN>), grid, dim3(kBlock), 0, s, G); break;
    case kEpiAct: hipLaunchKernelGGL((k_train_gemm<kEpiAct, kGN>), grid, dim3(kBlock), 0, s, G); break;
    case kEpiActGrad: hipLaunchKernelGGL((k_train_gemm<kEpiActGrad, kGN>), grid, dim3(kBlock), 0, s, G); break;
    default: hipLaunchKernelGGL((k_train_gemm<kEpiPartial, kGN>), grid, dim3(kBlock), 0, s, G); break;
    }
    return hipGetLastError();
}

hipError_t launch_sum_partials(const float *part, uint32_t nz, uint32_t M, uint32_t N, float *part2, float *dst,
                               uint32_t ld, hipStream_t s)
{
    const dim3 g1((M * N + kBlock - 1) / kBlock, kSumGroups);
    hipLaunchKernelGGL(k_sum_partials1, g1, dim3(kBlock), 0, s, part, nz, M * N, part2);
    hipLaunchKernelGGL(k_sum_partials2, dim3((M * N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part2, M, N, dst, ld);
    return hipGetLastError();
}

hipError_t launch_sum_copies(float *a, uint64_t n, uint32_t copies, hipStream_t s)
{
    if (copies <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_sum_copies, dim3(stream_blocks(n)), dim3(kBlock), 0, s, a, n, copies);
    return hipGetLastError();
}

hipError_t launch_train_loss(const TrainLossArgs &A, hipStream_t s)
{
    hipLaunchKernelGGL(k_train_loss, dim3((A.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_train_loss_final(const float *part, uint32_t n, float *loss, hipStream_t s)
{
    const uint32_t nparts = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_train_loss_final, dim3(1), dim3(kBlock), 0, s, part, nparts, n, loss);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &A, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(stream_blocks(A.count)), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

}  // namespace lsnif
