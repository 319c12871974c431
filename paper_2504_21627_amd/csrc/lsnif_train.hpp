// Arguments of the training kernels (one training step of Sec. 5.2, 5.3).
#pragma once
#include "lsnif_kernels.hpp"

namespace lsnif {

// Encoding of a batch (forward: features into x0) and its transpose
// (backward: dx0 scattered onto the table gradients).  Thread = (ray, point).
struct TrainEncArgs {
    Geom g;
    const float4 *rays;
    uint32_t n;
    const uint32_t *lists;    // walk output, entry j of ray r at lists[j n + r]
    const uint8_t *nvox;
    const float *tab;         // [L][T][F] parameters
    float *gtab;              // backward: `replicas` gradient copies of [L][T][F], back to back
    uint32_t replicas;        // block b adds into copy b % replicas (blocks alternate over the XCDs)
    uint64_t n_tab;           // floats of one copy
    float *x;                 // [n][H L F]: x0 (forward) or dx0 (backward)
};

// C(i, j) = sum_k A(i, k) B(k, j) over i < M, j < N, k < K, the operands read
// through strides; gridDim.z splits K in chunks of kchunk (partial epilogue).
struct GemmArgs {
    const float *A;
    int64_t sai, sak;
    const float *B;
    int64_t sbk, sbj;
    float *C;
    int64_t ldc;
    const float *aux;         // post-activation values for the derivative epilogue, ld = ldc
    uint32_t M, N, K, kchunk;
    float slope;              // activation slope below 0 (0 for ReLU)
};

// Output tile of a block (rows x columns) and the K slice staged per step.
constexpr uint32_t kGM = 64, kGN = 64, kGK = 32;

// kEpiPartial: K chunk z stores its partial product at C + z M ldc (summed afterwards).
enum GemmEpi : int { kEpiStore = 0, kEpiAct = 1, kEpiActGrad = 2, kEpiPartial = 3 };

struct TrainLossArgs {
    Geom g;
    const float4 *rays;
    const lsnif_train_target *gt;
    uint32_t n;
    const uint8_t *nvox;
    const float *z;           // [n][ldz] raw outputs
    float *dz;                // [n][ldz] d loss / d z
    uint32_t ldz, out_dim, n_mat, has_albedo;
    float *loss_part;         // per-block sums of the per-ray losses, one float per block
};

struct AdamArgs {
    float *p, *m, *v;
    const float *g;
    uint64_t count;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
};

hipError_t launch_train_fill(float *a, uint64_t na, float *b, uint64_t nb, hipStream_t s);
hipError_t launch_train_encode(const TrainEncArgs &A, bool backward, hipStream_t s);
hipError_t launch_train_gemm(const GemmArgs &G, int epi, hipStream_t s);
// dst[i ld + j] = sum over z < nz of part[(z M + i) N + j], i < M, j < N; part2 holds
// kSumGroups x M x N floats of scratch.
constexpr uint32_t kSumGroups = 16;
hipError_t launch_sum_partials(const float *part, uint32_t nz, uint32_t M, uint32_t N, float *part2, float *dst,
                               uint32_t ld, hipStream_t s);
// a[i] += sum over r = 1 .. copies-1 of a[r n + i], i < n.
hipError_t launch_sum_copies(float *a, uint64_t n, uint32_t copies, hipStream_t s);
hipError_t launch_train_loss(const TrainLossArgs &A, hipStream_t s);
hipError_t launch_train_loss_final(const float *part, uint32_t n, float *loss, hipStream_t s);
hipError_t launch_adam(const AdamArgs &A, hipStream_t s);

}  // namespace lsnif
