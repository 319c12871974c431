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
    float *gtab;              // [L][T][F] gradients (backward)
    float *x;                 // [n][H L F]: x0 (forward) or dx0 (backward)
};

// C(i, j) = sum_k A(i, k) B(k, j) over i < M, j < N, k < K, the operands read
// through strides; gridDim.z splits K in chunks of kchunk (atomic epilogue).
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

enum GemmEpi : int { kEpiStore = 0, kEpiAct = 1, kEpiActGrad = 2, kEpiAtomic = 3 };

struct TrainLossArgs {
    Geom g;
    const float4 *rays;
    const lsnif_train_target *gt;
    uint32_t n;
    const uint8_t *nvox;
    const float *z;           // [n][ldz] raw outputs
    float *dz;                // [n][ldz] d loss / d z
    uint32_t ldz, out_dim, n_mat, has_albedo;
    double *loss_acc;         // sum of the per-ray losses
};

struct AdamArgs {
    float *p, *m, *v;
    const float *g;
    uint64_t count;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
};

hipError_t launch_train_fill(float *a, uint64_t na, float *b, uint64_t nb, double *acc, hipStream_t s);
hipError_t launch_train_encode(const TrainEncArgs &A, bool backward, hipStream_t s);
hipError_t launch_train_gemm(const GemmArgs &G, int epi, hipStream_t s);
hipError_t launch_train_loss(const TrainLossArgs &A, hipStream_t s);
hipError_t launch_train_loss_final(const double *acc, uint32_t n, float *loss, hipStream_t s);
hipError_t launch_adam(const AdamArgs &A, hipStream_t s);

}  // namespace lsnif
