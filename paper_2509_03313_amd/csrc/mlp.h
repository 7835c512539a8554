// mlp.h -- launch helpers of the surrogate perceptron kernels (mlp.hip), used by
// the C ABI in mlp_api.cpp.  Internal: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct gsbs_mlp;

namespace gsbs {

// Architecture: 296 inputs, four hidden layers of 256 (GELU), 7 outputs.
constexpr int kMlpIn = 296;
constexpr int kMlpHidden = 256;
constexpr int kMlpOut = 7;
constexpr int kMlpLayers = 5;

// C = A B^T; work (work_elems floats, may be null) holds the partial products
// when the reduction is split.
void mlp_gemm_nt(hipStream_t st, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc, int M,
                 int N, int K, float* work, size_t work_elems);
void mlp_input(hipStream_t st, const float* x, int B, int n_in, uint16_t* X, uint16_t* XT, int Mp, int Kp);
// One forward layer: X W^T with the layer epilogue fused into the product's
// store (Z = XW^T + bias; hidden: A = BF16(GELU(Z)), Z and AT when not null;
// output: Y = Z as FP32 B x n_valid).
void mlp_gemm_layer(hipStream_t st, const uint16_t* A, const uint16_t* W, int Mp, int Np, int Kp, const float* bias,
                    int B, int n_valid, int hidden, float* Z, uint16_t* Aout, uint16_t* AT, float* Y);
void mlp_loss(hipStream_t st, const float* Y, const float* T, int B, int n_out, int Mp, int Np, float* dZ,
              uint16_t* dZb, uint16_t* dZT, float* loss);
void mlp_act_grad(hipStream_t st, const float* dA, const float* Z, int B, int Mp, int Np, int n_valid, float* dZ,
                  uint16_t* dZb, uint16_t* dZT);
// Column sums of dZ; work holds ceil(Mp / 512) x Np partial sums.
void mlp_colsum(hipStream_t st, const float* dZ, int Mp, int Np, float* db, float* work);
void mlp_adam(hipStream_t st, float* w, float* m1, float* m2, const float* grad, int64_t n, int rows, int cols,
              float lr, float beta1, float beta2, float eps, float c1, float c2, uint16_t* wb, uint16_t* wbt);
void mlp_cast(hipStream_t st, const float* w, int64_t n, int rows, int cols, uint16_t* wb, uint16_t* wbt);

// Forward pass of x[batch][296] (device) into y[batch][7] (device), synchronised.
int mlp_forward_sync(gsbs_mlp* m, const float* x, int batch, float* y);

}  // namespace gsbs
