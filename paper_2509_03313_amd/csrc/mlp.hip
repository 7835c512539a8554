// mlp.hip -- gfx950 kernels of the inter-pulse surrogate: a 296-256-256-256-256-7
// perceptron with erf-GELU hidden layers, BF16 weights and activations and FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), its backward pass
// and an Adam update on FP32 master weights.
//
// Every matrix product has the form C[M x N] = A[M x K] * B[N x K]^T with both
// operands K-contiguous in BF16 and M, N, K multiples of 32 (zero padded), so
// one kernel serves the forward product (X W^T), the input gradient
// (dZ (W^T)^T) and the weight gradient (dZ^T (X^T)^T): the producers also
// write the transposed copies the products need.
#include <algorithm>

#include "mlp.h"

namespace gsbs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpBlock = 256;

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU (erf form) and its derivative.  The normal CDF is taken as
// erfc(-z/sqrt 2)/2, which keeps its relative accuracy in the lower tail where
// 1 + erf(z/sqrt 2) would cancel in FP32.
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * erfcf(-z * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float z) {
    const float cdf = 0.5f * erfcf(-z * 0.70710678118654752f);
    const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// C = A B^T on the matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16).  A
// block of 4 waves computes a 64 x 64 tile of C, each wave a 32 x 32 quarter
// as 2 x 2 MFMA tiles.  Per K step of 32 the block stages A[64][32] and
// B[64][32] in LDS -- one 16-byte global load per thread and operand, rows
// padded by 16 bytes against bank conflicts -- and each wave reads its
// fragments from there: lane l feeds row l%16 of an A tile and of a B tile
// with the 8 values k = 8 (l/16) .. +7 and receives C[4 (l/16) + i][l%16],
// i = 0..3, of each tile.  M, N, K are multiples of 32 (zero padded); rows
// beyond M or N of a partial tile load zeros and store nothing.  With a split
// of the reduction (blockIdx.z > 0 possible) block z sums k in [z kc, z kc + kc)
// and writes its partial product to C + z M ldc; k_sum_splits adds them up.
constexpr int kGemmTile = 64;
constexpr int kGemmK = 32;
constexpr int kGemmPad = 8;  // BF16 values of row padding in LDS

// Layer epilogue applied to the product as it leaves the registers (forward
// pass; bias null: plain store of C): Z = C + bias; hidden layers A = BF16(GELU(Z))
// (Z and the transpose AT kept only when not null), rows >= B and columns
// >= n_valid 0; output layer Y = Z (FP32, B x n_valid).
struct MlpEpi {
    const float* bias;
    float* Z;
    uint16_t* A;
    uint16_t* AT;
    float* Y;
    int32_t B, n_valid, hidden, Mp;
};

__device__ __forceinline__ void epi_store(const MlpEpi& q, int row, int col, int Np, float v) {
    const bool valid = row < q.B && col < q.n_valid;
    const float z = valid ? v + q.bias[col] : 0.0f;
    const size_t e = (size_t)row * Np + col;
    if (q.hidden) {
        if (q.Z) q.Z[e] = z;
        const uint16_t h = to_bf16(valid ? gelu(z) : 0.0f);
        q.A[e] = h;
        if (q.AT) q.AT[(size_t)col * q.Mp + row] = h;
    } else if (valid) {
        q.Y[(size_t)row * q.n_valid + col] = z;
    }
}

__global__ __launch_bounds__(kMlpBlock) void k_gemm_nt(const uint16_t* __restrict__ A, int32_t lda,
                                                     const uint16_t* __restrict__ B, int32_t ldb,
                                                     float* __restrict__ C, int32_t ldc, int32_t M, int32_t N,
                                                     int32_t K, int32_t kc, MlpEpi epi) {
    __shared__ __align__(16) uint16_t sa[kGemmTile][kGemmK + kGemmPad];
    __shared__ __align__(16) uint16_t sb[kGemmTile][kGemmK + kGemmPad];
    const int bm = blockIdx.y * kGemmTile, bn = blockIdx.x * kGemmTile;
    const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
    C += (size_t)blockIdx.z * M * ldc;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = t >> 2, lq = (t & 3) * 8;  // loader: row and 8-value chunk of the K slice
    const bool va = bm + lr < M, vb = bn + lr < N;
    const uint16_t* pa = A + (size_t)(bm + lr) * lda + lq;
    const uint16_t* pb = B + (size_t)(bn + lr) * ldb + lq;
    const int r = lane & 15, g = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += kGemmK) {
        const uint4 ra = va ? *reinterpret_cast<const uint4*>(pa + k0) : make_uint4(0u, 0u, 0u, 0u);
        const uint4 rb = vb ? *reinterpret_cast<const uint4*>(pb + k0) : make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();  // the previous slice has been read
        *reinterpret_cast<uint4*>(&sa[lr][lq]) = ra;
        *reinterpret_cast<uint4*>(&sb[lr][lq]) = rb;
        __syncthreads();
        bf16x8 fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = *reinterpret_cast<const bf16x8*>(&sa[wm + 16 * i + r][g]);
#pragma unroll
        for (int j = 0; j < 2; ++j) fb[j] = *reinterpret_cast<const bf16x8*>(&sb[wn + 16 * j + r][g]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = bm + wm + 16 * i + 4 * (lane >> 4) + e, col = bn + wn + 16 * j + r;
                if (row < M && col < N) {
                    if (epi.bias) epi_store(epi, row, col, ldc, acc[i][j][e]);
                    else C[(size_t)row * ldc + col] = acc[i][j][e];
                }
            }
}

// Sum of ns partial products work[z][M][ldc] into C[M][ldc] (columns < N),
// in a fixed order.
__global__ void k_sum_splits(const float* __restrict__ work, int32_t ns, int32_t M, int32_t N, int32_t ldc,
                             float* __restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    const int r = (int)(e / N), c = (int)(e % N);
    float s = 0.0f;
    for (int z = 0; z < ns; ++z) s += work[((size_t)z * M + r) * ldc + c];
    C[(size_t)r * ldc + c] = s;
}

// Input features (FP32, rows of n_in) -> BF16 activations X [Mp x Kp] and,
// unless XT is null, X^T [Kp x Mp], zero padded.
__global__ void k_mlp_input(const float* __restrict__ x, int32_t B, int32_t n_in, uint16_t* __restrict__ X,
                            uint16_t* __restrict__ XT, int32_t Mp, int32_t Kp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Mp * Kp) return;
    const int m = (int)(e / Kp), k = (int)(e % Kp);
    const float v = (m < B && k < n_in) ? x[(size_t)m * n_in + k] : 0.0f;
    const uint16_t h = to_bf16(v);
    X[e] = h;
    if (XT) XT[(size_t)k * Mp + m] = h;
}

// Mean squared error over the B x n_out outputs and its gradient dY =
// 2 (Y - T) / (B n_out) as BF16 (and transpose) for the products, FP32 for
// the bias gradient.  loss accumulates the sum of squares (host divides).
__global__ void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int32_t B, int32_t n_out,
                           int32_t Mp, int32_t Np, float* __restrict__ dZ, uint16_t* __restrict__ dZb,
                           uint16_t* __restrict__ dZT, float* __restrict__ loss) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.0f;
    if (e < (int64_t)Mp * Np) {
        const int m = (int)(e / Np), n = (int)(e % Np);
        float d = 0.0f;
        if (m < B && n < n_out) {
            const float r = Y[(size_t)m * n_out + n] - T[(size_t)m * n_out + n];
            sq = r * r;
            d = 2.0f * r / (float)(B * n_out);
        }
        dZ[e] = d;
        const uint16_t h = to_bf16(d);
        dZb[e] = h;
        dZT[(size_t)n * Mp + m] = h;
    }
    for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0 && sq != 0.0f) atomicAdd(loss, sq);
}

// dZ = dA * GELU'(Z) on the valid part (FP32, BF16 and BF16 transpose).
__global__ void k_mlp_act_grad(const float* __restrict__ dA, const float* __restrict__ Z, int32_t B, int32_t Mp,
                               int32_t Np, int32_t n_valid, float* __restrict__ dZ, uint16_t* __restrict__ dZb,
                               uint16_t* __restrict__ dZT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Mp * Np) return;
    const int m = (int)(e / Np), n = (int)(e % Np);
    const float d = (m < B && n < n_valid) ? dA[e] * gelu_grad(Z[e]) : 0.0f;
    dZ[e] = d;
    const uint16_t h = to_bf16(d);
    dZb[e] = h;
    dZT[(size_t)n * Mp + m] = h;
}

// Bias gradient: column sums of dZ over the batch (one thread per column).
// Column sums of dZ [Mp][Np] over a chunk of rows per blockIdx.y: 64 columns
// per block, 4 rows at a time; the partial sums go to part[chunk][Np].
constexpr int kColRows = 512;
__global__ __launch_bounds__(kMlpBlock) void k_mlp_colsum(const float* __restrict__ dZ, int32_t Mp, int32_t Np,
                                                         float* __restrict__ part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
    const int r0 = blockIdx.y * kColRows, r1 = min(Mp, r0 + kColRows);
    float s = 0.0f;
    if (c < Np)
        for (int r = r0 + q; r < r1; r += 4) s += dZ[(size_t)r * Np + c];
    red[q][threadIdx.x & 63] = s;
    __syncthreads();
    if (q == 0 && c < Np) part[(size_t)blockIdx.y * Np + c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                             (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// Adam on one parameter block; the BF16 copy (and its transpose for weight
// matrices, rows x cols = Np x Kp) is refreshed from the FP32 master.
__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ m1, float* __restrict__ m2,
                           const float* __restrict__ grad, int64_t n, int32_t rows, int32_t cols, float lr,
                           float beta1, float beta2, float eps, float c1, float c2, uint16_t* __restrict__ wb,
                           uint16_t* __restrict__ wbt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gr = grad[e];
    const float a = beta1 * m1[e] + (1.0f - beta1) * gr;
    const float b = beta2 * m2[e] + (1.0f - beta2) * gr * gr;
    m1[e] = a;
    m2[e] = b;
    const float mh = a / c1, vh = b / c2;
    const float v = w[e] - lr * mh / (sqrtf(vh) + eps);
    w[e] = v;
    if (wb) {
        const uint16_t h = to_bf16(v);
        wb[e] = h;
        const int r = (int)(e / cols), c = (int)(e % cols);
        wbt[(size_t)c * rows + r] = h;
    }
}

// Refresh BF16 weights (and transpose) from the FP32 master, keeping padding 0.
__global__ void k_mlp_cast(const float* __restrict__ w, int64_t n, int32_t rows, int32_t cols,
                           uint16_t* __restrict__ wb, uint16_t* __restrict__ wbt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint16_t h = to_bf16(w[e]);
    wb[e] = h;
    wbt[(size_t)(e % cols) * rows + e / cols] = h;
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kMlpBlock - 1) / kMlpBlock); }

void mlp_gemm_nt(hipStream_t st, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc, int M,
                 int N, int K, float* work, size_t work_elems) {
    const int tiles = ((N + kGemmTile - 1) / kGemmTile) * ((M + kGemmTile - 1) / kGemmTile);
    // few output tiles over a long reduction (the weight gradients, K = batch):
    // split K so that the launch fills the device, partial products in work
    int ns = 1;
    if (work && tiles < 256 && K >= 1024) {
        ns = std::min(std::min(64, K / 512), std::max(1, 512 / tiles));
        ns = (int)std::min<size_t>((size_t)ns, work_elems / ((size_t)M * ldc));
        ns = std::max(ns, 1);
    }
    const int kc = ns > 1 ? ((K + ns - 1) / ns + kGemmK - 1) / kGemmK * kGemmK : K;
    ns = (K + kc - 1) / kc;
    const dim3 grid((N + kGemmTile - 1) / kGemmTile, (M + kGemmTile - 1) / kGemmTile, ns);
    const MlpEpi none{};
    if (ns == 1) {
        hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kMlpBlock), 0, st, A, lda, B, ldb, C, ldc, M, N, K, K, none);
        return;
    }
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kMlpBlock), 0, st, A, lda, B, ldb, work, ldc, M, N, K, kc, none);
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for((int64_t)M * N)), dim3(kMlpBlock), 0, st, work, ns, M, N, ldc, C);
}
void mlp_gemm_layer(hipStream_t st, const uint16_t* A, const uint16_t* W, int Mp, int Np, int Kp, const float* bias,
                    int B, int n_valid, int hidden, float* Z, uint16_t* Aout, uint16_t* AT, float* Y) {
    const dim3 grid((Np + kGemmTile - 1) / kGemmTile, (Mp + kGemmTile - 1) / kGemmTile, 1);
    const MlpEpi epi{bias, Z, Aout, AT, Y, B, n_valid, hidden, Mp};
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kMlpBlock), 0, st, A, Kp, W, Kp, (float*)nullptr, Np, Mp, Np, Kp, Kp, epi);
}
void mlp_input(hipStream_t st, const float* x, int B, int n_in, uint16_t* X, uint16_t* XT, int Mp, int Kp) {
    hipLaunchKernelGGL(k_mlp_input, dim3(blocks_for((int64_t)Mp * Kp)), dim3(kMlpBlock), 0, st, x, B, n_in, X, XT,
                       Mp, Kp);
}
void mlp_loss(hipStream_t st, const float* Y, const float* T, int B, int n_out, int Mp, int Np, float* dZ,
              uint16_t* dZb, uint16_t* dZT, float* loss) {
    hipLaunchKernelGGL(k_mlp_loss, dim3(blocks_for((int64_t)Mp * Np)), dim3(kMlpBlock), 0, st, Y, T, B, n_out, Mp,
                       Np, dZ, dZb, dZT, loss);
}
void mlp_act_grad(hipStream_t st, const float* dA, const float* Z, int B, int Mp, int Np, int n_valid, float* dZ,
                  uint16_t* dZb, uint16_t* dZT) {
    hipLaunchKernelGGL(k_mlp_act_grad, dim3(blocks_for((int64_t)Mp * Np)), dim3(kMlpBlock), 0, st, dA, Z, B, Mp, Np,
                       n_valid, dZ, dZb, dZT);
}
void mlp_colsum(hipStream_t st, const float* dZ, int Mp, int Np, float* db, float* work) {
    const int chunks = (Mp + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(k_mlp_colsum, dim3((Np + 63) / 64, chunks), dim3(kMlpBlock), 0, st, dZ, Mp, Np, work);
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(Np)), dim3(kMlpBlock), 0, st, work, chunks, 1, Np, Np, db);
}
void mlp_adam(hipStream_t st, float* w, float* m1, float* m2, const float* grad, int64_t n, int rows, int cols,
              float lr, float beta1, float beta2, float eps, float c1, float c2, uint16_t* wb, uint16_t* wbt) {
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(n)), dim3(kMlpBlock), 0, st, w, m1, m2, grad, n, rows, cols, lr,
                       beta1, beta2, eps, c1, c2, wb, wbt);
}
void mlp_cast(hipStream_t st, const float* w, int64_t n, int rows, int cols, uint16_t* wb, uint16_t* wbt) {
    hipLaunchKernelGGL(k_mlp_cast, dim3(blocks_for(n)), dim3(kMlpBlock), 0, st, w, n, rows, cols, wb, wbt);
}

}  // namespace gsbs
