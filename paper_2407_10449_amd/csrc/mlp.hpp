// The warm-start network: a fully connected stack with exact GELU between
// layers, trained with mean squared error and Adam, run on the matrix cores
// in bfloat16 with float32 accumulation and float32 master weights.
//
//   forward   Z_l = H_{l-1} W_l^T + c_l,  H_l = bf16(gelu(Z_l))   (H_{-1} = input)
//   output    Y = H_{L-2} W_{L-1}^T + c_{L-1}
//   loss      mean over all outputs of (Y - T)^2; dY = 2 (Y - T) / (B n_out)
//   backward  dW_l = dZ_l^T H_{l-1},  dc_l = column sums of dZ_l,
//             dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
// gelu(z) = z Phi(z) (Hendrycks & Gimpel), gelu'(z) = Phi(z) + z phi(z).
// Adam follows Kingma & Ba with bias corrections.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ess {

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // nearest, ties to even
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__device__ __forceinline__ float gelu_f(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

enum MlpEpiMode {
    EPI_STORE = 0,    // out_f = acc
    EPI_HIDDEN = 1,   // z = acc + bias -> out_f (Z), out_b = bf16(gelu(z))
    EPI_OUTPUT = 2,   // out_f = acc + bias
    EPI_DGELU = 3     // g = acc * gelu'(zin) -> out_f, out_b = bf16(g)
};

struct MlpGemm {
    int M, N, K;
    const uint16_t* A;   // A(i, k) = A[i * sa0 + k * sa1]
    long long sa0, sa1;
    const uint16_t* B;   // B(k, j) = B[k * sb0 + j * sb1]
    long long sb0, sb1;
    int mode;
    const float* bias;   // [N]
    const float* zin;    // [M][ldo]
    float* out_f;        // [M][ldo]
    uint16_t* out_b;     // [M][ldo]
    int ldo;
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

// C[i][j] = sum_k A(i, k) B(k, j) for strided bfloat16 operands (any layout),
// 64 x 64 tile per 256 threads, v_mfma_f32_16x16x16_bf16 (lane l supplies the
// four k values 4 (l / 16) .. + 3 of row / column l % 16), K staged 32 at a
// time through LDS; out-of-range elements load as zero.
__global__ __launch_bounds__(256) void mlp_gemm_kernel(MlpGemm g) {
    constexpr int BK = 32, LK = BK + 8;
    __shared__ __attribute__((aligned(16))) uint16_t As[64 * LK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int tiles_n = (g.N + 63) / 64;
    const int m0 = (blockIdx.x / tiles_n) * 64, n0 = (blockIdx.x % tiles_n) * 64;
    mf32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = mf32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        for (int e = tid; e < 64 * BK; e += 256) {
            const int r = e / BK, k = e % BK;
            const int gi = m0 + r, gk = k0 + k, gj = n0 + r;
            As[r * LK + k] = (gi < g.M && gk < g.K) ? g.A[gi * g.sa0 + gk * g.sa1] : uint16_t(0);
            Bs[r * LK + k] = (gj < g.N && gk < g.K) ? g.B[gk * g.sb0 + gj * g.sb1] : uint16_t(0);
        }
        __syncthreads();
        for (int kc = 0; kc < BK; kc += 16) {
            const int kofs = kc + (lane >> 4) * 4;
            bf16x4 a[2], b[2];
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x4*>(&As[(wm * 32 + i * 16 + (lane & 15)) * LK + kofs]);
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x4*>(&Bs[(wn * 32 + j * 16 + (lane & 15)) * LK + kofs]);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                const size_t o = static_cast<size_t>(row) * g.ldo + col;
                const float x = acc[i][j][v];
                if (g.mode == EPI_STORE) {
                    g.out_f[o] = x;
                } else if (g.mode == EPI_HIDDEN) {
                    const float z = x + g.bias[col];
                    g.out_f[o] = z;
                    g.out_b[o] = to_bf16(gelu_f(z));
                } else if (g.mode == EPI_OUTPUT) {
                    g.out_f[o] = x + g.bias[col];
                } else {
                    const float d = x * gelu_grad_f(g.zin[o]);
                    g.out_f[o] = d;
                    g.out_b[o] = to_bf16(d);
                }
            }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x)
        y[i] = to_bf16(x[i]);
}

// dY = 2 (Y - T) / n (float32 and bfloat16) and the block's partial loss.
__global__ void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                long long n, float* __restrict__ dy, uint16_t* __restrict__ dyb,
                                double* __restrict__ partial) {
    __shared__ double red[256];
    double s = 0.0;
    const float scale = 2.0f / static_cast<float>(n);
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const float e = Y[i] - T[i];
        s += static_cast<double>(e) * e;
        const float g = scale * e;
        dy[i] = g;
        dyb[i] = to_bf16(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dc[j] = sum_i dz[i][j] (rows strided by ld), one thread per column.
__global__ void colsum_kernel(const float* __restrict__ dz, int rows, int cols, int ld,
                              float* __restrict__ dc) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += dz[static_cast<size_t>(i) * ld + j];
    dc[j] = s;
}

// One Adam step over the flat parameter vector; c1 = 1 / (1 - b1^t),
// c2 = 1 / (1 - b2^t).
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

}  // namespace ess
