// Non-standard normal front end (Appendix A): N(mu, Sigma) truncated to
// {A x <= b} with Sigma = L L^T becomes u ~ N(0, I) truncated to
// {(A L) u <= b - A mu}, and samples map back as x = L u + mu.  These kernels
// run once per problem (A L, b - A mu) and once per trace (L u + mu); sums
// are float64.
#pragma once
#include <hip/hip_runtime.h>

namespace ess {

// C (m x n) = X (m x k) * B (k x n), or X * B^T when trans_b (B then n x k),
// plus add[j] on column j when add is given; row-major, float64 sums, C
// rounded to TC.  16 x 16 output tiles through LDS, one element per thread.
template <typename TX, typename TC>
__global__ __launch_bounds__(256) void gemm_tiled_f64(const TX* __restrict__ X,
                                                      const double* __restrict__ B, int m, int k,
                                                      int n, int trans_b,
                                                      const double* __restrict__ add,
                                                      TC* __restrict__ C) {
    __shared__ double xs[16][17];
    __shared__ double bs[16][17];
    const int tiles_n = (n + 15) / 16;   // one-dimensional grid over the tiles
    const int t_row = static_cast<int>(blockIdx.x) / tiles_n, t_col = static_cast<int>(blockIdx.x) % tiles_n;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = t_row * 16 + ty, col = t_col * 16 + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < k; k0 += 16) {
        const int xr = row, xc = k0 + tx;
        xs[ty][tx] = (xr < m && xc < k) ? static_cast<double>(X[static_cast<size_t>(xr) * k + xc]) : 0.0;
        const int br = k0 + ty, bc = col;   // element (br, bc) of B
        double bv = 0.0;
        if (br < k && bc < n)
            bv = trans_b ? B[static_cast<size_t>(bc) * k + br] : B[static_cast<size_t>(br) * n + bc];
        bs[ty][tx] = bv;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) acc = fma(xs[ty][j], bs[j][tx], acc);
        __syncthreads();
    }
    if (row < m && col < n) {
        if (add) acc += add[col];
        C[static_cast<size_t>(row) * n + col] = static_cast<TC>(acc);
    }
}

// out[i] = b[i] - sum_j A[i, j] mu[j]: one wave per row, float64 sums in a
// fixed order (lanes stride the row, then a butterfly).
template <typename TA>
__global__ __launch_bounds__(256) void shift_rhs(const TA* __restrict__ A,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ mu, int m, int d,
                                                 double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
    if (i >= m) return;   // whole waves leave together
    double s = 0.0;
    for (int j = lane; j < d; j += 64) s = fma(static_cast<double>(A[static_cast<size_t>(i) * d + j]), mu[j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[i] = b[i] - s;
}

}  // namespace ess
