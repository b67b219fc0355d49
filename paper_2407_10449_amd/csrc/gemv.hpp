// Row-parallel projections for small chain groups (few chains per context).
#pragma once
#include <hip/hip_runtime.h>

#include "gemm.hpp"

namespace ess {

// Projections of a few chains (at most NG CW in the group).  The tile GEMM
// pads the chain axis to whole tiles, so with one or ten chains nearly all of
// its matrix work is padding and its time is the latency of a long K loop.
//
// Here a 256-thread workgroup owns four rows of A.  Its four waves split the
// work as NG chain groups of CW chains times KS slices of K (NG KS = 4):
// - wave w takes chains [CW (w % NG), CW (w % NG) + CW) and every KS-th
//   256-column stretch of K starting at stretch w / NG;
// - its lanes read four consecutive columns (16-byte loads) and keep the
//   4 x 2 CW partial sums (x' and nu of every chain) in registers;
// - a butterfly over the wave, then a sum of the KS slices through LDS in
//   slice order, finishes every value in a fixed order.
// Splitting K over waves keeps four times as many loads in flight as one
// wave per row group would, which is what a launch over a few thousand rows
// needs to reach the memory bandwidth.  A is streamed once per launch; the
// chain rows come from the caches.  Rows are padded to mp (a multiple of 128)
// and K to a multiple of 32, so every read stays inside the buffers.
//
// The sums are kept in float64 for float storage too: a product of two floats
// is exact in float64, so the only rounding left is the final one to T.  At
// these chain counts the kernel waits on memory and latency, and the float64
// arithmetic costs little, while float32 sums over K = d terms of unscaled
// rows (|a_i| near sqrt(d)) move the arc ends by more than the trim and turn
// into safeguard rejections (Section 3.3).
// Four consecutive elements from a 16-byte aligned address.
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
    const double2 t0 = reinterpret_cast<const double2*>(p)[0];
    const double2 t1 = reinterpret_cast<const double2*>(p)[1];
    v[0] = t0.x;
    v[1] = t0.y;
    v[2] = t1.x;
    v[3] = t1.y;
}

template <typename T, int CW, int NG>
__global__ __launch_bounds__(256) void proj_gemv(const T* __restrict__ A,
                                                 const T* __restrict__ B0,
                                                 const T* __restrict__ B1, int K, int cols,
                                                 ProjOut o) {
    constexpr int R = 4, KS = 4 / NG;
    constexpr int UNROLL = CW <= 2 ? 2 : 1;   // two stretches in flight when registers allow
    static_assert(NG * KS == 4, "four waves per workgroup");
    __shared__ double red[KS][NG][2 * CW][R];
    const int lane = threadIdx.x & 63;
    const int w = static_cast<int>(threadIdx.x >> 6);
    const int grp = w % NG, slice = w / NG;
    const int i0 = blockIdx.x * R;   // the grid covers o.m rows exactly (rounded up to R)
    const int nch = min(o.C - o.c0, o.Cg);
    const int cb = grp * CW;         // the wave's first chain
    const bool do_x = cols != 1, do_n = cols != 0;   // 0: x' only, 1: nu only, 2: both
    double ax[R][CW], an[R][CW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            ax[r][c] = 0.0;
            an[r][c] = 0.0;
        }
    // Loads carry no branches: a chain past the group's end reads the last
    // chain's row (valid memory; its sums are never stored), and a column set
    // that is not asked for reads the other one.
    const T* bx = do_x ? B0 : B1;
    const T* bn = do_n ? B1 : B0;
    if (cb < nch) {
#pragma unroll UNROLL
        for (int k = 4 * lane + 256 * slice; k < K; k += 256 * KS) {
            T a[R][4], xv[CW][4], nv[CW][4];
#pragma unroll
            for (int r = 0; r < R; ++r) load4(A + static_cast<size_t>(i0 + r) * K + k, a[r]);
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const size_t off = static_cast<size_t>(min(cb + c, nch - 1)) * K + k;
                load4(bx + off, xv[c]);
                load4(bn + off, nv[c]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double ad[R];
#pragma unroll
                for (int r = 0; r < R; ++r) ad[r] = static_cast<double>(a[r][e]);
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const double xd = static_cast<double>(xv[c][e]);
                    const double nd = static_cast<double>(nv[c][e]);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        ax[r][c] = fma(ad[r], xd, ax[r][c]);
                        an[r][c] = fma(ad[r], nd, an[r][c]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                ax[r][c] += __shfl_xor(ax[r][c], off, 64);
                an[r][c] += __shfl_xor(an[r][c], off, 64);
            }
    // every lane holds the wave's sums; lane j keeps value j (column j / 2,
    // x' when j is even, nu when odd) of the four rows in LDS
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (lane == 2 * c) red[slice][grp][2 * c][r] = ax[r][c];
            if (lane == 2 * c + 1) red[slice][grp][2 * c + 1][r] = an[r][c];
        }
    __syncthreads();
    if (slice != 0 || lane >= 2 * CW) return;
    const int c = lane >> 1;
    if (cb + c >= nch) return;
    const bool is_x = (lane & 1) == 0;
    if (is_x ? !do_x : !do_n) return;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        v[r] = red[0][grp][lane][r];
#pragma unroll
        for (int sl = 1; sl < KS; ++sl) v[r] += red[sl][grp][lane][r];
    }
    // x' of chain cb + c is virtual column cb + c, nu is column Cg + cb + c
    proj_store4<T>(o, is_x ? cb + c : o.Cg + cb + c, i0, static_cast<T>(v[0]),
                   static_cast<T>(v[1]), static_cast<T>(v[2]), static_cast<T>(v[3]));
}

}  // namespace ess
