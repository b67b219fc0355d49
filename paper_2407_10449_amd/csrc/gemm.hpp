// Constraint projections for a block of chains: out[c][i] = a_i^T y_c.
//
// One launch covers a group of Cg chains starting at chain c0, as a "virtual"
// column axis of length 2 Cg: columns [0, Cg) read the proposals x' (their
// projections A x' are the safeguard check of Section 3.3 and, once accepted,
// the next step's A x_t), columns [Cg, 2 Cg) read the next ellipse directions
// nu (their projections A nu are the q_i of the trigonometric equation,
// Section 2).  The paper notes both products are the O(md) part of a step
// (Section 2.2).  B0 and B1 point at the group's first row.
//
// Layout (all padded by the host so no tile ever leaves its buffers):
//   A  [mp][dp]  row-major, rows >= m and columns >= d are zero
//   Y  [Cp][dp]  one row per chain (x' or nu), columns >= d are zero
//   P  [2][Cp][mp], Q [Cp][mp]: chain-major so a chain's m projections are
//   contiguous for the per-chain interval kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ess {

struct ProjOut {
    int m, C, Cp, mp;
    int c0, Cg;       // the group's first chain and its (padded) size
    const double* b;  // b of chain c starts at b + c * bstride
    int bstride;      // 0: one b for all chains, m: one b per chain
    void* P;          // [2][Cp][mp]: the committed projections live in P[sel[c]]
    void* Q;          // [Cp][mp]
    const int* sel;   // [Cp]
    int* flag;        // [Cp]: set to 1 when a checked row is violated
    int p_direct;     // 1: write P[sel[c]] (state replaced), 0: P[1 - sel[c]] (proposal)
    int strict;       // 1: violation is p >= b (start check), 0: p > b (safeguard)
};

// Four consecutive rows i0 .. i0 + 3 of virtual column n.  bpre, when given
// and b is shared by all chains, holds b of those rows (+inf past m), loaded
// by the caller ahead of time.
template <typename T>
__device__ __forceinline__ void proj_store4(const ProjOut& o, int n, int i0, T v0, T v1, T v2,
                                            T v3, const double* bpre = nullptr) {
    if (n < o.Cg) {
        const int c = o.c0 + n;
        const int s = o.sel[c];
        const int buf = o.p_direct ? s : 1 - s;
        T* dst = static_cast<T*>(o.P) + (static_cast<size_t>(buf) * o.Cp + c) * o.mp + i0;
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
        } else {
            dst[0] = v0; dst[1] = v1; dst[2] = v2; dst[3] = v3;
        }
        if (c < o.C) {
            const T vv[4] = {v0, v1, v2, v3};
            bool bad = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + r;
                const double pv = static_cast<double>(vv[r]);
                if (bpre != nullptr && o.bstride == 0) {
                    bad |= o.strict ? (pv >= bpre[r]) : (pv > bpre[r]);
                } else if (i < o.m) {
                    const double bi = o.b[static_cast<size_t>(c) * o.bstride + i];
                    bad |= o.strict ? (pv >= bi) : (pv > bi);
                }
            }
            if (bad) o.flag[c] = 1;   // every writer stores the same value
        }
    } else {
        const int c = o.c0 + n - o.Cg;
        T* dst = static_cast<T*>(o.Q) + static_cast<size_t>(c) * o.mp + i0;
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
        } else {
            dst[0] = v0; dst[1] = v1; dst[2] = v2; dst[3] = v3;
        }
    }
}

// blockIdx -> (tile row, tile column).  Workgroups are dispatched round-robin
// over the 8 XCDs, so consecutive ids land on different L2s.  The id is first
// regrouped so that each XCD receives a contiguous run of logical tiles, and
// logical tiles walk a band of group_m tile rows before moving right: the
// tiles one XCD holds share few A row panels and few chain panels.
__device__ __forceinline__ void tile_coords(int bid, int tiles_m, int tiles_n, int group_m,
                                            int& tm, int& tn) {
    const int nt = tiles_m * tiles_n;
    int logical = bid;
    if ((nt & 7) == 0) logical = (bid & 7) * (nt >> 3) + (bid >> 3);
    const int per_group = group_m * tiles_n;
    const int g = logical / per_group;
    const int first = g * group_m;
    const int rows = min(tiles_m - first, group_m);
    const int r = logical - g * per_group;
    tm = first + r % rows;
    tn = r / rows;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 projections on the matrix cores (v_mfma_f32_16x16x4_f32), float32
// accumulation.  NW_M x NW_N waves, each owning a (BM / NW_M) x (BN / NW_N)
// block of 16 x 16 MFMA tiles; 128 x 128 tiles use 4 x 2 waves (two per
// SIMD, which hides LDS and barrier latency behind the other wave's MFMAs).  K advances 32 at a time through a double-
// buffered LDS tile.  Inside each group of 16 k, lane l supplies the four k
// values 4 (l / 16) .. 4 (l / 16) + 3 of its row as one 16-byte LDS read, and
// MFMA number kk uses element kk: A and B use the same k for the same (lane
// group, kk), so the contraction covers all 16 k exactly once.  Rows in LDS
// are padded by PADK floats so that the rows of one fragment read fall on
// distinct banks; the padding never changes the order of the sums, so every
// tile shape and padding gives bit-identical products.
template <int BM, int BN, int PADK = 4>
struct GemmLds {
    static constexpr int BK = 32, LK = BK + PADK;
    float As[2][BM * LK];
    float Bs[2][BN * LK];
};

// One BM x BN output tile at (m0, n0) of the group described by `o`; B0 / B1
// point at the group's first x' / nu row.  All NW_M x NW_N waves of the block
// call it; the tile ends with the block synchronised.
template <int BM, int BN, int NW_M = 2, int NW_N = 2, int PADK = 4>
__device__ __forceinline__ void gemm_tile_f32(const float* __restrict__ A,
                                              const float* __restrict__ B0,
                                              const float* __restrict__ B1, int K, int m0, int n0,
                                              const ProjOut& o, GemmLds<BM, BN, PADK>& L) {
    constexpr int NT = 64 * NW_M * NW_N;
    constexpr int BK = GemmLds<BM, BN, PADK>::BK, LK = GemmLds<BM, BN, PADK>::LK;
    constexpr int WM = BM / NW_M, WN = BN / NW_N, TM = WM / 16, TN = WN / 16;
    constexpr int ALD = BM * BK / 4 / NT, BLD = BN * BK / 4 / NT;
    static_assert(ALD >= 1 && BLD >= 1 && TM >= 1 && TN >= 1, "tile too small for the waves");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NW_N, wn = wave % NW_N;
    const float* Ab = A + static_cast<size_t>(m0) * K;
    const float* Bb = (n0 < o.Cg) ? B0 + static_cast<size_t>(n0) * K
                                  : B1 + static_cast<size_t>(n0 - o.Cg) * K;

    f32x4 ra[ALD], rb[BLD];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < ALD; ++i) {
            const int idx = tid + i * NT, row = idx >> 3, kq = idx & 7;
            ra[i] = *reinterpret_cast<const f32x4*>(Ab + static_cast<size_t>(row) * K + k0 + kq * 4);
        }
#pragma unroll
        for (int i = 0; i < BLD; ++i) {
            const int idx = tid + i * NT, row = idx >> 3, kq = idx & 7;
            rb[i] = *reinterpret_cast<const f32x4*>(Bb + static_cast<size_t>(row) * K + k0 + kq * 4);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < ALD; ++i) {
            const int idx = tid + i * NT, row = idx >> 3, kq = idx & 7;
            *reinterpret_cast<f32x4*>(&L.As[buf][row * LK + kq * 4]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < BLD; ++i) {
            const int idx = tid + i * NT, row = idx >> 3, kq = idx & 7;
            *reinterpret_cast<f32x4*>(&L.Bs[buf][row * LK + kq * 4]) = rb[i];
        }
    };

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // b of this thread's output rows, read before the main loop so that its
    // latency hides there (with one b for all chains; a b per chain is read
    // per element in the epilogue).  Stores to P may alias b for the compiler,
    // which otherwise reloads it after every store.
    double brow[TM][4];
    if (n0 < o.Cg && o.bstride == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
                brow[i][r] = row < o.m ? o.b[row] : __builtin_inf();
            }
    }

    const int KT = K / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < KT) gload((kt + 1) * BK);
#pragma unroll
        for (int kc = 0; kc < BK / 16; ++kc) {
            f32x4 af[TM], bf[TN];
            const int kofs = kc * 16 + (lane >> 4) * 4;
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const f32x4*>(
                    &L.As[buf][(wm * WM + i * 16 + (lane & 15)) * LK + kofs]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bf[j] = *reinterpret_cast<const f32x4*>(
                    &L.Bs[buf][(wn * WN + j * 16 + (lane & 15)) * LK + kofs]);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][kk], bf[j][kk],
                                                                         acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < KT) lstore(buf ^ 1);
        __syncthreads();
    }

    // MFMA 16x16 output: lane l holds rows 4 (l / 16) .. + 3 of column l % 16.
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int i0 = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
            const int n = n0 + wn * WN + j * 16 + (lane & 15);
            proj_store4<float>(o, n, i0, acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3],
                               brow[i]);
        }
}

// One launch of gemm_tile_f32 tiles over a group of chains (see above), with
// the XCD-aware tile order of tile_coords.
template <int BM, int BN, int NW_M, int NW_N>
__global__ __launch_bounds__(64 * NW_M * NW_N) void proj_gemm_f32(const float* __restrict__ A,
                                                                  const float* __restrict__ B0,
                                                                  const float* __restrict__ B1,
                                                                  int K, int tiles_m, int tiles_n,
                                                                  int tn0, int group_m, ProjOut o) {
    // rows of 40 floats: measured free of LDS bank conflicts at the
    // benchmarked shape, where rows of 36 conflicted (about 3.2M conflict
    // cycles per launch) and cost 3 % of the kernel time
    __shared__ __attribute__((aligned(16))) GemmLds<BM, BN, 8> lds;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, group_m, tm, tn);
    tn += tn0;
    gemm_tile_f32<BM, BN, NW_M, NW_N, 8>(A, B0, B1, K, tm * BM, tn * BN, o, lds);
}

// ---------------------------------------------------------------------------
// float32 projections through exact bfloat16 splits on the bfloat16 matrix
// cores (v_mfma_f32_16x16x32_bf16), float32 accumulation.
//
// Every float32 operand x is split into three bfloat16 pieces,
//   hi = bf16(x), mid = bf16(x - hi), lo = x - hi - mid,
// each rounded to nearest: x - hi keeps at most 16 significant bits and
// x - hi - mid at most 8, so lo is exact and hi + mid + lo = x exactly.  Of
// the nine products of pieces, the six down to relative size 2^-16 are
// accumulated (hi hi, hi mid, mid hi, hi lo, mid mid, lo hi); the three
// dropped ones (mid lo, lo mid, lo lo) are below 2^-24 of |a x| together,
// the size of one float32 rounding, and carry random signs.  Measured on
// random 2000 x 2048 x 1000 products the error against float64 stays below
// that of a float32 sum of the same terms.  Products of bfloat16 pieces are
// exact in float32, so only the float32 accumulation rounds.
//
// A is split once at init (three [mp][dp] arrays of bfloat16); the x' and
// nu rows stay float32 in memory and are split while they are staged into
// LDS.  Tiles of 128 x 128 (eight waves) or 64 x 64 (four waves), K slabs of
// 32 (one MFMA deep), double-buffered LDS.
// A row of a slab is 32 bfloat16 = four 16-byte chunks, stored unpadded with
// chunk q of row r at position q ^ ((r >> 2) & 3): the 16 rows of a fragment
// read (one chunk each) and the 16 chunks of four rows a store covers both
// fall on 16 distinct 16-byte bank groups.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int BT>
struct SplitLds {
    static constexpr int BM = BT, BN = BT, BK = 32, LK = 32;
    uint16_t a[2][3][BM * LK];
    uint16_t b[2][3][BN * LK];
};

// element offset of chunk q (8 bfloat16) of row r in a swizzled slab
__device__ __forceinline__ int split_chunk(int r, int q) {
    return r * 32 + ((q ^ ((r >> 2) & 3)) << 3);
}

// bfloat16 rounding (to nearest, ties to even) of a float's bits, as the
// high half of a float32 pattern
__device__ __forceinline__ uint32_t bf16_round_bits(uint32_t u) {
    return (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
}

// the three pieces of two floats, packed two bfloat16 per word (low half first)
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t& h, uint32_t& m,
                                           uint32_t& l) {
    const uint32_t h0 = bf16_round_bits(__float_as_uint(x0));
    const uint32_t h1 = bf16_round_bits(__float_as_uint(x1));
    const float r0 = x0 - __uint_as_float(h0), r1 = x1 - __uint_as_float(h1);
    const uint32_t m0 = bf16_round_bits(__float_as_uint(r0));
    const uint32_t m1 = bf16_round_bits(__float_as_uint(r1));
    const float s0 = r0 - __uint_as_float(m0), s1 = r1 - __uint_as_float(m1);
    h = (h0 >> 16) | h1;
    m = (m0 >> 16) | m1;
    l = (__float_as_uint(s0) >> 16) | (__float_as_uint(s1) & 0xFFFF0000u);
}

__device__ __forceinline__ void split8(const float4 v, const float4 w, uint4& h, uint4& m, uint4& l) {
    split_pair(v.x, v.y, h.x, m.x, l.x);
    split_pair(v.z, v.w, h.y, m.y, l.y);
    split_pair(w.x, w.y, h.z, m.z, l.z);
    split_pair(w.z, w.w, h.w, m.w, l.w);
}

// A (mp x dp floats) into its three bfloat16 pieces, n = mp dp elements.
__global__ __launch_bounds__(256) void split_rows_kernel(const float* __restrict__ src, size_t n,
                                                         uint16_t* __restrict__ hi,
                                                         uint16_t* __restrict__ mid,
                                                         uint16_t* __restrict__ lo) {
    for (size_t e = 2 * (static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x); e < n;
         e += 2 * static_cast<size_t>(gridDim.x) * 256) {
        uint32_t h, m, l;
        split_pair(src[e], e + 1 < n ? src[e + 1] : 0.0f, h, m, l);
        hi[e] = static_cast<uint16_t>(h);
        mid[e] = static_cast<uint16_t>(m);
        lo[e] = static_cast<uint16_t>(l);
        if (e + 1 < n) {
            hi[e + 1] = static_cast<uint16_t>(h >> 16);
            mid[e + 1] = static_cast<uint16_t>(m >> 16);
            lo[e + 1] = static_cast<uint16_t>(l >> 16);
        }
    }
}

template <int BT, int NW_M, int NW_N>
__device__ __forceinline__ void gemm_tile_split(const uint16_t* __restrict__ A0,
                                                const uint16_t* __restrict__ A1,
                                                const uint16_t* __restrict__ A2,
                                                const float* __restrict__ B0,
                                                const float* __restrict__ B1, int K, int m0, int n0,
                                                const ProjOut& o, SplitLds<BT>& L) {
    constexpr int BM = BT, BN = BT, BK = SplitLds<BT>::BK, LK = SplitLds<BT>::LK;
    constexpr int NT = 64 * NW_M * NW_N;
    constexpr int WM = BM / NW_M, WN = BN / NW_N, TM = WM / 16, TN = WN / 16;
    constexpr int LD = BM * BK / 8 / NT;   // 16-byte chunks of 8 k per thread and piece
    static_assert(LD == 1 || LD == 2, "128 x 32 slab over 256 or 512 threads");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NW_N, wn = wave % NW_N;
    const float* Bb = (n0 < o.Cg) ? B0 + static_cast<size_t>(n0) * K
                                  : B1 + static_cast<size_t>(n0 - o.Cg) * K;
    // chunk u of this thread: row idx / 4, k offset 8 (idx % 4), idx = tid + u NT
    const int r0 = tid >> 2, q0 = (tid & 3) * 8;
    const int r1 = (tid + NT) >> 2, q1 = ((tid + NT) & 3) * 8;
    const size_t ao0 = static_cast<size_t>(m0 + r0) * K + q0, ao1 = static_cast<size_t>(m0 + r1) * K + q1;
    const size_t bo0 = static_cast<size_t>(r0) * K + q0, bo1 = static_cast<size_t>(r1) * K + q1;
    const int lo0 = split_chunk(r0, q0 >> 3), lo1 = split_chunk(r1, q1 >> 3);
    // one slab's staged operands; two sets, so a slab's loads are issued two
    // slabs before they are stored to LDS (the A pieces and x' / nu rows come
    // from L2 or the MALL, whose latency exceeds one slab of matrix work)
    // two register sets (suffix _0 and _1) of one slab's operands each
    uint4 a00_0, a01_0, a02_0, a10_0, a11_0, a12_0, a00_1, a01_1, a02_1, a10_1, a11_1, a12_1;
    float4 b0a_0, b0b_0, b1a_0, b1b_0, b0a_1, b0b_1, b1a_1, b1b_1;
#define ESS_SPLIT_GLOAD(S, k0)                                                     \
    do {                                                                           \
        a00##S = *reinterpret_cast<const uint4*>(A0 + ao0 + (k0));                 \
        a01##S = *reinterpret_cast<const uint4*>(A1 + ao0 + (k0));                 \
        a02##S = *reinterpret_cast<const uint4*>(A2 + ao0 + (k0));                 \
        b0a##S = *reinterpret_cast<const float4*>(Bb + bo0 + (k0));                \
        b0b##S = *reinterpret_cast<const float4*>(Bb + bo0 + (k0) + 4);            \
        if constexpr (LD == 2) {                                                   \
            a10##S = *reinterpret_cast<const uint4*>(A0 + ao1 + (k0));             \
            a11##S = *reinterpret_cast<const uint4*>(A1 + ao1 + (k0));             \
            a12##S = *reinterpret_cast<const uint4*>(A2 + ao1 + (k0));             \
            b1a##S = *reinterpret_cast<const float4*>(Bb + bo1 + (k0));            \
            b1b##S = *reinterpret_cast<const float4*>(Bb + bo1 + (k0) + 4);        \
        }                                                                          \
    } while (0)
#define ESS_SPLIT_LSTORE(S, buf)                                                   \
    do {                                                                           \
        uint4 h_, m_, l_;                                                          \
        split8(b0a##S, b0b##S, h_, m_, l_);                                        \
        *reinterpret_cast<uint4*>(&L.a[buf][0][lo0]) = a00##S;                     \
        *reinterpret_cast<uint4*>(&L.a[buf][1][lo0]) = a01##S;                     \
        *reinterpret_cast<uint4*>(&L.a[buf][2][lo0]) = a02##S;                     \
        *reinterpret_cast<uint4*>(&L.b[buf][0][lo0]) = h_;                         \
        *reinterpret_cast<uint4*>(&L.b[buf][1][lo0]) = m_;                         \
        *reinterpret_cast<uint4*>(&L.b[buf][2][lo0]) = l_;                         \
        if constexpr (LD == 2) {                                                   \
            split8(b1a##S, b1b##S, h_, m_, l_);                                    \
            *reinterpret_cast<uint4*>(&L.a[buf][0][lo1]) = a10##S;                 \
            *reinterpret_cast<uint4*>(&L.a[buf][1][lo1]) = a11##S;                 \
            *reinterpret_cast<uint4*>(&L.a[buf][2][lo1]) = a12##S;                 \
            *reinterpret_cast<uint4*>(&L.b[buf][0][lo1]) = h_;                     \
            *reinterpret_cast<uint4*>(&L.b[buf][1][lo1]) = m_;                     \
            *reinterpret_cast<uint4*>(&L.b[buf][2][lo1]) = l_;                     \
        }                                                                          \
    } while (0)

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    double brow[TM][4];
    if (n0 < o.Cg && o.bstride == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
                brow[i][r] = row < o.m ? o.b[row] : __builtin_inf();
            }
    }

    // slab kt: the six products of its fragments from LDS buffer kt & 1
    auto compute = [&](int buf) {
        // lane l supplies k = 8 (l / 16) .. + 7 of row l % 16 for A and of
        // column l % 16 for B; the output is rows 4 (l / 16) .. + 3 of column l % 16
        // (fragment rows start at multiples of 16, so the swizzle of row
        // l % 16 is that of the fragment's row)
        const int fa = split_chunk(wm * WM + (lane & 15), lane >> 4);
        const int fb = split_chunk(wn * WN + (lane & 15), lane >> 4);
        // read in the order the products below first need the pieces:
        // (lo A, hi B), (mid A, mid B), (hi A, lo B)
        bf16x8 af[3][TM], bfr[3][TN];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[2 - p][i] = *reinterpret_cast<const bf16x8*>(&L.a[buf][2 - p][fa + i * 16 * LK]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[p][j] = *reinterpret_cast<const bf16x8*>(&L.b[buf][p][fb + j * 16 * LK]);
        }
        // smallest products first
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                f32x4 c = acc[i][j];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], c, 0, 0, 0);
                acc[i][j] = c;
            }
    };

    // pipeline: slab kt in LDS, slab kt + 1 staged in registers, slab kt + 2
    // being fetched; two iterations per trip so the register sets keep their
    // roles (K is a multiple of 32; an odd slab count ends with one half trip)
    const int KT = K / BK;
    ESS_SPLIT_GLOAD(_0, 0);
    ESS_SPLIT_LSTORE(_0, 0);
    if (KT > 1) ESS_SPLIT_GLOAD(_1, BK);
    __syncthreads();
    for (int kt = 0; kt < KT; kt += 2) {
        // even slab kt: set _1 holds slab kt + 1, set _0 is free
        if (kt + 2 < KT) ESS_SPLIT_GLOAD(_0, (kt + 2) * BK);
        compute(0);
        if (kt + 1 < KT) ESS_SPLIT_LSTORE(_1, 1);
        __syncthreads();
        if (kt + 1 >= KT) break;
        // odd slab kt + 1: set _0 holds slab kt + 2, set _1 is free
        if (kt + 3 < KT) ESS_SPLIT_GLOAD(_1, (kt + 3) * BK);
        compute(1);
        if (kt + 2 < KT) ESS_SPLIT_LSTORE(_0, 0);
        __syncthreads();
    }
#undef ESS_SPLIT_GLOAD
#undef ESS_SPLIT_LSTORE
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int i0 = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
            const int n = n0 + wn * WN + j * 16 + (lane & 15);
            proj_store4<float>(o, n, i0, acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3],
                               brow[i]);
        }
}

template <int BT, int NW_M, int NW_N>
__global__ __launch_bounds__(64 * NW_M * NW_N) void proj_gemm_split(
    const uint16_t* __restrict__ A0, const uint16_t* __restrict__ A1,
    const uint16_t* __restrict__ A2, const float* __restrict__ B0, const float* __restrict__ B1,
    int K, int tiles_m, int tiles_n, int tn0, int group_m, ProjOut o) {
    __shared__ __attribute__((aligned(16))) SplitLds<BT> lds;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, group_m, tm, tn);
    tn += tn0;
    gemm_tile_split<BT, NW_M, NW_N>(A0, A1, A2, B0, B1, K, tm * BT, tn * BT, o, lds);
}

// float64 projections on the vector ALUs (MI355X runs float64 FMA on the
// vector units at the same rate as its float64 matrix cores).  64 x 64 tile,
// each thread a 4 x 4 block: rows 4 ty .. 4 ty + 3, columns tx + 16 u.
template <int BM, int BN>
__global__ __launch_bounds__(256) void proj_gemm_f64(const double* __restrict__ A,
                                                     const double* __restrict__ B0,
                                                     const double* __restrict__ B1, int K,
                                                     int tiles_m, int tiles_n, int tn0,
                                                     int group_m, ProjOut o) {
    static_assert(BM == 64 && BN == 64, "float64 projection tile is 64 x 64");
    constexpr int BK = 16;
    __shared__ double As[BK][BM + 1];
    __shared__ double Bs[BK][BN + 1];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, group_m, tm, tn);
    tn += tn0;
    const int m0 = tm * BM, n0 = tn * BN;
    const double* Ab = A + static_cast<size_t>(m0) * K;
    const double* Bb = (n0 < o.Cg) ? B0 + static_cast<size_t>(n0) * K
                                   : B1 + static_cast<size_t>(n0 - o.Cg) * K;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = tid + r * 256, row = idx / BK, k = idx % BK;
            As[k][row] = Ab[static_cast<size_t>(row) * K + k0 + k];
            Bs[k][row] = Bb[static_cast<size_t>(row) * K + k0 + k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            double a[4], bv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = As[k][ty * 4 + v];
#pragma unroll
            for (int u = 0; u < 4; ++u) bv[u] = Bs[k][tx + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[v][u] = fma(a[v], bv[u], acc[v][u]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        proj_store4<double>(o, n0 + tx + 16 * u, m0 + ty * 4, acc[0][u], acc[1][u], acc[2][u],
                            acc[3][u]);
}

}  // namespace ess
