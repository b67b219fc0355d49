// Per-chain part of one transition: commit the previous proposal, solve every
// constraint's intersection angles, build the active intervals, draw theta,
// move, and draw the next ellipse direction.  One workgroup of 256 or 512
// threads per chain.
//
// Roots (Appendix B): p = a_i^T x, q = a_i^T nu, r = hypot(p, q),
// tau = atan2(q, p), phi = acos(b / r); the ellipse leaves the halfspace on the
// arc (tau - phi, tau + phi).  alpha = (tau - phi) wrapped into [0, 2 pi),
// beta = min(alpha + 2 phi, 2 pi), so I_i = [0, alpha] U [beta, 2 pi].
// Rows with r = 0 or b / r >= 1 never meet the ellipse (Section 3.2): the paper
// pads them with alpha = beta = 0, which only adds zero-length candidates and
// leaves every cumulative max unchanged, so they are dropped here instead.
//
// Active intervals (Algorithm 3 / Proposition 1): order the rows by alpha
// (ties by row index) and let gamma be the running max of beta in that order;
// the candidates are [0, alpha_(1)], [gamma_(k-1), alpha_(k)] for k = 2..n and
// [gamma_(n), 2 pi]; a candidate whose upper end lies below its lower end is
// empty.  Trimming (Section 3.3) moves real ends inward by eps; the ends at 0
// and 2 pi are the seam through x_t and stay.  theta is drawn by inverse CDF
// over the candidates in ascending order.
//
// Two ways to produce the same non-empty candidates:
//
// * bucket path (sample_bucket_kernel): alpha is bucketed by angle into NB
//   equal arcs (a monotone map, so buckets are a first pass of the sort), with
//   the max beta of every bucket.  An exclusive max-scan over buckets gives
//   G[b], the running max of beta over all rows of earlier buckets.  A row with
//   alpha < G[its bucket] has gamma_(k-1) >= G > alpha: its candidate is empty
//   whatever the order inside the bucket, and the cumulative max leaving the
//   bucket does not depend on that order either.  Only the remaining rows
//   ("survivors", typically a handful) need their exact predecessor max inside
//   their own bucket, found by comparing against the bucket's rows in float64.
//   The survivors' candidates are then ranked by (alpha, row) and summed in
//   ascending order.  Crowded buckets are split again (refinement, below)
//   in the kernels for few chains and beyond 4096 rows.
// * full path (full_chain): a bitonic sort of all crossing rows in LDS, for
//   chains whose survivors still exceed SMAX (adversarial inputs such as many
//   disjoint arcs spread over the circle) or when the full sort is requested,
//   done in place by the same workgroup up to 4096 rows.  Keys are
//   alpha mapped monotonically to a 48-bit fixed-point turn fraction
//   floor(alpha * 2^48 / 2 pi) above a 16-bit slot (or row) index, so one
//   64-bit compare orders them; two alphas closer than 2 pi * 2^-48
//   (2.2e-14 rad) may swap, which moves the union by at most their distance.
//
// More than 4096 rows (up to 16384) take the same two paths with every pass
// over the rows made in chunks (sample_large_kernel, fallback_large_kernel),
// after large_roots_kernel has solved the roots over the whole device (which
// the kernels for few chains also use above 2048 rows).
// The quadratic comparators sit beside them: likelihood testing at midpoints
// (Section 2.2, sample_midpoint_kernel) and Algorithm 2's sequential
// intersection (sample_alg2_kernel).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace ess {

struct SampleArgs {
    int d, m, C, Cp, dp, mp;
    int c0;               // first chain of this launch (block b handles chain c0 + b)
    uint32_t problem;
    const double* b;      // [m], or [C][m] when bstride = m
    int bstride;
    const void* P;        // [2][Cp][mp] T
    const void* Q;        // [Cp][mp] T
    void* X;              // [Cp][dp] T, committed state
    void* Xprop;          // [Cp][dp] T, proposal
    void* N;              // [Cp][dp] T, nu of this step; replaced by the next step's
    int* sel;             // [Cp]
    int* flag;            // [Cp]
    long long* rej;       // [Cp]
    double eps;
    uint64_t seed;
    uint32_t step;        // step whose nu/u are used, relative to *step_base
    const uint32_t* step_base;   // nullable: device counter added to step
    int has_pending;      // commit the previous proposal first
    int gen_next;         // write nu(step + 1) into N after the move
    void* trace;          // nullable: committed state of the previous step, [C][d] T
    const double* u_explicit;   // nullable: u instead of the Philox draw
    double* intervals;    // nullable: [C][m + 1][2]
    int* n_intervals;     // nullable: [C]
    double* theta_out;    // nullable: [C]
    void* pq_out;         // nullable: [2][C][m] T
    int* rejected_out;    // nullable: [C] (commit kernel)
    int* fb_list;         // [C]: chains handed to the full path this step
    int* fb_count;        // [2]: list length, indexed by step parity
    int force_full;       // 1: every chain takes the full path
    void* ab;             // more than 4096 rows: [Cp][mp] double2, alpha and beta per row
    uint64_t* keys;       // more than 16384 rows: [Cp][kstride] sort keys of the full sort
    int kstride;          // a power of two >= m
};

__device__ __forceinline__ uint32_t abs_step(const SampleArgs& a) {
    return a.step + (a.step_base ? *a.step_base : 0u);
}

constexpr double kKeyScale = 281474976710656.0 / kTwoPi;   // 2^48 / (2 pi)
constexpr uint64_t kKeyMax = (1ull << 48) - 1;
constexpr int SMAX = 128;   // survivors the bucket path resolves in place

// T is the storage type of p and q.  With float storage, a float32 test of
// z = b / r >= 1.01 (as b^2 >= 1.0201 r^2, relative error a few 1e-7) first
// discards rows that certainly miss the ellipse, which saves the float64 work
// for about a third of the rows at the benchmarked shape.  For every other
// row z is float64, and the two angles come from float32 functions of
// well-conditioned float64 quantities:
// * tau = atan2 of the exact floats q, p, off by a few float ulps (< 1e-6 rad);
// * phi = acos z through the half-angle form 2 asin sqrt((1 - |z|) / 2),
//   mirrored to pi - that for z < 0.  1 - |z| is formed in float64, where it
//   is exact to the rounding of z, so the one float32 rounding of its half
//   moves phi by a relative 2^-24, and sqrt and asin (argument at most
//   sqrt(1/2), where asin's slope is at most sqrt(2)) add a few ulps: phi is
//   within a few 1e-7 rad everywhere, near tangency (z -> 1, a tiny arc)
//   included, inside the 1e-6 rad trim of the interval ends.  (acos of z
//   rounded to float32 amplifies that rounding by 1 / sqrt(1 - z^2) without
//   bound near tangency.)
// With double storage both angles are float64.  The wrap, alpha, beta and
// every later comparison are float64.
template <typename T>
__device__ __forceinline__ bool solve_roots(double p, double q, double bi, double& al,
                                            double& be) {
    if (sizeof(T) == 4) {
        // z >= 1.01 as b > 0 and b^2 >= 1.0201 r^2, without a root or a
        // divide (also r = 0 for b > 0).  b < 1e18 keeps b^2 finite, so an
        // overflowing right side only sends the row on to the float64 test.
        const float pf = static_cast<float>(p), qf = static_cast<float>(q);
        const float bf = static_cast<float>(bi);
        if (bf > 0.0f && bf < 1e18f && bf * bf >= 1.0201f * (pf * pf + qf * qf)) return false;
    }
    // float p, q: their squares are exact in float64 and their sum can
    // neither overflow nor underflow, so z = b rsqrt(p^2 + q^2) is within a
    // few ulps (one reciprocal square root instead of a root and a divide)
    double z;
    if (sizeof(T) == 4) {
        const double s2 = p * p + q * q;
        if (!(s2 > 0.0)) return false;
        z = bi * rsqrt(s2);
    } else {
        const double r = hypot(p, q);
        if (!(r > 0.0)) return false;
        z = bi / r;
    }
    if (!(z < 1.0)) return false;
    z = fmax(z, -1.0);
    double tau, phi;
    if (sizeof(T) == 4) {
        tau = static_cast<double>(atan2f(static_cast<float>(q), static_cast<float>(p)));
        const float w = static_cast<float>(0.5 * (1.0 - fabs(z)));
        const double h = 2.0 * static_cast<double>(asinf(sqrtf(w)));
        phi = z >= 0.0 ? h : kPi - h;
    } else {
        tau = atan2(q, p);
        phi = acos(z);
    }
    double a = tau - phi;
    if (a < 0.0) a += kTwoPi;
    if (a >= kTwoPi) a = 0.0;
    al = a;
    be = fmin(a + 2.0 * phi, kTwoPi);
    return true;
}

__device__ __forceinline__ uint64_t sort_key(double alpha, int slot) {
    uint64_t q = static_cast<uint64_t>(alpha * kKeyScale);
    q = q > kKeyMax ? kKeyMax : q;
    return (q << 16) | static_cast<uint64_t>(slot);
}

// bit pattern of a non-negative double: integer order equals numeric order
__device__ __forceinline__ unsigned long long obits(double v) {
    return static_cast<unsigned long long>(__double_as_longlong(v));
}
__device__ __forceinline__ double ofloat(unsigned long long v) {
    return __longlong_as_double(static_cast<long long>(v));
}

// ---- block-wide helpers (256 threads = 4 waves of 64) ----
template <int NW = 4>
__device__ __forceinline__ int block_count_prefix(bool pred, int* s_w, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(pred);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[w] = __popcll(mask);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int cnt = s_w[i];
        off += (i < w) ? cnt : 0;
        tot += cnt;
    }
    __syncthreads();
    total = tot;
    return off + before;
}

struct MaxOp {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct SumOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};

// Exclusive scan of one value per thread (thread order), identity `id`, over
// a block of NW waves; s_w holds NW values.
template <typename Op, int NW = 4>
__device__ __forceinline__ double block_excl_scan(double v, double id, Op op, double* s_w) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o, 64);
        if (lane >= o) x = op(y, x);
    }
    if (lane == 63) s_w[w] = x;
    double ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = id;
    __syncthreads();
    double pre = id;
#pragma unroll
    for (int i = 0; i < NW; ++i)
        if (i < w) pre = op(pre, s_w[i]);
    __syncthreads();
    return (lane == 0) ? pre : op(pre, ex);
}

// A 64-bit value moved across lanes by one DPP control, both halves with the
// same control: lanes whose source lies outside the row, or which the row
// mask leaves out, receive 0 (the bits of +0.0).
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROW_MASK, 0xf, BOUND);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf,
                                               BOUND);
    return __longlong_as_double(static_cast<long long>(
        (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
        static_cast<unsigned>(lo)));
}

// v of lane k (k the same in every lane), in every lane of the wave
__device__ __forceinline__ double lane_value(double v, int k) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), k));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), k));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Inclusive max over lanes 0 .. lane of a wave, for values >= 0 (0 is the
// identity, which is what lanes without a source receive).  Within each row
// of 16 lanes a Hillis-Steele scan with shifts 1, 2, 4, 8 (DPP row_shr); then
// lane 15 of a row is broadcast into the next row (rows 1 and 3) and lane 31
// into rows 2 and 3 (DPP row_bcast), as in AMD's published GCN cross-lane
// scan.  Register-to-register moves only: no LDS round trip per step.
__device__ __forceinline__ double wave_incl_max(double x) {
    x = fmax(x, dpp_f64<0x111, 0xf, true>(x));   // row_shr:1
    x = fmax(x, dpp_f64<0x112, 0xf, true>(x));   // row_shr:2
    x = fmax(x, dpp_f64<0x114, 0xf, true>(x));   // row_shr:4
    x = fmax(x, dpp_f64<0x118, 0xf, true>(x));   // row_shr:8
    x = fmax(x, dpp_f64<0x142, 0xa, false>(x));  // row_bcast:15 into rows 1, 3
    x = fmax(x, dpp_f64<0x143, 0xc, false>(x));  // row_bcast:31 into rows 2, 3
    return x;
}

// Exclusive max-scan of one value >= 0 per thread over a block of NW waves
// (0 for thread 0).  One barrier: s_w (NW values) must not be written again
// before the caller's next barrier.
template <int NW>
__device__ __forceinline__ double block_excl_max(double v, double* s_w) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double x = wave_incl_max(v);
    if (lane == 63) s_w[w] = x;
    double ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = 0.0;
    __syncthreads();
    double pre = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i)
        if (i < w) pre = fmax(pre, s_w[i]);
    return fmax(pre, ex);
}

// Ascending bitonic sort of key[0 .. n2), n2 a power of two >= 512, by BS threads.
template <int BS = 256>
__device__ __forceinline__ void bitonic_sort_lds(uint64_t* key, int n2) {
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (n2 >> 1); t += BS) {
                const int lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const int hi = lo | j;
                const bool up = (lo & k) == 0;
                const uint64_t a = key[lo], bb = key[hi];
                if ((a > bb) == up) {
                    key[lo] = bb;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Everything the per-chain code touches for one chain: its problem's sizes and
// right-hand side, its rows of the state, proposal, direction and projection
// buffers, its bookkeeping entries, and optional outputs.
template <typename T>
struct ChainRef {
    int d, m;
    uint32_t chain, problem, step;   // Philox counter words (chain index within its problem)
    int gen_next;
    double eps;
    uint64_t seed;
    const double* b;
    const T* P0;          // committed projections of buffer s start at P0 + s * pstride
    size_t pstride;
    const T* q;
    T* x;
    T* xp;
    T* nu;
    int* sel;
    int* flag;
    long long* rej;
    T* trace;             // nullable
    const double* u;      // nullable: explicit uniform
    double* intervals;    // nullable: (m + 1) x 2
    int* n_intervals;     // nullable
    double* theta_out;    // nullable
    T* p_out;             // nullable
    T* q_out;             // nullable
    int* rejected_out;    // nullable
};

template <typename T>
__device__ __forceinline__ ChainRef<T> make_ref(const SampleArgs& a, int c) {
    ChainRef<T> r;
    r.d = a.d;
    r.m = a.m;
    r.chain = static_cast<uint32_t>(c);
    r.problem = a.problem;
    r.step = abs_step(a);
    r.gen_next = a.gen_next;
    r.eps = a.eps;
    r.seed = a.seed;
    r.b = a.b + static_cast<size_t>(c) * a.bstride;
    r.P0 = static_cast<const T*>(a.P) + static_cast<size_t>(c) * a.mp;
    r.pstride = static_cast<size_t>(a.Cp) * a.mp;
    r.q = static_cast<const T*>(a.Q) + static_cast<size_t>(c) * a.mp;
    r.x = static_cast<T*>(a.X) + static_cast<size_t>(c) * a.dp;
    r.xp = static_cast<T*>(a.Xprop) + static_cast<size_t>(c) * a.dp;
    r.nu = static_cast<T*>(a.N) + static_cast<size_t>(c) * a.dp;
    r.sel = a.sel + c;
    r.flag = a.flag + c;
    r.rej = a.rej + c;
    r.trace = a.trace ? static_cast<T*>(a.trace) + static_cast<size_t>(c) * a.d : nullptr;
    r.u = a.u_explicit ? a.u_explicit + c : nullptr;
    r.intervals = a.intervals ? a.intervals + static_cast<size_t>(c) * (a.m + 1) * 2 : nullptr;
    r.n_intervals = a.n_intervals ? a.n_intervals + c : nullptr;
    r.theta_out = a.theta_out ? a.theta_out + c : nullptr;
    r.p_out = a.pq_out ? static_cast<T*>(a.pq_out) + static_cast<size_t>(c) * a.m : nullptr;
    r.q_out = a.pq_out ? static_cast<T*>(a.pq_out) + (static_cast<size_t>(a.C) + c) * a.m : nullptr;
    r.rejected_out = a.rejected_out ? a.rejected_out + c : nullptr;
    return r;
}

// Accept or reject the chain's pending proposal (Section 3.3: a proposal
// violating some constraint is dropped and the chain stays).  Returns the
// buffer index of the chain's committed projections.
template <typename T>
__device__ __forceinline__ int commit_chain(const ChainRef<T>& r) {
    const int fl = *r.flag;
    const int s = *r.sel;
    __syncthreads();   // all reads of flag / sel precede the writes below
    const int snew = fl ? s : (s ^ 1);
    if (threadIdx.x == 0) {
        if (fl) *r.rej += 1;
        *r.sel = snew;
        *r.flag = 0;
        if (r.rejected_out) *r.rejected_out = fl;
    }
    // four elements per thread and pass, all loaded before any store (the
    // stores may alias the loads for the compiler, which would otherwise wait
    // for memory once per element); a load past d reads element d - 1
    const T* src = fl ? r.x : r.xp;
    const int nt = static_cast<int>(blockDim.x);
    for (int k0 = threadIdx.x; k0 < r.d; k0 += 4 * nt) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[min(k0 + u * nt, r.d - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * nt;
            if (k < r.d) {
                if (!fl) r.x[k] = v[u];
                if (r.trace) r.trace[k] = v[u];
            }
        }
    }
    return snew;
}

template <typename T>
__global__ __launch_bounds__(256) void commit_kernel(SampleArgs a) {
    commit_chain<T>(make_ref<T>(a, a.c0 + blockIdx.x));
}

// nu for `step` into dst[c * ld + k], k < d (chains c0 .. c0 + gridDim.x - 1).
template <typename T>
__global__ __launch_bounds__(256) void draw_kernel(uint64_t seed, uint32_t step_rel,
                                                   const uint32_t* step_base, uint32_t problem,
                                                   int d, T* dst, long long ld, double* u, int c0) {
    const int c = c0 + blockIdx.x;
    const uint32_t step = step_rel + (step_base ? *step_base : 0u);
    const Rng rng(seed);
    T* row = dst ? dst + static_cast<size_t>(c) * ld : nullptr;
    if (row) {
        for (int j = threadIdx.x; 2 * j < d; j += 256) {
            double z0, z1;
            rng.normal_pair(j, c, step, problem, z0, z1);
            row[2 * j] = static_cast<T>(z0);
            if (2 * j + 1 < d) row[2 * j + 1] = static_cast<T>(z1);
        }
    }
    if (u && threadIdx.x == 0) u[c] = rng.theta_uniform(c, step, problem);
}

template <typename T>
__device__ __forceinline__ double theta_uniform(const ChainRef<T>& r) {
    return r.u ? *r.u : Rng(r.seed).theta_uniform(r.chain, r.step, r.problem);
}

// Move along the ellipse, x' = x cos(theta) + nu sin(theta), then (optionally)
// replace nu by the next step's draw.  Called by all threads of the block.
template <typename T>
__device__ __forceinline__ void move_chain(const ChainRef<T>& r, double theta) {
    if (threadIdx.x == 0 && r.theta_out) *r.theta_out = theta;
    double sd, cd;
    sincos(theta, &sd, &cd);
    const T ct = static_cast<T>(cd), st = static_cast<T>(sd);
    // loads of four elements per thread before their stores, as in the commit
    const int nt = static_cast<int>(blockDim.x);
    for (int k0 = threadIdx.x; k0 < r.d; k0 += 4 * nt) {
        T xv[4], nv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = min(k0 + u * nt, r.d - 1);
            xv[u] = r.x[k];
            nv[u] = r.nu[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * nt;
            // one explicit contraction, so that every kernel that moves a
            // chain rounds it the same way
            if (k < r.d) r.xp[k] = fma(xv[u], ct, nv[u] * st);
        }
    }
    if (r.gen_next) {
        __syncthreads();   // every read of this step's nu is done
        const Rng rng(r.seed);
        for (int j = threadIdx.x; 2 * j < r.d; j += blockDim.x) {
            double z0, z1;
            rng.normal_pair(j, r.chain, r.step + 1, r.problem, z0, z1);
            r.nu[2 * j] = static_cast<T>(z0);
            if (2 * j + 1 < r.d) r.nu[2 * j + 1] = static_cast<T>(z1);
        }
    }
}

// The next step's normals of element pair (2 tid, 2 tid + 1), drawn before
// the move: the draw needs no loaded value, so it can run while loads are in
// flight.  `valid` is false when the thread has no pair or nothing is drawn.
template <typename T>
struct NextPair {
    T z0, z1;
    bool valid;
};

template <typename T>
__device__ __forceinline__ NextPair<T> draw_next_pair(const ChainRef<T>& r) {
    NextPair<T> n{T(0), T(0), false};
    if (r.gen_next && 2 * static_cast<int>(threadIdx.x) < r.d) {
        double z0, z1;
        Rng(r.seed).normal_pair(threadIdx.x, r.chain, r.step + 1, r.problem, z0, z1);
        n = NextPair<T>{static_cast<T>(z0), static_cast<T>(z1), true};
    }
    return n;
}

// The bookkeeping half of a commit (Section 3.3): the decision on the pending
// proposal, the rejection count and the projection buffer the roots read.
// The rows are copied later, by move_pairs, in the same pass as the move.
// Returns the committed projection buffer; `from_prop` tells whether the
// proposal became the state.
// `next`, when given, receives the early draw of the next direction's pair,
// made while flag and sel are loaded.
template <typename T>
__device__ __forceinline__ int commit_flags(const ChainRef<T>& r, bool& from_prop,
                                            NextPair<T>* next = nullptr) {
    const int fl = *r.flag;
    const int s = *r.sel;
    if (next) *next = draw_next_pair<T>(r);
    __syncthreads();   // every read of flag / sel precedes the writes below
    const int snew = fl ? s : (s ^ 1);
    if (threadIdx.x == 0) {
        if (fl) *r.rej += 1;
        *r.sel = snew;
        *r.flag = 0;
        if (r.rejected_out) *r.rejected_out = fl;
    }
    from_prop = !fl;
    return snew;
}

// Element pairs (2 j, 2 j + 1), j = t, t + BS, ... belong to thread t in
// move_pairs, so a thread reads nu exactly where it writes the next nu.  The
// first pair is loaded ahead, while the roots' loads are in flight, and held
// in registers until the move.
template <typename T>
struct PairAhead {
    T v0, v1, n0, n1;   // the state's and nu's elements
};

template <typename T>
__device__ __forceinline__ PairAhead<T> pair_ahead(const ChainRef<T>& r, bool from_prop) {
    PairAhead<T> q{};
    const int k = 2 * static_cast<int>(threadIdx.x);
    if (k < r.d) {
        const T* src = from_prop ? r.xp : r.x;
        const bool two = k + 1 < r.d;
        q.v0 = src[k];
        q.n0 = r.nu[k];
        q.v1 = two ? src[k + 1] : T(0);
        q.n1 = two ? r.nu[k + 1] : T(0);
    }
    return q;
}

// The move of every element, x' = v cos(theta) + nu sin(theta), where v is
// the state (the proposal when it was accepted, else x), with the commit's
// copies on the way: the accepted proposal into x, the state into the trace;
// then nu replaced by the next step's draw.  Element pairs as in pair_ahead,
// the first taken from `q`.
template <typename T, int BS>
__device__ __forceinline__ void move_pairs(const ChainRef<T>& r, double theta, bool from_prop,
                                           bool copy_state, const PairAhead<T>* q,
                                           const NextPair<T>* next = nullptr,
                                           const double* sc = nullptr) {
    if (threadIdx.x == 0 && r.theta_out) *r.theta_out = theta;
    double sd, cd;
    if (sc) {   // sin theta, cos theta taken once by the bucket path
        sd = sc[0];
        cd = sc[1];
    } else {
        sincos(theta, &sd, &cd);
    }
    const T ct = static_cast<T>(cd), st = static_cast<T>(sd);
    const T* src = from_prop ? r.xp : r.x;
    for (int j = threadIdx.x; 2 * j < r.d; j += BS) {
        const int k = 2 * j;
        const bool two = k + 1 < r.d;
        T v0, v1, n0, n1;
        if (q && j < BS) {
            v0 = q->v0;
            v1 = q->v1;
            n0 = q->n0;
            n1 = q->n1;
        } else {
            v0 = src[k];
            n0 = r.nu[k];
            v1 = two ? src[k + 1] : T(0);
            n1 = two ? r.nu[k + 1] : T(0);
        }
        if (copy_state) {
            r.x[k] = v0;
            if (two) r.x[k + 1] = v1;
        }
        if (r.trace) {
            r.trace[k] = v0;
            if (two) r.trace[k + 1] = v1;
        }
        // one explicit contraction, as in move_chain
        r.xp[k] = fma(v0, ct, n0 * st);
        if (two) r.xp[k + 1] = fma(v1, ct, n1 * st);
    }
    // the next nu over the same pairs: each thread overwrites only the nu
    // elements it has read itself, so no barrier is needed
    if (r.gen_next) {
        int j = threadIdx.x;
        if (next) {   // the first pair, drawn ahead
            if (next->valid) {
                r.nu[2 * j] = next->z0;
                if (2 * j + 1 < r.d) r.nu[2 * j + 1] = next->z1;
            }
            j += BS;
        }
        const Rng rng(r.seed);
        for (; 2 * j < r.d; j += BS) {
            double z0, z1;
            rng.normal_pair(j, r.chain, r.step + 1, r.problem, z0, z1);
            r.nu[2 * j] = static_cast<T>(z0);
            if (2 * j + 1 < r.d) r.nu[2 * j + 1] = static_cast<T>(z1);
        }
    }
}

// ---------------------------------------------------------------------------
// Full path: bitonic sort of every crossing row, then the sweep.
// ---------------------------------------------------------------------------
struct FullLds {
    double* alpha;
    double* beta;
    uint64_t* key;
    double* red;      // [BS / 64]
    int* cnt;         // [BS / 64]
    double* bcast;    // [2]
    int* kstar;       // [1]
    double* theta;    // [1]
};

// Where the sweep finds alpha and beta of the k-th key in order.
enum FullKeys {
    KEYS_SLOT = 0,   // alpha and beta of every crossing row in LDS, keys carry the slot
    KEYS_ROW = 1,    // only the keys live in LDS (room for 16384 rows); they carry
                     // the row index and every sweep solves the row's roots again
    KEYS_ROW_AB = 2  // keys as KEYS_ROW; alpha and beta of each row come from `abg`
                     // (one double2 per row, beta = 0 where the ellipse does not
                     // cross), which the caller has filled
};

// BS threads (256 or 512) take part.
// Returns theta (the same in every thread); the caller moves the chain.
template <typename T, int KEYS = KEYS_SLOT, int BS = 256>
__device__ double full_chain(const ChainRef<T>& r, int sel, const FullLds& L,
                             const double2* abg = nullptr) {
    constexpr bool LARGE = KEYS != KEYS_SLOT;
    constexpr int NW = BS / 64;
    const int tid = threadIdx.x;
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    int n = 0;
    for (int i0 = 0; i0 < r.m; i0 += BS) {
        const int i = i0 + tid;
        double al = 0.0, be = 0.0;
        bool hit = false;
        if (i < r.m) {
            if constexpr (KEYS == KEYS_ROW_AB) {
                const double2 v = abg[i];
                al = v.x;
                be = v.y;
                hit = be > 0.0;
            } else {
                const T p = Pc[i], q = r.q[i];
                hit = solve_roots<T>(static_cast<double>(p), static_cast<double>(q), r.b[i], al, be);
                if (r.p_out) {
                    r.p_out[i] = p;
                    r.q_out[i] = q;
                }
            }
        }
        int tot;
        const int pos = block_count_prefix<NW>(hit, L.cnt, tot);
        if (hit) {
            const int slot = n + pos;
            if constexpr (LARGE) {
                L.key[slot] = sort_key(al, i);
            } else {
                L.alpha[slot] = al;
                L.beta[slot] = be;
                L.key[slot] = sort_key(al, slot);
            }
        }
        n += tot;
    }
    int n2 = 512;
    while (n2 < n) n2 <<= 1;
    for (int k = n + tid; k < n2; k += BS) L.key[k] = ~0ull;
    __syncthreads();
    bitonic_sort_lds<BS>(L.key, n2);

    // sweep: running max of beta in alpha order, candidate lengths
    const int per = n2 / BS;
    const int k0 = tid * per;
    const int k1 = min(k0 + per, n);
    const double eps = r.eps;
    // alpha and beta of the k-th key in order
    auto ab = [&](int k, double& a, double& bt) {
        const int s = static_cast<int>(L.key[k] & 0xFFFF);
        if constexpr (KEYS == KEYS_ROW_AB) {
            const double2 v = abg[s];
            a = v.x;
            bt = v.y;
        } else if constexpr (KEYS == KEYS_ROW) {
            solve_roots<T>(static_cast<double>(Pc[s]), static_cast<double>(r.q[s]), r.b[s], a, bt);
        } else {
            a = L.alpha[s];
            bt = L.beta[s];
        }
    };
    double tmax = 0.0;
    for (int k = k0; k < k1; ++k) {
        double a, bt;
        ab(k, a, bt);
        tmax = fmax(tmax, bt);
    }
    const double g_in = block_excl_scan<MaxOp, NW>(tmax, 0.0, MaxOp(), L.red);
    const bool owns_last = (tid == BS - 1);

    auto cand = [&](int k, double& g, double& lo, double& hi) {
        double a, bt;
        ab(k, a, bt);
        lo = g;
        hi = a;
        g = fmax(g, bt);
        if (lo > 0.0) lo += eps;
        if (hi < kTwoPi) hi -= eps;
    };
    double tsum = 0.0, gend;
    {
        double g = g_in;
        for (int k = k0; k < k1; ++k) {
            double lo, hi;
            cand(k, g, lo, hi);
            tsum += fmax(hi - lo, 0.0);
        }
        gend = g;
    }
    // The last candidate [gamma_n, 2 pi] belongs to the block's last thread, whose running
    // max at the end of its chunk is gamma_n.
    double last_lo = 0.0, last_len = 0.0;
    if (owns_last) {
        last_lo = gend > 0.0 ? gend + eps : gend;
        last_len = fmax(kTwoPi - last_lo, 0.0);
        tsum += last_len;
    }
    const double s_in = block_excl_scan<SumOp, NW>(tsum, 0.0, SumOp(), L.red);
    if (owns_last) L.bcast[0] = s_in + tsum;
    if (tid == 0) *L.kstar = 0x7FFFFFFF;
    __syncthreads();
    const double total = L.bcast[0];
    const double s = theta_uniform(r) * total;

    // theta: first candidate whose running sum exceeds s (inverse CDF)
    double my_theta = 0.0, last_hi = 0.0;
    int my_k = 0x7FFFFFFF, last_k = -1;
    if (total > 0.0) {
        double g = g_in, run = s_in;
        for (int k = k0; k < k1; ++k) {
            double lo, hi;
            cand(k, g, lo, hi);
            const double len = fmax(hi - lo, 0.0);
            if (len > 0.0) {
                if (my_k == 0x7FFFFFFF && run + len > s) {
                    my_k = k;
                    my_theta = fmax(lo, fmin(lo + (s - run), hi));
                }
                last_k = k;
                last_hi = hi;
            }
            run += len;
        }
        if (owns_last && last_len > 0.0) {
            if (my_k == 0x7FFFFFFF && run + last_len > s) {
                my_k = n;
                my_theta = fmax(last_lo, fmin(last_lo + (s - run), kTwoPi));
            }
            last_k = n;
            last_hi = kTwoPi;
        }
        if (my_k != 0x7FFFFFFF) atomicMin(L.kstar, my_k);
    }
    __syncthreads();
    const int kstar = *L.kstar;
    __syncthreads();   // every thread has read kstar before it is reused
    if (total > 0.0) {
        if (kstar == 0x7FFFFFFF) {
            // s rounded up to the total: take the upper end of the last piece
            if (tid == 0) *L.kstar = -1;
            __syncthreads();
            if (last_k >= 0) atomicMax(L.kstar, last_k);
            __syncthreads();
            if (last_k >= 0 && last_k == *L.kstar) L.theta[0] = last_hi;
        } else if (my_k == kstar) {
            L.theta[0] = my_theta;
        }
    } else if (tid == 0) {
        L.theta[0] = 0.0;
        *r.flag = 1;   // empty active set: stay, counted as a rejection
    }

    // optional: the non-empty trimmed intervals, ascending
    if (r.intervals) {
        int cnt = 0;
        {
            double g = g_in;
            for (int k = k0; k < k1; ++k) {
                double lo, hi;
                cand(k, g, lo, hi);
                cnt += (hi - lo > 0.0);
            }
            if (owns_last) cnt += (last_len > 0.0);
        }
        const double base = block_excl_scan<SumOp, NW>(static_cast<double>(cnt), 0.0, SumOp(), L.red);
        int w = static_cast<int>(base);
        double g = g_in;
        for (int k = k0; k < k1; ++k) {
            double lo, hi;
            cand(k, g, lo, hi);
            if (hi - lo > 0.0) {
                r.intervals[2 * w] = lo;
                r.intervals[2 * w + 1] = hi;
                ++w;
            }
        }
        if (owns_last) {
            if (last_len > 0.0) {
                r.intervals[2 * w] = last_lo;
                r.intervals[2 * w + 1] = kTwoPi;
                ++w;
            }
            if (r.n_intervals) *r.n_intervals = w;
        }
    }
    __syncthreads();
    return L.theta[0];
}

#define ESS_FULL_LDS(NMAX)                                  \
    __shared__ double s_alpha[NMAX];                        \
    __shared__ double s_beta[NMAX];                         \
    __shared__ uint64_t s_key[NMAX];                        \
    __shared__ double s_red[8];                             \
    __shared__ int s_cnt[8];                                \
    __shared__ double s_bcast[2];                           \
    __shared__ int s_kstar;                                 \
    __shared__ double s_theta[2];                           \
    const FullLds full_lds{s_alpha, s_beta, s_key, s_red, s_cnt, s_bcast, &s_kstar, s_theta};



__global__ void zero_ints(int* p, int n) {
    if (static_cast<int>(threadIdx.x) < n) p[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Bucket path.  BS threads per chain (256 or 512), RPT rows per thread
// (m <= BS RPT), NB angle buckets.
// ---------------------------------------------------------------------------
template <int NB>
struct BucketLds {
    unsigned long long G[NB];          // bucket max beta, then prefix max
    signed char head[NB];              // last survivor of each bucket, -1 if none
    double sa[SMAX];                   // survivors: alpha
    int si[SMAX], sk[SMAX];            // survivors: row, bucket
    signed char nxt[SMAX];             // previous survivor of the same bucket, -1 if none
    unsigned long long sm[SMAX];       // survivors: in-bucket predecessor max
    double lo[SMAX + 1], hi[SMAX + 1];
    double len[SMAX + 1], cum[SMAX + 1];   // candidate lengths, their running sums
    double red[8];
    double gtot, total, u;
    int scount, kstar, klast;
    int smin, smax;                    // bucket range of the survivors (refinement)
    double theta;
    double sc[2];                      // sin theta, cos theta (by the lane that set theta)
};

// Levels of bucket refinement before a chain goes to the full path, and the
// survivor count below which refinement stops.
constexpr int kRefineLevels = 3;
constexpr int kRefineTarget = 16;

// Refinement levels in use (block-uniform, kept in scalar registers).  Level
// l keeps the rows of buckets [lo[l], hi[l]] and maps them to the bucket
// coordinate (alpha NB / 2 pi - off[l]) sc[l], clamped to the f[l]
// sub-buckets of the row's bucket one level up, so rounding of the composed
// map cannot reorder buckets.
struct RefineMap {
    int n;
    int lo[kRefineLevels], hi[kRefineLevels], f[kRefineLevels];
    double off[kRefineLevels], sc[kRefineLevels];
};

__device__ __forceinline__ double uniform_double(double v) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(u)));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(u >> 32)));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Bucket of alpha at the current refinement level, -1 once the row has left
// the search.  Recomputed from alpha wherever it is needed, so no per-row
// bucket stays in registers.
template <int NB>
__device__ __forceinline__ int bucket_of(const RefineMap& R, double a) {
    constexpr double kBucket = NB / kTwoPi;
    int b = min(static_cast<int>(a * kBucket), NB - 1);
#pragma unroll
    for (int l = 0; l < kRefineLevels; ++l) {
        if (l >= R.n) break;
        if (b < R.lo[l] || b > R.hi[l]) return -1;
        const int first = (b - R.lo[l]) * R.f[l];
        const double t = (a * kBucket - R.off[l]) * R.sc[l];
        b = min(max(static_cast<int>(t), first), first + R.f[l] - 1);
    }
    return b;
}

// Roots of rows row0 + tid + BS j (j < RPT) of the chain; beta = 0 marks a
// row past m or one the ellipse does not cross.  With `out`, the chain's p
// and q of those rows go to the optional output.  Every row's p, q and b are
// loaded before any root is solved (a row past m reads row m - 1), so the
// thread waits for memory once instead of once per row behind the branches
// of the root solve.
template <typename T, int RPT, int BS>
__device__ __forceinline__ void block_roots(const ChainRef<T>& r, const T* Pc, int row0, bool out,
                                            double (&al)[RPT], double (&be)[RPT]) {
    T pv[RPT], qv[RPT];
    double bv[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = min(row0 + static_cast<int>(threadIdx.x) + BS * j, r.m - 1);
        pv[j] = Pc[i];
        qv[j] = r.q[i];
        bv[j] = r.b[i];
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = row0 + static_cast<int>(threadIdx.x) + BS * j;
        al[j] = 0.0;
        be[j] = 0.0;
        if (i < r.m) {
            double x0, x1;
            if (solve_roots<T>(static_cast<double>(pv[j]), static_cast<double>(qv[j]), bv[j], x0, x1)) {
                al[j] = x0;
                be[j] = x1;
            }
            if (out && r.p_out) {
                r.p_out[i] = pv[j];
                r.q_out[i] = qv[j];
            }
        }
    }
}

// alpha, beta of rows row0 + tid + BS j from a root array (beta = 0: no
// crossing, or past m).
template <int RPT, int BS>
__device__ __forceinline__ void block_ab(const double2* ab, int row0, int m, double (&al)[RPT],
                                         double (&be)[RPT]) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = row0 + static_cast<int>(threadIdx.x) + BS * j;
        const double2 v = i < m ? ab[i] : make_double2(0.0, 0.0);
        al[j] = v.x;
        be[j] = v.y;
    }
}

// The inverse of block_ab: alpha, beta of rows row0 + tid + BS j into ab.
template <int RPT, int BS>
__device__ __forceinline__ void store_ab(double2* ab, int row0, int m, const double (&al)[RPT],
                                         const double (&be)[RPT]) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = row0 + static_cast<int>(threadIdx.x) + BS * j;
        if (i < m) ab[i] = make_double2(al[j], be[j]);
    }
}

// G[b] = max beta of the rows in bucket b (G cleared before).
template <int RPT, int NB>
__device__ __forceinline__ void bucket_max_pass(BucketLds<NB>& L, const RefineMap& R,
                                                const double (&al)[RPT], const double (&be)[RPT]) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (be[j] > 0.0) {
            const int b = bucket_of<NB>(R, al[j]);
            if (b >= 0) atomicMax(&L.G[b], obits(be[j]));
        }
    }
    __syncthreads();
}

// Exclusive prefix max over buckets, in place: G[b] = max(g0, max beta of
// rows in buckets < b); thread t owns buckets [t NB/BS, (t+1) NB/BS).  With
// `top`, gamma_n (max beta over all rows) goes to gtot.
template <int NB, int BS>
__device__ __forceinline__ void bucket_prefix_max(BucketLds<NB>& L, double g0, bool top) {
    constexpr int BPT = NB / BS;
    static_assert(BPT >= 1, "at least one bucket per thread");
    const int tid = threadIdx.x;
    double tmax = 0.0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) tmax = fmax(tmax, ofloat(L.G[tid * BPT + j]));
    const double g_in = block_excl_max<BS / 64>(tmax, L.red);
    double run = fmax(g0, g_in);
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const double v = ofloat(L.G[tid * BPT + j]);
        L.G[tid * BPT + j] = obits(run);
        run = fmax(run, v);
    }
    if (top && tid == BS - 1) L.gtot = run;
    __syncthreads();
}

// Survivors among rows row0 + tid + BS j: rows whose candidate can be
// non-empty (alpha >= G of their bucket); the first SMAX of the chain are
// listed.  Returns the chain's count so far.
template <int RPT, int NB, int BS>
__device__ __forceinline__ int find_survivors(BucketLds<NB>& L, const RefineMap& R,
                                              const double (&al)[RPT], const double (&be)[RPT],
                                              int row0 = 0) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (be[j] > 0.0) {
            const int b = bucket_of<NB>(R, al[j]);
            if (b >= 0 && al[j] >= ofloat(L.G[b])) {
                const int k = atomicAdd(&L.scount, 1);
                if (k < SMAX) {
                    L.sa[k] = al[j];
                    L.si[k] = row0 + tid + BS * j;
                    L.sk[k] = b;
                    L.sm[k] = 0ull;
                }
            }
        }
    }
    __syncthreads();
    return L.scount;
}

// Survivors chained per bucket, so a row meets only its own bucket's
// survivors (a row-by-survivor scan cost tens of microseconds per chain):
// survivor s links to the previous survivor of its bucket, and the last one
// heads the bucket; meanwhile another wave draws this step's uniform.
template <typename T, int NB>
__device__ __forceinline__ void link_survivors(const ChainRef<T>& r, BucketLds<NB>& L, int S) {
    const int tid = threadIdx.x;
    static_assert(SMAX <= 128, "survivor links are bytes");
    if (tid < S) {
        const int b = L.sk[tid];
        int prev = -1;
        bool last = true;
        for (int s = 0; s < S; ++s) {
            if (L.sk[s] == b) {
                if (s < tid) prev = s;
                else if (s > tid) last = false;
            }
        }
        L.nxt[tid] = static_cast<signed char>(prev);
        if (last) L.head[b] = static_cast<signed char>(tid);
    }
    if (tid == 64) L.u = theta_uniform(r);
    __syncthreads();
}

// Exact predecessor max inside each survivor's bucket (ties by row index),
// for rows row0 + tid + BS j.  No barrier at the end.
template <int RPT, int NB, int BS>
__device__ __forceinline__ void pred_max_pass(BucketLds<NB>& L, const RefineMap& R,
                                              const double (&al)[RPT], const double (&be)[RPT],
                                              int row0) {
    const int tid = threadIdx.x;
    // every row's bucket head first: one LDS round trip, not one per row
    int head[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int b = be[j] > 0.0 ? bucket_of<NB>(R, al[j]) : -1;
        head[j] = b >= 0 ? L.head[b] : -1;
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = row0 + tid + BS * j;
        for (int s = head[j]; s >= 0; s = L.nxt[s]) {
            if (al[j] < L.sa[s] || (al[j] == L.sa[s] && i < L.si[s]))
                atomicMax(&L.sm[s], obits(be[j]));
        }
    }
}

// The survivors' candidates in ascending (alpha, row) order, theta by inverse
// CDF and the optional interval output.  Returns theta (the same in every
// thread); the caller moves the chain.
template <typename T, int NB>
__device__ __forceinline__ double finish_bucket(const ChainRef<T>& r, BucketLds<NB>& L, int S) {
    const int tid = threadIdx.x;
    // the survivors' candidates, placed in ascending (alpha, row) order
    const double eps = r.eps;
    if (tid < S) {
        const double alpha = L.sa[tid];
        const int row = L.si[tid];
        int rank = 0;
        for (int s = 0; s < S; ++s) {
            const double o = L.sa[s];
            rank += (o < alpha) || (o == alpha && L.si[s] < row);
        }
        double lo = fmax(ofloat(L.G[L.sk[tid]]), ofloat(L.sm[tid]));
        double hi = alpha;
        if (lo > 0.0) lo += eps;
        if (hi < kTwoPi) hi -= eps;
        L.lo[rank] = lo;
        L.hi[rank] = hi;
    }
    if (tid == 0) {
        const double g = L.gtot;
        L.lo[S] = g > 0.0 ? g + eps : g;
        L.hi[S] = kTwoPi;
        L.kstar = 1 << 30;
        L.klast = -1;
    }
    __syncthreads();

    // inverse CDF over the S + 1 candidates in order: the running sums are a
    // sequential left-to-right sum (those of a cumulative sum), and theta lies
    // in the first non-empty candidate whose running sum exceeds s = u L.  Up
    // to 64 candidates: lane k of the first wave holds candidate k, the
    // running sums pass from lane to lane through scalar registers (no LDS
    // round trip per candidate), and ballots find the candidate.  More: the
    // lengths are formed in parallel, one thread keeps the running sums in
    // LDS, and the search is parallel.  Both give the same theta bit for bit.
    const int Su = __builtin_amdgcn_readfirstlane(S);
    // the one lane that finds theta also takes its sine and cosine for the
    // move, once per chain instead of once per wave
    bool mine = false;
    double th = 0.0;
    if (Su < 64) {
        if (tid < 64) {
            const bool in = tid <= Su;
            const double lo = in ? L.lo[tid] : 0.0;
            const double hi = in ? L.hi[tid] : 0.0;
            const double len = in ? fmax(hi - lo, 0.0) : 0.0;
            double run = 0.0, before = 0.0, cum = 0.0;
            for (int k = 0; k <= Su; ++k) {
                if (tid == k) before = run;
                run += lane_value(len, k);
                if (tid == k) cum = run;
            }
            const double total = run;   // the same in every lane
            if (total > 0.0) {
                const double sv = L.u * total;
                const unsigned long long pos = __ballot(len > 0.0);
                const unsigned long long hit = __ballot(len > 0.0 && cum > sv);
                if (hit) {
                    if (tid == __ffsll(static_cast<long long>(hit)) - 1) {
                        th = fmax(lo, fmin(lo + (sv - before), hi));
                        mine = true;
                    }
                } else if (tid == 63 - __clzll(static_cast<long long>(pos))) {
                    th = hi;   // rounding put s at the total
                    mine = true;
                }
            } else if (tid == 0) {
                mine = true;   // theta 0
                *r.flag = 1;   // empty active set: stay, counted as a rejection
            }
        }
    } else {
        if (tid <= S) L.len[tid] = fmax(L.hi[tid] - L.lo[tid], 0.0);
        __syncthreads();
        if (tid == 0) {
            double run = 0.0;
            int k = 0;
            for (; k + 4 <= S + 1; k += 4) {
                const double l0 = L.len[k], l1 = L.len[k + 1], l2 = L.len[k + 2], l3 = L.len[k + 3];
                run += l0;
                L.cum[k] = run;
                run += l1;
                L.cum[k + 1] = run;
                run += l2;
                L.cum[k + 2] = run;
                run += l3;
                L.cum[k + 3] = run;
            }
            for (; k <= S; ++k) {
                run += L.len[k];
                L.cum[k] = run;
            }
            L.total = run;
        }
        __syncthreads();
        const double total = L.total;
        if (total > 0.0) {
            const double sv = L.u * total;
            if (tid <= S && L.len[tid] > 0.0) {
                if (L.cum[tid] > sv) atomicMin(&L.kstar, tid);
                atomicMax(&L.klast, tid);
            }
            __syncthreads();
            if (tid == 0) {
                const int k = L.kstar;
                if (k <= S) {
                    const double before = k > 0 ? L.cum[k - 1] : 0.0;
                    th = fmax(L.lo[k], fmin(L.lo[k] + (sv - before), L.hi[k]));
                } else {
                    th = L.hi[L.klast];   // rounding put s at the total
                }
                mine = true;
            }
        } else if (tid == 0) {
            mine = true;   // theta 0
            *r.flag = 1;   // empty active set: stay, counted as a rejection
        }
    }
    if (mine) {
        double sd, cd;
        sincos(th, &sd, &cd);
        L.theta = th;
        L.sc[0] = sd;
        L.sc[1] = cd;
    }
    if (tid == 0 && r.intervals) {
        int w = 0;
        for (int k = 0; k <= S; ++k) {
            if (L.hi[k] - L.lo[k] > 0.0) {
                r.intervals[2 * w] = L.lo[k];
                r.intervals[2 * w + 1] = L.hi[k];
                ++w;
            }
        }
        if (r.n_intervals) *r.n_intervals = w;
    }
    __syncthreads();
    return L.theta;
}

// When more than SMAX rows survive, the survivors' buckets [blo, bhi] are
// split again: every row whose bucket lies in that range moves to one of
// floor(NB / (bhi - blo + 1)) sub-buckets of its bucket (an affine map of its
// bucket coordinate, so the order of alpha is kept), every other row leaves
// the search (its candidate is empty already), and the max-scan restarts from
// G[blo].  Angles that crowd a few buckets (as on unnormalised instances whose
// state sits close to many constraints, where alpha piles up just above 0)
// then spread over all NB buckets again.  Returns false when the survivors
// still exceed SMAX once refinement stops (kRefineLevels levels, a level that
// did not halve them, or a range that cannot be split): the caller hands the
// chain to the full path.  On success theta holds the drawn angle and the
// caller moves the chain.
// With `ab`, the roots come from large_roots_kernel's output instead; with
// `spill`, a chain handed over leaves every row's alpha and beta there.
template <typename T, int RPT, int NB, int BS = 256, bool REFINE = false>
__device__ bool bucket_chain(const ChainRef<T>& r, int sel, BucketLds<NB>& L, double& theta,
                             const double2* ab = nullptr, double2* spill = nullptr) {
    static_assert(BS == 256 || BS == 512, "one chain per 256 or 512 threads");
    const int tid = threadIdx.x;
    for (int b = tid; b < NB; b += BS) {
        L.G[b] = 0ull;
        L.head[b] = -1;
    }
    if (tid == 0) L.scount = 0;

    // roots of this thread's rows (row i = tid + BS r); beta = 0 marks no crossing
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    double al[RPT], be[RPT];
    if (ab)
        block_ab<RPT, BS>(ab, 0, r.m, al, be);
    else
        block_roots<T, RPT, BS>(r, Pc, 0, true, al, be);
    __syncthreads();
    RefineMap R;
    R.n = 0;
    bucket_max_pass<RPT, NB>(L, R, al, be);
    bucket_prefix_max<NB, BS>(L, 0.0, true);
    int S = find_survivors<RPT, NB, BS>(L, R, al, be);

    // refinement (rare on well-scaled problems, so only the variants for few
    // chains and the second attempt on a chain carry its code and registers).
    // Beyond overflow it also pays when survivors crowd a few buckets: every
    // row then meets all survivors of its bucket in the predecessor pass.
    // Below overflow it stops once a level no longer halves the survivors.
    if (!REFINE && S > SMAX) {
        // the full sort takes over: every row's alpha and beta for it
        if (spill) store_ab<RPT, BS>(spill, 0, r.m, al, be);
        return false;
    }
    int s_prev = 1 << 30;
    while (REFINE && S > kRefineTarget) {
        if (R.n == kRefineLevels || (S <= SMAX && 2 * S > s_prev)) {
            if (S > SMAX) return false;
            break;
        }
        s_prev = S;
        if (tid == 0) {
            L.smin = NB;
            L.smax = -1;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            if (be[j] > 0.0) {
                const int b = bucket_of<NB>(R, al[j]);
                if (b >= 0 && al[j] >= ofloat(L.G[b])) {
                    atomicMin(&L.smin, b);
                    atomicMax(&L.smax, b);
                }
            }
        }
        __syncthreads();
        const int blo = __builtin_amdgcn_readfirstlane(L.smin);
        const int bhi = __builtin_amdgcn_readfirstlane(L.smax);
        const int f = NB / (bhi - blo + 1);
        if (f < 2) {
            if (S > SMAX) return false;
            break;
        }
        const double g0 = ofloat(L.G[blo]);
        double off = 0.0, sc = 1.0;   // the map one level up
#pragma unroll
        for (int l = 0; l < kRefineLevels; ++l) {
            if (l + 1 == R.n) {
                off = R.off[l];
                sc = R.sc[l];
            }
        }
        off = uniform_double(off + blo / sc);
        sc = uniform_double(sc * f);
#pragma unroll
        for (int l = 0; l < kRefineLevels; ++l) {
            if (l == R.n) {
                R.lo[l] = blo;
                R.hi[l] = bhi;
                R.f[l] = f;
                R.off[l] = off;
                R.sc[l] = sc;
            }
        }
        ++R.n;
        __syncthreads();   // every read of G and of the range precedes the reset
        for (int b = tid; b < NB; b += BS) {
            L.G[b] = 0ull;
            L.head[b] = -1;
        }
        if (tid == 0) L.scount = 0;
        __syncthreads();
        bucket_max_pass<RPT, NB>(L, R, al, be);
        bucket_prefix_max<NB, BS>(L, g0, false);
        S = find_survivors<RPT, NB, BS>(L, R, al, be);
    }

    link_survivors<T, NB>(r, L, S);
    pred_max_pass<RPT, NB, BS>(L, R, al, be, 0);
    __syncthreads();
    theta = finish_bucket<T, NB>(r, L, S);
    return true;
}

// Rows beyond what one pass holds in registers (m > BS RPT): the same bucket
// path with refinement, each pass over the rows in chunks of BS RPT, reading
// alpha and beta of every row from `ab` (16 bytes per row), which
// large_roots_kernel filled before this launch (three passes, plus three per
// refinement level).  Returns false, or true with theta, as bucket_chain
// does.
template <typename T, int RPT, int NB, int BS>
__device__ bool bucket_chain_large(const ChainRef<T>& r, int sel, BucketLds<NB>& L, double& theta,
                                   double2* ab) {
    const int tid = threadIdx.x;
    constexpr int CH = BS * RPT;
    for (int b = tid; b < NB; b += BS) {
        L.G[b] = 0ull;
        L.head[b] = -1;
    }
    if (tid == 0) L.scount = 0;
    __syncthreads();
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    double al[RPT], be[RPT];
    RefineMap R;
    R.n = 0;
    (void)Pc;
    for (int c0 = 0; c0 < r.m; c0 += CH) {
        block_ab<RPT, BS>(ab, c0, r.m, al, be);
        bucket_max_pass<RPT, NB>(L, R, al, be);
    }
    bucket_prefix_max<NB, BS>(L, 0.0, true);
    int S = 0;
    for (int c0 = 0; c0 < r.m; c0 += CH) {
        block_ab<RPT, BS>(ab, c0, r.m, al, be);
        S = find_survivors<RPT, NB, BS>(L, R, al, be, c0);
    }
    int s_prev = 1 << 30;
    while (S > kRefineTarget) {
        if (R.n == kRefineLevels || (S <= SMAX && 2 * S > s_prev)) {
            if (S > SMAX) return false;
            break;
        }
        s_prev = S;
        if (tid == 0) {
            L.smin = NB;
            L.smax = -1;
        }
        __syncthreads();
        for (int c0 = 0; c0 < r.m; c0 += CH) {
            block_ab<RPT, BS>(ab, c0, r.m, al, be);
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (be[j] > 0.0) {
                    const int b = bucket_of<NB>(R, al[j]);
                    if (b >= 0 && al[j] >= ofloat(L.G[b])) {
                        atomicMin(&L.smin, b);
                        atomicMax(&L.smax, b);
                    }
                }
            }
        }
        __syncthreads();
        const int blo = __builtin_amdgcn_readfirstlane(L.smin);
        const int bhi = __builtin_amdgcn_readfirstlane(L.smax);
        const int f = NB / (bhi - blo + 1);
        if (f < 2) {
            if (S > SMAX) return false;
            break;
        }
        const double g0 = ofloat(L.G[blo]);
        double off = 0.0, sc = 1.0;
#pragma unroll
        for (int l = 0; l < kRefineLevels; ++l) {
            if (l + 1 == R.n) {
                off = R.off[l];
                sc = R.sc[l];
            }
        }
        off = uniform_double(off + blo / sc);
        sc = uniform_double(sc * f);
#pragma unroll
        for (int l = 0; l < kRefineLevels; ++l) {
            if (l == R.n) {
                R.lo[l] = blo;
                R.hi[l] = bhi;
                R.f[l] = f;
                R.off[l] = off;
                R.sc[l] = sc;
            }
        }
        ++R.n;
        __syncthreads();   // every read of G and of the range precedes the reset
        for (int b = tid; b < NB; b += BS) {
            L.G[b] = 0ull;
            L.head[b] = -1;
        }
        if (tid == 0) L.scount = 0;
        __syncthreads();
        for (int c0 = 0; c0 < r.m; c0 += CH) {
            block_ab<RPT, BS>(ab, c0, r.m, al, be);
            bucket_max_pass<RPT, NB>(L, R, al, be);
        }
        bucket_prefix_max<NB, BS>(L, g0, false);
        for (int c0 = 0; c0 < r.m; c0 += CH) {
            block_ab<RPT, BS>(ab, c0, r.m, al, be);
            S = find_survivors<RPT, NB, BS>(L, R, al, be, c0);
        }
    }
    if (S > SMAX) return false;
    link_survivors<T, NB>(r, L, S);
    for (int c0 = 0; c0 < r.m; c0 += CH) {
        block_ab<RPT, BS>(ab, c0, r.m, al, be);
        pred_max_pass<RPT, NB, BS>(L, R, al, be, c0);
    }
    __syncthreads();
    theta = finish_bucket<T, NB>(r, L, S);
    return true;
}

// LDS of the bucket kernels for many chains: the bucket path's arrays or, for
// a chain the bucket path hands back, the keys of the full sort done in
// place.  The keys carry the row index and every sweep solves the row's
// roots again (as beyond 4096 rows), so the union is no larger than the
// bucket arrays up to 2048 rows and occupancy is unchanged.
template <int NB, int NK>
struct BucketOrKeys {
    union {
        BucketLds<NB> bucket;
        uint64_t key[NK];
    };
    double red[8];
    int cnt[8];
    double bcast[2];
    int kstar;
    double theta[2];
};

template <typename T, int RPT, int NB, int BS = 256, bool REFINE = false, bool PRE = false>
__global__ __launch_bounds__(BS, (BS == 512 && RPT <= 4 && !REFINE) ? 8 : 1) void sample_bucket_kernel(SampleArgs a) {
    const int c = a.c0 + blockIdx.x;
    const ChainRef<T> r = make_ref<T>(a, c);
    if constexpr (REFINE) {
        const int sel = a.has_pending ? commit_chain<T>(r) : *r.sel;
        // the variants for few chains refine crowded buckets and keep alpha
        // and beta of a chain they sort in LDS (occupancy does not matter
        // with no more chains than compute units)
        // PRE: large_roots_kernel has solved this step's roots into a.ab
        const double2* ab = PRE ? static_cast<const double2*>(a.ab) + static_cast<size_t>(c) * a.mp : nullptr;
        double theta = 0.0;
        if constexpr (PRE && RPT * BS > 4096) {
            // up to 16384 rows held in registers across every pass; a chain
            // the buckets cannot resolve sorts keys only, in the bucket
            // arrays' LDS, with alpha and beta read back from a.ab
            __shared__ BucketOrKeys<NB, RPT * BS> lds;
            const bool done = !a.force_full && bucket_chain<T, RPT, NB, BS, true>(r, sel, lds.bucket, theta, ab);
            if (!done) {
                __syncthreads();
                const FullLds L{nullptr, nullptr, lds.key, lds.red, lds.cnt, lds.bcast, &lds.kstar, lds.theta};
                theta = full_chain<T, KEYS_ROW_AB, BS>(r, sel, L, ab);
            }
        } else {
            __shared__ BucketLds<NB> lds;
            const bool done = !a.force_full && bucket_chain<T, RPT, NB, BS, true>(r, sel, lds, theta, ab);
            if (!done) {
                ESS_FULL_LDS(RPT * BS)
                theta = full_chain<T, KEYS_SLOT, BS>(r, sel, full_lds);
            }
        }
        move_chain<T>(r, theta);
    } else {
        // a chain whose survivors overflow (or every chain, with the full
        // sort requested) is sorted in place by the same workgroup, so no
        // second launch follows.  Its roots go to the chain's row of a.ab
        // first, so the full sort reads them instead of solving them again
        // (which would hold the kernel's registers above the bucket path's).
        constexpr int NK = RPT * BS > 512 ? RPT * BS : 512;
        __shared__ BucketOrKeys<NB, NK> lds;
        double2* abg = static_cast<double2*>(a.ab) + static_cast<size_t>(c) * a.mp;
        bool done = false;
        // the commit's bookkeeping now, its row copies with the move
        bool from_prop = false;
        // the next direction's first pair, drawn while flag and sel load;
        // 512-thread chains (registers capped at 64) park it in LDS
        NextPair<T> next;
        int sel;
        if (a.has_pending) {
            sel = commit_flags<T>(r, from_prop, &next);
        } else {
            next = draw_next_pair<T>(r);
            sel = *r.sel;
        }
        __shared__ T next_lds[BS == 512 ? 2 * BS : 1];
        if constexpr (BS == 512) {
            next_lds[2 * threadIdx.x] = next.z0;
            next_lds[2 * threadIdx.x + 1] = next.z1;
        }
        const PairAhead<T> ahead = pair_ahead<T>(r, from_prop);
        double theta = 0.0;
        if (!a.force_full) {
            if constexpr (PRE)
                done = bucket_chain<T, RPT, NB, BS, false>(r, sel, lds.bucket, theta, abg, nullptr);
            else
                done = bucket_chain<T, RPT, NB, BS, false>(r, sel, lds.bucket, theta, nullptr, abg);
        } else if constexpr (!PRE) {
            double al[RPT], be[RPT];
            block_roots<T, RPT, BS>(r, r.P0 + static_cast<size_t>(sel) * r.pstride, 0, true, al, be);
            store_ab<RPT, BS>(abg, 0, r.m, al, be);
        }
        if (!done) {
            __syncthreads();   // every row's alpha and beta is in a.ab
            const FullLds L{nullptr, nullptr, lds.key, lds.red, lds.cnt, lds.bcast, &lds.kstar, lds.theta};
            theta = full_chain<T, KEYS_ROW_AB, BS>(r, sel, L, abg);
        }
        if constexpr (BS == 512) {   // each thread reads back its own pair
            next.z0 = next_lds[2 * threadIdx.x];
            next.z1 = next_lds[2 * threadIdx.x + 1];
        }
        move_pairs<T, BS>(r, theta, from_prop, from_prop && a.has_pending, &ahead, &next,
                          done ? lds.bucket.sc : nullptr);
    }
}

// ---------------------------------------------------------------------------
// Comparator: likelihood testing at midpoints (Section 2.2), O(m^2) per chain.
// The 2n intersection angles of the n crossing rows are sorted (48-bit keys
// carrying 2 row + end); each gap between consecutive angles, with 0 and
// 2 pi as the outer ends, is active when x(theta) at its midpoint satisfies
// all m constraints, tested from the cached projections.  Active gaps of
// positive length are the active intervals: consecutive gaps share an angle
// that is a crossing of some row, which is violated on one side, so two
// active gaps never touch except across a gap of length zero (tied angles),
// where this kernel keeps two pieces of the same set.
// ---------------------------------------------------------------------------
constexpr int kMidpointMaxRows = 4096;

template <typename T>
struct MidLds {
    uint64_t key[2 * kMidpointMaxRows];   // sort keys, then the angles' bits
    T p[kMidpointMaxRows], q[kMidpointMaxRows];
    unsigned char ok[2 * kMidpointMaxRows + 1];
    double red[4];
    int cnt[4];
    double bcast[2];
    int kstar;
    double theta;
};

template <typename T>
__device__ void midpoint_chain(const ChainRef<T>& r, int sel, MidLds<T>& L) {
    const int tid = threadIdx.x;
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    // roots, both angles of each crossing row as keys; p and q kept in LDS
    int n = 0;
    for (int i0 = 0; i0 < r.m; i0 += 256) {
        const int i = i0 + tid;
        double al = 0.0, be = 0.0;
        bool hit = false;
        if (i < r.m) {
            const T p = Pc[i], q = r.q[i];
            L.p[i] = p;
            L.q[i] = q;
            hit = solve_roots<T>(static_cast<double>(p), static_cast<double>(q), r.b[i], al, be);
            if (r.p_out) {
                r.p_out[i] = p;
                r.q_out[i] = q;
            }
        }
        int tot;
        const int pos = block_count_prefix(hit, L.cnt, tot);
        if (hit) {
            L.key[n + 2 * pos] = sort_key(al, 2 * i);
            L.key[n + 2 * pos + 1] = sort_key(be, 2 * i + 1);
        }
        n += 2 * tot;
    }
    int n2 = 512;
    while (n2 < n) n2 <<= 1;
    for (int k = n + tid; k < n2; k += 256) L.key[k] = ~0ull;
    __syncthreads();
    bitonic_sort_lds(L.key, n2);
    // the exact angle of every key, in place of the key
    for (int k = tid; k < n; k += 256) {
        const int s = static_cast<int>(L.key[k] & 0xFFFF);
        const int i = s >> 1;
        double al, be;
        solve_roots<T>(static_cast<double>(L.p[i]), static_cast<double>(L.q[i]), r.b[i], al, be);
        L.key[k] = static_cast<uint64_t>(__double_as_longlong((s & 1) ? be : al));
    }
    __syncthreads();
    auto ang = [&](int k) { return __longlong_as_double(static_cast<long long>(L.key[k])); };
    // gap g runs from angle g - 1 (0 for g = 0) to angle g (2 pi for g = n)
    auto gap = [&](int g, double& lo, double& hi) {
        lo = g == 0 ? 0.0 : ang(g - 1);
        hi = g == n ? kTwoPi : ang(g);
    };
    // the likelihood at every gap's midpoint: all m rows, no early exit
    for (int g = tid; g <= n; g += 256) {
        double lo, hi;
        gap(g, lo, hi);
        bool ok = false;
        if (hi > lo) {
            double sm, cm;
            sincos(0.5 * (lo + hi), &sm, &cm);
            bool inside = true;
            for (int i = 0; i < r.m; ++i)
                inside &= static_cast<double>(L.p[i]) * cm + static_cast<double>(L.q[i]) * sm <= r.b[i];
            ok = inside;
        }
        L.ok[g] = ok ? 1 : 0;
    }
    if (tid == 0) L.kstar = 0x7FFFFFFF;
    __syncthreads();

    // inverse CDF over the active gaps in ascending order (trimmed at real
    // ends), each thread a contiguous range of gaps
    const double eps = r.eps;
    const int per = (n + 1 + 255) / 256;
    const int g0 = tid * per, g1 = min(g0 + per, n + 1);
    auto piece = [&](int g, double& lo, double& hi) {
        gap(g, lo, hi);
        if (!L.ok[g]) {
            hi = lo;
            return;
        }
        if (lo > 0.0) lo += eps;
        if (hi < kTwoPi) hi -= eps;
    };
    double tsum = 0.0;
    for (int g = g0; g < g1; ++g) {
        double lo, hi;
        piece(g, lo, hi);
        tsum += fmax(hi - lo, 0.0);
    }
    const double s_in = block_excl_scan(tsum, 0.0, SumOp(), L.red);
    if (tid == 255) L.bcast[0] = s_in + tsum;
    __syncthreads();
    const double total = L.bcast[0];
    const double sv = theta_uniform(r) * total;
    double my_theta = 0.0, last_hi = 0.0;
    int my_g = 0x7FFFFFFF, last_g = -1;
    if (total > 0.0) {
        double run = s_in;
        for (int g = g0; g < g1; ++g) {
            double lo, hi;
            piece(g, lo, hi);
            const double len = fmax(hi - lo, 0.0);
            if (len > 0.0) {
                if (my_g == 0x7FFFFFFF && run + len > sv) {
                    my_g = g;
                    my_theta = fmax(lo, fmin(lo + (sv - run), hi));
                }
                last_g = g;
                last_hi = hi;
            }
            run += len;
        }
        if (my_g != 0x7FFFFFFF) atomicMin(&L.kstar, my_g);
    }
    __syncthreads();
    const int kstar = L.kstar;
    __syncthreads();   // every thread has read kstar before it is reused
    if (total > 0.0) {
        if (kstar == 0x7FFFFFFF) {
            // s rounded up to the total: the upper end of the last piece
            if (tid == 0) L.kstar = -1;
            __syncthreads();
            if (last_g >= 0) atomicMax(&L.kstar, last_g);
            __syncthreads();
            if (last_g >= 0 && last_g == L.kstar) L.theta = last_hi;
        } else if (my_g == kstar) {
            L.theta = my_theta;
        }
    } else if (tid == 0) {
        L.theta = 0.0;
        *r.flag = 1;   // empty active set: stay, counted as a rejection
    }

    // optional: the active trimmed pieces, ascending
    if (r.intervals) {
        int cnt = 0;
        for (int g = g0; g < g1; ++g) {
            double lo, hi;
            piece(g, lo, hi);
            cnt += (hi - lo > 0.0);
        }
        const double base = block_excl_scan(static_cast<double>(cnt), 0.0, SumOp(), L.red);
        int w = static_cast<int>(base);
        for (int g = g0; g < g1; ++g) {
            double lo, hi;
            piece(g, lo, hi);
            if (hi - lo > 0.0) {
                r.intervals[2 * w] = lo;
                r.intervals[2 * w + 1] = hi;
                ++w;
            }
        }
        if (tid == 255 && r.n_intervals) *r.n_intervals = w;
    }
    __syncthreads();
    move_chain<T>(r, L.theta);
}

template <typename T>
__global__ __launch_bounds__(256) void sample_midpoint_kernel(SampleArgs a) {
    __shared__ MidLds<T> lds;
    const int c = a.c0 + blockIdx.x;
    const ChainRef<T> r = make_ref<T>(a, c);
    const int sel = a.has_pending ? commit_chain<T>(r) : *r.sel;
    midpoint_chain<T>(r, sel, lds);
}

// ---------------------------------------------------------------------------
// Comparator: Algorithm 2, the active set by its definition.  Starting from
// [0, 2 pi], the set is intersected with I_i = [0, alpha_i] U [beta_i, 2 pi]
// one row at a time, in row order: every piece [l, h] leaves
// [l, min(h, alpha_i)] and [max(l, beta_i), h].  Pieces of zero length are
// dropped where they appear (they carry no length, and no later
// intersection can lengthen them), and a row the ellipse does not cross
// (I_i the whole circle) leaves the set as it is.  The arc (alpha_i, beta_i)
// splits at most one piece, so the list holds at most m + 1 pieces; the work
// per row is linear in their number, O(m^2) at worst (Appendix D's input).
// The pieces come out in ascending order, the same non-empty intervals as
// Algorithm 3's candidates, and theta is drawn from them in the same way.
// One wave per chain; the list lives in LDS as two buffers of m + 2 pieces
// (dynamic shared memory).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void sample_alg2_kernel(SampleArgs a) {
    extern __shared__ double2 alg2_lists[];
    __shared__ double s_theta;
    const int lane = threadIdx.x;
    const int c = a.c0 + blockIdx.x;
    const ChainRef<T> r = make_ref<T>(a, c);
    const int sel = a.has_pending ? commit_chain<T>(r) : *r.sel;
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    double2* cur = alg2_lists;
    double2* nxt = alg2_lists + (r.m + 2);
    if (lane == 0) cur[0] = make_double2(0.0, kTwoPi);
    int n = 1;   // pieces in cur (the same in every lane)
    __syncthreads();
    for (int i0 = 0; i0 < r.m; i0 += 64) {
        // the roots of 64 rows at once, then the rows one after another
        const int i = i0 + lane;
        double al = 0.0, be = 0.0;
        if (i < r.m) {
            const T p = Pc[i], q = r.q[i];
            double x0, x1;
            if (solve_roots<T>(static_cast<double>(p), static_cast<double>(q), r.b[i], x0, x1)) {
                al = x0;
                be = x1;
            }
            if (r.p_out) {
                r.p_out[i] = p;
                r.q_out[i] = q;
            }
        }
        const int rows = min(64, r.m - i0);
        for (int j = 0; j < rows; ++j) {
            const double aj = __shfl(al, j, 64), bj = __shfl(be, j, 64);
            if (!(bj > 0.0)) continue;   // no crossing: I_j is the whole circle
            int total = 0;
            for (int k0 = 0; k0 < n; k0 += 64) {
                const int k = k0 + lane;
                const double2 v = k < n ? cur[k] : make_double2(0.0, 0.0);
                const double h1 = fmin(v.y, aj), l2 = fmax(v.x, bj);
                const bool p1 = k < n && h1 > v.x;
                const bool p2 = k < n && v.y > l2;
                const int cnt = static_cast<int>(p1) + static_cast<int>(p2);
                int incl = cnt;   // inclusive prefix sum of the counts over the wave
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += y;
                }
                const int pos = total + incl - cnt;
                if (p1) nxt[pos] = make_double2(v.x, h1);
                if (p2) nxt[pos + (p1 ? 1 : 0)] = make_double2(l2, v.y);
                total += __shfl(incl, 63, 64);
            }
            n = total;
            double2* t = cur;
            cur = nxt;
            nxt = t;
            __syncthreads();
        }
    }
    // trim real ends by eps, theta by inverse CDF over the pieces in order
    if (lane == 0) {
        const double eps = r.eps;
        auto piece = [&](int k, double& lo, double& hi) {
            lo = cur[k].x;
            hi = cur[k].y;
            if (lo > 0.0) lo += eps;
            if (hi < kTwoPi) hi -= eps;
        };
        double total = 0.0;
        for (int k = 0; k < n; ++k) {
            double lo, hi;
            piece(k, lo, hi);
            total += fmax(hi - lo, 0.0);
        }
        double theta = 0.0;
        if (total > 0.0) {
            const double sv = theta_uniform(r) * total;
            double run = 0.0;
            int last = -1;
            bool found = false;
            for (int k = 0; k < n; ++k) {
                double lo, hi;
                piece(k, lo, hi);
                const double len = fmax(hi - lo, 0.0);
                if (len > 0.0) {
                    last = k;
                    if (!found && run + len > sv) {
                        theta = fmax(lo, fmin(lo + (sv - run), hi));
                        found = true;
                    }
                }
                run += len;
            }
            if (!found) {   // rounding put s at the total
                double lo, hi;
                piece(last, lo, hi);
                theta = hi;
            }
        } else {
            *r.flag = 1;   // empty active set: stay, counted as a rejection
        }
        if (r.intervals) {
            int w = 0;
            for (int k = 0; k < n; ++k) {
                double lo, hi;
                piece(k, lo, hi);
                if (hi - lo > 0.0) {
                    r.intervals[2 * w] = lo;
                    r.intervals[2 * w + 1] = hi;
                    ++w;
                }
            }
            if (r.n_intervals) *r.n_intervals = w;
        }
        s_theta = theta;
    }
    __syncthreads();
    move_chain<T>(r, s_theta);
}

// Rows beyond 4096: 512 threads per chain, the chunked bucket path with
// refinement; chains it cannot resolve go to the full sort of keys only, in
// LDS up to kMaxRowsLds rows and in global memory beyond (the keys carry the
// row in 16 bits).
constexpr int kMaxRowsLds = 16384;
constexpr int kMaxRowsLarge = 65536;

// Roots of every row of every chain ahead of sample_large_kernel: one thread
// per row and many workgroups per chain, so the float64 solves spread over
// the device instead of one workgroup per chain.  The projections are those
// the per-chain kernel's commit will select (P[sel] after a rejection,
// P[1 - sel] after an acceptance); flag and sel are only read here.  Also
// writes the optional p, q output.
template <typename T>
__global__ __launch_bounds__(256) void large_roots_kernel(SampleArgs a) {
    const int slabs = (a.m + 255) / 256;
    const int c = a.c0 + static_cast<int>(blockIdx.x) / slabs;
    const int i = (static_cast<int>(blockIdx.x) % slabs) * 256 + static_cast<int>(threadIdx.x);
    if (i >= a.m) return;
    const ChainRef<T> r = make_ref<T>(a, c);
    const int s = *r.sel;
    const int sel = a.has_pending ? (*r.flag ? s : (s ^ 1)) : s;
    const T* Pc = r.P0 + static_cast<size_t>(sel) * r.pstride;
    const T p = Pc[i], q = r.q[i];
    double al = 0.0, be = 0.0, x0, x1;
    if (solve_roots<T>(static_cast<double>(p), static_cast<double>(q), r.b[i], x0, x1)) {
        al = x0;
        be = x1;
    }
    static_cast<double2*>(a.ab)[static_cast<size_t>(c) * a.mp + i] = make_double2(al, be);
    if (r.p_out) {
        r.p_out[i] = p;
        r.q_out[i] = q;
    }
}

template <typename T>
__global__ __launch_bounds__(512) void sample_large_kernel(SampleArgs a) {
    __shared__ BucketLds<2048> lds;
    const int c = a.c0 + blockIdx.x;
    const ChainRef<T> r = make_ref<T>(a, c);
    const int sel = a.has_pending ? commit_chain<T>(r) : *r.sel;
    const uint32_t step = r.step;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.fb_count[(step + 1) & 1] = 0;   // next step's list
    double2* ab = static_cast<double2*>(a.ab) + static_cast<size_t>(c) * a.mp;
    double theta = 0.0;
    const bool done = !a.force_full && bucket_chain_large<T, 8, 2048, 512>(r, sel, lds, theta, ab);
    if (done) move_chain<T>(r, theta);
    else if (threadIdx.x == 0) a.fb_list[atomicAdd(a.fb_count + (step & 1), 1)] = c;
}

// The chains sample_large_kernel handed over: the full sort of their keys,
// with alpha and beta of every row read back from a.ab (large_roots_kernel
// solved them this step).  GLOBAL: the keys live in the chain's row of a.keys
// instead of LDS, for more than kMaxRowsLds rows (a bitonic network over
// global memory, slow but only for chains whose survivors overflow).
template <typename T, bool GLOBAL = false>
__global__ __launch_bounds__(256) void fallback_large_kernel(SampleArgs a) {
    __shared__ uint64_t s_key[GLOBAL ? 1 : kMaxRowsLds];
    __shared__ double s_red[4];
    __shared__ int s_cnt[4];
    __shared__ double s_bcast[2];
    __shared__ int s_kstar;
    __shared__ double s_theta[2];
    const int count = a.fb_count[abs_step(a) & 1];
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int c = a.fb_list[idx];
        uint64_t* key = GLOBAL ? a.keys + static_cast<size_t>(c) * a.kstride : s_key;
        const FullLds L{nullptr, nullptr, key, s_red, s_cnt, s_bcast, &s_kstar, s_theta};
        const ChainRef<T> r = make_ref<T>(a, c);
        const double2* abg = static_cast<const double2*>(a.ab) + static_cast<size_t>(c) * a.mp;
        move_chain<T>(r, full_chain<T, KEYS_ROW_AB>(r, *r.sel, L, abg));
        __syncthreads();
    }
}

}  // namespace ess

namespace ess {

__global__ void step_counter_kernel(uint32_t* counter, uint32_t value, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = add ? *counter + value : value;
}

}  // namespace ess
