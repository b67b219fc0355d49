// Per-chain part of one transition: commit the previous proposal, solve every
// constraint's intersection angles, build the active intervals with a sort and
// a cumulative max, draw theta, move, and draw the next ellipse direction.
//
// One 256-thread workgroup per chain; the chain's angles live in LDS.
//
// Roots (Appendix B): p = a_i^T x, q = a_i^T nu, r = hypot(p, q),
// tau = atan2(q, p), phi = acos(b / r); the ellipse leaves the halfspace on the
// arc (tau - phi, tau + phi).  alpha = (tau - phi) wrapped into [0, 2 pi),
// beta = min(alpha + 2 phi, 2 pi), so I_i = [0, alpha] U [beta, 2 pi].
// Rows with r = 0 or b / r >= 1 never meet the ellipse (Section 3.2): the paper
// pads them with alpha = beta = 0, which only adds zero-length candidates and
// leaves every cumulative max unchanged, so they are dropped here instead.
//
// Active intervals (Algorithm 3 / Proposition 1): sort the alphas, carry the
// betas; with gamma the running max of the betas in that order, the candidates
// are [0, alpha_(1)], [gamma_(k-1), alpha_(k)] for k = 2..n and
// [gamma_(n), 2 pi]; a candidate with its upper end below its lower end is
// empty.  Trimming (Section 3.3) moves real ends inward by eps; the ends at 0
// and 2 pi are the seam through x_t and stay.
//
// Sort keys: alpha is mapped monotonically to a 48-bit fixed-point turn
// fraction floor(alpha * 2^48 / 2 pi) and packed above the 16-bit slot index,
// so a single 64-bit compare orders the pairs.  Two alphas closer than
// 2 pi * 2^-48 (2.2e-14 rad) may come out in either order, which moves the
// union by at most their distance.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace ess {

struct SampleArgs {
    int d, m, C, Cp, dp, mp;
    uint32_t problem;
    const double* b;      // [m]
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
    uint32_t step;        // step whose nu/u are used
    int has_pending;      // commit the previous proposal first
    int gen_next;         // write nu(step + 1) into N after the move
    void* trace;          // nullable: committed state of the previous step, [C][d] T
    const double* u_explicit;   // nullable: u instead of the Philox draw
    double* intervals;    // nullable: [C][m + 1][2]
    int* n_intervals;     // nullable: [C]
    double* theta_out;    // nullable: [C]
    void* pq_out;         // nullable: [2][C][m] T
    int* rejected_out;    // nullable: [C] (commit kernel)
};

constexpr double kKeyScale = 281474976710656.0 / kTwoPi;   // 2^48 / (2 pi)
constexpr uint64_t kKeyMax = (1ull << 48) - 1;

__device__ __forceinline__ bool solve_roots(double p, double q, double bi, double& al,
                                            double& be) {
    const double r = hypot(p, q);
    if (!(r > 0.0)) return false;
    double z = bi / r;
    if (!(z < 1.0)) return false;
    z = fmax(z, -1.0);
    const double tau = atan2(q, p);
    const double phi = acos(z);
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

// ---- block-wide helpers (256 threads = 4 waves of 64) ----
// Position of this thread's element among the block's true predicates, and
// the block total.
__device__ __forceinline__ int block_count_prefix(bool pred, int* s_w, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(pred);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[w] = __popcll(mask);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
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

// Exclusive scan of one value per thread (thread order), identity `id`.
template <typename Op>
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
    for (int i = 0; i < 4; ++i)
        if (i < w) pre = op(pre, s_w[i]);
    __syncthreads();
    return (lane == 0) ? pre : op(pre, ex);
}

// Ascending bitonic sort of key[0 .. n2), n2 a power of two >= 512.
__device__ __forceinline__ void bitonic_sort_lds(uint64_t* key, int n2) {
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (n2 >> 1); t += 256) {
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

// Accept or reject the pending proposal of chain c (Section 3.3: a proposal
// violating some constraint is dropped and the chain stays).  Returns the
// buffer index of the chain's committed projections.
template <typename T>
__device__ __forceinline__ int commit_chain(const SampleArgs& a, int c) {
    const int fl = a.flag[c];
    const int s = a.sel[c];
    __syncthreads();   // all reads of flag / sel precede the writes below
    const int snew = fl ? s : (s ^ 1);
    if (threadIdx.x == 0) {
        if (fl) a.rej[c] += 1;
        a.sel[c] = snew;
        a.flag[c] = 0;
        if (a.rejected_out) a.rejected_out[c] = fl;
    }
    T* x = static_cast<T*>(a.X) + static_cast<size_t>(c) * a.dp;
    const T* xp = static_cast<const T*>(a.Xprop) + static_cast<size_t>(c) * a.dp;
    T* tr = a.trace ? static_cast<T*>(a.trace) + static_cast<size_t>(c) * a.d : nullptr;
    for (int k = threadIdx.x; k < a.d; k += 256) {
        T v;
        if (!fl) {
            v = xp[k];
            x[k] = v;
        } else {
            v = x[k];
        }
        if (tr) tr[k] = v;
    }
    return snew;
}

template <typename T>
__global__ __launch_bounds__(256) void commit_kernel(SampleArgs a) {
    commit_chain<T>(a, blockIdx.x);
}

// nu for `step` into dst[c * ld + k], k < d (chains 0 .. C-1).
template <typename T>
__global__ __launch_bounds__(256) void draw_kernel(uint64_t seed, uint32_t step, uint32_t problem,
                                                   int d, T* dst, long long ld, double* u) {
    const int c = blockIdx.x;
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

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void sample_kernel(SampleArgs a) {
    __shared__ double s_alpha[NMAX];
    __shared__ double s_beta[NMAX];
    __shared__ uint64_t s_key[NMAX];
    __shared__ double s_red[4];
    __shared__ int s_cnt[4];
    __shared__ double s_bcast[2];
    __shared__ int s_kstar;
    __shared__ double s_theta[2];

    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    int sel = a.sel[c];
    if (a.has_pending) sel = commit_chain<T>(a, c);

    // ---- roots of every constraint; keep the rows the ellipse crosses ----
    const T* Pc = static_cast<const T*>(a.P) + (static_cast<size_t>(sel) * a.Cp + c) * a.mp;
    const T* Qc = static_cast<const T*>(a.Q) + static_cast<size_t>(c) * a.mp;
    int n = 0;
    for (int i0 = 0; i0 < a.m; i0 += 256) {
        const int i = i0 + tid;
        double al = 0.0, be = 0.0;
        bool hit = false;
        if (i < a.m) {
            const T p = Pc[i], q = Qc[i];
            hit = solve_roots(static_cast<double>(p), static_cast<double>(q), a.b[i], al, be);
            if (a.pq_out) {
                T* pq = static_cast<T*>(a.pq_out);
                pq[static_cast<size_t>(c) * a.m + i] = p;
                pq[(static_cast<size_t>(a.C) + c) * a.m + i] = q;
            }
        }
        int tot;
        const int pos = block_count_prefix(hit, s_cnt, tot);
        if (hit) {
            const int slot = n + pos;
            s_alpha[slot] = al;
            s_beta[slot] = be;
            s_key[slot] = sort_key(al, slot);
        }
        n += tot;
    }
    int n2 = 512;
    while (n2 < n) n2 <<= 1;
    for (int k = n + tid; k < n2; k += 256) s_key[k] = ~0ull;
    __syncthreads();
    bitonic_sort_lds(s_key, n2);

    // ---- sweep: running max of beta in alpha order, candidate lengths ----
    const int per = n2 >> 8;
    const int k0 = tid * per;
    const int k1 = min(k0 + per, n);
    const double eps = a.eps;
    double tmax = 0.0;
    for (int k = k0; k < k1; ++k) tmax = fmax(tmax, s_beta[s_key[k] & 0xFFFF]);
    const double g_in = block_excl_scan(tmax, 0.0, MaxOp(), s_red);
    const bool owns_last = (tid == 255);

    auto cand = [&](int k, double& g, double& lo, double& hi) {
        const int slot = static_cast<int>(s_key[k] & 0xFFFF);
        lo = g;
        hi = s_alpha[slot];
        g = fmax(g, s_beta[slot]);
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
    // The last candidate [gamma_n, 2 pi] belongs to thread 255, whose running
    // max at the end of its chunk is gamma_n.
    double last_lo = 0.0, last_len = 0.0;
    if (owns_last) {
        last_lo = gend > 0.0 ? gend + eps : gend;
        last_len = fmax(kTwoPi - last_lo, 0.0);
        tsum += last_len;
    }
    const double s_in = block_excl_scan(tsum, 0.0, SumOp(), s_red);
    if (owns_last) s_bcast[0] = s_in + tsum;
    if (tid == 0) s_kstar = 0x7FFFFFFF;
    __syncthreads();
    const double total = s_bcast[0];
    const double u = a.u_explicit ? a.u_explicit[c] : Rng(a.seed).theta_uniform(c, a.step, a.problem);
    const double s = u * total;

    // ---- theta: first candidate whose running sum exceeds s (inverse CDF) ----
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
        if (my_k != 0x7FFFFFFF) atomicMin(&s_kstar, my_k);
    }
    __syncthreads();
    const int kstar = s_kstar;
    __syncthreads();   // every thread has read s_kstar before it is reused
    if (total > 0.0) {
        if (kstar == 0x7FFFFFFF) {
            // s rounded up to the total: take the upper end of the last piece
            if (tid == 0) s_kstar = -1;
            __syncthreads();
            if (last_k >= 0) atomicMax(&s_kstar, last_k);
            __syncthreads();
            if (last_k >= 0 && last_k == s_kstar) s_theta[0] = last_hi;
        } else if (my_k == kstar) {
            s_theta[0] = my_theta;
        }
    } else if (tid == 0) {
        s_theta[0] = 0.0;
        a.flag[c] = 1;   // empty active set: stay, counted as a rejection
    }

    // ---- optional: the non-empty trimmed intervals, ascending ----
    if (a.intervals) {
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
        const double base = block_excl_scan(static_cast<double>(cnt), 0.0, SumOp(), s_red);
        int w = static_cast<int>(base);
        double* out = a.intervals + static_cast<size_t>(c) * (a.m + 1) * 2;
        double g = g_in;
        for (int k = k0; k < k1; ++k) {
            double lo, hi;
            cand(k, g, lo, hi);
            if (hi - lo > 0.0) {
                out[2 * w] = lo;
                out[2 * w + 1] = hi;
                ++w;
            }
        }
        if (owns_last) {
            if (last_len > 0.0) {
                out[2 * w] = last_lo;
                out[2 * w + 1] = kTwoPi;
                ++w;
            }
            if (a.n_intervals) a.n_intervals[c] = w;
        }
    }
    __syncthreads();
    const double theta = s_theta[0];
    if (tid == 0 && a.theta_out) a.theta_out[c] = theta;

    // ---- move along the ellipse: x' = x cos(theta) + nu sin(theta) ----
    double sd, cd;
    sincos(theta, &sd, &cd);
    const T ct = static_cast<T>(cd), st = static_cast<T>(sd);
    const T* x = static_cast<const T*>(a.X) + static_cast<size_t>(c) * a.dp;
    T* xp = static_cast<T*>(a.Xprop) + static_cast<size_t>(c) * a.dp;
    T* nu = static_cast<T*>(a.N) + static_cast<size_t>(c) * a.dp;
    for (int k = tid; k < a.d; k += 256) xp[k] = x[k] * ct + nu[k] * st;

    // ---- the next step's ellipse direction ----
    if (a.gen_next) {
        __syncthreads();   // every read of this step's nu is done
        const Rng rng(a.seed);
        for (int j = tid; 2 * j < a.d; j += 256) {
            double z0, z1;
            rng.normal_pair(j, c, a.step + 1, a.problem, z0, z1);
            nu[2 * j] = static_cast<T>(z0);
            if (2 * j + 1 < a.d) nu[2 * j + 1] = static_cast<T>(z1);
        }
    }
}

}  // namespace ess
