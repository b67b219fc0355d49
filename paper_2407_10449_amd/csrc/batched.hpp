// Many independent polytopes of uneven size advanced together.
//
// One persistent launch per step.  Its work queue holds first every projection
// tile of every problem (A x' for the previous proposals and A nu for this
// step, Section 2 and 3.3), then one item per chain (commit the previous
// proposal; roots, active intervals, theta and move as in the single-problem
// kernels).  Workgroups take items from a device counter in queue order.  A
// chain item waits until all tiles of its problem have been released: every
// tile is taken before any chain item, and a taken tile belongs to a running
// workgroup, so the wait ends (a spin limit turns a broken invariant into an
// error flag instead of a hang).  Queue and tile counters are indexed by step
// parity; each launch clears the other parity's counters for the next one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm.hpp"
#include "sample.hpp"

namespace ess {

constexpr int kBatchBM = 64, kBatchBN = 64;

struct ProbDesc {
    int d, m, C, dp, mp, Cp;
    int ntiles;          // projection tiles of this problem (both column halves)
    int chain_off;       // first padded chain index (sel / flag / rej)
    long long a_off;     // A pack: mp x dp block
    long long b_off;     // b pack: m
    long long x_off;     // X / X' / nu packs: Cp x dp block
    long long p_off;     // P pack: 2 x Cp x mp block
    long long q_off;     // Q pack: Cp x mp block
    long long t_off;     // caller state / trace layout: C x d block
    double eps;
    uint64_t seed;
};

struct BatchArgs {
    int n_probs, NT, NC;
    const ProbDesc* descs;
    const int4* tiles;     // (problem, tile row, tile column, 0)
    const int2* chains;    // (problem, chain)
    const float* A;
    const double* b;
    float* X;
    float* Xprop;
    float* N;
    float* P;
    float* Q;
    int* sel;
    int* flag;
    long long* rej;
    int* queue;            // [2]
    int* done;             // [2][n_probs]
    int* fb_list;          // [total chains]: global chain-table indices
    int* fb_count;         // [2]
    int* error;            // [1]: set when a wait exceeds its spin limit
    uint32_t step;         // relative to *step_base
    const uint32_t* step_base;   // nullable device counter
    int has_pending;       // commit the previous proposals
    int do_sample;         // chain items also sample (0: commit only)
    int gen_next;
    int cols;              // tiles computed: 0 x' half, 1 nu half, 2 both
    int p_direct, strict;  // projection epilogue mode
    float* trace;          // nullable: committed states of the previous step
};

__device__ __forceinline__ uint32_t abs_step(const BatchArgs& a) {
    return a.step + (a.step_base ? *a.step_base : 0u);
}

__device__ __forceinline__ ProjOut batch_proj_out(const BatchArgs& a, const ProbDesc& pd) {
    ProjOut o;
    o.m = pd.m;
    o.C = pd.C;
    o.Cp = pd.Cp;
    o.mp = pd.mp;
    o.c0 = 0;
    o.Cg = pd.Cp;
    o.b = a.b + pd.b_off;
    o.bstride = 0;
    o.P = a.P + pd.p_off;
    o.Q = a.Q + pd.q_off;
    o.sel = a.sel + pd.chain_off;
    o.flag = a.flag + pd.chain_off;
    o.p_direct = a.p_direct;
    o.strict = a.strict;
    return o;
}

__device__ __forceinline__ ChainRef<float> batch_ref(const BatchArgs& a, const ProbDesc& pd,
                                                     int p, int c) {
    ChainRef<float> r;
    r.d = pd.d;
    r.m = pd.m;
    r.chain = static_cast<uint32_t>(c);
    r.problem = static_cast<uint32_t>(p);
    r.step = abs_step(a);
    r.gen_next = a.gen_next;
    r.eps = pd.eps;
    r.seed = pd.seed;
    r.b = a.b + pd.b_off;
    r.P0 = a.P + pd.p_off + static_cast<size_t>(c) * pd.mp;
    r.pstride = static_cast<size_t>(pd.Cp) * pd.mp;
    r.q = a.Q + pd.q_off + static_cast<size_t>(c) * pd.mp;
    r.x = a.X + pd.x_off + static_cast<size_t>(c) * pd.dp;
    r.xp = a.Xprop + pd.x_off + static_cast<size_t>(c) * pd.dp;
    r.nu = a.N + pd.x_off + static_cast<size_t>(c) * pd.dp;
    r.sel = a.sel + pd.chain_off + c;
    r.flag = a.flag + pd.chain_off + c;
    r.rej = a.rej + pd.chain_off + c;
    r.trace = a.trace ? a.trace + pd.t_off + static_cast<size_t>(c) * pd.d : nullptr;
    r.u = nullptr;
    r.intervals = nullptr;
    r.n_intervals = nullptr;
    r.theta_out = nullptr;
    r.p_out = nullptr;
    r.q_out = nullptr;
    r.rejected_out = nullptr;
    return r;
}

// Tile `t` of the batch (skipped when outside the selected column half).
__device__ __forceinline__ void batch_tile(const BatchArgs& a, int4 t,
                                           GemmLds<kBatchBM, kBatchBN>& L) {
    const ProbDesc& pd = a.descs[t.x];
    const int n0 = t.z * kBatchBN;
    const bool nu_half = n0 >= pd.Cp;
    if ((a.cols == 0 && nu_half) || (a.cols == 1 && !nu_half)) return;
    const ProjOut o = batch_proj_out(a, pd);
    gemm_tile_f32<kBatchBM, kBatchBN>(a.A + pd.a_off, a.Xprop + pd.x_off, a.N + pd.x_off, pd.dp,
                                      t.y * kBatchBM, n0, o, L);
}

template <int NB>
union BatchLds {
    GemmLds<kBatchBM, kBatchBN> g;
    BucketLds<NB> b;
};

template <int RPT, int NB>
__global__ __launch_bounds__(256) void batched_step_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) BatchLds<NB> lds;
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int par = static_cast<int>(abs_step(a) & 1u);
    const int total = a.NT + a.NC;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.queue + par, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        if (item == 0 && tid == 0) {
            a.queue[par ^ 1] = 0;            // the next launch's queue
            a.fb_count[par ^ 1] = 0;         // and its full-sort list
        }
        if (item < a.NT) {
            const int4 t = a.tiles[item];
            batch_tile(a, t, lds.g);
            if (tid == 0) {
                __threadfence();
                atomicAdd(a.done + par * a.n_probs + t.x, 1);
            }
        } else {
            const int2 ch = a.chains[item - a.NT];
            const ProbDesc& pd = a.descs[ch.x];
            if (tid == 0) {
                int* cnt = a.done + par * a.n_probs + ch.x;
                long spins = 0;
                while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < pd.ntiles) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > (1l << 26)) {
                        atomicExch(a.error, 1);
                        break;
                    }
                }
                __threadfence();
                if (ch.y == 0) a.done[(par ^ 1) * a.n_probs + ch.x] = 0;   // next launch
            }
            __syncthreads();
            const ChainRef<float> r = batch_ref(a, pd, ch.x, ch.y);
            const int sel = a.has_pending ? commit_chain<float>(r) : *r.sel;
            if (a.do_sample) {
                const bool ok = bucket_chain<float, RPT, NB>(r, sel, lds.b);
                if (!ok && tid == 0) a.fb_list[atomicAdd(a.fb_count + par, 1)] = item - a.NT;
            }
        }
        __syncthreads();
    }
}

// Chains the batched step handed over, sorted in full.
template <int NMAX>
__global__ __launch_bounds__(256) void batched_fallback_kernel(BatchArgs a) {
    ESS_FULL_LDS(NMAX)
    const int par = static_cast<int>(abs_step(a) & 1u);
    const int count = a.fb_count[par];
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int2 ch = a.chains[a.fb_list[idx]];
        const ChainRef<float> r = batch_ref(a, a.descs[ch.x], ch.x, ch.y);
        full_chain<float>(r, *r.sel, full_lds);
        __syncthreads();
    }
}

// Projection tiles only, one block per tile (state checks outside a run).
__global__ __launch_bounds__(256) void batched_proj_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) GemmLds<kBatchBM, kBatchBN> lds;
    batch_tile(a, a.tiles[blockIdx.x], lds);
}

// nu of `step` for every chain of the batch (one block per chain).
__global__ __launch_bounds__(256) void batched_draw_kernel(BatchArgs a) {
    const int2 ch = a.chains[blockIdx.x];
    const ProbDesc& pd = a.descs[ch.x];
    const Rng rng(pd.seed);
    float* nu = a.N + pd.x_off + static_cast<size_t>(ch.y) * pd.dp;
    for (int j = threadIdx.x; 2 * j < pd.d; j += 256) {
        double z0, z1;
        rng.normal_pair(j, ch.y, abs_step(a), ch.x, z0, z1);
        nu[2 * j] = static_cast<float>(z0);
        if (2 * j + 1 < pd.d) nu[2 * j + 1] = static_cast<float>(z1);
    }
}

// Caller layout (problem blocks of C x d) <-> library rows (Cp x dp blocks),
// one block per chain.
__global__ __launch_bounds__(256) void batched_copy_rows(BatchArgs a, const float* src, float* dst,
                                                         int to_library) {
    const int2 ch = a.chains[blockIdx.x];
    const ProbDesc& pd = a.descs[ch.x];
    const size_t lrow = pd.x_off + static_cast<size_t>(ch.y) * pd.dp;
    const size_t crow = pd.t_off + static_cast<size_t>(ch.y) * pd.d;
    for (int k = threadIdx.x; k < pd.d; k += 256) {
        if (to_library) dst[lrow + k] = src[crow + k];
        else dst[crow + k] = src[lrow + k];
    }
}

__global__ void zero_ints_n(int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace ess
