// Many independent polytopes of uneven size advanced together.
//
// Work per step: every projection tile of every problem (A x' for the
// previous proposals and A nu for this step, Section 2 and 3.3), then one item
// per chain (commit the previous proposal; roots, active intervals, theta and
// move as in the single-problem kernels).  Two launch forms give the same
// results:
//
// * split (batched_proj_kernel, then batched_chain_kernel): the kernel
//   boundary makes the tiles' projections visible to the chains.  The tile
//   order keeps each row panel of a problem's A on one XCD.
// * fused (batched_step_kernel): one launch.  Every problem owns a run of
//   workgroups, one per tile and one per chain; the tile runs of all problems
//   come first in the grid, then the chain runs.  A workgroup takes its item
//   from its problem's own ticket counter when it starts: tickets below the
//   problem's tile count are tiles, the rest chains.  A chain waits until all
//   tiles of its problem are released.  The tiles hold smaller tickets, and a
//   ticket is only ever held by a running workgroup, so the wait ends whatever
//   order the hardware starts workgroups in (a spin limit turns a broken
//   invariant into an error flag instead of a hang).  Counters per problem
//   keep the atomics spread out.  Ticket and tile counters are indexed by step
//   parity; the workgroup holding a problem's ticket 0 clears that problem's
//   counters of the other parity for the next launch.
//
// The fused form pays for its device-scope release / acquire pairs: on a part
// whose XCDs have separate L2 caches they write back and invalidate L2, per
// workgroup.  The split form pays one kernel boundary instead and is the
// default; the autotuner times both.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gemm.hpp"
#include "sample.hpp"

namespace ess {

// Projection tile shapes, chosen per problem: 0 = 64 x 64, 1 = 32 x 64,
// 2 = 64 x 32, 3 = 32 x 32 (rows of A x chain columns) on the float32
// matrix cores, and 4 = 64 x 64 split bfloat16 tiles (problems with more than
// 192 columns, as single-problem contexts take them).  Rows are padded to 64
// and chains to 64, so every shape tiles the padded blocks exactly.
constexpr int kBatchShapes = 4;   // the float32 shapes the autotuner picks from
constexpr int kBatchSplitShape = 4;
constexpr int kBatchPadM = 64, kBatchPadC = 64;
__host__ __device__ constexpr int shape_bm(int s) { return (s & 1) ? 32 : 64; }
__host__ __device__ constexpr int shape_bn(int s) { return (s & 2) ? 32 : 64; }

struct ProbDesc {
    int d, m, C, dp, mp, Cp;
    int shape;           // projection tile shape (see shape_bm / shape_bn)
    int cls;             // chain class: m <= 256 2^cls
    int tiles_n;         // tile columns: 2 Cp / shape_bn(shape)
    int ntiles;          // tiles: ceil(m / shape_bm(shape)) x tiles_n
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
    const int* wg_prob;    // [NT + NC]: the problem of each workgroup of the step launch
    const int4* tiles;     // [NTL]: (problem, tile row, tile column, 0) or (-1, ...) padding
    int NTL;               // entries of the tile table (NT plus padding)
    const int2* chains;    // [NC]: (problem, chain), larger chain classes first
    const float* A;
    const uint16_t* A3;    // [3][a_elems] bfloat16 pieces of A (piece p at A3 + p a_elems)
    size_t a_elems;
    const double* b;
    float* X;
    float* Xprop;
    float* N;
    float* P;
    float* Q;
    int* sel;
    int* flag;
    long long* rej;
    int* tickets;          // [2][n_probs]
    int* done;             // [2][n_probs]: released tiles
    int2* fb_list;         // unused since chains are sorted in place (kept for the layout)
    int* fb_count;         // [2]
    double2* ab;           // alpha, beta of a chain sorted in full: problem p's chain c
                           // owns ab[q_off + c mp ..) (the Q pack's layout)
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

// rows of 40 floats (conflict-free fragment reads, as in the single-problem
// kernel); the largest float32 shape takes 40 KB and the split tile 48 KB, so
// three workgroups share a CU
constexpr int kBatchPadK = 8;
union BatchGemmLds {
    GemmLds<64, 64, kBatchPadK> s0;
    GemmLds<32, 64, kBatchPadK> s1;
    GemmLds<64, 32, kBatchPadK> s2;
    GemmLds<32, 32, kBatchPadK> s3;
    SplitLds<64> s4;
};

// Tile (tm, tn) of problem pd in its own shape (skipped when outside the
// selected column half).
__device__ __forceinline__ void batch_tile(const BatchArgs& a, const ProbDesc& pd, int tm, int tn,
                                           BatchGemmLds& L) {
    const int bm = shape_bm(pd.shape), bn = shape_bn(pd.shape);
    const int n0 = tn * bn;
    const bool nu_half = n0 >= pd.Cp;
    if ((a.cols == 0 && nu_half) || (a.cols == 1 && !nu_half)) return;
    const ProjOut o = batch_proj_out(a, pd);
    const float* A = a.A + pd.a_off;
    const float* B0 = a.Xprop + pd.x_off;
    const float* B1 = a.N + pd.x_off;
    const int m0 = tm * bm;
    switch (pd.shape) {
        case 0: gemm_tile_f32<64, 64, 2, 2, kBatchPadK>(A, B0, B1, pd.dp, m0, n0, o, L.s0); break;
        case 1: gemm_tile_f32<32, 64, 2, 2, kBatchPadK>(A, B0, B1, pd.dp, m0, n0, o, L.s1); break;
        case 2: gemm_tile_f32<64, 32, 2, 2, kBatchPadK>(A, B0, B1, pd.dp, m0, n0, o, L.s2); break;
        case 3: gemm_tile_f32<32, 32, 2, 2, kBatchPadK>(A, B0, B1, pd.dp, m0, n0, o, L.s3); break;
        default: {
            const uint16_t* A3 = a.A3 + pd.a_off;
            gemm_tile_split<64, 2, 2>(A3, A3 + a.a_elems, A3 + 2 * a.a_elems, B0, B1, pd.dp, m0, n0,
                                      o, L.s4);
            break;
        }
    }
}

// LDS of a chain item: the bucket arrays of its class or, for a chain the
// bucket path hands back, the keys of the full sort done in place.  The
// fused form adds the projection tiles' arrays to the union.
template <int NK, bool GEMM>
struct BatchLds {
    union {
        BucketLds<256> b0;
        BucketLds<512> b1;
        BucketLds<1024> b2;
        BucketLds<2048> b3;
        uint64_t key[NK];
        typename std::conditional<GEMM, BatchGemmLds, char>::type g;
    };
    double red[8];
    int cnt[8];
    double bcast[2];
    int kstar;
    double theta[2];
};

// A chain after the commit's decision: the committed projection buffer,
// whether the proposal became the state (its row copies then happen in the
// move's pass, as in the single-problem kernel), and the next direction's
// first pair, drawn already.
struct ChainStart {
    int sel;
    bool from_prop;
    NextPair<float> next;
};

// The per-chain part of a batched step after the commit: the bucket path, and
// for a chain whose survivors overflow the full sort in place from its roots,
// which the bucket path leaves in a.ab (keys in the bucket arrays' LDS).
template <int RPT, int NB>
__device__ __forceinline__ void batch_sample(const BatchArgs& a, const ProbDesc& pd, int c,
                                             const ChainRef<float>& r, const ChainStart& st,
                                             BucketLds<NB>& bucket, const FullLds& L) {
    double2* abg = a.ab + pd.q_off + static_cast<size_t>(c) * pd.mp;
    double theta = 0.0;
    const bool done = bucket_chain<float, RPT, NB>(r, st.sel, bucket, theta, nullptr, abg);
    if (!done) {
        __syncthreads();   // every row's alpha and beta is in a.ab
        theta = full_chain<float, KEYS_ROW_AB, 256>(r, st.sel, L, abg);
    }
    move_pairs<float, 256>(r, theta, st.from_prop, st.from_prop && a.has_pending, nullptr,
                           &st.next, done ? bucket.sc : nullptr);
}

// The chain's class picks the rows per thread and the bucket count, so a
// chain of a small problem runs no more passes and bucket sweeps than its
// rows need, whatever the largest problem of the batch: up to 256 rows one
// row per thread and 256 buckets, up to 1024 rows four and 1024 buckets (two
// and 512 when no problem is larger), the rest the batch's largest.  When
// some problem has more than 2048 rows, only the first class is kept apart.
// A further variant inlined beside these has put the row arrays of every
// variant in scratch memory.  The bucket path's result does not depend on
// the bucket count (survivors that coarser buckets add have empty
// candidates), so the chains are those of the single-problem kernels.
template <int RPT_MAX, typename Lds>
__device__ __forceinline__ void batch_sample_class(const BatchArgs& a, const ProbDesc& pd, int c,
                                                   const ChainRef<float>& r, const ChainStart& st,
                                                   Lds& lds) {
    const FullLds L{nullptr, nullptr, lds.key, lds.red, lds.cnt, lds.bcast, &lds.kstar, lds.theta};
    const int cls = __builtin_amdgcn_readfirstlane(pd.cls);
    constexpr int MID = RPT_MAX > 8 ? 1 : (RPT_MAX < 4 ? RPT_MAX : 4);
    constexpr int TOP = RPT_MAX > 8 ? 1 : 3;   // first class of the largest variant
    if constexpr (RPT_MAX > 4) {
        if (cls >= TOP) return batch_sample<RPT_MAX, 2048>(a, pd, c, r, st, lds.b3, L);
    }
    if constexpr (MID > 1) {
        if (cls >= 1) {
            if constexpr (MID == 4) return batch_sample<4, 1024>(a, pd, c, r, st, lds.b2, L);
            else return batch_sample<2, 512>(a, pd, c, r, st, lds.b1, L);
        }
    }
    batch_sample<1, 256>(a, pd, c, r, st, lds.b0, L);
}

// One chain's share of a step: the commit of its pending proposal, then
// (unless this launch only commits) Algorithm 3's step and the move.  The
// next direction's first pair is drawn while flag and sel load.
template <int RPT_MAX, typename Lds>
__device__ __forceinline__ void batch_chain_item(const BatchArgs& a, const ProbDesc& pd, int p,
                                                 int c, Lds& lds) {
    const ChainRef<float> r = batch_ref(a, pd, p, c);
    if (!a.do_sample) {
        if (a.has_pending) commit_chain<float>(r);
        return;
    }
    ChainStart st;
    st.from_prop = false;
    if (a.has_pending) {
        st.sel = commit_flags<float>(r, st.from_prop, &st.next);
    } else {
        st.next = draw_next_pair<float>(r);
        st.sel = *r.sel;
    }
    batch_sample_class<RPT_MAX>(a, pd, c, r, st, lds);
}

template <int RPT>
constexpr int batch_keys() { return RPT * 256 > 512 ? RPT * 256 : 512; }

template <int RPT_MAX>
__global__ __launch_bounds__(256) void batched_step_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) BatchLds<batch_keys<RPT_MAX>(), true> lds;
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int par = static_cast<int>(abs_step(a) & 1u);
    const int p = a.wg_prob[blockIdx.x];
    const ProbDesc& pd = a.descs[p];
    if (tid == 0) s_item = atomicAdd(a.tickets + par * a.n_probs + p, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item == 0 && tid == 0) {                                 // the next launch's counters
        a.tickets[(par ^ 1) * a.n_probs + p] = 0;
        a.done[(par ^ 1) * a.n_probs + p] = 0;
    }
    if (item < pd.ntiles) {
        batch_tile(a, pd, item / pd.tiles_n, item % pd.tiles_n, lds.g);
        // every wave publishes its own stores before the barrier (a barrier
        // alone does not wait for them), then one release counts the tile
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0)
            __hip_atomic_fetch_add(a.done + par * a.n_probs + p, 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int c = item - pd.ntiles;
    if (c >= pd.C) return;   // the grid holds exactly ntiles + C workgroups per problem
    if (tid == 0) {
        int* cnt = a.done + par * a.n_probs + p;
        long spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < pd.ntiles) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1l << 26)) {
                atomicExch(a.error, 1);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // one acquire, after the wait
    }
    __syncthreads();
    batch_chain_item<RPT_MAX>(a, pd, p, c, lds);
}

// Split form, second launch: one workgroup per chain (the caller's order).
// Chains of the larger classes come first in a.chains, so the longest items
// start early.
template <int RPT_MAX>
__global__ __launch_bounds__(256, RPT_MAX <= 8 ? 6 : 1) void batched_chain_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) BatchLds<batch_keys<RPT_MAX>(), false> lds;
    const int2 ch = a.chains[blockIdx.x];
    batch_chain_item<RPT_MAX>(a, a.descs[ch.x], ch.x, ch.y, lds);
}

// Projection tiles, one block per entry of the tile table (split form, and
// the state checks outside a run).
__global__ __launch_bounds__(256) void batched_proj_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) BatchGemmLds lds;
    const int4 t = a.tiles[blockIdx.x];
    if (t.x < 0) return;   // padding that keeps the XCD assignment of the order
    batch_tile(a, a.descs[t.x], t.y, t.z, lds);
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
