// libess host side: problem validation, library-owned device memory, and the
// launch sequence of each transition.
//
// Per step the device runs two kernels:
//   sample_kernel  (one workgroup per chain): commit the previous proposal,
//                  roots, sort + cumulative max, theta, x', next nu
//   proj_gemm      (matrix cores): A x' for the safeguard check together with
//                  A nu for the next step, in one launch over 2 Cp columns
// so a run of T steps is 2 T + 3 launches.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ess.h"
#include "gemm.hpp"
#include "gemv.hpp"
#include "philox.hpp"
#include "sample.hpp"
#include "batched.hpp"
#include "mlp.hpp"
#include "gauss.hpp"

using namespace ess;

namespace {

thread_local std::string g_err;

ess_status fail(ess_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? ESS_ERR_OOM : ESS_ERR_HIP, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                  \
    } while (0)

#define ESS_TRY(expr)                    \
    do {                                 \
        ess_status s_ = (expr);          \
        if (s_ != ESS_OK) return s_;     \
    } while (0)

int round_up(int v, int q) { return (v + q - 1) / q * q; }

// One d-vector copied into every chain row (ESS_X0_BROADCAST).
template <typename T>
__global__ void broadcast_rows(const T* __restrict__ src, T* __restrict__ dst, int d, int dp) {
    T* row = dst + static_cast<size_t>(blockIdx.x) * dp;
    for (int k = threadIdx.x; k < d; k += blockDim.x) row[k] = src[k];
}

}  // namespace

constexpr int kMaxGroups = 4;
// size classes of batched problems for the tile-shape choice:
// d <= 64, d <= 192, d > 192, each split at m <= 256
constexpr int kTileBuckets = 6;

// A contiguous block of chains with its own stream during ess_run: chains
// [c0, c0 + n) valid, padded to Cg (a multiple of every projection tile width).
struct Group {
    int c0, n, Cg;
};

struct ess_ctx {
    int d = 0, m = 0, C = 0, prec = 32, esz = 4;
    int dp = 0, mp = 0, Cp = 0;
    uint64_t seed = 0;
    double eps = 0.0;
    uint32_t flags = 0;
    int bstride = 0;   // 0: one b for every chain; m: a b per chain (ESS_PER_CHAIN_B)
    hipStream_t st = nullptr;
    void* A = nullptr;
    double* b = nullptr;
    void* X = nullptr;
    void* Xprop = nullptr;
    void* N = nullptr;
    void* P = nullptr;
    void* Q = nullptr;
    int* sel = nullptr;
    int* flag = nullptr;
    long long* rej = nullptr;
    int* fb_list = nullptr;    // chains handed to the full-sort path
    uint64_t* keys = nullptr;  // more than 16384 rows: [Cp][kstride] full-sort keys
    int kstride = 0;
    uint16_t* A3 = nullptr;    // [3][mp][dp] bfloat16 pieces of A (split projections)
    bool split_proj = false;   // float32 projections through exact bfloat16 splits
    void* AB = nullptr;        // [Cp][mp] double2: alpha, beta of every row (m > 4096, or
                               // m > 2048 with at most 256 chains), and of a chain the
                               // bucket path hands to the full sort
    int* fb_count = nullptr;   // [2 per group]: list lengths by step parity
    int* accepted = nullptr;   // [Cp]: gated starts taken
    uint32_t* d_step = nullptr;   // device copy of the step counter, read by the kernels
    uint64_t step = 0;
    // graph replay of ess_run: a capture stream and executables keyed by the run shape
    hipStream_t cs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    struct GraphEntry {
        int64_t n_steps, thin;
        void* trace;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    bool use_graphs = true;
    int bm = 128, bn = 128, group_m = 4;
    // chain groups: each runs its own sample -> project pipeline on its own
    // stream, so one group's matrix-core work overlaps another's vector work
    int G = 1;
    hipStream_t gs[kMaxGroups] = {};
    hipEvent_t fork = nullptr, join[kMaxGroups] = {};
    hipEvent_t stagger[kMaxGroups] = {};   // group g's per-chain kernel of a step is done
    std::vector<void*> allocs;
    // kernel timing (ess_profile)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
    double prof_ms[4] = {0, 0, 0, 0};
    long long prof_n[4] = {0, 0, 0, 0};
    // many problems advanced together (ess_init_batched)
    struct Batch {
        int n = 0, NT = 0, NTL = 0, NC = 0, rpt = 1;
        bool fused = false;          // one launch per step instead of tiles, then chains
        long long state_elems = 0;   // sum of C d (caller layout)
        int chains_padded = 0;
        int max_tiles = 0;           // NT with the smallest tiles everywhere
        int max_table = 0;           // tile table capacity (max_tiles plus XCD padding)
        int bucket_shape[kTileBuckets] = {};   // tile shape of each size class
        // problem sets advanced on streams of their own (split launch form):
        // set k's tiles are tiles[set_toff[k] ..) (set_ntl[k] entries) and its
        // chains chains[set_coff[k] ..) (set_nc[k])
        int nsets = 1;
        std::vector<int> set_of;     // [n] the set of each problem
        int set_toff[kMaxGroups] = {}, set_ntl[kMaxGroups] = {};
        int set_coff[kMaxGroups] = {}, set_nc[kMaxGroups] = {};
        std::vector<ProbDesc> h;
        std::vector<int> order;      // problems by decreasing projection work
        ProbDesc* descs = nullptr;
        int* wg_prob = nullptr;      // [max_tiles + NC]
        int4* tiles = nullptr;       // [max_table]
        int2* chains = nullptr;      // [NC], the caller's order
        float* A = nullptr;
        uint16_t* A3 = nullptr;      // [3][sum mp dp] bfloat16 pieces of A (split tiles)
        size_t a_elems = 0;          // sum over problems of mp dp
        float* X = nullptr;
        float* Xprop = nullptr;
        float* N = nullptr;
        float* P = nullptr;
        float* Q = nullptr;
        double* b = nullptr;
        int* counters = nullptr;   // fb_count[2], error[1], tickets[2 n], done[2 n]
        int2* fb_list = nullptr;
        double2* ab = nullptr;       // alpha, beta of chains sorted in full (the Q pack's layout)
    };
    std::unique_ptr<Batch> batch;

    Group whole() const { return Group{0, C, Cp}; }
    // G groups of whole 128-chain panels, as even as the panels allow
    Group group(int g) const {
        const int panels = Cp / 128;
        const int p0 = g * panels / G, p1 = (g + 1) * panels / G;
        const int c0 = p0 * 128, Cg = (p1 - p0) * 128;
        return Group{c0, std::max(0, std::min(C - c0, Cg)), Cg};
    }
};

namespace {

ess_status dalloc(ess_ctx* c, void** p, size_t bytes) {
    HIP_TRY(hipMalloc(p, bytes));
    c->allocs.push_back(*p);
    HIP_TRY(hipMemsetAsync(*p, 0, bytes, c->st));
    return ESS_OK;
}

// The group streams and their events (every one exists from the start: the
// autotuner and cached choices may raise the group count later).
ess_status create_group_streams(ess_ctx* c) {
    hipError_t ee = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    for (int g = 0; g < kMaxGroups && ee == hipSuccess; ++g) {
        ee = hipStreamCreateWithFlags(&c->gs[g], hipStreamNonBlocking);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&c->join[g], hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&c->stagger[g], hipEventDisableTiming);
    }
    if (ee != hipSuccess) return fail(ESS_ERR_HIP, "creating group streams: %s", hipGetErrorString(ee));
    return ESS_OK;
}

ess_status create_run_streams(ess_ctx* c) {
    HIP_TRY(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    c->use_graphs = !(c->flags & ESS_EAGER) && !std::getenv("ESS_EAGER");
    return ESS_OK;
}

hipEvent_t take_event(ess_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches issued by `fn` on stream st with an event pair when
// profiling.
template <typename F>
ess_status timed(ess_ctx* c, int kind, hipStream_t st, F&& fn) {
    if (!c->profiling) return fn();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return fail(ESS_ERR_HIP, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(a, st));
    ess_status s = fn();
    HIP_TRY(hipEventRecord(b, st));
    c->ev_open.push_back({kind, {a, b}});
    return s;
}

ess_status drain_events(ess_ctx* c) {
    if (c->ev_open.empty()) return ESS_OK;
    HIP_TRY(hipStreamSynchronize(c->st));
    for (auto& e : c->ev_open) {
        HIP_TRY(hipEventSynchronize(e.second.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.second.first, e.second.second));
        c->prof_ms[e.first] += ms;
        c->prof_n[e.first] += 1;
        c->ev_pool.push_back(e.second.first);
        c->ev_pool.push_back(e.second.second);
    }
    c->ev_open.clear();
    return ESS_OK;
}

ProjOut proj_out(const ess_ctx* c, const Group& g, int p_direct, int strict) {
    ProjOut o;
    o.m = c->m;
    o.C = c->C;
    o.Cp = c->Cp;
    o.mp = c->mp;
    o.c0 = g.c0;
    o.Cg = g.Cg;
    o.b = c->b;
    o.bstride = c->bstride;
    o.P = c->P;
    o.Q = c->Q;
    o.sel = c->sel;
    o.flag = c->flag;
    o.p_direct = p_direct;
    o.strict = strict;
    return o;
}

enum Cols { COLS_X = 0, COLS_NU = 1, COLS_BOTH = 2 };

template <int BM, int BN, int NW_M = 2, int NW_N = 2>
void launch_f32(const ess_ctx* c, const Group& g, hipStream_t st, const float* B0, int cols,
                const ProjOut& o) {
    const int tiles_m = c->mp / BM, half = g.Cg / BN;
    const int tn0 = (cols == COLS_NU) ? half : 0;
    const int tiles_n = (cols == COLS_BOTH) ? 2 * half : half;
    const float* B1 = static_cast<const float*>(c->N) + static_cast<size_t>(g.c0) * c->dp;
    hipLaunchKernelGGL((proj_gemm_f32<BM, BN, NW_M, NW_N>), dim3(tiles_m * tiles_n),
                       dim3(64 * NW_M * NW_N), 0, st,
                       static_cast<const float*>(c->A), B0, B1, c->dp, tiles_m, tiles_n, tn0,
                       c->group_m, o);
}

// Projections of group g's columns selected by `cols`: rows of Y (x or x')
// and/or the current nu rows.  One workgroup per four rows.
template <typename T, int CW, int NG>
void launch_gemv(const ess_ctx* c, hipStream_t st, const T* B0, const T* B1, int cols,
                 const ProjOut& o) {
    hipLaunchKernelGGL((proj_gemv<T, CW, NG>), dim3((c->m + 3) / 4), dim3(256), 0, st,
                       static_cast<const T*>(c->A), B0, B1, c->dp, cols, o);
}

// Groups of at most kGemvChains chains take the row-parallel kernel: up to 4
// chains with the four waves splitting K, 5 to 12 as four waves of 3 chains
// over the whole of K (measured 10 % faster than two waves of 6 chains with
// K split in two: 7.7 against 8.5 ms for 10 chains x 100 steps at d = 4000).
// The four waves of 3 chains each stream the workgroup's rows of A, which
// the caches absorb while A fits in them; above kGemvCachedBytes (the
// last-level cache is 256 MB) two waves of 6 chains read A half as often.
constexpr int kGemvChains = 12;
constexpr size_t kGemvCachedBytes = static_cast<size_t>(128) << 20;

ess_status launch_proj(const ess_ctx* c, const Group& g, hipStream_t st, const void* Y, int cols,
                       int p_direct, int strict) {
    const ProjOut o = proj_out(c, g, p_direct, strict);
    const size_t off = static_cast<size_t>(g.c0) * c->dp;
    if (g.n <= kGemvChains) {
        if (c->prec == 32) {
            const float* B0 = static_cast<const float*>(Y) + off;
            const float* B1 = static_cast<const float*>(c->N) + off;
            const bool big = static_cast<size_t>(c->mp) * c->dp * c->esz > kGemvCachedBytes;
            if (g.n <= 2) launch_gemv<float, 2, 1>(c, st, B0, B1, cols, o);
            else if (g.n <= 4) launch_gemv<float, 4, 1>(c, st, B0, B1, cols, o);
            else if (big) launch_gemv<float, kGemvChains / 2, 2>(c, st, B0, B1, cols, o);
            else launch_gemv<float, kGemvChains / 4, 4>(c, st, B0, B1, cols, o);
        } else {
            const double* B0 = static_cast<const double*>(Y) + off;
            const double* B1 = static_cast<const double*>(c->N) + off;
            const bool big = static_cast<size_t>(c->mp) * c->dp * c->esz > kGemvCachedBytes;
            if (g.n <= 2) launch_gemv<double, 2, 1>(c, st, B0, B1, cols, o);
            else if (g.n <= 4) launch_gemv<double, 4, 1>(c, st, B0, B1, cols, o);
            else if (big) launch_gemv<double, kGemvChains / 2, 2>(c, st, B0, B1, cols, o);
            else launch_gemv<double, kGemvChains / 4, 4>(c, st, B0, B1, cols, o);
        }
        HIP_TRY(hipGetLastError());
        return ESS_OK;
    }
    if (c->prec == 32 && c->split_proj) {
        const float* B0 = static_cast<const float*>(Y) + off;
        const float* B1 = static_cast<const float*>(c->N) + off;
        const size_t plane = static_cast<size_t>(c->mp) * c->dp;
        const int bt = c->bm;   // 128 or 64 (bm = bn)
        const int tiles_m = c->mp / bt, half = g.Cg / bt;
        const int tn0 = (cols == COLS_NU) ? half : 0;
        const int tiles_n = (cols == COLS_BOTH) ? 2 * half : half;
        if (bt == 128)
            hipLaunchKernelGGL((proj_gemm_split<128, 4, 2>), dim3(tiles_m * tiles_n), dim3(512), 0,
                               st, c->A3, c->A3 + plane, c->A3 + 2 * plane, B0, B1, c->dp, tiles_m,
                               tiles_n, tn0, c->group_m, o);
        else
            hipLaunchKernelGGL((proj_gemm_split<64, 2, 2>), dim3(tiles_m * tiles_n), dim3(256), 0,
                               st, c->A3, c->A3 + plane, c->A3 + 2 * plane, B0, B1, c->dp, tiles_m,
                               tiles_n, tn0, c->group_m, o);
    } else if (c->prec == 32) {
        const float* B0 = static_cast<const float*>(Y) + off;
        if (c->bm == 128 && c->bn == 128) launch_f32<128, 128, 4, 2>(c, g, st, B0, cols, o);
        else if (c->bm == 128 && c->bn == 64) launch_f32<128, 64>(c, g, st, B0, cols, o);
        else if (c->bm == 64 && c->bn == 128) launch_f32<64, 128>(c, g, st, B0, cols, o);
        else launch_f32<64, 64>(c, g, st, B0, cols, o);
    } else {
        const int tiles_m = c->mp / 64, half = g.Cg / 64;
        const int tn0 = (cols == COLS_NU) ? half : 0;
        const int tiles_n = (cols == COLS_BOTH) ? 2 * half : half;
        hipLaunchKernelGGL((proj_gemm_f64<64, 64>), dim3(tiles_m * tiles_n), dim3(256), 0, st,
                           static_cast<const double*>(c->A), static_cast<const double*>(Y) + off,
                           static_cast<const double*>(c->N) + off, c->dp, tiles_m, tiles_n, tn0,
                           c->group_m, o);
    }
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

SampleArgs sample_args(const ess_ctx* c, const Group& g, int gi) {
    SampleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.d = c->d;
    a.m = c->m;
    a.C = c->C;
    a.Cp = c->Cp;
    a.dp = c->dp;
    a.mp = c->mp;
    a.c0 = g.c0;
    a.problem = 0;
    a.b = c->b;
    a.bstride = c->bstride;
    a.P = c->P;
    a.Q = c->Q;
    a.X = c->X;
    a.Xprop = c->Xprop;
    a.N = c->N;
    a.sel = c->sel;
    a.flag = c->flag;
    a.rej = c->rej;
    a.eps = c->eps;
    a.seed = c->seed;
    a.fb_list = c->fb_list + g.c0;
    a.fb_count = c->fb_count + 2 * gi;
    a.step_base = c->d_step;
    a.force_full = (c->flags & ESS_SORT_FULL) ? 1 : 0;
    a.ab = c->AB;
    a.keys = c->keys;
    a.kstride = c->kstride;
    return a;
}

// Dynamic LDS of Algorithm 2's kernel: two lists of m + 2 pieces.
size_t alg2_lds_bytes(int m) { return 2 * sizeof(double2) * static_cast<size_t>(m + 2); }

// The per-chain kernel of one step over the group's chains (beyond 4096 rows:
// the root pre-pass, the chunked bucket path and the full sort of the chains
// it hands over).
template <typename T>
void launch_sample_t(const ess_ctx* c, const Group& g, hipStream_t st, const SampleArgs& a) {
    const dim3 grid(g.n), b(256), b2(512);
    const int rpt = (c->m + 255) / 256;
    if (c->flags & ESS_LIKELIHOOD_MIDPOINT) {
        hipLaunchKernelGGL((sample_midpoint_kernel<T>), grid, b, 0, st, a);
        return;
    }
    if (c->flags & ESS_BRUTE_FORCE) {
        hipLaunchKernelGGL((sample_alg2_kernel<T>), grid, dim3(64), alg2_lds_bytes(c->m), st, a);
        return;
    }
    if (c->m > 4096) {
        // the roots over the whole device first
        const long long blocks = static_cast<long long>((c->m + 255) / 256) * g.n;
        hipLaunchKernelGGL((large_roots_kernel<T>), dim3(static_cast<unsigned>(blocks)), b, 0, st, a);
        if (g.n <= 256 && c->m <= 16384) {
            // few chains: every row's alpha and beta in registers, 16 or 32
            // per thread, for all passes (the chunked passes reload a.ab and
            // wait on it once per chunk), the full sort in place from a.ab
            if (c->m <= 8192)
                hipLaunchKernelGGL((sample_bucket_kernel<T, 16, 2048, 512, true, true>), grid, b2, 0, st, a);
            else
                hipLaunchKernelGGL((sample_bucket_kernel<T, 32, 2048, 512, true, true>), grid, b2, 0, st, a);
            return;
        }
        // then rows in chunks of 4096 per pass; the full sort keeps keys only
        const dim3 fg(a.force_full ? std::min(g.n, 768) : std::min(g.n, 32));
        hipLaunchKernelGGL((sample_large_kernel<T>), grid, b2, 0, st, a);
        if (c->m > kMaxRowsLds)
            hipLaunchKernelGGL((fallback_large_kernel<T, true>), fg, b, 0, st, a);
        else
            hipLaunchKernelGGL((fallback_large_kernel<T>), fg, b, 0, st, a);
        return;
    }
    // more than 1024 rows: 512 threads per chain (measured 12 % faster at
    // m = 2000: the latency-bound phases have half the rows per thread)
    // With no more chains than compute units, occupancy does not matter and
    // the kernel carries the bucket refinement itself, so a chain with crowded
    // buckets is resolved in place instead of by the full sort.
    // Few chains also take 512 threads at every m: the phases are latency-bound
    // and halving the rows per thread shortens them (one chain at m = 1000:
    // 22 -> 16 us).
    // Every variant sorts a chain it cannot resolve in place, so one launch
    // per step does all of the per-chain work.
    if (g.n <= 256) {
        if (rpt <= 2) hipLaunchKernelGGL((sample_bucket_kernel<T, 1, 2048, 512, true>), grid, b2, 0, st, a);
        else if (rpt <= 4) hipLaunchKernelGGL((sample_bucket_kernel<T, 2, 2048, 512, true>), grid, b2, 0, st, a);
        else if (rpt <= 8) hipLaunchKernelGGL((sample_bucket_kernel<T, 4, 2048, 512, true>), grid, b2, 0, st, a);
        else if (c->m > 2048) {
            // above 2048 rows the roots go over the whole device first (one
            // chain at m = 4000: 11 us of solves inside one workgroup)
            const long long blocks = static_cast<long long>((c->m + 255) / 256) * g.n;
            hipLaunchKernelGGL((large_roots_kernel<T>), dim3(static_cast<unsigned>(blocks)), b, 0, st, a);
            hipLaunchKernelGGL((sample_bucket_kernel<T, 8, 2048, 512, true, true>), grid, b2, 0, st, a);
        } else {
            hipLaunchKernelGGL((sample_bucket_kernel<T, 8, 2048, 512, true>), grid, b2, 0, st, a);
        }
    } else if (rpt <= 1) {
        hipLaunchKernelGGL((sample_bucket_kernel<T, 1, 256>), grid, b, 0, st, a);
    } else if (rpt <= 2) {
        hipLaunchKernelGGL((sample_bucket_kernel<T, 2, 2048>), grid, b, 0, st, a);
    } else if (rpt <= 4) {
        hipLaunchKernelGGL((sample_bucket_kernel<T, 4, 2048>), grid, b, 0, st, a);
    } else if (rpt <= 8) {
        if (std::getenv("ESS_ROOTS_PREPASS")) {
            const long long blocks = static_cast<long long>((c->m + 255) / 256) * g.n;
            hipLaunchKernelGGL((large_roots_kernel<T>), dim3(static_cast<unsigned>(blocks)), b, 0, st, a);
            hipLaunchKernelGGL((sample_bucket_kernel<T, 4, 2048, 512, false, true>), grid, b2, 0, st, a);
        } else
            hipLaunchKernelGGL((sample_bucket_kernel<T, 4, 2048, 512>), grid, b2, 0, st, a);
    } else {
        hipLaunchKernelGGL((sample_bucket_kernel<T, 8, 2048, 512>), grid, b2, 0, st, a);
    }
}

ess_status launch_sample(const ess_ctx* c, const Group& g, hipStream_t st, const SampleArgs& a) {
    if (c->prec == 32) launch_sample_t<float>(c, g, st, a);
    else launch_sample_t<double>(c, g, st, a);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status clear_fallback_lists(const ess_ctx* c, hipStream_t st, int gi) {
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, st, c->fb_count + 2 * gi, 2);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status launch_commit(const ess_ctx* c, const Group& g, hipStream_t st, const SampleArgs& a) {
    if (c->prec == 32) hipLaunchKernelGGL((commit_kernel<float>), dim3(g.n), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((commit_kernel<double>), dim3(g.n), dim3(256), 0, st, a);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

// nu of `step` for chains [c0, c0 + n) into dst rows (leading dimension ld),
// and/or their theta uniforms.
// step is relative to *step_base when step_base is given, else absolute.
ess_status launch_draw(const ess_ctx* c, int c0, int n, hipStream_t st, uint64_t step,
                       const uint32_t* step_base, void* dst, long long ld, double* u) {
    if (c->prec == 32)
        hipLaunchKernelGGL((draw_kernel<float>), dim3(n), dim3(256), 0, st, c->seed,
                           static_cast<uint32_t>(step), step_base, 0u, c->d,
                           static_cast<float*>(dst), ld, u, c0);
    else
        hipLaunchKernelGGL((draw_kernel<double>), dim3(n), dim3(256), 0, st, c->seed,
                           static_cast<uint32_t>(step), step_base, 0u, c->d,
                           static_cast<double*>(dst), ld, u, c0);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

// caller rows (C x d, dense) -> library rows (Cp x dp, padded), or back.
ess_status copy_rows_in(const ess_ctx* c, void* dst, const void* src) {
    HIP_TRY(hipMemcpy2DAsync(dst, static_cast<size_t>(c->dp) * c->esz, src,
                             static_cast<size_t>(c->d) * c->esz, static_cast<size_t>(c->d) * c->esz,
                             c->C, hipMemcpyDefault, c->st));
    return ESS_OK;
}

ess_status copy_rows_out(const ess_ctx* c, void* dst, const void* src) {
    HIP_TRY(hipMemcpy2DAsync(dst, static_cast<size_t>(c->d) * c->esz, src,
                             static_cast<size_t>(c->dp) * c->esz, static_cast<size_t>(c->d) * c->esz,
                             c->C, hipMemcpyDefault, c->st));
    return ESS_OK;
}

// Strict feasibility check (a_i^T x < b_i) of the rows in c->X (staged = 0:
// their projections go to the committed buffers, for ess_init) or of rows
// staged in c->Xprop (staged = 1: projections into the proposal buffers; on
// success every chain adopts its staged row as an accepted proposal, so a
// failed call leaves the state as it was).
ess_status check_rows(ess_ctx* c, const char* what, int staged) {
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * c->Cp, c->st));
    ESS_TRY(launch_proj(c, c->whole(), c->st, staged ? c->Xprop : c->X, COLS_X, !staged, 1));
    std::vector<int> fl(c->C);
    HIP_TRY(hipMemcpyAsync(fl.data(), c->flag, sizeof(int) * c->C, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    for (int ch = 0; ch < c->C; ++ch) {
        if (!fl[ch]) continue;
        int sel = 0;
        HIP_TRY(hipMemcpy(&sel, c->sel + ch, sizeof(int), hipMemcpyDeviceToHost));
        if (staged) sel ^= 1;
        std::vector<double> bh(c->m), ph(c->m);
        HIP_TRY(hipMemcpy(bh.data(), c->b + static_cast<size_t>(ch) * c->bstride,
                          sizeof(double) * c->m, hipMemcpyDeviceToHost));
        const size_t off = (static_cast<size_t>(sel) * c->Cp + ch) * c->mp;
        if (c->prec == 32) {
            std::vector<float> pf(c->m);
            HIP_TRY(hipMemcpy(pf.data(), static_cast<float*>(c->P) + off, sizeof(float) * c->m,
                              hipMemcpyDeviceToHost));
            for (int i = 0; i < c->m; ++i) ph[i] = pf[i];
        } else {
            HIP_TRY(hipMemcpy(ph.data(), static_cast<double*>(c->P) + off, sizeof(double) * c->m,
                              hipMemcpyDeviceToHost));
        }
        int row = -1;
        for (int i = 0; i < c->m && row < 0; ++i)
            if (ph[i] >= bh[i]) row = i;
        HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * c->Cp, c->st));
        return fail(ESS_ERR_INFEASIBLE_START,
                    "%s: chain %d is not strictly feasible: row %d has a^T x = %.9g >= b = %.9g",
                    what, ch, row, row >= 0 ? ph[row] : 0.0, row >= 0 ? bh[row] : 0.0);
    }
    if (staged) ESS_TRY(launch_commit(c, c->whole(), c->st, sample_args(c, c->whole(), 0)));
    return ESS_OK;
}

// nu of the current step (the device counter) into N and A nu into Q, which
// every run expects to find there.
ess_status prime_direction(ess_ctx* c) {
    ESS_TRY(launch_draw(c, 0, c->C, c->st, 0, c->d_step, c->N, c->dp, nullptr));
    return launch_proj(c, c->whole(), c->st, c->Xprop, COLS_NU, 0, 0);
}

ess_status check_ctx(const ess_ctx* c) {
    if (!c) return fail(ESS_ERR_INVALID_ARG, "null context");
    return ESS_OK;
}

ess_status sum_rejections(const ess_ctx* c, long long& total) {
    const int n = c->batch ? c->batch->chains_padded : c->C;
    std::vector<long long> r(n);
    HIP_TRY(hipMemcpyAsync(r.data(), c->rej, sizeof(long long) * n, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    total = 0;
    for (long long v : r) total += v;
    return ESS_OK;
}

ess_status launch_step_counter(const ess_ctx* c, hipStream_t st, uint64_t value, int add) {
    hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(64), 0, st, c->d_step,
                       static_cast<uint32_t>(value), add);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

// Issues n_steps transitions of every group on stream `base` (groups run on
// their own streams between a fork and a join event) and advances the device
// step counter.  Steps are relative to that counter, so the same launches can
// be captured once and replayed.
ess_status issue_run(ess_ctx* c, int64_t n_steps, int64_t thin, void* trace, hipStream_t base) {
    const size_t trace_row = static_cast<size_t>(c->C) * c->d * c->esz;
    const bool split = c->G > 1;
    hipStream_t sts[kMaxGroups];
    Group gr[kMaxGroups];
    for (int g = 0; g < c->G; ++g) {
        sts[g] = split ? c->gs[g] : base;
        gr[g] = split ? c->group(g) : c->whole();
    }
    if (split) {
        HIP_TRY(hipEventRecord(c->fork, base));
        for (int g = 0; g < c->G; ++g) HIP_TRY(hipStreamWaitEvent(sts[g], c->fork, 0));
    }
    // N and Q already hold nu of the current step and A nu (prime_direction
    // after every change of state or counter, and each run's last step draws
    // and projects the next run's first direction), so every step of the run
    // is the same pair of launches
    SampleArgs a[kMaxGroups];
    for (int g = 0; g < c->G; ++g) {
        if (gr[g].n == 0) continue;
        if (c->m > 4096) ESS_TRY(clear_fallback_lists(c, sts[g], g));
        a[g] = sample_args(c, gr[g], g);
    }
    for (int64_t s = 0; s < n_steps; ++s) {
        for (int g = 0; g < c->G; ++g) {
            if (gr[g].n == 0) continue;
            a[g].step = static_cast<uint32_t>(s);
            a[g].has_pending = s > 0;
            a[g].gen_next = 1;
            a[g].trace = (trace && s > 0 && s % thin == 0)
                             ? static_cast<char*>(trace) + (s / thin - 1) * trace_row
                             : nullptr;
            // staggered groups: group g's per-chain kernel of step s starts after
            // group g-1's, so it runs beside group g-1's projections (vector work
            // beside matrix-core work) instead of beside its per-chain kernel
            if (split && g > 0) HIP_TRY(hipStreamWaitEvent(sts[g], c->stagger[g - 1], 0));
            ESS_TRY(timed(c, ESS_KERNEL_SAMPLE, sts[g],
                          [&] { return launch_sample(c, gr[g], sts[g], a[g]); }));
            if (split && g + 1 < c->G) HIP_TRY(hipEventRecord(c->stagger[g], sts[g]));
            ESS_TRY(timed(c, ESS_KERNEL_PROJECT, sts[g], [&] {
                return launch_proj(c, gr[g], sts[g], c->Xprop, COLS_BOTH, 0, 0);
            }));
        }
    }
    for (int g = 0; g < c->G; ++g) {
        if (gr[g].n == 0) continue;
        SampleArgs f = sample_args(c, gr[g], g);
        f.trace = (trace && n_steps % thin == 0)
                      ? static_cast<char*>(trace) + (n_steps / thin - 1) * trace_row
                      : nullptr;
        ESS_TRY(timed(c, ESS_KERNEL_OTHER, sts[g], [&] { return launch_commit(c, gr[g], sts[g], f); }));
    }
    if (split) {
        for (int g = 0; g < c->G; ++g) {
            HIP_TRY(hipEventRecord(c->join[g], sts[g]));
            HIP_TRY(hipStreamWaitEvent(base, c->join[g], 0));
        }
    }
    return launch_step_counter(c, base, static_cast<uint64_t>(n_steps), 1);
}

// ---------------------------------------------------------------- batched
BatchArgs batch_args(const ess_ctx* c) {
    const ess_ctx::Batch& B = *c->batch;
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_probs = B.n;
    a.NT = B.NT;
    a.NC = B.NC;
    a.descs = B.descs;
    a.wg_prob = B.wg_prob;
    a.tiles = B.tiles;
    a.NTL = B.NTL;
    a.chains = B.chains;
    a.A = B.A;
    a.A3 = B.A3;
    a.a_elems = B.a_elems;
    a.b = B.b;
    a.X = B.X;
    a.Xprop = B.Xprop;
    a.N = B.N;
    a.P = B.P;
    a.Q = B.Q;
    a.sel = c->sel;
    a.flag = c->flag;
    a.rej = c->rej;
    a.fb_count = B.counters;
    a.error = B.counters + 2;
    a.tickets = B.counters + 3;
    a.done = B.counters + 3 + 2 * B.n;
    a.fb_list = B.fb_list;
    a.ab = B.ab;
    a.step_base = c->d_step;
    return a;
}

template <int RPT_MAX>
ess_status launch_step_t(ess_ctx* c, const BatchArgs& a, hipStream_t st) {
    const ess_ctx::Batch& B = *c->batch;
    if (B.fused)
        return timed(c, ESS_KERNEL_BATCHED, st, [&] {
            hipLaunchKernelGGL((batched_step_kernel<RPT_MAX>), dim3(a.NT + a.NC), dim3(256), 0, st, a);
            HIP_TRY(hipGetLastError());
            return ESS_OK;
        });
    ESS_TRY(timed(c, ESS_KERNEL_PROJECT, st, [&] {
        hipLaunchKernelGGL(batched_proj_kernel, dim3(a.NTL), dim3(256), 0, st, a);
        HIP_TRY(hipGetLastError());
        return ESS_OK;
    }));
    return timed(c, ESS_KERNEL_SAMPLE, st, [&] {
        hipLaunchKernelGGL((batched_chain_kernel<RPT_MAX>), dim3(a.NC), dim3(256), 0, st, a);
        HIP_TRY(hipGetLastError());
        return ESS_OK;
    });
}

// The kernels carry the chain classes up to the largest problem's.
ess_status launch_batched_step(ess_ctx* c, const BatchArgs& a, hipStream_t st) {
    const ess_ctx::Batch& B = *c->batch;
    if (B.rpt <= 1) return launch_step_t<1>(c, a, st);
    if (B.rpt <= 2) return launch_step_t<2>(c, a, st);
    if (B.rpt <= 4) return launch_step_t<4>(c, a, st);
    if (B.rpt <= 8) return launch_step_t<8>(c, a, st);
    return launch_step_t<16>(c, a, st);
}

// A x for the rows in `rows` (X unless given; p_direct) with the strict start
// check, then the flags.
ess_status batched_set_state_from_X(ess_ctx* c, const char* what, float* rows = nullptr) {
    ess_ctx::Batch& B = *c->batch;
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * B.chains_padded, c->st));
    BatchArgs a = batch_args(c);
    a.Xprop = rows ? rows : B.X;    // tiles read the rows to be committed
    a.cols = 0;
    a.p_direct = 1;
    a.strict = 1;
    hipLaunchKernelGGL(batched_proj_kernel, dim3(B.NTL), dim3(256), 0, c->st, a);
    HIP_TRY(hipGetLastError());
    std::vector<int> fl(B.chains_padded);
    HIP_TRY(hipMemcpyAsync(fl.data(), c->flag, sizeof(int) * B.chains_padded, hipMemcpyDeviceToHost,
                           c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    for (int p = 0; p < B.n; ++p)
        for (int ch = 0; ch < B.h[p].C; ++ch)
            if (fl[B.h[p].chain_off + ch]) {
                HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * B.chains_padded, c->st));
                return fail(ESS_ERR_INFEASIBLE_START,
                            "%s: problem %d chain %d is not strictly feasible", what, p, ch);
            }
    return ESS_OK;
}

ess_status batched_issue(ess_ctx* c, int64_t n_steps, int64_t thin, void* trace, hipStream_t st) {
    ess_ctx::Batch& B = *c->batch;
    const int ncnt = 3 + 4 * B.n;
    hipLaunchKernelGGL(zero_ints_n, dim3(std::min((ncnt + 255) / 256, 64)), dim3(256), 0, st,
                       B.counters, ncnt);
    HIP_TRY(hipGetLastError());
    BatchArgs a = batch_args(c);
    a.step = 0;
    ESS_TRY(timed(c, ESS_KERNEL_OTHER, st, [&] {
        hipLaunchKernelGGL(batched_draw_kernel, dim3(B.NC), dim3(256), 0, st, a);
        HIP_TRY(hipGetLastError());
        return ESS_OK;
    }));
    const size_t row = static_cast<size_t>(B.state_elems);
    // the split form with several problem sets: each set's steps on a stream
    // of its own, forked from st after the draw and joined before the counter
    const bool sets = !B.fused && B.nsets > 1;
    if (sets) {
        HIP_TRY(hipEventRecord(c->fork, st));
        for (int k = 0; k < B.nsets; ++k) HIP_TRY(hipStreamWaitEvent(c->gs[k], c->fork, 0));
    }
    for (int64_t s = 0; s <= n_steps; ++s) {
        a.step = static_cast<uint32_t>(s);
        a.has_pending = s > 0;
        a.do_sample = s < n_steps;
        a.gen_next = s + 1 < n_steps;
        a.cols = (s == 0) ? 1 : (s == n_steps ? 0 : 2);
        a.p_direct = 0;
        a.strict = 0;
        a.trace = (trace && s > 0 && s % thin == 0)
                      ? static_cast<float*>(trace) + (s / thin - 1) * row
                      : nullptr;
        if (!sets) {
            ESS_TRY(launch_batched_step(c, a, st));
            continue;
        }
        for (int k = 0; k < B.nsets; ++k) {
            BatchArgs ak = a;
            ak.tiles = B.tiles + B.set_toff[k];
            ak.NTL = B.set_ntl[k];
            ak.chains = B.chains + B.set_coff[k];
            ak.NC = B.set_nc[k];
            ESS_TRY(launch_batched_step(c, ak, c->gs[k]));
        }
    }
    if (sets) {
        for (int k = 0; k < B.nsets; ++k) {
            HIP_TRY(hipEventRecord(c->join[k], c->gs[k]));
            HIP_TRY(hipStreamWaitEvent(st, c->join[k], 0));
        }
    }
    return launch_step_counter(c, st, static_cast<uint64_t>(n_steps), 1);
}

ess_status batched_check_error(ess_ctx* c) {
    ess_ctx::Batch& B = *c->batch;
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, B.counters + 2, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    if (err) return fail(ESS_ERR_HIP, "batched step: a chain waited past its spin limit");
    return ESS_OK;
}

int tile_bucket(const ProbDesc& d) {
    const int db = d.d <= 64 ? 0 : (d.d <= 192 ? 1 : 2);
    return 2 * db + (d.m > 256 ? 1 : 0);
}

// Tile counts, the workgroup -> problem table of the fused launch (all tile
// runs, then all chain runs, problems by decreasing work) and the tile table
// of the split launch and the state check, from the current shape of every
// size class.  Workgroups go to the 8 XCDs round-robin by index, so table
// entry 8 k + x runs on XCD x: each row panel of a problem (the tiles that
// share its rows of A) is given whole to the XCD with the fewest tiles so
// far, and the eight lists are padded to one length and interleaved.
// Problem sets, each advanced on a stream of its own: a set's chains wait
// only for its own tiles, so one set's chain kernel runs beside another set's
// tiles instead of after every tile of the batch.  Problems go, largest
// first, to the set with the least work so far (rows x chains x (columns +
// 128), projections plus per-row chain work); within a set, chains of the
// larger classes come first, so the longest chain items start early.  The
// chains do not depend on the set count (only the launches' order does).
// Rebuilds the chain list (and leaves the tile table to batched_layout).
ess_status batched_sets(ess_ctx* c, int nsets) {
    ess_ctx::Batch& B = *c->batch;
    const int n = B.n;
    B.nsets = std::max(1, std::min(std::min(nsets, kMaxGroups), n));
    B.set_of.assign(n, 0);
    double load[kMaxGroups] = {};
    for (int p : B.order) {
        int k = 0;
        for (int j = 1; j < B.nsets; ++j)
            if (load[j] < load[k]) k = j;
        B.set_of[p] = k;
        load[k] += static_cast<double>(B.h[p].m) * B.h[p].C * (B.h[p].d + 128);
    }
    std::vector<int2> chains;
    for (int k = 0; k < B.nsets; ++k) {
        B.set_coff[k] = static_cast<int>(chains.size());
        for (int cls = 4; cls >= 0; --cls)
            for (int p = 0; p < n; ++p)
                if (B.set_of[p] == k && B.h[p].cls == cls)
                    for (int ch = 0; ch < B.h[p].C; ++ch) chains.push_back(make_int2(p, ch));
        B.set_nc[k] = static_cast<int>(chains.size()) - B.set_coff[k];
    }
    if (static_cast<int>(chains.size()) != B.NC) return fail(ESS_ERR_INVALID_ARG, "batched sets: chain count");
    HIP_TRY(hipMemcpyAsync(B.chains, chains.data(), sizeof(int2) * B.NC, hipMemcpyHostToDevice, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));   // the host list goes away at return
    return ESS_OK;
}

ess_status batched_layout(ess_ctx* c) {
    constexpr int kXcds = 8;
    ess_ctx::Batch& B = *c->batch;
    for (auto& d : B.h) {
        // the split tiles for d > 192, whatever the class shapes (as in a
        // single-problem context, so a problem's chains are the same alone)
        d.shape = d.d > 192 ? kBatchSplitShape : B.bucket_shape[tile_bucket(d)];
        d.tiles_n = 2 * d.Cp / shape_bn(d.shape);
        d.ntiles = ((d.m + shape_bm(d.shape) - 1) / shape_bm(d.shape)) * d.tiles_n;
    }
    std::vector<int> wg;
    std::vector<int4> table;
    B.NT = 0;
    for (const int p : B.order) {
        wg.insert(wg.end(), B.h[p].ntiles, p);
        B.NT += B.h[p].ntiles;
    }
    for (int p : B.order) wg.insert(wg.end(), B.h[p].C, p);
    // one XCD-interleaved segment of the tile table per problem set
    for (int k = 0; k < B.nsets; ++k) {
        std::vector<int4> lists[kXcds];
        for (int p : B.order) {
            if (B.set_of[p] != k) continue;
            const ProbDesc& d = B.h[p];
            for (int tm = 0; tm < d.ntiles / d.tiles_n; ++tm) {
                int x = 0;
                for (int y = 1; y < kXcds; ++y)
                    if (lists[y].size() < lists[x].size()) x = y;
                for (int tn = 0; tn < d.tiles_n; ++tn) lists[x].push_back(make_int4(p, tm, tn, 0));
            }
        }
        size_t len = 0;
        for (auto& l : lists) len = std::max(len, l.size());
        B.set_toff[k] = static_cast<int>(table.size());
        B.set_ntl[k] = static_cast<int>(kXcds * len);
        table.resize(table.size() + kXcds * len, make_int4(-1, 0, 0, 0));
        for (int x = 0; x < kXcds; ++x)
            for (size_t j = 0; j < lists[x].size(); ++j) table[B.set_toff[k] + kXcds * j + x] = lists[x][j];
    }
    if (B.NT > B.max_tiles || static_cast<long long>(table.size()) > B.max_table)
        return fail(ESS_ERR_INVALID_ARG, "batched layout: tile table overflow");
    B.NTL = static_cast<int>(table.size());
    HIP_TRY(hipMemcpyAsync(B.descs, B.h.data(), sizeof(ProbDesc) * B.n, hipMemcpyHostToDevice, c->st));
    HIP_TRY(hipMemcpyAsync(B.wg_prob, wg.data(), sizeof(int) * wg.size(), hipMemcpyHostToDevice, c->st));
    HIP_TRY(hipMemcpyAsync(B.tiles, table.data(), sizeof(int4) * table.size(), hipMemcpyHostToDevice,
                           c->st));
    // the host vectors go away at return: wait for the copies
    HIP_TRY(hipStreamSynchronize(c->st));
    return ESS_OK;
}

ess_status batched_init(ess_ctx* c, const ess_problem* pr, int n) {
    c->batch.reset(new ess_ctx::Batch());
    ess_ctx::Batch& B = *c->batch;
    B.n = n;
    B.h.resize(n);
    long long a_off = 0, b_off = 0, x_off = 0, p_off = 0, q_off = 0, t_off = 0;
    int chain_off = 0, max_m = 1;
    long long max_tiles = 0;
    int max_panel = 0;
    for (int p = 0; p < n; ++p) {
        ProbDesc& d = B.h[p];
        d.d = pr[p].d;
        d.m = pr[p].m;
        d.C = pr[p].n_chains;
        d.dp = round_up(d.d, 32);
        d.mp = round_up(d.m, kBatchPadM);
        d.Cp = round_up(d.C, kBatchPadC);
        d.chain_off = chain_off;
        d.cls = 0;
        while ((256 << d.cls) < d.m) ++d.cls;
        d.a_off = a_off;
        d.b_off = b_off;
        d.x_off = x_off;
        d.p_off = p_off;
        d.q_off = q_off;
        d.t_off = t_off;
        d.eps = pr[p].trim_eps;
        d.seed = pr[p].seed;
        a_off += static_cast<long long>(d.mp) * d.dp;
        b_off += d.m;
        x_off += static_cast<long long>(d.Cp) * d.dp;
        p_off += 2ll * d.Cp * d.mp;
        q_off += static_cast<long long>(d.Cp) * d.mp;
        t_off += static_cast<long long>(d.C) * d.d;
        chain_off += d.Cp;
        max_m = std::max(max_m, d.m);
        max_tiles += static_cast<long long>(d.mp / 32) * (2 * d.Cp / 32);
        max_panel = std::max(max_panel, 2 * d.Cp / 32);
        if (max_tiles + chain_off > (1ll << 31) - 1)
            return fail(ESS_ERR_UNSUPPORTED, "ess_init_batched: more than 2^31 - 1 work items");
    }
    B.state_elems = t_off;
    B.chains_padded = chain_off;
    B.max_tiles = static_cast<int>(max_tiles);
    // greedy by count: list lengths differ by at most one panel (per set)
    B.max_table = static_cast<int>(max_tiles + 8ll * kMaxGroups * (max_panel + 1));
    B.rpt = (max_m + 255) / 256;
    // problems with the most projection work first, so their tiles start early
    B.order.resize(n);
    std::iota(B.order.begin(), B.order.end(), 0);
    std::stable_sort(B.order.begin(), B.order.end(), [&](int x, int y) {
        return static_cast<long long>(B.h[x].mp) * B.h[x].dp * B.h[x].Cp >
               static_cast<long long>(B.h[y].mp) * B.h[y].dp * B.h[y].Cp;
    });
    int nchains = 0;
    for (int p = 0; p < n; ++p) nchains += B.h[p].C;
    B.NC = nchains;

    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.descs), sizeof(ProbDesc) * n));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.wg_prob), sizeof(int) * (max_tiles + B.NC)));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.tiles), sizeof(int4) * B.max_table));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.chains), sizeof(int2) * B.NC));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.A), sizeof(float) * a_off));
    B.a_elems = static_cast<size_t>(a_off);
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.A3), 3 * sizeof(uint16_t) * B.a_elems));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.b), sizeof(double) * b_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.X), sizeof(float) * x_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.Xprop), sizeof(float) * x_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.N), sizeof(float) * x_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.P), sizeof(float) * p_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.Q), sizeof(float) * q_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.counters), sizeof(int) * (3 + 4 * n)));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.fb_list), sizeof(int2) * B.NC));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&B.ab), sizeof(double2) * q_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&c->sel), sizeof(int) * chain_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&c->flag), sizeof(int) * chain_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&c->rej), sizeof(long long) * chain_off));
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&c->d_step), sizeof(uint32_t)));
    ESS_TRY(create_run_streams(c));
    ESS_TRY(create_group_streams(c));
    {
        int ns = 2;
        if (const char* e = std::getenv("ESS_BATCH_SETS")) ns = std::atoi(e);
        ESS_TRY(batched_sets(c, ns));
    }
    for (int p = 0; p < n; ++p) {
        const ProbDesc& d = B.h[p];
        HIP_TRY(hipMemcpy2DAsync(B.A + d.a_off, sizeof(float) * d.dp, pr[p].A, sizeof(float) * d.d,
                                 sizeof(float) * d.d, d.m, hipMemcpyDefault, c->st));
        HIP_TRY(hipMemcpyAsync(B.b + d.b_off, pr[p].b, sizeof(double) * d.m, hipMemcpyDefault, c->st));
        if (pr[p].flags & ESS_X0_BROADCAST) {
            hipLaunchKernelGGL((broadcast_rows<float>), dim3(d.C), dim3(256), 0, c->st,
                               static_cast<const float*>(pr[p].x0), B.X + d.x_off, d.d, d.dp);
            HIP_TRY(hipGetLastError());
        } else {
            HIP_TRY(hipMemcpy2DAsync(B.X + d.x_off, sizeof(float) * d.dp, pr[p].x0,
                                     sizeof(float) * d.d, sizeof(float) * d.d, d.C,
                                     hipMemcpyDefault, c->st));
        }
    }
    {   // A's bfloat16 pieces for the split tiles (padding stays zero)
        const size_t n_el = B.a_elems;
        const unsigned grid = static_cast<unsigned>(std::min<size_t>((n_el / 2 + 255) / 256, 4096));
        hipLaunchKernelGGL(split_rows_kernel, dim3(grid), dim3(256), 0, c->st, B.A, n_el, B.A3,
                           B.A3 + n_el, B.A3 + 2 * n_el);
        HIP_TRY(hipGetLastError());
    }
    ESS_TRY(batched_layout(c));   // synchronises: the host chain table is copied
    return batched_set_state_from_X(c, "ess_init_batched");
}

ess_status batched_copy_state(const ess_ctx* c, const float* src, float* dst, int to_library) {
    BatchArgs a = batch_args(c);
    hipLaunchKernelGGL(batched_copy_rows, dim3(c->batch->NC), dim3(256), 0, c->st, a, src, dst,
                       to_library);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

// ---------------------------------------------------------------- runs
// Kernel by kernel on the caller's stream (while profiling, or with
// ESS_EAGER), otherwise by replaying a graph captured once per run shape on
// the library's capture stream, ordered after the caller's stream by events.
ess_status run_dispatch(ess_ctx* c, int64_t n_steps, int64_t thin, void* trace) {
    auto issue = [&](hipStream_t st) {
        return c->batch ? batched_issue(c, n_steps, thin, trace, st)
                        : issue_run(c, n_steps, thin, trace, st);
    };
    if (!c->use_graphs || c->profiling) {
        ESS_TRY(issue(c->st));
    } else {
        hipGraphExec_t exec = nullptr;
        for (auto& g : c->graphs)
            if (g.n_steps == n_steps && g.thin == thin && g.trace == trace) exec = g.exec;
        if (!exec) {
            HIP_TRY(hipStreamBeginCapture(c->cs, hipStreamCaptureModeRelaxed));
            const ess_status s = issue(c->cs);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cs, &graph);
            if (s != ESS_OK) {
                if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
                return s;
            }
            HIP_TRY(e);
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_TRY(ei);
            if (c->graphs.size() >= 8) {
                // the oldest graph may still be queued or running on the
                // capture stream: wait for it before destroying it
                HIP_TRY(hipStreamSynchronize(c->cs));
                (void)hipGraphExecDestroy(c->graphs.front().exec);
                c->graphs.erase(c->graphs.begin());
            }
            c->graphs.push_back({n_steps, thin, trace, exec});
        }
        HIP_TRY(hipEventRecord(c->ev_in, c->st));
        HIP_TRY(hipStreamWaitEvent(c->cs, c->ev_in, 0));
        HIP_TRY(hipGraphLaunch(exec, c->cs));
        HIP_TRY(hipEventRecord(c->ev_out, c->cs));
        HIP_TRY(hipStreamWaitEvent(c->st, c->ev_out, 0));
    }
    if (c->batch) ESS_TRY(batched_check_error(c));
    return ESS_OK;
}

ess_status drop_graphs(ess_ctx* c) {
    if (!c->graphs.empty()) HIP_TRY(hipStreamSynchronize(c->cs));
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    return ESS_OK;
}

// A's three bfloat16 pieces for the split projections (allocated once).
ess_status split_A(ess_ctx* c) {
    if (c->A3) return ESS_OK;
    const size_t plane = static_cast<size_t>(c->mp) * c->dp;
    ESS_TRY(dalloc(c, reinterpret_cast<void**>(&c->A3), 3 * plane * sizeof(uint16_t)));
    const unsigned grid = static_cast<unsigned>(std::min<size_t>((plane / 2 + 255) / 256, 4096));
    hipLaunchKernelGGL(split_rows_kernel, dim3(grid), dim3(256), 0, c->st,
                       static_cast<const float*>(c->A), plane, c->A3, c->A3 + plane,
                       c->A3 + 2 * plane);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ESS_ERR_HIP, "splitting A: %s", hipGetErrorString(e));
    return ESS_OK;
}

// ---------------------------------------------------------------- autotuning
// Tile choices per batched workload, cached in a small JSON file:
//   {"<key>": {"shape_code": 1365, "fused": 0, "us_per_step": 162.5}, ...}
std::string tune_cache_path() {
    if (const char* p = std::getenv("ESS_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : ".") + "/.cache/ess_tune.json";
}

std::string tune_key(const ess_ctx* c) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::ostringstream k;
    if (c->batch) {
        long long work = 0;
        for (const auto& d : c->batch->h) work += static_cast<long long>(d.m) * d.d * d.C;
        k << arch << " batched n=" << c->batch->n << " chains=" << c->batch->NC << " work=" << work;
    } else {
        k << arch << " single p=" << c->prec << " d=" << c->d << " m=" << c->m << " C=" << c->C
          << (c->bstride ? " perchainb" : "");
    }
    return k.str();
}

std::string read_file(const std::string& path) {
    std::ifstream f(path);
    std::stringstream ss;
    ss << f.rdbuf();
    return ss.str();
}

// The object stored under `key`, or "".
std::string cache_entry(const std::string& text, const std::string& key) {
    const std::string q = "\"" + key + "\"";
    const size_t at = text.find(q);
    if (at == std::string::npos) return "";
    const size_t open = text.find('{', at + q.size());
    const size_t close = text.find('}', open);
    if (open == std::string::npos || close == std::string::npos) return "";
    return text.substr(open, close - open + 1);
}

double field(const std::string& obj, const char* name, double dflt) {
    const std::string q = std::string("\"") + name + "\"";
    const size_t at = obj.find(q);
    if (at == std::string::npos) return dflt;
    const size_t colon = obj.find(':', at);
    return colon == std::string::npos ? dflt : std::atof(obj.c_str() + colon + 1);
}

// A batched context's tile shape per size class, as one base-4 number
// (class k in digit k).
struct TuneChoice {
    int shape_code = 0;
    int fused = 0;
    int sets = 0;   // problem sets of the split form (0: keep)
    double us = 0;
};

int encode_shapes(const ess_ctx* c) {
    int code = 0;
    for (int k = kTileBuckets - 1; k >= 0; --k) code = code * kBatchShapes + c->batch->bucket_shape[k];
    return code;
}

void set_choice(ess_ctx* c, const TuneChoice& t) {
    c->batch->fused = t.fused != 0;
    int code = t.shape_code;
    for (int k = 0; k < kTileBuckets; ++k) {
        c->batch->bucket_shape[k] = code % kBatchShapes;
        code /= kBatchShapes;
    }
}

ess_status apply_choice(ess_ctx* c, const TuneChoice& t) {
    set_choice(c, t);
    if (t.sets > 0 && t.sets != c->batch->nsets) ESS_TRY(batched_sets(c, t.sets));
    return batched_layout(c);
}

TuneChoice current_choice(const ess_ctx* c) {
    TuneChoice t;
    t.shape_code = encode_shapes(c);
    t.fused = c->batch->fused ? 1 : 0;
    t.sets = c->batch->nsets;
    return t;
}

int max_shape_code() {
    int v = 1;
    for (int k = 0; k < kTileBuckets; ++k) v *= kBatchShapes;
    return v;
}

// The cached choice for this workload, then the overrides ESS_BATCH_TILE
// ("BMxBN" for every size class) and ESS_BATCH_LAUNCH ("split" or "fused").
ess_status load_tuned(ess_ctx* c) {
    if (!c->batch) return ESS_OK;   // single problems: load_tuned_single at init
    const std::string obj = cache_entry(read_file(tune_cache_path()), tune_key(c));
    if (!obj.empty()) {
        TuneChoice t;
        t.shape_code = static_cast<int>(field(obj, "shape_code", -1));
        t.fused = field(obj, "fused", 0) != 0 ? 1 : 0;
        const int sets = static_cast<int>(field(obj, "sets", 0));
        if (t.shape_code >= 0 && t.shape_code < max_shape_code()) set_choice(c, t);
        if (sets >= 1 && sets <= kMaxGroups && !std::getenv("ESS_BATCH_SETS"))
            ESS_TRY(batched_sets(c, sets));
    }
    if (const char* env = std::getenv("ESS_BATCH_TILE")) {
        int bm = 0, bn = 0, shape = -1;
        if (std::sscanf(env, "%dx%d", &bm, &bn) == 2)
            for (int sh = 0; sh < kBatchShapes; ++sh)
                if (shape_bm(sh) == bm && shape_bn(sh) == bn) shape = sh;
        if (shape < 0)
            return fail(ESS_ERR_INVALID_ARG, "ESS_BATCH_TILE must be 64x64, 32x64, 64x32 or 32x32");
        for (int k = 0; k < kTileBuckets; ++k) c->batch->bucket_shape[k] = shape;
    }
    if (const char* env = std::getenv("ESS_BATCH_LAUNCH")) {
        const std::string v(env);
        if (v != "split" && v != "fused")
            return fail(ESS_ERR_INVALID_ARG, "ESS_BATCH_LAUNCH must be split or fused");
        c->batch->fused = v == "fused";
    }
    return batched_layout(c);
}

// Writes `"key": value` into the cache file, replacing the key's old entry.
void store_entry(const std::string& key, const std::string& value) {
    const std::string path = tune_cache_path();
    std::string text = read_file(path);
    const std::string e = "\"" + key + "\": " + value;
    const std::string q = "\"" + key + "\"";
    const size_t at = text.find(q);
    if (at != std::string::npos) {
        const size_t close = text.find('}', at);
        text.replace(at, close - at + 1, e);
    } else {
        const size_t last = text.rfind('}');
        if (text.empty() || last == std::string::npos) text = "{\n" + e + "\n}\n";
        else {
            const bool empty_obj = text.find('"') == std::string::npos;
            text.insert(last, (empty_obj ? "" : ",\n") + e + "\n");
        }
    }
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        // create the directory one level at a time (no shell)
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    std::ofstream f(path);
    f << text;
}

void store_tuned(const ess_ctx* c, const TuneChoice& t) {
    std::ostringstream v;
    v << "{\"shape_code\": " << t.shape_code << ", \"fused\": " << t.fused
      << ", \"sets\": " << t.sets << ", \"us_per_step\": " << t.us << "}";
    store_entry(tune_key(c), v.str());
}

// ---------------------------------------------------------- single problems
// A single-problem context's projection kernel: float32 through the split
// bfloat16 tiles (128 x 128) or float32 matrix-core tiles of 128 or 64 rows
// by 128 or 64 chain columns (float64: its one 64 x 64 tile), and the band
// height of the XCD-aware tile order.  Cached under the context's key as
//   {"split": 1, "bm": 128, "bn": 128, "group_m": 4, "us_per_step": 80.1}.
// Chain groups, their streams and events are never changed here.
struct SingleChoice {
    int split = 0, bm = 64, bn = 64, group_m = 4;
    double us = 0;
};

SingleChoice single_current(const ess_ctx* c) {
    SingleChoice t;
    t.split = c->split_proj ? 1 : 0;
    t.bm = c->bm;
    t.bn = c->bn;
    t.group_m = c->group_m;
    return t;
}

bool single_valid(const ess_ctx* c, const SingleChoice& t) {
    const bool tile = (t.bm == 64 || t.bm == 128) && (t.bn == 64 || t.bn == 128);
    if (t.group_m < 1 || t.group_m > 64 || !tile) return false;
    if (c->prec == 64) return t.split == 0 && t.bm == 64 && t.bn == 64;
    return !t.split || t.bm == t.bn;   // split tiles: 128 x 128 or 64 x 64
}

// The cached choice for this shape, if any; ESS_PROJ_TILE keeps its tile.
void load_tuned_single(ess_ctx* c) {
    const std::string obj = cache_entry(read_file(tune_cache_path()), tune_key(c));
    if (obj.empty()) return;
    SingleChoice t;
    t.split = field(obj, "split", 0) != 0 ? 1 : 0;
    t.bm = static_cast<int>(field(obj, "bm", 0));
    t.bn = static_cast<int>(field(obj, "bn", 0));
    t.group_m = static_cast<int>(field(obj, "group_m", 0));
    if (!single_valid(c, t)) return;
    if (!std::getenv("ESS_PROJ_TILE")) {
        c->bm = t.bm;
        c->bn = t.bn;
        c->split_proj = t.split != 0;
    }
    c->group_m = t.group_m;
}

ess_status single_apply(ess_ctx* c, const SingleChoice& t) {
    c->bm = t.bm;
    c->bn = t.bn;
    c->group_m = t.group_m;
    c->split_proj = t.split != 0;
    if (c->split_proj) ESS_TRY(split_A(c));
    return drop_graphs(c);
}

void store_tuned_single(const ess_ctx* c, const SingleChoice& t) {
    std::ostringstream v;
    v << "{\"split\": " << t.split << ", \"bm\": " << t.bm << ", \"bn\": " << t.bn
      << ", \"group_m\": " << t.group_m << ", \"us_per_step\": " << t.us << "}";
    store_entry(tune_key(c), v.str());
}

// Times the candidates on graph replays of steps_per_trial steps each
// (one pass over the kernel shapes at the current band height, then the
// band heights for the best shape), keeps the fastest, and puts the chains
// back where they were: state, step and rejection counts.
ess_status autotune_single(ess_ctx* c, int32_t steps_per_trial, std::ostringstream& rep,
                           SingleChoice& best) {
    struct Scratch {
        hipStream_t st = nullptr;
        void* saved = nullptr;
        long long* rej = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Scratch() {
            if (saved || rej) (void)hipStreamSynchronize(st);   // no copy still uses them
            if (saved) (void)hipFree(saved);
            if (rej) (void)hipFree(rej);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } scr;
    scr.st = c->st;
    const size_t bytes = static_cast<size_t>(c->C) * c->d * c->esz;
    HIP_TRY(hipMalloc(&scr.saved, bytes));
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&scr.rej), sizeof(long long) * c->Cp));
    ESS_TRY(copy_rows_out(c, scr.saved, c->X));
    HIP_TRY(hipMemcpyAsync(scr.rej, c->rej, sizeof(long long) * c->Cp, hipMemcpyDeviceToDevice,
                           c->st));
    const uint64_t step0 = c->step;
    HIP_TRY(hipEventCreate(&scr.e0));
    HIP_TRY(hipEventCreate(&scr.e1));

    auto trial = [&](SingleChoice& t) -> ess_status {
        ESS_TRY(single_apply(c, t));
        ESS_TRY(run_dispatch(c, steps_per_trial, 1, nullptr));   // capture and warm
        c->step += steps_per_trial;
        HIP_TRY(hipEventRecord(scr.e0, c->st));
        ESS_TRY(run_dispatch(c, steps_per_trial, 1, nullptr));
        c->step += steps_per_trial;
        HIP_TRY(hipEventRecord(scr.e1, c->st));
        HIP_TRY(hipEventSynchronize(scr.e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, scr.e0, scr.e1));
        t.us = 1e3 * ms / steps_per_trial;
        rep << (t.split ? "split" : "f32") << " " << t.bm << "x" << t.bn << ", band "
            << t.group_m << ": " << t.us << " us/step\n";
        return ESS_OK;
    };
    const SingleChoice before = single_current(c);
    std::vector<SingleChoice> shapes;
    if (c->prec == 64) {
        shapes.push_back(before);
    } else {
        const int tiles[4][2] = {{128, 128}, {128, 64}, {64, 128}, {64, 64}};
        for (const int bt : {128, 64}) {
            SingleChoice sp;
            sp.split = 1;
            sp.bm = sp.bn = bt;
            sp.group_m = before.group_m;
            shapes.push_back(sp);
        }
        for (const auto& tb : tiles) {
            SingleChoice t;
            t.bm = tb[0];
            t.bn = tb[1];
            t.group_m = before.group_m;
            shapes.push_back(t);
        }
    }
    ess_status st = ESS_OK;
    best = before;
    best.us = 1e30;
    for (auto& t : shapes) {
        if (st != ESS_OK) break;
        st = trial(t);
        if (st == ESS_OK && t.us < best.us) best = t;
    }
    for (const int gm : {1, 2, 4, 8, 16}) {
        if (st != ESS_OK) break;
        if (gm == best.group_m) continue;
        SingleChoice t = best;
        t.group_m = gm;
        st = trial(t);
        if (st == ESS_OK && t.us < best.us) best = t;
    }
    // the chains go back to where they were, on the chosen kernels
    ess_status fin = single_apply(c, st == ESS_OK ? best : before);
    if (fin == ESS_OK) fin = copy_rows_in(c, c->Xprop, scr.saved);
    if (fin == ESS_OK) fin = check_rows(c, "ess_autotune", 1);
    if (fin == ESS_OK) fin = launch_step_counter(c, c->st, step0, 0);
    if (fin == ESS_OK) fin = prime_direction(c);
    c->step = step0;
    if (fin == ESS_OK) {
        const hipError_t e = hipMemcpyAsync(c->rej, scr.rej, sizeof(long long) * c->Cp,
                                            hipMemcpyDeviceToDevice, c->st);
        if (e != hipSuccess) fin = fail(ESS_ERR_HIP, "restoring rejections: %s", hipGetErrorString(e));
    }
    if (st != ESS_OK) return st;
    return fin;
}

// ---------------------------------------------------------------- network
}  // namespace

struct ess_mlp {
    int L = 0;                      // layers
    std::vector<int> w;             // widths, L + 1
    std::vector<long long> w_off, c_off;   // offsets of W_l and c_l in the flat vector
    long long n_params = 0, n_weights = 0;
    hipStream_t st = nullptr;
    float* params = nullptr;        // flat: W_0, c_0, W_1, c_1, ...
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    uint16_t* wb = nullptr;         // bfloat16 copies of the weights (same offsets minus biases)
    std::vector<long long> wb_off;
    long long adam_t = 0;
    int cap = 0;                    // batch capacity of the activation buffers
    uint16_t* xin = nullptr;        // [cap][w0]
    std::vector<float*> z;          // hidden pre-activations [cap][w_{l+1}]
    std::vector<uint16_t*> h;       // hidden activations, bfloat16
    float* y = nullptr;             // [cap][wL]
    float* dzf = nullptr;           // [cap][max width]
    uint16_t* dzb = nullptr;
    float* dzf2 = nullptr;
    uint16_t* dzb2 = nullptr;
    double* partial = nullptr;      // [256]
    std::vector<void*> allocs;
};

namespace {

ess_status mlp_alloc(ess_mlp* n, void** p, size_t bytes) {
    HIP_TRY(hipMalloc(p, bytes));
    n->allocs.push_back(*p);
    HIP_TRY(hipMemsetAsync(*p, 0, bytes, n->st));
    return ESS_OK;
}

ess_status mlp_reserve(ess_mlp* n, int batch) {
    if (batch <= n->cap) return ESS_OK;
    if (n->cap > 0) HIP_TRY(hipStreamSynchronize(n->st));   // old buffers may still be in use
    auto drop = [&](void* q) {
        if (!q) return;
        (void)hipFree(q);
        n->allocs.erase(std::remove(n->allocs.begin(), n->allocs.end(), q), n->allocs.end());
    };
    drop(n->xin); drop(n->y); drop(n->dzf); drop(n->dzb); drop(n->dzf2); drop(n->dzb2);
    for (auto* q : n->z) drop(q);
    for (auto* q : n->h) drop(q);
    n->z.assign(n->L - 1, nullptr);
    n->h.assign(n->L - 1, nullptr);
    const int wmax = *std::max_element(n->w.begin(), n->w.end());
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->xin), sizeof(uint16_t) * batch * n->w[0]));
    for (int l = 0; l + 1 < n->L; ++l) {
        ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->z[l]), sizeof(float) * batch * n->w[l + 1]));
        ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->h[l]), sizeof(uint16_t) * batch * n->w[l + 1]));
    }
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->y), sizeof(float) * batch * n->w[n->L]));
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->dzf), sizeof(float) * batch * wmax));
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->dzb), sizeof(uint16_t) * batch * wmax));
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->dzf2), sizeof(float) * batch * wmax));
    ESS_TRY(mlp_alloc(n, reinterpret_cast<void**>(&n->dzb2), sizeof(uint16_t) * batch * wmax));
    n->cap = batch;
    return ESS_OK;
}

ess_status mlp_gemm(const ess_mlp* n, const MlpGemm& g) {
    const int tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
    hipLaunchKernelGGL(mlp_gemm_kernel, dim3(tiles), dim3(256), 0, n->st, g);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status mlp_refresh_bf16(const ess_mlp* n) {
    for (int l = 0; l < n->L; ++l) {
        const long long cnt = static_cast<long long>(n->w[l + 1]) * n->w[l];
        hipLaunchKernelGGL(to_bf16_kernel, dim3(std::min<long long>((cnt + 255) / 256, 1024)),
                           dim3(256), 0, n->st, n->params + n->w_off[l], n->wb + n->wb_off[l], cnt);
    }
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status mlp_forward(ess_mlp* n, const float* in, int B) {
    ESS_TRY(mlp_reserve(n, B));
    const long long cnt = static_cast<long long>(B) * n->w[0];
    hipLaunchKernelGGL(to_bf16_kernel, dim3(std::min<long long>((cnt + 255) / 256, 1024)), dim3(256),
                       0, n->st, in, n->xin, cnt);
    HIP_TRY(hipGetLastError());
    const uint16_t* hprev = n->xin;
    for (int l = 0; l < n->L; ++l) {
        const int din = n->w[l], dout = n->w[l + 1];
        MlpGemm g{};
        g.M = B;
        g.N = dout;
        g.K = din;
        g.A = hprev;
        g.sa0 = din;
        g.sa1 = 1;
        g.B = n->wb + n->wb_off[l];   // B(k, j) = W_l[j][k]
        g.sb0 = 1;
        g.sb1 = din;
        g.bias = n->params + n->c_off[l];
        g.ldo = dout;
        if (l + 1 < n->L) {
            g.mode = EPI_HIDDEN;
            g.out_f = n->z[l];
            g.out_b = n->h[l];
            hprev = n->h[l];
        } else {
            g.mode = EPI_OUTPUT;
            g.out_f = n->y;
        }
        ESS_TRY(mlp_gemm(n, g));
    }
    return ESS_OK;
}

ess_status mlp_backward(ess_mlp* n, const float* target, int B, double* loss) {
    const int L = n->L, dout = n->w[L];
    const long long cnt = static_cast<long long>(B) * dout;
    const int nb = static_cast<int>(std::min<long long>((cnt + 255) / 256, 256));
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, n->st, n->y, target, cnt, n->dzf,
                       n->dzb, n->partial);
    HIP_TRY(hipGetLastError());
    float* dzf = n->dzf;
    uint16_t* dzb = n->dzb;
    float* dzf_next = n->dzf2;
    uint16_t* dzb_next = n->dzb2;
    for (int l = L - 1; l >= 0; --l) {
        const int din = n->w[l], dw = n->w[l + 1];
        const uint16_t* hin = l > 0 ? n->h[l - 1] : n->xin;
        MlpGemm g{};   // dW_l[i][j] = sum_b dZ[b][i] H[b][j]
        g.M = dw;
        g.N = din;
        g.K = B;
        g.A = dzb;
        g.sa0 = 1;
        g.sa1 = dw;
        g.B = hin;
        g.sb0 = din;
        g.sb1 = 1;
        g.mode = EPI_STORE;
        g.out_f = n->grads + n->w_off[l];
        g.ldo = din;
        ESS_TRY(mlp_gemm(n, g));
        hipLaunchKernelGGL(colsum_kernel, dim3((dw + 255) / 256), dim3(256), 0, n->st, dzf, B, dw, dw,
                           n->grads + n->c_off[l]);
        HIP_TRY(hipGetLastError());
        if (l > 0) {
            MlpGemm d{};   // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
            d.M = B;
            d.N = din;
            d.K = dw;
            d.A = dzb;
            d.sa0 = dw;
            d.sa1 = 1;
            d.B = n->wb + n->wb_off[l];   // B(k, j) = W_l[k][j]
            d.sb0 = din;
            d.sb1 = 1;
            d.mode = EPI_DGELU;
            d.zin = n->z[l - 1];
            d.out_f = dzf_next;
            d.out_b = dzb_next;
            d.ldo = din;
            ESS_TRY(mlp_gemm(n, d));
            std::swap(dzf, dzf_next);
            std::swap(dzb, dzb_next);
        }
    }
    if (loss) {
        std::vector<double> part(nb);
        HIP_TRY(hipMemcpyAsync(part.data(), n->partial, sizeof(double) * nb, hipMemcpyDeviceToHost, n->st));
        HIP_TRY(hipStreamSynchronize(n->st));
        double s = 0.0;
        for (double v : part) s += v;
        *loss = s / static_cast<double>(cnt);
    }
    return ESS_OK;
}

// Start states for every chain: the candidate row where it is strictly
// feasible, the fallback row elsewhere.
// Float32 projections go through the split bfloat16 tiles at 128 x 128, and
// at 64 x 64 once A has more than 192 columns (K of 224 or more, where the
// matrix work dominates the tile); float32 matrix-core tiles otherwise.
// Batched contexts follow the same rule per problem, so a problem's chains
// are the same in a batch and alone.
bool default_split(const ess_ctx* c) {
    if (c->prec != 32 || c->bm != c->bn) return false;
    return c->bm == 128 || c->d > 192;
}

// Projection tile shape of a single-problem context.
void choose_tiles(ess_ctx* c) {
    if (c->prec == 32) {
        // 128 x 128 tiles when they fill the 256 CUs (one tile each), else
        // 64 x 64: measured fastest at d=1000, m=2000, 1024 chains (256
        // tiles) and at d=256, m=768 with 2048 chains (192 large tiles: 64 x 64
        // took 64.7 us per step against 73.8 to 76.0 for the larger shapes)
        const long long big = static_cast<long long>(c->mp / 128) * (2 * c->Cp / 128);
        c->bm = c->bn = big >= 256 ? 128 : 64;
    } else {
        c->bm = c->bn = 64;
    }
    if (const char* e = std::getenv("ESS_PROJ_TILE")) {   // "BMxBN", e.g. 64x128
        int bm = 0, bn = 0;
        if (std::sscanf(e, "%dx%d", &bm, &bn) == 2 && (bm == 64 || bm == 128) &&
            (bn == 64 || bn == 128) && c->prec == 32) {
            c->bm = bm;
            c->bn = bn;
        }
    }
}

// ---------------------------------------------------------------- no allocation
// ess_transition_explicit_static keeps every buffer a context would own in
// one file-scope array per device.  Host code never passes `scratch` itself
// to a kernel or copy: its address on the current device comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = static_cast<size_t>(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

ess_status scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ESS_ERR_UNSUPPORTED, "device %d: the static buffer serves devices 0 .. %d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ESS_ERR_HIP, "hipGetSymbolAddress gave a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ESS_OK;
}

// rows x cols (dense, row-major) into rows_p x ld, zero everywhere else.
template <typename T>
__global__ __launch_bounds__(256) void pad_copy_kernel(const T* __restrict__ src, int rows, int cols,
                                                       T* __restrict__ dst, int rows_p, int ld) {
    const size_t n = static_cast<size_t>(rows_p) * ld;
    for (size_t e = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * 256) {
        const int r = static_cast<int>(e / ld), k = static_cast<int>(e % ld);
        dst[e] = (r < rows && k < cols) ? src[static_cast<size_t>(r) * cols + k] : T(0);
    }
}

__global__ __launch_bounds__(256) void fill_ints_kernel(int* __restrict__ p, int n, int v) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

// The lowest chain whose strict feasibility check flagged a row (first
// starts at C).
__global__ __launch_bounds__(256) void first_flag_kernel(const int* __restrict__ flag, int C,
                                                         int* __restrict__ first) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < C && flag[c]) atomicMin(first, c);
}

template <typename T>
ess_status pad_copy(const void* src, int rows, int cols, void* dst, int rows_p, int ld,
                    hipStream_t st) {
    const size_t n = static_cast<size_t>(rows_p) * ld;
    const unsigned grid = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL((pad_copy_kernel<T>), dim3(grid), dim3(256), 0, st,
                       static_cast<const T*>(src), rows, cols, static_cast<T*>(dst), rows_p, ld);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status fill_ints(int* p, int n, int v, hipStream_t st) {
    const unsigned grid = static_cast<unsigned>(std::min((n + 255) / 256, 1024));
    hipLaunchKernelGGL(fill_ints_kernel, dim3(grid), dim3(256), 0, st, p, n, v);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

__global__ __launch_bounds__(256) void gate_rows_kernel(const int* __restrict__ flag,
                                                        const void* fallback, void* X, int d, int dp,
                                                        int esz, int* accepted) {
    const int c = blockIdx.x;
    const int bad = flag[c];
    if (threadIdx.x == 0) accepted[c] = !bad;
    if (!bad) return;
    if (esz == 4) {
        const float* src = static_cast<const float*>(fallback) + static_cast<size_t>(c) * d;
        float* dst = static_cast<float*>(X) + static_cast<size_t>(c) * dp;
        for (int k = threadIdx.x; k < d; k += 256) dst[k] = src[k];
    } else {
        const double* src = static_cast<const double*>(fallback) + static_cast<size_t>(c) * d;
        double* dst = static_cast<double*>(X) + static_cast<size_t>(c) * dp;
        for (int k = threadIdx.x; k < d; k += 256) dst[k] = src[k];
    }
}

}  // namespace

extern "C" {

const char* ess_last_error(void) { return g_err.c_str(); }

ess_status ess_init(const ess_problem* pr, void* stream, ess_ctx** out) {
    g_err.clear();
    if (!pr || !out) return fail(ESS_ERR_INVALID_ARG, "null problem or output pointer");
    *out = nullptr;
    if (!pr->A || !pr->b || !pr->x0) return fail(ESS_ERR_INVALID_ARG, "null A, b or x0");
    if (pr->d < 1 || pr->m < 1 || pr->n_chains < 1)
        return fail(ESS_ERR_INVALID_ARG, "d, m and n_chains must be >= 1 (got %d, %d, %d)", pr->d,
                    pr->m, pr->n_chains);
    if (pr->precision != 32 && pr->precision != 64)
        return fail(ESS_ERR_INVALID_ARG, "precision must be 32 or 64 (got %d)", pr->precision);
    if (!(pr->trim_eps >= 0.0) || pr->trim_eps > 1.0)
        return fail(ESS_ERR_INVALID_ARG, "trim_eps must lie in [0, 1] (got %g)", pr->trim_eps);
    if (pr->m > kMaxRowsLarge)
        return fail(ESS_ERR_UNSUPPORTED, "m = %d exceeds the %d rows one workgroup sorts", pr->m,
                    kMaxRowsLarge);
    if ((pr->flags & (ESS_LIKELIHOOD_MIDPOINT | ESS_BRUTE_FORCE)) && pr->m > kMidpointMaxRows)
        return fail(ESS_ERR_UNSUPPORTED, "the quadratic comparators take m <= %d (got %d)",
                    kMidpointMaxRows, pr->m);
    if ((pr->flags & ESS_LIKELIHOOD_MIDPOINT) && (pr->flags & ESS_BRUTE_FORCE))
        return fail(ESS_ERR_INVALID_ARG, "choose one of ESS_LIKELIHOOD_MIDPOINT and ESS_BRUTE_FORCE");
    if (pr->flags & ESS_BRUTE_FORCE) {
        // Algorithm 2's lists take more LDS than the default limit above 2046 rows
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(pr->precision == 32 ? &sample_alg2_kernel<float>
                                                              : &sample_alg2_kernel<double>),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(alg2_lds_bytes(pr->m)));
        if (e != hipSuccess)
            return fail(ESS_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    if (pr->d > (1 << 20) || pr->n_chains > (1 << 24))
        return fail(ESS_ERR_UNSUPPORTED, "d or n_chains too large");

    ess_ctx* c = new ess_ctx();
    c->d = pr->d;
    c->m = pr->m;
    c->C = pr->n_chains;
    c->prec = pr->precision;
    c->esz = pr->precision == 32 ? 4 : 8;
    c->seed = pr->seed;
    c->eps = pr->trim_eps;
    c->flags = pr->flags;
    c->bstride = (pr->flags & ESS_PER_CHAIN_B) ? pr->m : 0;
    c->st = static_cast<hipStream_t>(stream);
    // One chain group by default: splitting the chains into two concurrent
    // sample -> projection pipelines measured slower at d=1000, m=2000, 1024
    // chains (two half-size projection launches took 141 us per step against
    // 93 us for one).  ESS_CHAIN_GROUPS=2 selects the split.
    c->G = 1;
    if (const char* e = std::getenv("ESS_CHAIN_GROUPS")) {
        const int g = std::atoi(e);
        if (g >= 1 && g <= 2) c->G = g;   // more than two groups has not been exercised
    }
    c->mp = round_up(c->m, 128);
    c->Cp = round_up(c->C, 128);
    c->G = std::min(c->G, c->Cp / 128);
    c->dp = round_up(c->d, 32);
    choose_tiles(c);
    auto bail = [&](ess_status s) {
        std::string keep = g_err;
        ess_destroy(c);
        g_err = keep;
        return s;
    };
    const size_t rows = static_cast<size_t>(c->Cp) * c->dp * c->esz;
    ess_status s;
    if ((s = dalloc(c, &c->A, static_cast<size_t>(c->mp) * c->dp * c->esz)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->b),
                    sizeof(double) * c->m * (c->bstride ? c->C : 1))) != ESS_OK ||
        (s = dalloc(c, &c->X, rows)) != ESS_OK || (s = dalloc(c, &c->Xprop, rows)) != ESS_OK ||
        (s = dalloc(c, &c->N, rows)) != ESS_OK ||
        (s = dalloc(c, &c->P, 2 * static_cast<size_t>(c->Cp) * c->mp * c->esz)) != ESS_OK ||
        (s = dalloc(c, &c->Q, static_cast<size_t>(c->Cp) * c->mp * c->esz)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->sel), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->flag), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->rej), sizeof(long long) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->fb_list), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->accepted), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->d_step), sizeof(uint32_t))) != ESS_OK ||
        (s = create_run_streams(c)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->fb_count), sizeof(int) * 2 * kMaxGroups)) != ESS_OK ||
        (s = dalloc(c, &c->AB, 2 * sizeof(double) * static_cast<size_t>(c->Cp) * c->mp)) != ESS_OK)
        return bail(s);
    if (c->m > kMaxRowsLds) {
        c->kstride = 512;
        while (c->kstride < c->m) c->kstride <<= 1;
        if ((s = dalloc(c, reinterpret_cast<void**>(&c->keys),
                        sizeof(uint64_t) * static_cast<size_t>(c->Cp) * c->kstride)) != ESS_OK)
            return bail(s);
    }
    if ((s = create_group_streams(c)) != ESS_OK) return bail(s);

    hipError_t e = hipMemcpy2DAsync(c->A, static_cast<size_t>(c->dp) * c->esz, pr->A,
                                    static_cast<size_t>(c->d) * c->esz,
                                    static_cast<size_t>(c->d) * c->esz, c->m, hipMemcpyDefault, c->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->b, pr->b, sizeof(double) * c->m * (c->bstride ? c->C : 1),
                           hipMemcpyDefault, c->st);
    if (e == hipSuccess) {
        if (pr->flags & ESS_X0_BROADCAST) {
            if (c->prec == 32)
                hipLaunchKernelGGL((broadcast_rows<float>), dim3(c->C), dim3(256), 0, c->st,
                                   static_cast<const float*>(pr->x0), static_cast<float*>(c->X),
                                   c->d, c->dp);
            else
                hipLaunchKernelGGL((broadcast_rows<double>), dim3(c->C), dim3(256), 0, c->st,
                                   static_cast<const double*>(pr->x0), static_cast<double*>(c->X),
                                   c->d, c->dp);
            e = hipGetLastError();
        } else
            e = hipMemcpy2DAsync(c->X, static_cast<size_t>(c->dp) * c->esz, pr->x0,
                                 static_cast<size_t>(c->d) * c->esz,
                                 static_cast<size_t>(c->d) * c->esz, c->C, hipMemcpyDefault, c->st);
    }
    if (e != hipSuccess) {
        fail(ESS_ERR_HIP, "copying the problem: %s", hipGetErrorString(e));
        return bail(ESS_ERR_HIP);
    }
    // float32 projections through exact bfloat16 splits where default_split
    // says so, unless a tuned choice for this shape is cached (ess_autotune);
    // ESS_PROJ=f32 keeps the float32 matrix cores and ESS_PROJ_TILE a tile
    // shape whatever the cache holds
    c->split_proj = default_split(c);
    load_tuned_single(c);
    {
        const char* pe = std::getenv("ESS_PROJ");
        if (pe && std::strcmp(pe, "f32") == 0) c->split_proj = false;
    }
    if (c->split_proj && (s = split_A(c)) != ESS_OK) return bail(s);
    if ((s = check_rows(c, "ess_init", 0)) != ESS_OK || (s = prime_direction(c)) != ESS_OK)
        return bail(s);
    *out = c;
    return ESS_OK;
}

ess_status ess_profile(ess_ctx* c, int enable) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    ESS_TRY(drain_events(c));
    c->profiling = enable != 0;
    for (int k = 0; k < 4; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    return ESS_OK;
}

ess_status ess_profile_read(ess_ctx* c, int kind, double* total_ms, int64_t* count) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (kind < 0 || kind > 3) return fail(ESS_ERR_INVALID_ARG, "unknown kernel kind %d", kind);
    ESS_TRY(drain_events(c));
    if (total_ms) *total_ms = c->prof_ms[kind];
    if (count) *count = c->prof_n[kind];
    c->prof_ms[kind] = 0.0;
    c->prof_n[kind] = 0;
    return ESS_OK;
}

void ess_destroy(ess_ctx* c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    else (void)hipDeviceSynchronize();
    for (auto& e : c->ev_open) {
        c->ev_pool.push_back(e.second.first);
        c->ev_pool.push_back(e.second.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (int g = 0; g < kMaxGroups; ++g) {
        if (c->gs[g]) (void)hipStreamSynchronize(c->gs[g]);
        if (c->gs[g]) (void)hipStreamDestroy(c->gs[g]);
        if (c->join[g]) (void)hipEventDestroy(c->join[g]);
        if (c->stagger[g]) (void)hipEventDestroy(c->stagger[g]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    (void)drop_graphs(c);
    if (c->cs) (void)hipStreamDestroy(c->cs);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

ess_status ess_run(ess_ctx* c, int64_t n_steps, int64_t thin, void* trace, int64_t* n_rejected) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (n_steps < 0 || thin < 1) return fail(ESS_ERR_INVALID_ARG, "n_steps >= 0 and thin >= 1 required");
    if (c->step + static_cast<uint64_t>(n_steps) >= (1ull << 32))
        return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    long long before = 0;
    if (n_rejected) ESS_TRY(sum_rejections(c, before));
    if (n_steps > 0) {
        ESS_TRY(run_dispatch(c, n_steps, thin, trace));
        c->step += static_cast<uint64_t>(n_steps);
    }
    if (n_rejected) {
        long long after = 0;
        ESS_TRY(sum_rejections(c, after));
        *n_rejected = after - before;
    }
    return ESS_OK;
}

ess_status ess_step(ess_ctx* c, void* x_out) {
    ESS_TRY(ess_run(c, 1, 1, nullptr, nullptr));
    if (x_out) ESS_TRY(ess_get_state(c, x_out, nullptr));
    return ESS_OK;
}

ess_status ess_get_state(ess_ctx* c, void* x_out, uint64_t* step_out) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (x_out) {
        if (c->batch) ESS_TRY(batched_copy_state(c, c->batch->X, static_cast<float*>(x_out), 0));
        else ESS_TRY(copy_rows_out(c, x_out, c->X));
    }
    if (step_out) *step_out = c->step;
    return ESS_OK;
}

ess_status ess_set_state(ess_ctx* c, const void* x_in, uint64_t step) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (!x_in) return fail(ESS_ERR_INVALID_ARG, "null state");
    if (step >= (1ull << 32)) return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    if (c->batch) {
        // staged in X' and checked there; a state that fails the strict check
        // leaves the context where it was (its projections recomputed from X)
        ess_ctx::Batch& B = *c->batch;
        ESS_TRY(batched_copy_state(c, static_cast<const float*>(x_in), B.Xprop, 1));
        const ess_status st = batched_set_state_from_X(c, "ess_set_state", B.Xprop);
        if (st != ESS_OK) {
            const std::string msg = g_err;
            (void)batched_set_state_from_X(c, "ess_set_state", B.X);
            g_err = msg;
            return st;
        }
        const size_t bytes = sizeof(float) * (B.h.back().x_off +
                                              static_cast<size_t>(B.h.back().Cp) * B.h.back().dp);
        HIP_TRY(hipMemcpyAsync(B.X, B.Xprop, bytes, hipMemcpyDeviceToDevice, c->st));
        ESS_TRY(launch_step_counter(c, c->st, step, 0));
    } else {
        ESS_TRY(copy_rows_in(c, c->Xprop, x_in));
        ESS_TRY(check_rows(c, "ess_set_state", 1));
        ESS_TRY(launch_step_counter(c, c->st, step, 0));
        ESS_TRY(prime_direction(c));
    }
    c->step = step;
    return ESS_OK;
}

ess_status ess_rejections(ess_ctx* c, int64_t* per_chain) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (!per_chain) return fail(ESS_ERR_INVALID_ARG, "null output");
    if (c->batch) {
        const ess_ctx::Batch& B = *c->batch;
        std::vector<long long> r(B.chains_padded);
        HIP_TRY(hipMemcpyAsync(r.data(), c->rej, sizeof(long long) * B.chains_padded,
                               hipMemcpyDeviceToHost, c->st));
        HIP_TRY(hipStreamSynchronize(c->st));
        long long k = 0;
        for (int p = 0; p < B.n; ++p)
            for (int ch = 0; ch < B.h[p].C; ++ch) per_chain[k++] = r[B.h[p].chain_off + ch];
        return ESS_OK;
    }
    HIP_TRY(hipMemcpyAsync(per_chain, c->rej, sizeof(long long) * c->C, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return ESS_OK;
}

ess_status ess_init_batched(const ess_problem* pr, int32_t n_problems, void* stream, ess_ctx** out) {
    g_err.clear();
    if (!pr || !out) return fail(ESS_ERR_INVALID_ARG, "null problems or output pointer");
    *out = nullptr;
    if (n_problems < 1 || n_problems > (1 << 23))
        return fail(ESS_ERR_INVALID_ARG, "n_problems must lie in [1, 2^23] (got %d)", n_problems);
    long long total_chains = 0;
    for (int p = 0; p < n_problems; ++p) {
        const ess_problem& q = pr[p];
        if (!q.A || !q.b || !q.x0) return fail(ESS_ERR_INVALID_ARG, "problem %d: null A, b or x0", p);
        if (q.d < 1 || q.m < 1 || q.n_chains < 1)
            return fail(ESS_ERR_INVALID_ARG, "problem %d: d, m and n_chains must be >= 1", p);
        if (q.precision != 32)
            return fail(ESS_ERR_UNSUPPORTED, "problem %d: batched problems run in precision 32", p);
        if (!(q.trim_eps >= 0.0) || q.trim_eps > 1.0)
            return fail(ESS_ERR_INVALID_ARG, "problem %d: trim_eps must lie in [0, 1]", p);
        if (q.m > 4096) return fail(ESS_ERR_UNSUPPORTED, "problem %d: m = %d exceeds 4096", p, q.m);
        if (q.d > (1 << 20)) return fail(ESS_ERR_UNSUPPORTED, "problem %d: d too large", p);
        if (q.flags & (ESS_SORT_FULL | ESS_LIKELIHOOD_MIDPOINT | ESS_BRUTE_FORCE))
            return fail(ESS_ERR_UNSUPPORTED,
                        "problem %d: ESS_SORT_FULL and the comparators are not offered for batches", p);
        total_chains += q.n_chains;
    }
    if (total_chains > (1 << 24)) return fail(ESS_ERR_UNSUPPORTED, "too many chains in the batch");
    ess_ctx* c = new ess_ctx();
    c->prec = 32;
    c->esz = 4;
    c->st = static_cast<hipStream_t>(stream);
    c->C = static_cast<int>(total_chains);
    ess_status s = batched_init(c, pr, n_problems);
    if (s == ESS_OK) s = load_tuned(c);
    if (s != ESS_OK) {
        std::string keep = g_err;
        ess_destroy(c);
        g_err = keep;
        return s;
    }
    *out = c;
    return ESS_OK;
}

ess_status ess_transition_explicit(ess_ctx* c, const void* x, const void* nu, const double* u,
                                   void* x_new, double* intervals, int32_t* n_intervals,
                                   double* theta, int32_t* rejected, void* pq) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (c->batch) return fail(ESS_ERR_UNSUPPORTED, "explicit transitions take single-problem contexts");
    if (!x || !nu || !u || !x_new) return fail(ESS_ERR_INVALID_ARG, "null x, nu, u or x_new");
    ESS_TRY(copy_rows_in(c, c->Xprop, x));
    ESS_TRY(check_rows(c, "ess_transition_explicit", 1));
    ESS_TRY(copy_rows_in(c, c->N, nu));
    const Group w = c->whole();
    if (c->m > 4096) ESS_TRY(clear_fallback_lists(c, c->st, 0));
    ESS_TRY(launch_proj(c, w, c->st, c->Xprop, COLS_NU, 0, 0));
    SampleArgs a = sample_args(c, w, 0);
    a.step = 0;   // the device counter holds the current step
    a.u_explicit = u;
    a.intervals = intervals;
    a.n_intervals = n_intervals;
    a.theta_out = theta;
    a.pq_out = pq;
    ESS_TRY(launch_sample(c, w, c->st, a));
    ESS_TRY(launch_proj(c, w, c->st, c->Xprop, COLS_X, 0, 0));
    SampleArgs f = sample_args(c, w, 0);
    f.rejected_out = rejected;
    ESS_TRY(launch_commit(c, w, c->st, f));
    ESS_TRY(copy_rows_out(c, x_new, c->X));
    // N and Q back to the current step's direction for later runs
    return prime_direction(c);
}

ess_status ess_transition_explicit_static(int32_t d, int32_t m, int32_t n_chains,
                                          int32_t precision, const void* A, const double* b,
                                          double trim_eps, const void* x, const void* nu,
                                          const double* u, void* x_new, double* intervals,
                                          int32_t* n_intervals, double* theta, int32_t* rejected,
                                          void* stream) {
    g_err.clear();
    if (!A || !b || !x || !nu || !u || !x_new)
        return fail(ESS_ERR_INVALID_ARG, "null A, b, x, nu, u or x_new");
    if (d < 1 || m < 1 || n_chains < 1)
        return fail(ESS_ERR_INVALID_ARG, "d, m and n_chains must be >= 1 (got %d, %d, %d)", d, m,
                    n_chains);
    if (precision != 32 && precision != 64)
        return fail(ESS_ERR_INVALID_ARG, "precision must be 32 or 64 (got %d)", precision);
    if (!(trim_eps >= 0.0) || trim_eps > 1.0)
        return fail(ESS_ERR_INVALID_ARG, "trim_eps must lie in [0, 1] (got %g)", trim_eps);
    if (m > kMaxRowsLarge || d > (1 << 20) || n_chains > (1 << 24))
        return fail(ESS_ERR_UNSUPPORTED, "d, m or n_chains too large");
    void* base = nullptr;
    ESS_TRY(scratch_address(&base));

    // the buffers of a context, carved from the static array (256-byte aligned)
    ess_ctx c;
    c.d = d;
    c.m = m;
    c.C = n_chains;
    c.prec = precision;
    c.esz = precision == 32 ? 4 : 8;
    c.eps = trim_eps;
    c.st = static_cast<hipStream_t>(stream);
    c.mp = round_up(m, 128);
    c.Cp = round_up(n_chains, 128);
    c.dp = round_up(d, 32);
    c.use_graphs = false;
    choose_tiles(&c);
    {
        // the projections ess_init would choose, so the values agree
        const char* pe = std::getenv("ESS_PROJ");
        c.split_proj = default_split(&c) && !(pe && std::strcmp(pe, "f32") == 0);
    }
    if (m > kMaxRowsLds) {
        c.kstride = 512;
        while (c.kstride < m) c.kstride <<= 1;
    }
    const size_t plane = static_cast<size_t>(c.mp) * c.dp;
    const size_t rows = static_cast<size_t>(c.Cp) * c.dp * c.esz;
    const size_t proj = static_cast<size_t>(c.Cp) * c.mp * c.esz;
    const int n_ints = 3 * c.Cp + 2 * kMaxGroups + 2;   // sel, flag, fb_list, fb_count, step, first
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t oA = carve(static_cast<size_t>(c.mp) * c.dp * c.esz);
    const size_t oX = carve(rows), oXp = carve(rows), oN = carve(rows);
    const size_t oP = carve(2 * proj), oQ = carve(proj);
    const size_t oAB = carve(2 * sizeof(double) * static_cast<size_t>(c.Cp) * c.mp);
    const size_t oRej = carve(sizeof(long long) * c.Cp);
    const size_t oInts = carve(sizeof(int) * n_ints);
    const size_t oKeys = carve(sizeof(uint64_t) * static_cast<size_t>(c.Cp) * c.kstride);
    const size_t oA3 = carve(c.split_proj ? 3 * plane * sizeof(uint16_t) : 0);
    if (off > kStaticScratchBytes)
        return fail(ESS_ERR_UNSUPPORTED,
                    "this shape needs %zu bytes of device memory; the static buffer holds %zu", off,
                    kStaticScratchBytes);
    unsigned char* mem = static_cast<unsigned char*>(base);
    c.A = mem + oA;
    c.b = const_cast<double*>(b);   // read only
    c.X = mem + oX;
    c.Xprop = mem + oXp;
    c.N = mem + oN;
    c.P = mem + oP;
    c.Q = mem + oQ;
    c.AB = mem + oAB;
    c.rej = reinterpret_cast<long long*>(mem + oRej);
    c.keys = c.kstride ? reinterpret_cast<uint64_t*>(mem + oKeys) : nullptr;
    c.A3 = c.split_proj ? reinterpret_cast<uint16_t*>(mem + oA3) : nullptr;
    int* ints = reinterpret_cast<int*>(mem + oInts);
    c.sel = ints;
    c.flag = ints + c.Cp;
    c.fb_list = ints + 2 * c.Cp;
    c.fb_count = ints + 3 * c.Cp;
    c.d_step = reinterpret_cast<uint32_t*>(ints + 3 * c.Cp + 2 * kMaxGroups);
    int* first = ints + 3 * c.Cp + 2 * kMaxGroups + 1;

    // the array keeps the previous call's contents: clear what starts at zero
    // (fill kernels, so the call can be captured), pad A, x and nu with zeros
    ESS_TRY(fill_ints(ints, n_ints - 1, 0, c.st));
    ESS_TRY(fill_ints(first, 1, n_chains, c.st));
    ESS_TRY(fill_ints(reinterpret_cast<int*>(c.rej), 2 * c.Cp, 0, c.st));
    const Group w = c.whole();
    if (precision == 32) {
        ESS_TRY(pad_copy<float>(A, m, d, c.A, c.mp, c.dp, c.st));
        ESS_TRY(pad_copy<float>(x, n_chains, d, c.X, c.Cp, c.dp, c.st));
        ESS_TRY(pad_copy<float>(nu, n_chains, d, c.N, c.Cp, c.dp, c.st));
        if (c.split_proj) {
            const unsigned grid = static_cast<unsigned>(std::min<size_t>((plane / 2 + 255) / 256, 4096));
            hipLaunchKernelGGL(split_rows_kernel, dim3(grid), dim3(256), 0, c.st,
                               static_cast<const float*>(c.A), plane, c.A3, c.A3 + plane,
                               c.A3 + 2 * plane);
            HIP_TRY(hipGetLastError());
        }
    } else {
        ESS_TRY(pad_copy<double>(A, m, d, c.A, c.mp, c.dp, c.st));
        ESS_TRY(pad_copy<double>(x, n_chains, d, c.X, c.Cp, c.dp, c.st));
        ESS_TRY(pad_copy<double>(nu, n_chains, d, c.N, c.Cp, c.dp, c.st));
    }
    // strict feasibility of x (a_i^T x < b_i): A x into the committed buffers
    ESS_TRY(launch_proj(&c, w, c.st, c.X, COLS_X, 1, 1));
    hipLaunchKernelGGL(first_flag_kernel, dim3((n_chains + 255) / 256), dim3(256), 0, c.st, c.flag,
                       n_chains, first);
    HIP_TRY(hipGetLastError());
    int bad = n_chains;
    HIP_TRY(hipMemcpyAsync(&bad, first, sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (bad < n_chains)
        return fail(ESS_ERR_INFEASIBLE_START,
                    "ess_transition_explicit_static: chain %d is not strictly feasible", bad);
    // the transition, as ess_transition_explicit runs it
    ESS_TRY(fill_ints(c.flag, c.Cp, 0, c.st));
    ESS_TRY(launch_proj(&c, w, c.st, c.Xprop, COLS_NU, 0, 0));
    SampleArgs a = sample_args(&c, w, 0);
    a.step = 0;
    a.u_explicit = u;
    a.intervals = intervals;
    a.n_intervals = n_intervals;
    a.theta_out = theta;
    ESS_TRY(launch_sample(&c, w, c.st, a));
    ESS_TRY(launch_proj(&c, w, c.st, c.Xprop, COLS_X, 0, 0));
    SampleArgs f = sample_args(&c, w, 0);
    f.rejected_out = rejected;
    ESS_TRY(launch_commit(&c, w, c.st, f));
    return copy_rows_out(&c, x_new, c.X);
}

ess_status ess_draw(ess_ctx* c, uint64_t step, void* nu, double* u) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (c->batch) return fail(ESS_ERR_UNSUPPORTED, "ess_draw takes single-problem contexts");
    if (step >= (1ull << 32)) return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    return launch_draw(c, 0, c->C, c->st, step, nullptr, nu, c->d, u);
}


ess_status ess_set_state_gated(ess_ctx* c, const void* x_candidate, const void* x_fallback,
                               uint64_t step, int32_t* accepted) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (c->batch) return fail(ESS_ERR_UNSUPPORTED, "gated starts take single-problem contexts");
    if (!x_candidate || !x_fallback) return fail(ESS_ERR_INVALID_ARG, "null candidate or fallback");
    if (step >= (1ull << 32)) return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    // candidates staged in Xprop, checked strictly (projections into the
    // proposal buffers), rejected rows replaced by their fallback; the state
    // changes only once every staged row has passed the check
    ESS_TRY(copy_rows_in(c, c->Xprop, x_candidate));
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * c->Cp, c->st));
    ESS_TRY(launch_proj(c, c->whole(), c->st, c->Xprop, COLS_X, 0, 1));   // strict check
    hipLaunchKernelGGL(gate_rows_kernel, dim3(c->C), dim3(256), 0, c->st, c->flag, x_fallback,
                       c->Xprop, c->d, c->dp, c->esz, c->accepted);
    HIP_TRY(hipGetLastError());
    std::vector<int> acc(c->C);
    HIP_TRY(hipMemcpyAsync(acc.data(), c->accepted, sizeof(int) * c->C, hipMemcpyDeviceToHost, c->st));
    ESS_TRY(check_rows(c, "ess_set_state_gated (fallback rows)", 1));
    if (accepted)
        for (int i = 0; i < c->C; ++i) accepted[i] = acc[i];
    ESS_TRY(launch_step_counter(c, c->st, step, 0));
    ESS_TRY(prime_direction(c));
    c->step = step;
    return ESS_OK;
}

// ---- Appendix A: non-standard normal front end ----

ess_status ess_cholesky(const double* sigma, int32_t d, double* L) {
    g_err.clear();
    if (!sigma || !L || d < 1) return fail(ESS_ERR_INVALID_ARG, "need sigma, L and d >= 1");
    const size_t n = static_cast<size_t>(d);
    std::vector<double> out(n * n, 0.0);
    for (size_t j = 0; j < n; ++j) {
        double s = sigma[j * n + j];
        for (size_t k = 0; k < j; ++k) s -= out[j * n + k] * out[j * n + k];
        if (!(s > 0.0))
            return fail(ESS_ERR_INVALID_ARG, "sigma is not positive definite (pivot %zu is %g)", j, s);
        const double ljj = std::sqrt(s);
        out[j * n + j] = ljj;
        for (size_t i = j + 1; i < n; ++i) {
            double t = sigma[i * n + j];
            for (size_t k = 0; k < j; ++k) t -= out[i * n + k] * out[j * n + k];
            out[i * n + j] = t / ljj;
        }
    }
    std::memcpy(L, out.data(), sizeof(double) * n * n);
    return ESS_OK;
}

ess_status ess_whiten(const void* A, const double* b, const double* L, const double* mu, int32_t m,
                      int32_t d, int32_t precision, void* A_out, double* b_out, void* stream) {
    g_err.clear();
    if (!A || !b || !L || !mu || !A_out || !b_out)
        return fail(ESS_ERR_INVALID_ARG, "null argument to ess_whiten");
    if (m < 1 || d < 1) return fail(ESS_ERR_INVALID_ARG, "m and d must be >= 1 (got %d, %d)", m, d);
    if (precision != 32 && precision != 64)
        return fail(ESS_ERR_INVALID_ARG, "precision must be 32 or 64 (got %d)", precision);
    if (A_out == A) return fail(ESS_ERR_INVALID_ARG, "A_out must not alias A");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const long long tiles = static_cast<long long>((d + 15) / 16) * ((m + 15) / 16);
    if (tiles > (1ll << 31) - 1) return fail(ESS_ERR_UNSUPPORTED, "A too large for one launch");
    const dim3 g(static_cast<unsigned>(tiles)), blk(256);
    if (precision == 32) {
        hipLaunchKernelGGL((gemm_tiled_f64<float, float>), g, blk, 0, st, static_cast<const float*>(A), L,
                           m, d, d, 0, nullptr, static_cast<float*>(A_out));
        hipLaunchKernelGGL((shift_rhs<float>), dim3((m + 3) / 4), blk, 0, st, static_cast<const float*>(A),
                           b, mu, m, d, b_out);
    } else {
        hipLaunchKernelGGL((gemm_tiled_f64<double, double>), g, blk, 0, st, static_cast<const double*>(A),
                           L, m, d, d, 0, nullptr, static_cast<double*>(A_out));
        hipLaunchKernelGGL((shift_rhs<double>), dim3((m + 3) / 4), blk, 0, st,
                           static_cast<const double*>(A), b, mu, m, d, b_out);
    }
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status ess_unwhiten(const void* U, int64_t n, int32_t d, const double* L, const double* mu,
                        int32_t precision, void* X_out, void* stream) {
    g_err.clear();
    if (!U || !L || !mu || !X_out) return fail(ESS_ERR_INVALID_ARG, "null argument to ess_unwhiten");
    if (n < 1 || d < 1 || n > (1ll << 31) - 16)
        return fail(ESS_ERR_INVALID_ARG, "need 1 <= n < 2^31 and d >= 1 (got %lld, %d)",
                    static_cast<long long>(n), d);
    if (precision != 32 && precision != 64)
        return fail(ESS_ERR_INVALID_ARG, "precision must be 32 or 64 (got %d)", precision);
    if (X_out == U) return fail(ESS_ERR_INVALID_ARG, "X_out must not alias U");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int rows = static_cast<int>(n);
    const long long tiles = static_cast<long long>((d + 15) / 16) * ((rows + 15) / 16);
    if (tiles > (1ll << 31) - 1) return fail(ESS_ERR_UNSUPPORTED, "too many rows for one launch");
    const dim3 g(static_cast<unsigned>(tiles)), blk(256);
    if (precision == 32)
        hipLaunchKernelGGL((gemm_tiled_f64<float, float>), g, blk, 0, st, static_cast<const float*>(U), L,
                           rows, d, d, 1, mu, static_cast<float*>(X_out));
    else
        hipLaunchKernelGGL((gemm_tiled_f64<double, double>), g, blk, 0, st, static_cast<const double*>(U),
                           L, rows, d, d, 1, mu, static_cast<double*>(X_out));
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status ess_mlp_create(int32_t n_layers, const int32_t* widths, void* stream, ess_mlp** out) {
    g_err.clear();
    if (!out || !widths || n_layers < 1 || n_layers > 16)
        return fail(ESS_ERR_INVALID_ARG, "need 1..16 layers, widths and an output pointer");
    *out = nullptr;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 65536)
            return fail(ESS_ERR_INVALID_ARG, "width %d out of range", widths[l]);
    ess_mlp* n = new ess_mlp();
    n->L = n_layers;
    n->w.assign(widths, widths + n_layers + 1);
    n->st = static_cast<hipStream_t>(stream);
    long long off = 0, woff = 0;
    for (int l = 0; l < n_layers; ++l) {
        n->w_off.push_back(off);
        n->wb_off.push_back(woff);
        off += static_cast<long long>(n->w[l + 1]) * n->w[l];
        woff += static_cast<long long>(n->w[l + 1]) * n->w[l];
        n->c_off.push_back(off);
        off += n->w[l + 1];
    }
    n->n_params = off;
    n->n_weights = woff;
    ess_status s;
    if ((s = mlp_alloc(n, reinterpret_cast<void**>(&n->params), sizeof(float) * off)) != ESS_OK ||
        (s = mlp_alloc(n, reinterpret_cast<void**>(&n->grads), sizeof(float) * off)) != ESS_OK ||
        (s = mlp_alloc(n, reinterpret_cast<void**>(&n->m), sizeof(float) * off)) != ESS_OK ||
        (s = mlp_alloc(n, reinterpret_cast<void**>(&n->v), sizeof(float) * off)) != ESS_OK ||
        (s = mlp_alloc(n, reinterpret_cast<void**>(&n->wb), sizeof(uint16_t) * woff)) != ESS_OK ||
        (s = mlp_alloc(n, reinterpret_cast<void**>(&n->partial), sizeof(double) * 256)) != ESS_OK) {
        std::string keep = g_err;
        ess_mlp_destroy(n);
        g_err = keep;
        return s;
    }
    *out = n;
    return ESS_OK;
}

int64_t ess_mlp_num_params(const ess_mlp* n) { return n ? n->n_params : 0; }

ess_status ess_mlp_set_params(ess_mlp* n, const float* params) {
    g_err.clear();
    if (!n || !params) return fail(ESS_ERR_INVALID_ARG, "null network or parameters");
    HIP_TRY(hipMemcpyAsync(n->params, params, sizeof(float) * n->n_params, hipMemcpyDefault, n->st));
    HIP_TRY(hipMemsetAsync(n->m, 0, sizeof(float) * n->n_params, n->st));
    HIP_TRY(hipMemsetAsync(n->v, 0, sizeof(float) * n->n_params, n->st));
    n->adam_t = 0;
    return mlp_refresh_bf16(n);
}

ess_status ess_mlp_get_params(ess_mlp* n, float* params) {
    g_err.clear();
    if (!n || !params) return fail(ESS_ERR_INVALID_ARG, "null network or parameters");
    HIP_TRY(hipMemcpyAsync(params, n->params, sizeof(float) * n->n_params, hipMemcpyDefault, n->st));
    return ESS_OK;
}

ess_status ess_mlp_forward(ess_mlp* n, const float* in, int32_t batch, float* out) {
    g_err.clear();
    if (!n || !in || !out || batch < 1) return fail(ESS_ERR_INVALID_ARG, "bad forward arguments");
    ESS_TRY(mlp_forward(n, in, batch));
    HIP_TRY(hipMemcpyAsync(out, n->y, sizeof(float) * batch * n->w[n->L], hipMemcpyDefault, n->st));
    return ESS_OK;
}

ess_status ess_mlp_gradients(ess_mlp* n, const float* in, const float* target, int32_t batch,
                             float* grads, double* loss) {
    g_err.clear();
    if (!n || !in || !target || batch < 1) return fail(ESS_ERR_INVALID_ARG, "bad gradient arguments");
    ESS_TRY(mlp_forward(n, in, batch));
    ESS_TRY(mlp_backward(n, target, batch, loss));
    if (grads)
        HIP_TRY(hipMemcpyAsync(grads, n->grads, sizeof(float) * n->n_params, hipMemcpyDefault, n->st));
    return ESS_OK;
}

ess_status ess_mlp_adam(ess_mlp* n, double lr, double beta1, double beta2, double eps) {
    g_err.clear();
    if (!n || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
        return fail(ESS_ERR_INVALID_ARG, "bad Adam settings");
    n->adam_t += 1;
    const double c1 = 1.0 / (1.0 - std::pow(beta1, static_cast<double>(n->adam_t)));
    const double c2 = 1.0 / (1.0 - std::pow(beta2, static_cast<double>(n->adam_t)));
    hipLaunchKernelGGL(adam_kernel, dim3(std::min<long long>((n->n_params + 255) / 256, 2048)),
                       dim3(256), 0, n->st, n->params, n->grads, n->m, n->v, n->n_params,
                       static_cast<float>(lr), static_cast<float>(beta1), static_cast<float>(beta2),
                       static_cast<float>(eps), static_cast<float>(c1), static_cast<float>(c2));
    HIP_TRY(hipGetLastError());
    return mlp_refresh_bf16(n);
}

void ess_mlp_destroy(ess_mlp* n) {
    if (!n) return;
    if (n->st) (void)hipStreamSynchronize(n->st);
    else (void)hipDeviceSynchronize();
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
}


ess_status ess_autotune(ess_ctx* c, int32_t steps_per_trial, char* report, int32_t report_len) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (steps_per_trial < 1) return fail(ESS_ERR_INVALID_ARG, "steps_per_trial must be >= 1");
    if (!c->batch) {
        std::ostringstream rep;
        if (c->G == 1 && c->C <= kGemvChains) {
            rep << "chosen: nothing to tune (the projections of at most " << kGemvChains
                << " chains take the row-parallel kernel)\n";
        } else {
            SingleChoice best;
            ESS_TRY(autotune_single(c, steps_per_trial, rep, best));
            store_tuned_single(c, best);
            rep << "chosen: " << (best.split ? "split" : "f32") << " " << best.bm << "x" << best.bn
                << ", band " << best.group_m << " (" << best.us << " us/step)\n";
        }
        if (report && report_len > 0) {
            const std::string r = rep.str();
            const size_t n = std::min(r.size(), static_cast<size_t>(report_len - 1));
            std::memcpy(report, r.data(), n);
            report[n] = 0;
        }
        return ESS_OK;
    }
    ess_ctx::Batch& B = *c->batch;
    // the saved state and the two timing events, released on every return
    struct Scratch {
        hipStream_t st = nullptr;
        float* saved = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Scratch() {
            if (saved) {
                (void)hipStreamSynchronize(st);   // no copy still reads or writes it
                (void)hipFree(saved);
            }
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } scr;
    scr.st = c->st;
    // keep the chains where they are: save the state, restore it afterwards
    const size_t bytes = sizeof(float) * (B.h.back().x_off +
                                          static_cast<size_t>(B.h.back().Cp) * B.h.back().dp);
    HIP_TRY(hipMalloc(&scr.saved, bytes));
    float* const saved = scr.saved;
    HIP_TRY(hipMemcpyAsync(saved, B.X, bytes, hipMemcpyDeviceToDevice, c->st));
    const uint64_t step0 = c->step;
    bool present[kTileBuckets] = {};
    for (const auto& d : B.h)   // problems above 192 columns keep the split tiles
        if (d.d <= 192) present[tile_bucket(d)] = true;

    HIP_TRY(hipEventCreate(&scr.e0));
    HIP_TRY(hipEventCreate(&scr.e1));
    hipEvent_t e0 = scr.e0, e1 = scr.e1;
    std::ostringstream rep;
    ess_status st = ESS_OK;
    // time the current choice: capture and warm, then time a replay
    auto trial = [&](TuneChoice& t) -> ess_status {
        ESS_TRY(apply_choice(c, t));
        ESS_TRY(drop_graphs(c));
        ESS_TRY(run_dispatch(c, steps_per_trial, 1, nullptr));
        c->step += steps_per_trial;
        HIP_TRY(hipEventRecord(e0, c->st));
        ESS_TRY(run_dispatch(c, steps_per_trial, 1, nullptr));
        c->step += steps_per_trial;
        HIP_TRY(hipEventRecord(e1, c->st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        t.us = 1e3 * ms / steps_per_trial;
        rep << (t.fused ? "fused" : "split") << ", " << c->batch->nsets << " sets, shapes";
        int code = t.shape_code;
        for (int k = 0; k < kTileBuckets; ++k, code /= kBatchShapes)
            rep << " " << shape_bm(code % kBatchShapes) << "x" << shape_bn(code % kBatchShapes);
        rep << ": " << t.us << " us/step\n";
        return ESS_OK;
    };
    const TuneChoice before = current_choice(c);
    TuneChoice best = before;
    st = trial(best);
    // one pass of coordinate descent: each size class in turn, the others fixed
    int place = 1;
    for (int k = 0; k < kTileBuckets && st == ESS_OK; ++k, place *= kBatchShapes) {
        if (!present[k]) continue;
        const int digit = (best.shape_code / place) % kBatchShapes;
        for (int sh = 0; sh < kBatchShapes && st == ESS_OK; ++sh) {
            if (sh == digit) continue;
            TuneChoice t = best;
            t.shape_code = best.shape_code + (sh - digit) * place;
            st = trial(t);
            if (st == ESS_OK && t.us < best.us) best = t;
        }
    }
    if (st == ESS_OK) {   // the other launch form with the chosen shapes
        TuneChoice t = best;
        t.fused = best.fused ? 0 : 1;
        st = trial(t);
        if (st == ESS_OK && t.us < best.us) best = t;
    }
    // the split form's problem-set count (the chains do not depend on it)
    for (int ns = 1; ns <= std::min(kMaxGroups, B.n) && st == ESS_OK && !best.fused; ++ns) {
        if (ns == best.sets) continue;
        TuneChoice t = best;
        t.sets = ns;
        st = trial(t);
        if (st == ESS_OK && t.us < best.us) best = t;
    }
    ess_status fin = apply_choice(c, st == ESS_OK ? best : before);
    if (fin == ESS_OK) fin = drop_graphs(c);
    HIP_TRY(hipMemcpyAsync(B.X, saved, bytes, hipMemcpyDeviceToDevice, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    ESS_TRY(fin);
    ESS_TRY(batched_set_state_from_X(c, "ess_autotune"));
    ESS_TRY(launch_step_counter(c, c->st, step0, 0));
    c->step = step0;
    if (st != ESS_OK) return st;
    store_tuned(c, best);
    rep << "chosen: " << (best.fused ? "fused" : "split") << ", " << best.sets << " sets, shape_code "
        << best.shape_code
        << " (" << best.us << " us/step)\n";
    if (report && report_len > 0) {
        const std::string r = rep.str();
        const size_t n = std::min(r.size(), static_cast<size_t>(report_len - 1));
        std::memcpy(report, r.data(), n);
        report[n] = 0;
    }
    return ESS_OK;
}

}  // extern "C"
