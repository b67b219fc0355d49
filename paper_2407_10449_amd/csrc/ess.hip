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

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ess.h"
#include "gemm.hpp"
#include "philox.hpp"
#include "sample.hpp"

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

struct ess_ctx {
    int d = 0, m = 0, C = 0, prec = 32, esz = 4;
    int dp = 0, mp = 0, Cp = 0;
    uint64_t seed = 0;
    double eps = 0.0;
    uint32_t flags = 0;
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
    uint64_t step = 0;
    int bm = 128, bn = 128, group_m = 4;
    int nmax = 512;
    std::vector<void*> allocs;
};

namespace {

ess_status dalloc(ess_ctx* c, void** p, size_t bytes) {
    HIP_TRY(hipMalloc(p, bytes));
    c->allocs.push_back(*p);
    HIP_TRY(hipMemsetAsync(*p, 0, bytes, c->st));
    return ESS_OK;
}

ProjOut proj_out(const ess_ctx* c, int p_direct, int strict) {
    ProjOut o;
    o.m = c->m;
    o.C = c->C;
    o.Cp = c->Cp;
    o.mp = c->mp;
    o.b = c->b;
    o.P = c->P;
    o.Q = c->Q;
    o.sel = c->sel;
    o.flag = c->flag;
    o.p_direct = p_direct;
    o.strict = strict;
    return o;
}

enum Cols { COLS_X = 0, COLS_NU = 1, COLS_BOTH = 2 };

template <int BM, int BN>
void launch_f32(const ess_ctx* c, const void* B0, int cols, const ProjOut& o) {
    const int tiles_m = c->mp / BM, half = c->Cp / BN;
    const int tn0 = (cols == COLS_NU) ? half : 0;
    const int tiles_n = (cols == COLS_BOTH) ? 2 * half : half;
    hipLaunchKernelGGL((proj_gemm_f32<BM, BN>), dim3(tiles_m * tiles_n), dim3(256), 0, c->st,
                       static_cast<const float*>(c->A), static_cast<const float*>(B0),
                       static_cast<const float*>(c->N), c->dp, tiles_m, tiles_n, tn0,
                       c->group_m, o);
}

// Projections of the columns selected by `cols`: B0 rows (x or x') and/or the
// current nu rows.
ess_status launch_proj(const ess_ctx* c, const void* B0, int cols, int p_direct, int strict) {
    const ProjOut o = proj_out(c, p_direct, strict);
    if (c->prec == 32) {
        if (c->bm == 128 && c->bn == 128) launch_f32<128, 128>(c, B0, cols, o);
        else if (c->bm == 128 && c->bn == 64) launch_f32<128, 64>(c, B0, cols, o);
        else if (c->bm == 64 && c->bn == 128) launch_f32<64, 128>(c, B0, cols, o);
        else launch_f32<64, 64>(c, B0, cols, o);
    } else {
        const int tiles_m = c->mp / 64, half = c->Cp / 64;
        const int tn0 = (cols == COLS_NU) ? half : 0;
        const int tiles_n = (cols == COLS_BOTH) ? 2 * half : half;
        hipLaunchKernelGGL((proj_gemm_f64<64, 64>), dim3(tiles_m * tiles_n), dim3(256), 0, c->st,
                           static_cast<const double*>(c->A), static_cast<const double*>(B0),
                           static_cast<const double*>(c->N), c->dp, tiles_m, tiles_n, tn0,
                           c->group_m, o);
    }
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

SampleArgs sample_args(const ess_ctx* c) {
    SampleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.d = c->d;
    a.m = c->m;
    a.C = c->C;
    a.Cp = c->Cp;
    a.dp = c->dp;
    a.mp = c->mp;
    a.problem = 0;
    a.b = c->b;
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
    return a;
}

template <typename T>
void launch_sample_t(const ess_ctx* c, const SampleArgs& a) {
    const dim3 g(c->C), b(256);
    switch (c->nmax) {
        case 512: hipLaunchKernelGGL((sample_kernel<T, 512>), g, b, 0, c->st, a); break;
        case 1024: hipLaunchKernelGGL((sample_kernel<T, 1024>), g, b, 0, c->st, a); break;
        case 2048: hipLaunchKernelGGL((sample_kernel<T, 2048>), g, b, 0, c->st, a); break;
        default: hipLaunchKernelGGL((sample_kernel<T, 4096>), g, b, 0, c->st, a); break;
    }
}

ess_status launch_sample(const ess_ctx* c, const SampleArgs& a) {
    if (c->prec == 32) launch_sample_t<float>(c, a);
    else launch_sample_t<double>(c, a);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status launch_commit(const ess_ctx* c, const SampleArgs& a) {
    if (c->prec == 32) hipLaunchKernelGGL((commit_kernel<float>), dim3(c->C), dim3(256), 0, c->st, a);
    else hipLaunchKernelGGL((commit_kernel<double>), dim3(c->C), dim3(256), 0, c->st, a);
    HIP_TRY(hipGetLastError());
    return ESS_OK;
}

ess_status launch_draw(const ess_ctx* c, uint64_t step, void* dst, long long ld, double* u) {
    if (c->prec == 32)
        hipLaunchKernelGGL((draw_kernel<float>), dim3(c->C), dim3(256), 0, c->st, c->seed,
                           static_cast<uint32_t>(step), 0u, c->d, static_cast<float*>(dst), ld, u);
    else
        hipLaunchKernelGGL((draw_kernel<double>), dim3(c->C), dim3(256), 0, c->st, c->seed,
                           static_cast<uint32_t>(step), 0u, c->d, static_cast<double*>(dst), ld, u);
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

// Replace the state by the rows already in c->X: A x into the committed
// projection buffers and a strict feasibility check (a_i^T x < b_i).
ess_status set_state_from_X(ess_ctx* c, const char* what) {
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int) * c->Cp, c->st));
    ESS_TRY(launch_proj(c, c->X, COLS_X, 1, 1));
    std::vector<int> fl(c->C);
    HIP_TRY(hipMemcpyAsync(fl.data(), c->flag, sizeof(int) * c->C, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    for (int ch = 0; ch < c->C; ++ch) {
        if (!fl[ch]) continue;
        std::vector<int> sel(1);
        HIP_TRY(hipMemcpy(sel.data(), c->sel + ch, sizeof(int), hipMemcpyDeviceToHost));
        std::vector<double> bh(c->m), ph(c->m);
        HIP_TRY(hipMemcpy(bh.data(), c->b, sizeof(double) * c->m, hipMemcpyDeviceToHost));
        const size_t off = (static_cast<size_t>(sel[0]) * c->Cp + ch) * c->mp;
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
    return ESS_OK;
}

ess_status check_ctx(const ess_ctx* c) {
    if (!c) return fail(ESS_ERR_INVALID_ARG, "null context");
    return ESS_OK;
}

ess_status sum_rejections(const ess_ctx* c, long long& total) {
    std::vector<long long> r(c->C);
    HIP_TRY(hipMemcpyAsync(r.data(), c->rej, sizeof(long long) * c->C, hipMemcpyDeviceToHost,
                           c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    total = 0;
    for (long long v : r) total += v;
    return ESS_OK;
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
    if (pr->m > 4096) return fail(ESS_ERR_UNSUPPORTED, "m = %d exceeds the 4096 rows one workgroup sorts", pr->m);
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
    c->st = static_cast<hipStream_t>(stream);
    c->mp = round_up(c->m, 128);
    c->Cp = round_up(c->C, 128);
    c->dp = round_up(c->d, 32);
    if (c->prec == 32) {
        c->bm = c->m > 1024 ? 128 : 64;
        c->bn = c->C > 512 ? 128 : 64;
    } else {
        c->bm = c->bn = 64;
    }
    c->nmax = 512;
    while (c->nmax < c->m) c->nmax <<= 1;

    auto bail = [&](ess_status s) {
        std::string keep = g_err;
        ess_destroy(c);
        g_err = keep;
        return s;
    };
    const size_t rows = static_cast<size_t>(c->Cp) * c->dp * c->esz;
    ess_status s;
    if ((s = dalloc(c, &c->A, static_cast<size_t>(c->mp) * c->dp * c->esz)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->b), sizeof(double) * c->m)) != ESS_OK ||
        (s = dalloc(c, &c->X, rows)) != ESS_OK || (s = dalloc(c, &c->Xprop, rows)) != ESS_OK ||
        (s = dalloc(c, &c->N, rows)) != ESS_OK ||
        (s = dalloc(c, &c->P, 2 * static_cast<size_t>(c->Cp) * c->mp * c->esz)) != ESS_OK ||
        (s = dalloc(c, &c->Q, static_cast<size_t>(c->Cp) * c->mp * c->esz)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->sel), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->flag), sizeof(int) * c->Cp)) != ESS_OK ||
        (s = dalloc(c, reinterpret_cast<void**>(&c->rej), sizeof(long long) * c->Cp)) != ESS_OK)
        return bail(s);

    hipError_t e = hipMemcpy2DAsync(c->A, static_cast<size_t>(c->dp) * c->esz, pr->A,
                                    static_cast<size_t>(c->d) * c->esz,
                                    static_cast<size_t>(c->d) * c->esz, c->m, hipMemcpyDefault, c->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->b, pr->b, sizeof(double) * c->m, hipMemcpyDefault, c->st);
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
    if ((s = set_state_from_X(c, "ess_init")) != ESS_OK) return bail(s);
    *out = c;
    return ESS_OK;
}

void ess_destroy(ess_ctx* c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    else (void)hipDeviceSynchronize();
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
        const size_t trace_row = static_cast<size_t>(c->C) * c->d * c->esz;
        ESS_TRY(launch_draw(c, c->step, c->N, c->dp, nullptr));
        ESS_TRY(launch_proj(c, c->Xprop, COLS_NU, 0, 0));
        SampleArgs a = sample_args(c);
        for (int64_t s = 0; s < n_steps; ++s) {
            a.step = static_cast<uint32_t>(c->step + s);
            a.has_pending = s > 0;
            a.gen_next = s + 1 < n_steps;
            a.trace = (trace && s > 0 && s % thin == 0)
                          ? static_cast<char*>(trace) + (s / thin - 1) * trace_row
                          : nullptr;
            ESS_TRY(launch_sample(c, a));
            ESS_TRY(launch_proj(c, c->Xprop, s + 1 < n_steps ? COLS_BOTH : COLS_X, 0, 0));
        }
        SampleArgs f = sample_args(c);
        f.trace = (trace && n_steps % thin == 0)
                      ? static_cast<char*>(trace) + (n_steps / thin - 1) * trace_row
                      : nullptr;
        ESS_TRY(launch_commit(c, f));
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
    if (x_out) ESS_TRY(copy_rows_out(c, x_out, c->X));
    return ESS_OK;
}

ess_status ess_get_state(ess_ctx* c, void* x_out, uint64_t* step_out) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (x_out) ESS_TRY(copy_rows_out(c, x_out, c->X));
    if (step_out) *step_out = c->step;
    return ESS_OK;
}

ess_status ess_set_state(ess_ctx* c, const void* x_in, uint64_t step) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (!x_in) return fail(ESS_ERR_INVALID_ARG, "null state");
    if (step >= (1ull << 32)) return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    ESS_TRY(copy_rows_in(c, c->X, x_in));
    ESS_TRY(set_state_from_X(c, "ess_set_state"));
    c->step = step;
    return ESS_OK;
}

ess_status ess_rejections(ess_ctx* c, int64_t* per_chain) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (!per_chain) return fail(ESS_ERR_INVALID_ARG, "null output");
    HIP_TRY(hipMemcpyAsync(per_chain, c->rej, sizeof(long long) * c->C, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return ESS_OK;
}

ess_status ess_transition_explicit(ess_ctx* c, const void* x, const void* nu, const double* u,
                                   void* x_new, double* intervals, int32_t* n_intervals,
                                   double* theta, int32_t* rejected, void* pq) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (!x || !nu || !u || !x_new) return fail(ESS_ERR_INVALID_ARG, "null x, nu, u or x_new");
    ESS_TRY(copy_rows_in(c, c->X, x));
    ESS_TRY(set_state_from_X(c, "ess_transition_explicit"));
    ESS_TRY(copy_rows_in(c, c->N, nu));
    ESS_TRY(launch_proj(c, c->Xprop, COLS_NU, 0, 0));
    SampleArgs a = sample_args(c);
    a.step = static_cast<uint32_t>(c->step);
    a.u_explicit = u;
    a.intervals = intervals;
    a.n_intervals = n_intervals;
    a.theta_out = theta;
    a.pq_out = pq;
    ESS_TRY(launch_sample(c, a));
    ESS_TRY(launch_proj(c, c->Xprop, COLS_X, 0, 0));
    SampleArgs f = sample_args(c);
    f.rejected_out = rejected;
    ESS_TRY(launch_commit(c, f));
    ESS_TRY(copy_rows_out(c, x_new, c->X));
    return ESS_OK;
}

ess_status ess_draw(ess_ctx* c, uint64_t step, void* nu, double* u) {
    g_err.clear();
    ESS_TRY(check_ctx(c));
    if (step >= (1ull << 32)) return fail(ESS_ERR_UNSUPPORTED, "the step counter is limited to 2^32");
    return launch_draw(c, step, nu, c->d, u);
}

}  // extern "C"
