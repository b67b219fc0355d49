/*
 * libess: linear elliptical slice sampling on MI355X (gfx950).
 *
 * Samples N(0, I_d) restricted to the polytope {x : A x <= b} (Wu & Gardner,
 * arXiv 2407.10449, Section 1) with many independent Markov chains.  One
 * transition (Algorithm 1) draws nu ~ N(0, I), forms the ellipse
 * x cos(theta) + nu sin(theta) (Section 2), solves every constraint's
 * intersection angles (Appendix B, with the edge cases of Section 3.2), builds
 * the active intervals by sorting and a cumulative max (Algorithm 3,
 * Proposition 1), draws theta uniformly on them, moves, and applies the
 * safeguards of Section 3.3 (trimming by trim_eps, reject-and-stay).
 * Non-standard normals reduce to this form by whitening (Appendix A).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers unless marked "host".
 *  - Arrays are dense row-major; "T" is float when precision = 32 and double
 *    when precision = 64.  b and the interval outputs are always double.
 *  - Work is enqueued on the stream given to ess_init (a hipStream_t passed as
 *    void*, NULL = the null stream).  Calls return once the work is queued,
 *    except those that fill host memory, which synchronise the stream first.
 *  - Errors are returned as ess_status; ess_last_error() gives a message for
 *    the calling thread.  No call aborts the process.
 *  - The library owns the memory behind an ess_ctx; callers own every pointer
 *    they pass and may free inputs as soon as the call returns.
 *  - Random numbers: Philox4x32-10 keyed by the seed, counter
 *    (pair index, chain, step, stream | problem << 8); Box-Muller in float64.
 */
#ifndef ESS_H
#define ESS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ess_ctx ess_ctx;

typedef enum {
    ESS_OK = 0,
    ESS_ERR_INVALID_ARG = 1,      /* null pointer, bad size, bad precision ...   */
    ESS_ERR_INFEASIBLE_START = 2, /* some chain has a_i^T x0 >= b_i             */
    ESS_ERR_HIP = 3,              /* a HIP runtime call failed                   */
    ESS_ERR_OOM = 4,              /* device allocation failed                    */
    ESS_ERR_UNSUPPORTED = 5       /* size beyond what the kernels support        */
} ess_status;

/* ess_problem.flags */
#define ESS_X0_BROADCAST 1u   /* x0 holds one d-vector used by every chain */
#define ESS_PER_CHAIN_B 4u    /* b holds n_chains x m values: chain c samples the
                                 polytope {A x <= b_c} (a family sharing A) */
#define ESS_EAGER 8u          /* ess_run launches kernel by kernel instead of
                                 replaying a captured HIP graph */
#define ESS_SORT_FULL 2u      /* build every chain's active intervals with a full
                                 sort of all crossing rows instead of the bucketed
                                 sort (same intervals; for comparison) */
#define ESS_LIKELIHOOD_MIDPOINT 16u  /* comparator, not Algorithm 3: find the
                                 active intervals by likelihood testing at the
                                 midpoints between sorted intersection angles
                                 (Section 2.2), O(m^2) per chain; m <= 4096,
                                 single-problem contexts only */
#define ESS_BRUTE_FORCE 32u   /* comparator, not Algorithm 3: intersect the rows'
                                 sets one at a time (Algorithm 2), O(m^2) per chain
                                 at worst (Appendix D); m <= 4096, single-problem
                                 contexts only */

/* A whitened problem: N(0, I_d) truncated to {x : A x <= b} (Section 1).
 * The polytope must have a non-empty interior; x0 must be strictly inside
 * (a_i^T x0 < b_i for all i), since a start on the boundary leaves the
 * zero-length single-root case of Figure 2(d). */
typedef struct {
    int32_t d;            /* dimension, >= 1                                  */
    int32_t m;            /* number of constraints, 1 .. 65536 (1 .. 4096 in a
                             batched context); above 4096 every pass over the
                             rows is made in chunks of 4096 and the full sort
                             keeps keys only, in LDS up to 16384 rows and in
                             device memory (8 bytes per row and chain) beyond */
    int32_t n_chains;     /* independent chains, >= 1                         */
    int32_t precision;    /* 32: float storage and projections, float64 roots,
                             interval ends and sampling; 64: float64 throughout */
    const void* A;        /* device, m x d row-major, T                       */
    const double* b;      /* device, m (n_chains x m with ESS_PER_CHAIN_B)    */
    const void* x0;       /* device, n_chains x d (or d with ESS_X0_BROADCAST), T */
    uint64_t seed;        /* Philox key                                       */
    double trim_eps;      /* >= 0, radians; every active interval [l, u] becomes
                             [l + eps, u - eps] at its real ends (Section 3.3) */
    uint32_t flags;
} ess_problem;

/* Validates the problem, copies A, b and x0 into library memory, computes
 * A x0 and checks strict feasibility of every chain.  On success *out holds a
 * new context at step 0.  ESS_ERR_INFEASIBLE_START names the first offending
 * chain and row in ess_last_error(). */
ess_status ess_init(const ess_problem* problem, void* stream, ess_ctx** out);

/* Many independent problems in one context (a batch of polytopes of uneven
 * d and m).  problems[p] is read as for ess_init; precision must be 32 and
 * ESS_SORT_FULL is not offered.  Problem p's chains use p as the Philox problem
 * word.  Every step of ess_run advances all chains of all problems with one
 * persistent launch: the projection tiles of every problem, then every chain,
 * each chain starting once its problem's tiles are done.
 * For a batched context, state and trace arrays hold the problems one after
 * another, each as n_chains x d (float); ess_rejections lists chains in the same
 * order.  ess_transition_explicit and ess_draw return ESS_ERR_UNSUPPORTED. */
ess_status ess_init_batched(const ess_problem* problems, int32_t n_problems, void* stream,
                            ess_ctx** out);

/* One transition of Algorithm 1 for every chain.  x_out (nullable): n_chains x d,
 * T, receives the state after the step. */
ess_status ess_step(ess_ctx* ctx, void* x_out);

/* n_steps transitions of Algorithm 1 (Section 2: ellipse through x_t and
 * nu_t, active intervals by Algorithm 3, theta uniform over them, Section
 * 3.3's trim and reject-and-stay safeguard).  The first call with a given (n_steps, thin, trace)
 * captures the launches into a HIP graph; later calls with the same shape
 * replay it (unless ESS_EAGER or profiling is on).  A trace buffer that is
 * freed and reallocated at the same address is fine; the graph only stores
 * the pointer.
 * Every thin-th state is written to trace (nullable):
 * (n_steps / thin) x n_chains x d, T.  n_rejected (host, nullable) receives the
 * number of proposals rejected by the safeguard during this call (summed over
 * chains; a zero-length active set counts as a rejection). */
ess_status ess_run(ess_ctx* ctx, int64_t n_steps, int64_t thin, void* trace,
                   int64_t* n_rejected);

/* Current state x_t of Algorithm 1 (n_chains x d, T) and step counter t
 * (host). Either may be NULL. */
ess_status ess_get_state(ess_ctx* ctx, void* x_out, uint64_t* step_out);

/* Replaces the state x_t of Algorithm 1 (n_chains x d, T; strictly feasible,
 * as Section 3.2's edge cases require of a start) and the step counter.
 * Running n steps after ess_set_state(x, s) reproduces the run that reached
 * (x, s), bit for bit. */
ess_status ess_set_state(ess_ctx* ctx, const void* x_in, uint64_t step);

/* Gated start (the learned warm start's feasibility gate): every chain whose
 * candidate row (n_chains x d, T) is strictly feasible, a_i^T x < b_i for all i,
 * starts there; every other chain starts at its fallback row (n_chains x d, T),
 * which must be strictly feasible.  accepted (host, nullable, n_chains int32)
 * receives 1 where the candidate was taken.  Sets the step counter. */
ess_status ess_set_state_gated(ess_ctx* ctx, const void* x_candidate, const void* x_fallback,
                               uint64_t step, int32_t* accepted);

/* Per-chain rejection counters since ess_init (host, n_chains int64). */
ess_status ess_rejections(ess_ctx* ctx, int64_t* per_chain);

/* One transition of Algorithm 1 from explicit inputs (Section 2's ellipse,
 * Algorithm 3's active intervals, Section 3.3's trim and safeguard), for
 * testing against a reference.
 *  x (n_chains x d, T) becomes the state first (it must be feasible), nu
 *  (n_chains x d, T) is the ellipse direction and u (n_chains, double, in
 *  (0, 1)) picks theta.  Afterwards the context holds the new state and its
 *  step counter is unchanged.
 *  x_new      (n_chains x d, T): state after the transition
 *  intervals  (nullable, n_chains x (m + 1) x 2 double): the non-empty active
 *             intervals after trimming, ascending; n_intervals (nullable,
 *             n_chains int32) their count
 *  theta      (nullable, n_chains double): the drawn angle
 *  rejected   (nullable, n_chains int32): 1 if the safeguard kept x
 *  pq         (nullable, 2 x n_chains x m, T): the projections A x and A nu
 *             the kernels used. */
ess_status ess_transition_explicit(ess_ctx* ctx, const void* x, const void* nu,
                                   const double* u, void* x_new, double* intervals,
                                   int32_t* n_intervals, double* theta,
                                   int32_t* rejected, void* pq);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transition of ess_transition_explicit without a context.  It calls no
 * hipMalloc or hipFree; every buffer a context would own lives in one static
 * array of 64 MiB per device, which the library holds until the process ends.
 * A (m x d, T), b (m, double) and x, nu, u are read as by ess_init and
 * ess_transition_explicit (precision 32: float T; 64: double); x must be
 * strictly feasible (ESS_ERR_INFEASIBLE_START names the first chain that is
 * not; this check synchronises `stream`).  Outputs as for
 * ess_transition_explicit, with the same values: x_new (n_chains x d, T),
 * intervals (nullable, n_chains x (m + 1) x 2 double), n_intervals
 * (nullable, n_chains int32), theta (nullable, n_chains double), rejected
 * (nullable, n_chains int32).  The remaining work is queued on `stream` (a
 * hipStream_t as void*, NULL = the null stream).  ESS_ERR_UNSUPPORTED when the
 * shape needs more than the static array: about
 *   4 (mp dp + 3 Cp dp + 3 Cp mp) + 16 Cp mp bytes in precision 32 (8 in
 *   place of 4 in precision 64), mp = m and Cp = n_chains rounded up to 128,
 *   dp = d rounded up to 32; plus 6 mp dp bytes where precision 32 takes the
 *   split projections (as ess_init would: 128 x 128 tiles, or 64 x 64 tiles
 *   with d > 192), and 8 Cp m2
 *   bytes above 16384 rows (m2 = m rounded up to a power of two).
 * Every call on a device shares that device's array and keeps the last
 * call's contents there (the call clears what it needs): calls that overlap
 * on one device, from several streams or threads, race. */
ess_status ess_transition_explicit_static(int32_t d, int32_t m, int32_t n_chains,
                                          int32_t precision, const void* A, const double* b,
                                          double trim_eps, const void* x, const void* nu,
                                          const double* u, void* x_new, double* intervals,
                                          int32_t* n_intervals, double* theta, int32_t* rejected,
                                          void* stream);

/* The random numbers step `step` uses: nu (n_chains x d, T, nullable) and the
 * theta uniforms u (n_chains double, nullable).  Does not change the context. */
ess_status ess_draw(ess_ctx* ctx, uint64_t step, void* nu, double* u);

/* Autotuner of the projection kernels (Section 2's products A x and A nu;
 * the sampled chains do not depend on the choice in a batched context).
 * Every trial runs 2 x steps_per_trial steps (the first captures and warms
 * the graph, the second is timed); the fastest choice is kept and stored in
 * a JSON cache keyed by GPU architecture and workload ($ESS_TUNE_CACHE,
 * default ~/.cache/ess_tune.json), which later contexts of the same workload
 * load at init.  The chains' state, step counter and rejection counts are
 * restored afterwards.  report (host, nullable) receives one line per trial
 * and a last line "chosen: ...".
 * Batched contexts (ess_init_batched): problems fall into six size classes
 *   (d <= 64, d <= 192, d > 192, each split at m <= 256); the classes up to
 *   192 columns each take a float32 tile shape (64x64, 32x64, 64x32 or
 *   32x32 rows x chain columns), tuned by one pass of coordinate descent over
 *   the classes present, then the other launch form, then (split form) the
 *   number of problem sets run on streams of their own (1 to 4).  Problems
 *   above 192 columns keep the split bfloat16 64 x 64 tiles.
 * Single-problem contexts: in precision 32 the split bfloat16 tiles (128 x
 *   128 and 64 x 64) and the float32 tiles 128x128, 128x64, 64x128 and
 *   64x64, then the band height (1 to 16 tile rows) of the XCD-aware tile
 *   order; precision 64 tunes the band height only.  A context of at most 12 chains (the
 *   row-parallel projection) has nothing to tune and reports so.  The chains
 *   continue from the restored state on the chosen kernels, whose float32
 *   sums may round differently from the previous choice. */
ess_status ess_autotune(ess_ctx* ctx, int32_t steps_per_trial, char* report, int32_t report_len);

/* Kernel timing for measurement.  While enabled, every launch made by ess_run
 * is bracketed by a pair of HIP events on the context's stream; ess_profile_read
 * synchronises the stream and returns, for one kernel kind, the summed duration
 * (host, milliseconds) and the number of launches since profiling was enabled
 * or last read.  Kinds: ESS_KERNEL_PROJECT (projection GEMMs covering both the
 * proposals and the next directions), ESS_KERNEL_SAMPLE (per-chain roots, sort,
 * sweep, theta and move), ESS_KERNEL_OTHER (everything else). */
#define ESS_KERNEL_PROJECT 0
#define ESS_KERNEL_SAMPLE 1
#define ESS_KERNEL_OTHER 2
#define ESS_KERNEL_BATCHED 3   /* the persistent step of a batched context */
ess_status ess_profile(ess_ctx* ctx, int enable);
ess_status ess_profile_read(ess_ctx* ctx, int kind, double* total_ms, int64_t* count);

void ess_destroy(ess_ctx* ctx);

/* ---- Non-standard normal front end (Appendix A) ----------------------------
 * x ~ N(mu, Sigma) truncated to {A x <= b}, with Sigma = L L^T, is x = L u + mu
 * for u ~ N(0, I_d) truncated to {(A L) u <= b - A mu}: whiten the problem,
 * sample u with ess_init / ess_run, and map the states or traces back.
 * Matrices are row-major; L is lower triangular, d x d, float64. */

/* L = the Cholesky factor of sigma (both host, d x d, float64; only the lower
 * triangle of sigma is read, the upper triangle of L is zero).
 * ESS_ERR_INVALID_ARG when sigma is not positive definite. */
ess_status ess_cholesky(const double* sigma, int32_t d, double* L);

/* A_out (m x d, T) = A (m x d, T) L and b_out (m, float64) = b - A mu, float64
 * sums; T is float for precision 32, double for 64.  All pointers device;
 * A_out must not alias A.  Work is queued on `stream` (nullable). */
ess_status ess_whiten(const void* A, const double* b, const double* L, const double* mu,
                      int32_t m, int32_t d, int32_t precision, void* A_out, double* b_out,
                      void* stream);

/* X_out (n x d, T) = U (n x d, T) L^T + mu: every row u of U becomes L u + mu
 * (states, or traces flattened to rows).  Device pointers; X_out must not
 * alias U. */
ess_status ess_unwhiten(const void* U, int64_t n, int32_t d, const double* L, const double* mu,
                        int32_t precision, void* X_out, void* stream);

/* ---- The warm-start network ------------------------------------------------
 * A fully connected network y = W_L g(... g(W_1 x + c_1) ...) + c_L with the
 * exact GELU g(z) = z Phi(z) between layers, run on the matrix cores in
 * bfloat16 with float32 accumulation; float32 master weights, trained with the
 * mean squared error over all outputs and Adam (Kingma & Ba).  The flat
 * parameter vector holds W_0 (w1 x w0, row-major), c_0, W_1, c_1, ...
 * All arrays are device float32 unless marked host. */
typedef struct ess_mlp ess_mlp;
ess_status ess_mlp_create(int32_t n_layers, const int32_t* widths /* host, n_layers + 1 */,
                          void* stream, ess_mlp** out);
int64_t ess_mlp_num_params(const ess_mlp* net);
/* Copies parameters in (and resets the Adam moments) or out. */
ess_status ess_mlp_set_params(ess_mlp* net, const float* params);
ess_status ess_mlp_get_params(ess_mlp* net, float* params);
/* out (batch x w_L) = network(in (batch x w_0)). */
ess_status ess_mlp_forward(ess_mlp* net, const float* in, int32_t batch, float* out);
/* Forward and backward on one batch; keeps the gradients for ess_mlp_adam.
 * grads (nullable) receives them in the flat layout; loss (host, nullable) the
 * mean squared error. */
ess_status ess_mlp_gradients(ess_mlp* net, const float* in, const float* target, int32_t batch,
                             float* grads, double* loss);
/* One Adam step with the gradients of the last ess_mlp_gradients call. */
ess_status ess_mlp_adam(ess_mlp* net, double lr, double beta1, double beta2, double eps);
void ess_mlp_destroy(ess_mlp* net);

/* Message for the last failed call on this thread ("" if none). */
const char* ess_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ESS_H */
