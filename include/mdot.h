/*
 * mdot.h -- C ABI of the MI355X MDOT-PNCG optimal-transport library (libmdot.so).
 *
 * The library solves the discrete optimal transport problem
 *     OT(r, c, C) = min { <P, C> : P >= 0, P 1 = r, P^T 1 = c }
 * for a square cost C in [0,1]^{n x n} and marginals r, c on the simplex (paper Sec. 2.1),
 * with MDOT (Alg. 1: gamma annealing read as mirror descent, entropy-aware tolerance,
 * variable marginal smoothing, Taylor warm start eq. (approx-znext)), the PNCG projector
 * (Alg. 2 with the Sinkhorn direction eq. (sinkhorn-direction), the preconditioned
 * Hestenes-Stiefel beta eq. (beta_PPR_OT) and the App. B hybrid line search on the
 * approximate Wolfe conditions eq. (approximate-wolfe)), and the Round step (Alg. 3).
 *
 * Notation: gamma is the inverse temperature, P_ij = exp(u_i + v_j - gamma C_ij)
 * (eq. (lagrangian-closed-form)); u, v are potentials in nats. Cost-unit potentials are
 * f = u / gamma, g = v / gamma.
 *
 * Certified gap: every solve reports UB = <G, C> for the rounded plan G in U(r, c) and a
 * lower bound LB <= OT(r, c, C) obtained from the double c-transform of cost-unit
 * potentials (dual feasible, so weak LP duality applies). The potentials tried are u/gamma
 * and the finite difference (u^t - u^{t-1}) / (gamma^t - gamma^{t-1}) along the annealing
 * path. gap = UB - LB >= UB - OT. The lower bound is not part of the paper, which measures
 * error against an exact CPU solver.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device pointers on the context's device; the caller
 *     owns them. The library keeps no pointer after a synchronous call returns.
 *   - Calls are issued on the context's HIP stream. Synchronous calls return after the
 *     stream work they queued has completed.
 *   - Return value: 0 (MDOT_OK) on success; < 0 on error, in which case outputs are left
 *     untouched and mdot_last_error() describes the failure; > 0 is a warning with valid
 *     outputs (MDOT_W_NOT_CONVERGED: the budget or gamma cap was hit with gap > target;
 *     MDOT_W_RANGE: a sweep input put some row or column outside the exponent range the
 *     kernel can represent, see mdot_lse2).
 *   - One host thread per context.
 */
#ifndef MDOT_H
#define MDOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MDOT_OK = 0,
    MDOT_W_NOT_CONVERGED = 1,
    MDOT_W_RANGE = 2,
    MDOT_E_ARG = -1,      /* bad size, NULL pointer, bad enum or parameter */
    MDOT_E_MARGINAL = -2, /* r or c negative, non-finite, or |sum - 1| > 1e-9 max(m, n) */
    MDOT_E_COST = -3,     /* scaled cost outside [0, 1] or non-finite */
    MDOT_E_NOMEM = -4,    /* device allocation failed, or the request exceeds the HBM budget */
    MDOT_E_DEVICE = -5,   /* a HIP call failed */
    MDOT_E_BUSY = -6      /* no free serving slot */
};

/* How C is given. C is m x n: row i is source i (marginal r_i), column j is target j (marginal
 * c_j); the paper's problems are square (m = n), rectangular ones take the same path.
 * DENSE: data is an m*n row-major array of dtype. POINTS_* (d = 1..8): data holds X (m*d FP32,
 * row-major) followed by Y (n*d FP32); C_ij = scale * dist(x_i, y_j), computed on the fly in
 * FP64 inside the sweep (paper Sec. 3: O(n) memory when entries of C can be computed in O(1)).
 * Everywhere below, vectors indexed by rows (r, u, log r(P), shift) have m entries and vectors
 * indexed by columns (c, v, log c(P)) have n. */
typedef enum { MDOT_COST_DENSE = 0, MDOT_COST_POINTS_SQEUCLID = 1, MDOT_COST_POINTS_L1 = 2 } mdot_cost_kind;
typedef enum { MDOT_DT_F64 = 0, MDOT_DT_F32 = 1, MDOT_DT_F16 = 2, MDOT_DT_BF16 = 3 } mdot_dtype;

/* Arithmetic of the O(n^2) sweeps. F64: FP64 exponent arguments, FP64 exp and sums.
 * F32: FP64 exponent arguments, hardware FP32 exp2, FP32 partial sums of <= 4 terms,
 * FP64 everything else (dual objective, marginals, dot products, line search, gap
 * certificate); rows or columns whose shifted sums fall outside the FP32 range are
 * re-evaluated in F64. Round and certificate sweeps always accumulate in FP64. */
/* MIXED (a DENSE FP32 or FP64 cost; mdot_solve or mdot_submit): the library keeps an FP16 copy of the cost
 * in its workspace and runs the early stages (F32 arithmetic) on that copy while
 * gamma * scale * delta <= mixed_switch, delta = max_ij |C16_ij - C_ij| (raw units); the
 * remaining stages run on the exact cost. Any potentials start the next stage (Prop. 1.2),
 * so the stages on the copy only provide warm starts: every Round / certificate sweep reads
 * the exact cost, and the certified gap refers to it. */
typedef enum { MDOT_PREC_F64 = 0, MDOT_PREC_F32 = 1, MDOT_PREC_MIXED = 2 } mdot_precision;

#define MDOT_MAX_N 131072 /* largest n; larger sizes return MDOT_E_ARG */
#define MDOT_NOALLOC_MAX_N 4096 /* largest n of mdot_lse2_noalloc */

typedef struct {
    int32_t n;            /* columns (targets, marginal c), 1..MDOT_MAX_N */
    int32_t d;            /* point dimension for POINTS_* (1..8), ignored for DENSE */
    mdot_cost_kind kind;
    mdot_dtype dtype;     /* DENSE only: element type of data (POINTS_* use FP32 coordinates) */
    const void* data;     /* device */
    double scale;         /* C = scale * raw; > 0. For POINTS_*, 0 means 1 / max_ij raw. */
    int32_t m;            /* rows (sources, marginal r), 1..MDOT_MAX_N; 0 means m = n (square) */
    int32_t reserved;     /* must be 0 */
} mdot_cost_desc;

typedef struct {
    double p;             /* eps_d = H_min / gamma^p (Alg. 1); paper: 1.5 */
    double q;             /* gamma_{t+1} = q gamma_t (Alg. 1); paper: 2^(1/3) */
    double gamma_i;       /* first gamma (Alg. 1); paper: 2^4 */
    double gamma_f;       /* > 0: run the paper's schedule to gamma_f, round and certify once.
                             0: adaptive, certify after every stage, stop at gap <= target */
    double gamma_cap;     /* adaptive cap; 0 => 5 H_min / (2 target) (Remark 1) */
    double ls_c1, ls_c2;  /* approximate Wolfe constants; the paper leaves them open,
                             defaults 0.1 and 0.9 (Hager-Zhang) */
    int32_t max_ls_trials;    /* per line search (default 50) */
    int32_t max_pncg_iters;   /* per stage (default 100000) */
    int64_t max_sweeps;       /* LSE sweeps per solve, 0 = unlimited */
    mdot_precision precision; /* default MDOT_PREC_F32 */
    int32_t warm_start;       /* 1: Taylor warm start eq. (approx-znext); 0: reuse z^t;
                                 2: epsilon-scaling z' = (gamma^{t+1} / gamma^t) z^t (Sec. 4.2.1) */
    double mixed_switch;      /* MIXED: largest gamma * scale * delta run on the FP16 copy (default 0.05) */
    /* The variants the paper compares against (defaults 0 = the method as in Alg. 1 and 2). */
    int32_t projector;        /* 0: PNCG (Alg. 2); 1: log-domain Sinkhorn (Alg. 4): per iteration the
                                 row update u += log r~ - log r(P), then the column update
                                 v += log c~ - log c(P), two sweeps; the stage ends when
                                 ||r(P) - r~||_1 <= eps_d / 2 after a column update */
    int32_t precond;          /* 0: Sinkhorn direction eq. (sinkhorn-direction); 1: diagonal-Hessian
                                 direction eq. (s-tilde) (r~ / r(P) - 1, c~ / c(P) - 1), taken at an
                                 iteration only when every ratio lies in [0.01, 100], otherwise the
                                 Sinkhorn direction (Sec. 4.3); the choice also enters the numerator
                                 of beta. PNCG only */
    int32_t smoothing;        /* 0: variable weight eps_d / 4 per stage (Alg. 1); 1: fixed weight, the
                                 final stage's H / (4 gamma_f^p) in every stage (App. D); in adaptive
                                 mode gamma_f is the gamma cap */
    int32_t tol_log_n;        /* 0: eps_d = H_min / gamma^p (Alg. 1); 1: log n in place of H_min in
                                 eps_d, tolerance and smoothing (App. C); the gamma cap keeps H_min */
} mdot_params;

typedef struct {
    double primal_cost;   /* UB = <G, C>, G = Round(P) in U(r, c) (Alg. 3), best over checked stages */
    double dual_bound;    /* LB <= OT(r, c, C), best over checked stages */
    double gap;           /* UB - LB */
    double gamma_final;   /* gamma of the stage whose plan gave UB (potentials returned for it) */
    double marg_err_l1;   /* rounding-error estimate of ||r(G) - r||_1 + ||c(G) - c||_1 */
    double grad_norm;     /* ||grad g||_1 on the smoothed marginals when the solve stopped */
    double seconds;       /* device time of the solve (HIP events) */
    int32_t stages;
    int32_t status;       /* same value the call returns */
    int64_t pncg_iters, ls_trials, sweeps, cg_resets, ls_failures;
    int64_t fp64_retries; /* F32 sweeps re-run in F64 because of range */
    int64_t cert_sweeps;  /* Round/certificate sweeps */
    int64_t prec_switches; /* F32 stages continued with FP64 exp after the gradient norm stalled */
    int64_t proxy_stages;  /* MIXED: stages run on the FP16 copy of the cost */
    int64_t tilde_iters;   /* precond = 1: iterations whose direction was the diagonal-Hessian one */
} mdot_result;

typedef struct mdot_ctx mdot_ctx;

/* Create a context on HIP device `device`, issuing work on `hip_stream` (a hipStream_t,
 * NULL = the default stream). hbm_budget_bytes bounds the workspace the context may hold
 * (0 = no bound). Returns MDOT_OK, MDOT_E_ARG or MDOT_E_DEVICE. */
int mdot_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, mdot_ctx** out);

/* Free the context and its workspace. NULL is accepted. */
int mdot_ctx_destroy(mdot_ctx* ctx);

/* Fill *out with the defaults (paper Sec. 5.2: p = 1.5, q = 2^(1/3), gamma_i = 2^4;
 * adaptive mode, F32 sweeps). */
void mdot_default_params(mdot_params* out);

/* Solve OT(r, c, C) to a certified gap <= target_gap (adaptive mode), or run the paper's
 * schedule to params->gamma_f (schedule mode).
 *   cost       : cost descriptor (device data)
 *   r, c       : device FP64[m] and FP64[n], on the simplex: non-negative, finite,
 *                |sum - 1| <= 1e-9 max(m, n)
 *   target_gap : > 0 in adaptive mode (ignored in schedule mode)
 *   params     : NULL = mdot_default_params()
 *   u_out,v_out: device FP64[m] / FP64[n] or NULL: potentials (nats) of the reported stage,
 *                gauge fixed so that sum(u) = sum(v)
 *   res        : host, required
 * Synchronous. Returns MDOT_OK, MDOT_W_NOT_CONVERGED or an error. */
int mdot_solve(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* r, const double* c,
               double target_gap, const mdot_params* params, double* u_out, double* v_out,
               mdot_result* res);

/* One fused two-sided LogSumExp sweep (Alg. 2, the lines forming log r(P) and log c(P)):
 *   lr_i = log sum_j exp(u_i + v_j - gamma C_ij),   lc_j = log sum_i exp(u_i + v_j - gamma C_ij)
 * in one pass over C. u, lr_out: device FP64[m]; v, lc_out: device FP64[n].
 * shift: device FP64[m] prediction of lr used as the per-row exponent shift, or NULL, in
 * which case the library first runs a row-max pass. Columns are exact to FP32/FP64 range
 * when their log-sum lies within ~60 (F32) / ~700 (F64) nats of the largest row shift of
 * each 64-row tile; otherwise MDOT_W_RANGE is returned (values then may be -inf).
 * precision: MDOT_PREC_F32 or MDOT_PREC_F64. Synchronous. */
int mdot_lse2(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
              const double* shift, mdot_precision precision, double* lr_out, double* lc_out);

/* Allocation-free variant of mdot_lse2, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and return values as mdot_lse2 (the same kernels run; lr_out and
 * lc_out are bit-identical to mdot_lse2's), with these limits:
 *   - m, n <= MDOT_NOALLOC_MAX_N (4096), else MDOT_E_ARG;
 *   - cost->scale > 0 for point costs too (scale 0 asks for a max pass, which this call does
 *     not run), else MDOT_E_ARG.
 * Its partials, state and control block live in one static device array per GPU (about
 * 9.7 MB, held from library load until the process ends), not in the context's workspace;
 * the context supplies only its stream and the pinned host block created by mdot_ctx_create.
 * It calls no hipMalloc/hipFree and no allocating library routine. Every call on one GPU
 * uses that GPU's array, so calls that overlap on one GPU (two contexts or threads, or
 * streams that run concurrently) race and must be serialised by the caller; the array keeps
 * the last call's contents, and the call clears what must start at zero itself.
 * Synchronous. */
int mdot_lse2_noalloc(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v,
                      double gamma, const double* shift, mdot_precision precision, double* lr_out,
                      double* lc_out);

/* Round (Alg. 3) and certify the plan P(u, v; gamma) without materialising it: two sweeps
 * give UB = <G, C> with G = Round(P, r, c), and LB = the larger double c-transform bound of
 * (u/gamma, v/gamma) and, when u_prev/v_prev are non-NULL, of
 * ((u - u_prev)/(gamma - gamma_prev), (v - v_prev)/(gamma - gamma_prev)).
 * u, u_prev, r: device FP64[m]; v, v_prev, c: device FP64[n]. ub, lb, marg_err: host. Synchronous. */
int mdot_round_certify(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v,
                       double gamma, const double* u_prev, const double* v_prev, double gamma_prev,
                       const double* r, const double* c, double* ub, double* lb, double* marg_err);

/* ---- Serving: continuous batching ----
 * A context keeps up to 64 solves in flight. Each engine step advances every admitted solve by
 * one solver step (one sweep each) in shared kernel launches, in chunks of 16 steps; a solve
 * that finishes frees its slot and workspace when its chunk is read back (see mdot_run), where
 * further requests can be admitted. Solves of any cost kinds and dtypes can be in flight
 * together: a step launches one sweep kernel per cost type present (and one finalize and one
 * decision kernel for all). Each solve's arithmetic is independent of the others in flight
 * (own workspace, state and fixed-order reductions), so its result is the same alone and in
 * any mix.
 *
 * mdot_submit: admit one solve (arguments as mdot_solve). The inputs and u_out/v_out are
 * borrowed until mdot_poll reports the ticket done. Returns MDOT_OK with *ticket set,
 * MDOT_E_BUSY when no slot is free or the context's HBM budget (hbm_budget_bytes of
 * mdot_ctx_create; workspace of n ~ 17 n^2 / 32 + 200 n bytes, plus 2 n^2 for MIXED's FP16
 * copy) would be exceeded -- retry after mdot_run -- or an error (intake validation as in
 * mdot_solve). Synchronous intake. A MIXED solve switches to the exact cost at the chunk
 * boundary after it reaches the switch point; its result equals mdot_solve's. */
int mdot_submit(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* r, const double* c,
                double target_gap, const mdot_params* params, double* u_out, double* v_out,
                uint64_t* ticket);

/* Advance every solve in flight by `steps` solver steps (rounded up to whole chunks of 16) and
 * retire the finished ones (potentials written to their u_out/v_out, results kept for
 * mdot_poll). Chunks are pipelined: each chunk is launched before the previous one is read
 * back, so a call retires the solves finished by the chunks read back during it, and the last
 * chunk it launched is read back by the next call (or by mdot_poll with wait != 0). A solve
 * that finished stays in flight, doing nothing, until its chunk is read back. *n_done (host,
 * may be NULL) receives the number retired. Returns after the chunks it read back have
 * completed; the last chunk launched may still be running. */
int mdot_run(mdot_ctx* ctx, int steps, int* n_done);

/* Result of a submitted solve. Returns MDOT_OK (res filled, ticket released) or 2 when still in
 * flight and wait == 0; with wait != 0 it runs the engine until the ticket is done.
 * res->seconds is 0 for engine solves (latency is the caller's clock). */
int mdot_poll(mdot_ctx* ctx, uint64_t ticket, int wait, mdot_result* res);

/* Number of solves in flight and the workspace bytes they hold (host pointers, may be NULL). */
int mdot_inflight(mdot_ctx* ctx, int* n_active, size_t* bytes_in_use);

/* Measurement hook: run the solver's fused LSE sweep kernel `iters` times back-to-back on the
 * context stream at the potentials (u, v) and gamma (shifts set to the exact log-sums first,
 * as in a line-search trial near the solution) and return the mean duration per sweep in
 * milliseconds, taken with HIP events on that stream. u, v: device FP64[m], FP64[n]; ms_per_sweep: host.
 * Synchronous. */
int mdot_bench_sweep(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
                     mdot_precision precision, int iters, double* ms_per_sweep);

/* Measurement hook: as mdot_bench_sweep, but each of the `iters` sweeps (1..256) is timed alone
 * with HIP events after a kernel reads the caller's buffer `flush` (device, flush_bytes; make it
 * larger than the last-level cache, e.g. 512 MiB), so every sweep finds the cost evicted from
 * the L2 and last-level caches and streams it from HBM. The buffer is read, not written (one
 * element is written only if the buffer's sum is exactly -1.2345e300). Synchronous. */
int mdot_bench_sweep_flushed(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v,
                             double gamma, mdot_precision precision, int iters, const void* flush,
                             size_t flush_bytes, double* ms_per_sweep);

/* ---- Launch-variant tuning ----
 * The sweep kernel exists in variants that compute the same values bit for bit and differ only
 * in speed: capped at 4 waves per SIMD (128 VGPRs) or 2 (256 VGPRs), and, for FP32 costs, with or
 * without staging its second batch of cost rows in LDS. mdot_ctx_create reads the choice per
 * cost type and size from a table: the file named by the environment variable MDOT_TUNING, else
 * tuning.json in the directory above the one holding libmdot.so (written by the package's
 * tuner, tune.py, from measurements on the GPU); without a table every size uses 4 waves per
 * SIMD and staging above 2048 tiles.
 *
 * mdot_tune_override: force a variant for the later calls on this context (the tuner uses it):
 * occ = 2 or 4 (0 = the table's), stage = 0 (never stage), 1 (always stage) or -1 (the
 * table's). Returns MDOT_OK or MDOT_E_ARG.
 * mdot_tune_variant: the variant a call on `cost` would take: *occ (2 or 4) and
 * *stage_min_tiles (FP32 costs stage with more tiles than this). Host pointers. */
int mdot_tune_override(mdot_ctx* ctx, int occ, int stage);
int mdot_tune_variant(mdot_ctx* ctx, const mdot_cost_desc* cost, int* occ, int* stage_min_tiles);

/* Text of the last error on this context (never NULL). */
const char* mdot_last_error(const mdot_ctx* ctx);

/* Library version string. */
const char* mdot_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MDOT_H */
