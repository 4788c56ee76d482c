/*
 * bmc.h - C ABI of the MI355X (gfx950) nested continuation-value Monte Carlo
 * for multi-asset Bermudan options: the data-generation phase shared by the
 * two pricers of Doan, Gaikwad, Bossy, Baude & Stokes-Rees, "Parallel Pricing
 * Algorithms for Multi-Dimensional Bermudan/American Options using Monte Carlo
 * methods" (INRIA RR-6530, 2008), around which sit the rule fits (I&Z boundary
 * regression, CMC boosting classifier) and the final pricing pass.
 *
 * Conventions
 *  - Every entry point returns a bmc_status and never throws.  On error the
 *    outputs are untouched and bmc_last_error() returns a thread-local message.
 *  - Spec arrays (bmc_spec) are HOST memory owned by the caller and read only
 *    during the call.
 *  - Arrays documented as "device" are HIP device memory owned by the caller
 *    (e.g. torch tensors' data_ptr()).  Calls taking device arrays are
 *    asynchronous on the context's stream unless stated otherwise; the caller
 *    synchronises (bmc_sync or its own stream sync) before reading outputs.
 *  - Point sets are structure-of-arrays FP64: x[i*N + j] is asset i of point j.
 *  - bmc_ctx and bmc_rules are opaque, library-owned, freed by their destroy
 *    calls.  A context is not thread-safe; use one per host thread.
 *  - Random numbers: Philox4x32-10 keyed by (seed, stream << 16 | date), with
 *    counters (step-block, path, point, region): region is the I&Z exercise
 *    region of a boundary-search point, 0 everywhere else; seeds must fit in
 *    32 bits.
 */
#ifndef BMC_H
#define BMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMC_D_MAX 64      /* assets */
#define BMC_NT_MAX 512    /* exercise dates */

typedef enum {
    BMC_OK = 0,
    BMC_EINVAL = -1,        /* invalid argument or spec */
    BMC_ENOTSPD = -2,       /* correlation matrix not positive definite */
    BMC_ENOMEM = -3,        /* device allocation failed or budget exceeded */
    BMC_EDEVICE = -4,       /* HIP runtime error */
    BMC_EUNSUPPORTED = -5,  /* combination not supported */
    BMC_ENOCONV = -6,       /* reserved (I&Z drops and counts non-converged points) */
    BMC_EBUSY = -7,         /* request not finished yet */
    BMC_ECANCELED = -8      /* request cancelled (bmc_server_cancel) */
} bmc_status;

/* Payoffs (Section 2.1-2.2, Section 3.2): arithmetic-basket put
 * (K - mean S)^+, call on the maximum (max S - K)^+, geometric-average put
 * (K - (prod S)^(1/d))^+, call on the minimum (min S - K)^+.  For d = 1 the
 * two puts coincide, and so do the two calls. */
typedef enum { BMC_PUT_BASKET = 0, BMC_CALL_MAX = 1, BMC_PUT_GEO = 2, BMC_CALL_MIN = 3 } bmc_payoff;

/* I&Z boundary-point search: the plain fixed point s <- G(s) (Section 2.4), or
 * secant steps on its residual r(s) = G(s) - s (the paper's "Newton
 * iterations", Section 2.3): first step plain, then
 * s - r(s) (s - s_prev) / (r(s) - r(s_prev)) limited to 20 |r(s)|, the plain
 * step where that is undefined or not positive.  Both stop at the first
 * evaluated s with |r(s)| < eps and return G(s). */
typedef enum { BMC_SEARCH_PLAIN = 0, BMC_SEARCH_SECANT = 1 } bmc_search;

/* Pricers: Classification-Monte Carlo (Section 3) with the LogitBoost linear
 * classifier (BMC_CMC) or AdaBoost with decision stumps (BMC_CMC_ADA; Section
 * 3.2 names both boosters), and Ibanez-Zapatero boundary computation
 * (Section 2). */
typedef enum { BMC_CMC = 0, BMC_IZ = 1, BMC_CMC_ADA = 2 } bmc_method;

/* Arithmetic of the inner paths.  FP64: everything in double.  FP32: path
 * stepping, exp and the uniform-to-normal map in float, per-lane payoff sums
 * in double.  FP32_KAHAN: as FP32 with per-lane Kahan-compensated float sums
 * merged in double.  Rule fits, Cholesky and final reductions are always FP64. */
typedef enum { BMC_FP64 = 0, BMC_FP32 = 1, BMC_FP32_KAHAN = 2 } bmc_precision;

/* Random-number streams (second key word, high half). */
typedef enum { BMC_STREAM_OUTER = 1, BMC_STREAM_INNER = 2, BMC_STREAM_FINAL = 3 } bmc_stream;

/* Market model of Section 2.2 / 3.2: d assets under risk-neutral GBM with
 * rate r, dividend yields delta_i, volatilities sigma_i, correlation rho, and
 * N_T exercise dates 0 < t_1 < ... < t_NT = T (t_0 = 0 is not a date). */
typedef struct {
    int32_t d;              /* 1..BMC_D_MAX */
    const double *S0;       /* [d] spot prices, > 0 */
    const double *delta;    /* [d] dividend yields */
    const double *sigma;    /* [d] volatilities, >= 0 */
    const double *rho;      /* [d*d] row-major, symmetric, unit diagonal, SPD */
    double K, r, T;         /* strike > 0, rate, maturity > 0 */
    int32_t n_dates;        /* N_T, 1..BMC_NT_MAX */
    const double *dates;    /* [n_dates] strictly increasing, last == T */
    int32_t payoff;         /* bmc_payoff */
} bmc_spec;

typedef struct {
    int32_t method;         /* bmc_method */
    int32_t precision;      /* bmc_precision */
    int64_t N;              /* sample points per date (CMC training points, I&Z lattice points) */
    int64_t n;              /* inner paths per point */
    int64_t n_final;        /* final-pricing paths */
    uint64_t seed;          /* < 2^32 */
    int32_t cls_rounds;     /* boosting rounds, <= 64 (0: 8 for BMC_CMC, 64 for BMC_CMC_ADA) */
    int32_t iz_max_iter;    /* I&Z iteration cap (default 100 when 0) */
    double iz_eps;          /* I&Z tolerance in price units (default 0.01 when 0) */
    int32_t iz_search;      /* bmc_search (BMC_SEARCH_PLAIN when 0) */
} bmc_opts;

typedef struct {
    double price, variance, std_err, ci95;   /* ci95 = 1.96 std_err */
    int64_t inner_path_steps;                /* executed continuation path-steps */
    int64_t final_path_steps;                /* executed final-pricing path-steps */
    int64_t iz_unconverged;                  /* I&Z points dropped or not converged */
    int64_t iz_iterations;                   /* I&Z continuation evaluations per point, summed */
    double seconds;                          /* wall time of the call */
    double calc_seconds;                     /* continuation (data generation) */
    double fit_seconds;                      /* rule fits */
    double final_seconds;                    /* final pricing */
    double refine_seconds;                   /* FP32 forms: FP64 re-estimates of near ties */
} bmc_result;

typedef struct bmc_ctx bmc_ctx;
typedef struct bmc_rules bmc_rules;

/* Library version (major*10000 + minor*100 + patch). */
int32_t bmc_version(void);
/* Message of the last failing call on this thread ("" if none). */
const char *bmc_last_error(void);

/* Context on HIP device `device`, issuing work on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  Owns scratch memory. */
bmc_status bmc_ctx_create(int32_t device, void *hip_stream, bmc_ctx **out);
void bmc_ctx_destroy(bmc_ctx *ctx);
/* Batched date sweeps as HIP graphs (default off): bmc_price_batch captures
 * its planned launch sequence once and replays it while the launch
 * signature (every launch's shape and the context buffers it addresses) is
 * unchanged; spec values, seeds and task tables are device data, so a
 * repeated book of the same shapes replays with new inputs.  Results are
 * identical with and without graphs; the phase times of a graph run are
 * reported as one calc phase.  bmc_ctx_graph_stats counts captures and
 * replays. */
bmc_status bmc_ctx_set_graphs(bmc_ctx *ctx, int32_t enable);
bmc_status bmc_ctx_graph_stats(bmc_ctx *ctx, int64_t *captures, int64_t *replays);
/* Blocks until all work issued through ctx has finished. */
bmc_status bmc_sync(bmc_ctx *ctx);

/* Whole pricer, synchronous (Algorithm 1 for BMC_IZ, Algorithm 2 for BMC_CMC):
 * backward sweep over the dates (sample points, continuation estimates, rule
 * fit), then final pricing on an independent stream.  If rules_out is not
 * NULL it receives the learned rules (caller destroys them). */
bmc_status bmc_price(bmc_ctx *ctx, const bmc_spec *spec, const bmc_opts *opts,
                     bmc_rules **rules_out, bmc_result *out);

/* Many options priced together by the CMC pricer (Algorithm 2 for each),
 * synchronous.  specs[count], opts[count] (host; method must be BMC_CMC; each
 * option has its own d, dates, N, n, n_final, seed and precision) and
 * results[count] (host).  The options share every launch: round r learns
 * date N_T - 1 - r of each option that has one (bridge step, one persistent
 * continuation launch per dimension bucket and precision carrying the
 * (option, point, path-chunk) jobs, the boosting fits one block per option),
 * and an option's final pricing joins the round after its last date.  Each
 * result, and each rule table, is bit-identical to bmc_price on the same
 * spec and options.  seconds and the phase times are those of the whole
 * batch.  If rules_out is not NULL it receives count rule tables (caller
 * destroys them).  On error nothing is written. */
bmc_status bmc_price_batch(bmc_ctx *ctx, int32_t count, const bmc_spec *specs, const bmc_opts *opts,
                           bmc_rules **rules_out, bmc_result *results);

/* Launch shape of the continuation kernel: each workgroup job takes 256*ppt
 * paths of one point (ppt = paths per lane, 1..64).  The shape fixes the
 * order of the floating-point sums, so prices with different shapes agree to
 * the parity tolerance but not bit for bit; every call on a context uses
 * the context's table, so a price is the same alone and in a batch.
 * bmc_tuning_set keys an entry by dimension bucket (d = 0: any), precision
 * (-1: any) and n rounded up to a power of two (n = 0: any); ppt = 0 removes
 * the entry.  Without an entry a heuristic picks ppt from N and n.
 * bmc_tuning_get returns the shape a call with (d, precision, N, n) uses. */
bmc_status bmc_tuning_set(bmc_ctx *ctx, int32_t d, int32_t precision, int64_t n, int32_t ppt);
bmc_status bmc_tuning_get(bmc_ctx *ctx, int32_t d, int32_t precision, int64_t N, int64_t n, int32_t *ppt);
/* Autotuner: times the continuation kernel of spec with N points and n
 * paths for every shape ppt = 1, 2, 4, .. up to one job per point (at most
 * 64), at the first, middle and last dates (CMC points, exercise rules from
 * a small CMC pricing of the spec: at most 4096 points, n/8 paths), and
 * stores the shape with the most executed path-steps per
 * second over those dates in ctx's table for the spec's dimension bucket,
 * precision and n class; *ppt_out (may be NULL) receives it.  N = 1 tunes
 * the final pricing (date 0).  Synchronous. */
bmc_status bmc_autotune(bmc_ctx *ctx, const bmc_spec *spec, int32_t precision, int64_t N, int64_t n,
                        int32_t *ppt_out);

/* Serving loop (continuous batching).  A server owns a device arena of
 * hbm_budget bytes and a thread that runs rounds of the batched engine: each
 * round advances every request on the device by one stage (one date to
 * learn, or the final pricing) in shared launches.  Between rounds, queued
 * requests are admitted first come first served while their device
 * footprint (points, paths' partial sums, fit scratch, rule tables) fits
 * the arena and fewer than max_inflight are on the device; requests that
 * arrive while others run join them as memory and slots free up.  Learned
 * rule tables stay on the device in an LRU cache (rule_cache entries, in the
 * arena) keyed by spec, precision, N, n, seed, boosting rounds and launch
 * shape; a request that hits it runs only its final pricing.  Requests are
 * CMC (bmc_opts.method = BMC_CMC).  Every result is bit-identical to
 * bmc_price on the server's context; in a result, seconds = submission to
 * completion and calc_seconds = time queued before admission.  The server
 * uses ctx's device and launch-shape table (copied at creation) and its own
 * stream; ctx stays usable.  Thread-safe: any thread may submit, poll and
 * wait.  Destroy waits for every submitted request to finish. */
typedef struct bmc_server bmc_server;
typedef struct {
    int64_t hbm_budget;     /* device bytes for requests and cached rules (0: 4 GiB) */
    int32_t max_inflight;   /* requests on the device at once (0: 256) */
    int32_t rule_cache;     /* learned rule tables kept (0: 256; -1: no cache) */
} bmc_server_opts;
typedef struct {
    int64_t submitted, rejected, completed, failed;
    int64_t cache_hits, cache_misses, cached_rules;
    int64_t rounds, inner_path_steps, final_path_steps;
    int64_t queued, inflight, hbm_in_use, hbm_peak;
    double busy_seconds;    /* wall time of the server's rounds */
    int64_t canceled;       /* requests ended by bmc_server_cancel */
} bmc_server_stats;
bmc_status bmc_server_create(bmc_ctx *ctx, const bmc_server_opts *opts, bmc_server **out);
void bmc_server_destroy(bmc_server *server);
/* Queues a request (spec and opts are copied); BMC_ENOMEM if its footprint
 * exceeds the whole arena.  *ticket identifies it. */
bmc_status bmc_server_submit(bmc_server *server, const bmc_spec *spec, const bmc_opts *opts, uint64_t *ticket);
/* BMC_EBUSY while the request is queued or running; otherwise its status
 * (the result is written on BMC_OK) and the ticket is released. */
bmc_status bmc_server_poll(bmc_server *server, uint64_t ticket, bmc_result *out);
/* As poll, blocking up to timeout_s seconds (< 0: no limit). */
bmc_status bmc_server_wait(bmc_server *server, uint64_t ticket, double timeout_s, bmc_result *out);
/* Cancels a request, which then ends with BMC_ECANCELED (poll and wait
 * return it and release the ticket).  A queued request leaves the queue at
 * once.  For a request on the device a one-thread kernel on a control stream
 * sets a cancel word in its device memory: the continuation jobs of its
 * pricing read the word while they load their tables and stop before their
 * paths, so the launch in flight skips the request's remaining work, and at
 * the end of the round the server frees its device memory and slot and
 * caches none of its rules.  The other requests' results are unchanged.
 * BMC_EINVAL for an unknown ticket or a request that has already finished
 * (its result stays available). */
bmc_status bmc_server_cancel(bmc_server *server, uint64_t ticket);
bmc_status bmc_server_stats_get(bmc_server *server, bmc_server_stats *out);

/* Exercise-rule table of one spec and method: one row of width w per date
 * (rows 1..N_T-1 used).  CMC (Section 3.2): F(x) = sum_f w_f phi_f(x) with
 * phi = [1, u_1..u_d, u_1^2..u_d^2, g, g^2], u_i = ln(S_i/K), g = Phi(S)/K;
 * exercise iff Phi > 0 and F > 0.  CMC_ADA: AdaBoost stumps on
 * psi = [u_1..u_d, g] folded into per-feature threshold tables, row
 * [base, c_0..c_d, then per feature f (in order) its c_f thresholds theta in
 * ascending order followed by the c_f running sums R of their increments
 * delta = 2 alpha s in that order, zeros] of 1 + (d + 1) + 2 * 64 entries;
 * F(x) = base + sum over f of R_f[k_f - 1], k_f the number of thresholds
 * with psi_f(x) >= theta (no term when k_f = 0); exercise iff Phi > 0 and
 * F > 0.  I&Z (Section 2.2): one boundary block of
 * p = 1 + q + q(q+1)/2 coefficients (q = d - 1) per exercise region, region r
 * at offset r p of the row; b_r(x) = sum_f w_f xi_f with
 * xi = [1, v_1..v_q, v_a v_c (a <= c)] over v = ln(S_i/K) of the assets
 * i != r in increasing order.  The put family has one region (r = 0): it
 * exercises iff Phi > 0 and ln S_1 < b_0.  The max-call has d regions: with
 * r the largest asset (the first on ties) it exercises iff Phi > 0 and
 * ln S_r > b_r.  A new table never exercises. */
bmc_status bmc_rules_create(bmc_ctx *ctx, const bmc_spec *spec, int32_t method, bmc_rules **out);
void bmc_rules_destroy(bmc_rules *rules);
int32_t bmc_rules_width(const bmc_rules *rules);
/* Row `date` (1..N_T-1) from/to host memory (synchronous). */
bmc_status bmc_rules_set(bmc_rules *rules, int32_t date, const double *w_host);
bmc_status bmc_rules_get(const bmc_rules *rules, int32_t date, double *w_host);
/* Serialised form (header + FP64 rows).  *bytes: in = capacity, out = size;
 * buf = NULL queries the size. */
bmc_status bmc_rules_export(const bmc_rules *rules, void *buf, size_t *bytes);
bmc_status bmc_rules_import(bmc_ctx *ctx, const void *buf, size_t bytes, bmc_rules **out);

/* Number of I&Z exercise regions of a spec (Section 2.2): d for the
 * max-call, 1 for the put family; 0 for a NULL or empty spec. */
int32_t bmc_iz_regions(const bmc_spec *spec);

/* Sample points at `date` (1..N_T) into device x[d*N].  CMC: training points
 * from the Brownian bridge run back from T (Section 3.2-3.3); region must be
 * 0.  I&Z: rank-1 lattice points (Section 2.3, [glp]) over the assets other
 * than the region's own one (0 <= region < bmc_iz_regions), whose row is set
 * to K. */
bmc_status bmc_sample_points(bmc_ctx *ctx, const bmc_spec *spec, int32_t method, int32_t date,
                             int32_t region, int64_t N, uint64_t seed, double *x);

/* Continuation values at `date` m (0..N_T-1) of the N device points x: n inner
 * paths per point from t_m to T under the rules of later dates (Section 3.2,
 * the "small BA option"; Section 2.3 [calc]).  Writes device cont[N],
 * std_err[N] and, if not NULL, steps[N] (executed path-steps).  m = 0 with a
 * single point is the final-pricing pass (use bmc_final_price). */
bmc_status bmc_estimate_continuation(bmc_ctx *ctx, const bmc_spec *spec, const bmc_rules *rules,
                                     int32_t date, const double *x, int64_t N, int64_t n,
                                     uint64_t seed, int32_t precision,
                                     double *cont, double *std_err, int64_t *steps);

/* Fits the rule row of `date` from N device points.  CMC: region 0,
 * values = device continuation estimates; boosting on the in-the-money points
 * (Section 3.2 [class]): LogitBoost with a linear base learner (BMC_CMC) or
 * AdaBoost with stumps (BMC_CMC_ADA: labels sign(Phi - C), initial weights
 * |Phi - C|, 64 uniform bins per feature between its extremes over the
 * training points, weights rounded to a fixed-point grid so that the stump
 * errors are exact integers; bit-reproducible).  I&Z: fits the boundary block of `region`;
 * x[region*N + j] holds the converged boundary coordinate s*_j (<= 0 marks a
 * dropped point) and values is ignored; quadratic least squares of ln s*
 * (Section 2.3 [reg]).  rounds: boosting rounds, <= 64 (0: 8 for BMC_CMC, 64
 * for BMC_CMC_ADA).  A BMC_CMC fit runs as one launch whose blocks (at most one
 * per CU) meet at grid barriers; the call waits for it and returns
 * BMC_EDEVICE if a barrier gave up because its blocks were not all resident
 * (bmc_price reports the same). */
bmc_status bmc_fit_rule(bmc_ctx *ctx, const bmc_spec *spec, bmc_rules *rules, int32_t date,
                        int32_t region, const double *x, const double *values, int64_t N,
                        int32_t rounds);

/* I&Z boundary-point search of one region at `date` (Section 2.1 eq. (1),
 * Sections 2.2 and 2.4): for each of the J device points x (the region's own
 * asset ignored) iterate s <- Phi^{-1}(C(s)) on that asset from s = K with
 * common random numbers (the region is the fourth Philox counter word) until
 * |s' - s| < eps or max_iter.  Phi^{-1}: (K - c)^d / prod_{i>=2} x_i for the
 * geometric put, d (K - c) - sum_{i>=2} x_i for the arithmetic put, K + c for
 * the max-call.  Writes device s_out[J] (<= 0: dropped, not converged, or a
 * max-call fixed point not above every other asset) and iters[J]; *steps
 * (host, may be NULL) receives the executed path-steps.  Synchronous. */
bmc_status bmc_iz_search(bmc_ctx *ctx, const bmc_spec *spec, const bmc_rules *rules, int32_t date,
                         int32_t region, const double *x, int64_t J, int64_t n, uint64_t seed,
                         int32_t precision, double eps, int32_t max_iter, int32_t mode,
                         double *s_out, int32_t *iters, int64_t *steps);

/* Final pricing [mc] (Algorithms 1-2): n_final paths from S0 on the FINAL
 * stream under the rules; FP64 merge to price, sample variance, standard
 * error and 95% half-width.  Synchronous. */
bmc_status bmc_final_price(bmc_ctx *ctx, const bmc_spec *spec, const bmc_rules *rules,
                           int64_t n_final, uint64_t seed, int32_t precision, bmc_result *out);

/* Continuation values as bmc_estimate_continuation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The call allocates nothing: the device
 * spec tables and the per-job partial sums live in a static device array of
 * BMC_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  The
 * caller passes device x, cont, std_err (and steps or NULL) and rules made
 * beforehand.  Same arguments and results as bmc_estimate_continuation on
 * the same context (identical values); synchronous (it waits for the spec
 * upload, then enqueues on the context's stream).  BMC_ENOMEM if the
 * partial sums, 24 bytes per (point, path chunk) of the launch shape,
 * exceed the array less 256 KB.  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (several contexts or threads) race. */
#define BMC_NOALLOC_SCRATCH_BYTES (16u << 20)
bmc_status bmc_estimate_continuation_noalloc(bmc_ctx *ctx, const bmc_spec *spec, const bmc_rules *rules,
                                             int32_t date, const double *x, int64_t N, int64_t n,
                                             uint64_t seed, int32_t precision, double *cont,
                                             double *std_err, int64_t *steps);

/* Raw generator access for verification: M Philox4x32-10 blocks at device
 * counters ctr[4*M] -> device out[4*M]; and the four Box-Muller normals of
 * each block in the given precision (FP32 results widened to double). */
bmc_status bmc_philox(bmc_ctx *ctx, uint32_t k0, uint32_t k1, const uint32_t *ctr, int64_t M,
                      uint32_t *out);
bmc_status bmc_normals(bmc_ctx *ctx, uint32_t k0, uint32_t k1, const uint32_t *ctr, int64_t M,
                       int32_t precision, double *out);

#ifdef __cplusplus
}
#endif
#endif /* BMC_H */
