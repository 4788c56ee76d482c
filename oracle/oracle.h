/*
 * Plain FP64 CPU oracle for the nested continuation-value Monte Carlo of
 * Doan, Gaikwad, Bossy, Baude & Stokes-Rees, "Parallel Pricing Algorithms for
 * Multi-Dimensional Bermudan/American Options using Monte Carlo methods"
 * (INRIA RR-6530, 2008).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library; the two agree only through the written definitions of the method
 * (random-number layout, payoffs, features, fit and search rules).
 *
 * All arrays are host memory owned by the caller.  Point sets are
 * structure-of-arrays: x[i*N + j] is asset i of point j.
 * Functions return 0 on success and a negative code on bad input.
 */
#ifndef BMC_ORACLE_H
#define BMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PUT_BASKET = 0, ORC_CALL_MAX = 1, ORC_PUT_GEO = 2, ORC_CALL_MIN = 3 };
/* I&Z boundary-point search: plain fixed point, or secant steps on its residual */
enum { ORC_SEARCH_PLAIN = 0, ORC_SEARCH_SECANT = 1 };
enum { ORC_CMC = 0, ORC_IZ = 1, ORC_CMC_ADA = 2 };
/* AdaBoost stumps (ORC_CMC_ADA): bins per feature and the largest number of
 * boosting rounds a rule row holds. */
enum { ORC_ADA_BINS = 64, ORC_ADA_TMAX = 64 };
enum { ORC_STREAM_OUTER = 1, ORC_STREAM_INNER = 2, ORC_STREAM_FINAL = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOTSPD = -2, ORC_ENOMEM = -3,
       ORC_EUNSUPPORTED = -5 };

/* Market model of Section 2.2 / 3.2: d assets under risk-neutral GBM. */
typedef struct {
    int32_t d;
    const double *S0;     /* [d] */
    const double *delta;  /* [d] dividend yields */
    const double *sigma;  /* [d] volatilities */
    const double *rho;    /* [d*d] correlation, row-major */
    double K, r, T;
    int32_t n_dates;      /* N_T exercise dates t_1 < ... < t_NT = T */
    const double *dates;  /* [n_dates] */
    int32_t payoff;       /* ORC_PUT_BASKET / ORC_CALL_MAX / ORC_PUT_GEO / ORC_CALL_MIN */
} orc_spec;

/* Number of rule coefficients per date for a method and dimension (for I&Z:
 * one region's boundary). */
int orc_rule_width(int method, int d);
/* I&Z exercise regions (Section 2.2): d for the calls on the maximum and the
 * minimum, 1 otherwise. */
int orc_iz_regions(const orc_spec *s);
/* Width of a rule row: CMC weights, or the I&Z boundary blocks of every
 * region, region r at offset r * orc_rule_width(ORC_IZ, d). */
int orc_rule_width_spec(const orc_spec *s, int method);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);
/* Four standard normals from one Philox block (Box-Muller on word pairs). */
void orc_normal_block(uint32_t k0, uint32_t k1, const uint32_t ctr[4], double z[4]);

int orc_cholesky(int d, const double *rho, double *L);

/* Payoff of a price vector given in log coordinates. */
double orc_payoff(const orc_spec *s, const double *logS);

/* CMC training points at date m (Brownian bridge run back from T). */
int orc_points_cmc(const orc_spec *s, int m, int64_t N, uint32_t seed, double *x);

/* Korobov generator maximising the minimal toroidal distance. */
int64_t orc_korobov(int64_t J, int q);
/* I&Z lattice points at date m for a region's boundary: the lattice spans
 * the other assets; the region's own asset (asset 0 for the put family) is
 * set to K. */
int orc_points_iz(const orc_spec *s, int m, int region, int64_t J, double *x);

/*
 * Continuation estimate at date m (0 <= m < N_T) for N points x, n inner paths
 * each, under the rule table `rules` ([(N_T+1) * width], row k = date k).
 * m = 0 with stream FINAL and the single point S0 is the final pricing pass.
 * ids (may be NULL) gives each point's index in the random-number counters
 * (default: its position j), so that a subset of a larger point set can be
 * re-evaluated with its original draws.
 * Outputs cont[N], se[N], steps[N] (executed path-steps), sum[N], sumsq[N].
 */
int orc_continuation(const orc_spec *s, int method, const double *rules, int m,
                     const double *x, int64_t N, const uint32_t *ids, int64_t n,
                     uint32_t seed, int stream, int nthreads, double *cont, double *se,
                     int64_t *steps, double *sum, double *sumsq);

/* CMC LogitBoost fit of the exercise rule at one date (folded weights). */
int orc_fit_cmc(const orc_spec *s, const double *x, const double *cont,
                int64_t N, int rounds, double *w);

/* CMC AdaBoost fit with decision stumps at one date (1 <= rounds <= ORC_ADA_TMAX),
 * written as a folded rule row of orc_rule_width(ORC_CMC_ADA, d) entries:
 * [base, count_0..count_d, then per feature f its count_f thresholds in
 * ascending order and the running sums of their increments 2 alpha s]; a
 * point's score is base plus, per feature, the running sum at the number of
 * thresholds its feature value reaches.
 * Optional trace (any pointer may be NULL): *n_stumps, and per stump its
 * feature, first bin of the upper side, sign, weighted error eps and alpha;
 * lo[d+1], hi[d+1]: the feature ranges over the in-the-money points. */
int orc_fit_ada(const orc_spec *s, const double *x, const double *cont, int64_t N,
                int rounds, double *row, int *n_stumps, int *feat, int *bin, int *sign,
                double *eps, double *alpha, double *lo, double *hi);

/* I&Z fixed-point search of a region's boundary coordinate for J points at
 * date m; the inner paths of region r use r as the fourth counter word.
 * mode: ORC_SEARCH_PLAIN or ORC_SEARCH_SECANT.
 * Writes s_out[J] (<= 0 if dropped or unconverged) and iters[J]. */
int orc_iz_search(const orc_spec *s, const double *rules, int m, int region,
                  const double *x, int64_t J, int64_t n, uint32_t seed, double eps,
                  int max_iter, int mode, int nthreads, double *s_out, int32_t *iters,
                  int64_t *steps_total);

/* I&Z quadratic boundary regression of one region over its converged points;
 * b holds orc_rule_width(ORC_IZ, d) coefficients. */
int orc_fit_iz(const orc_spec *s, int region, const double *x, const double *sstar,
               int64_t J, double *b);

/*
 * Whole pricer (Algorithm 1 for ORC_IZ, Algorithm 2 for ORC_CMC).
 * rules_out: [(N_T+1) * orc_rule_width_spec(s, method)] or NULL.
 * result[8] = {price, variance, std_err, ci95, inner_steps, final_steps,
 *              iz_unconverged, iz_iterations}.
 */
int orc_price(const orc_spec *s, int method, int64_t N, int64_t n, int64_t n_final,
              uint32_t seed, int rounds, double eps, int max_iter, int search_mode,
              int nthreads, double *rules_out, double *result);

#ifdef __cplusplus
}
#endif
#endif
