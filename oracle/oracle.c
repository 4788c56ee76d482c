/*
 * Plain FP64 CPU oracle of the nested continuation-value Monte Carlo
 * (Doan et al., INRIA RR-6530, 2008).  TEST INFRASTRUCTURE ONLY: it checks the
 * GPU library and is never part of the product path.
 *
 * Written for a reader holding the paper: every routine follows the method's
 * steps in the paper's order, with no blocking, fusion or reordering.  Build
 * with -ffp-contract=off so that every product and sum rounds as written.
 *
 * Paper map:
 *   GBM market model, payoffs ............ Section 2.2 and Section 3.2
 *   continuation ("small BA option") ...... Section 3.2, data-generation step
 *   CMC stopping rule tau = min{F > 0} .... Section 3.2
 *   CMC training points by Brownian bridge  Section 3.2 and Section 3.3
 *   boosting classification [class] ....... Section 3.2, Algorithm 2
 *   I&Z matched condition P_t(S*) = I(S*) . Section 2.1, eq. (1)
 *   I&Z boundary-point iteration, eps ..... Section 2.4
 *   lattice points [glp], regression [reg]  Section 2.3, Algorithm 1
 *   final pricing [mc] and merge .......... Algorithms 1 and 2
 * Readings where the paper is silent (random-number layout, features, the
 * boosting base learner, lattice choice) are the written definitions the GPU
 * library also follows; each is stated at the routine that implements it.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The paper names no
 * generator; a counter-based one lets every (date, point, path, step) draw be
 * addressed directly.                                                        */

void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): u = (x + 1/2) / 2^32, exact in double. */
static double word_to_uniform(uint32_t x)
{
    return ((double)x + 0.5) * 0x1p-32;
}

/* Box-Muller on word pairs (0,1) and (2,3):
 *   z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1),
 *   z2, z3 likewise from (u2, u3). */
void orc_normal_block(uint32_t k0, uint32_t k1, const uint32_t ctr[4], double z[4])
{
    uint32_t w[4];
    orc_philox(k0, k1, ctr, w);
    const double two_pi = 2.0 * 3.14159265358979323846;
    for (int h = 0; h < 2; ++h) {
        double ua = word_to_uniform(w[2 * h]);
        double ub = word_to_uniform(w[2 * h + 1]);
        double radius = sqrt(-2.0 * log(ua));
        z[2 * h] = radius * cos(two_pi * ub);
        z[2 * h + 1] = radius * sin(two_pi * ub);
    }
}

/* Key: (seed, stream << 16 | date).  The date field keeps the draws of
 * different dates independent. */
static uint32_t key_hi(int stream, int date)
{
    return ((uint32_t)stream << 16) | ((uint32_t)date & 0xFFFFu);
}

/* The d normals of one GBM step.  Step k (absolute date index 1..N_T) of path
 * p from point j uses B = ceil(d/4) blocks with counters (k*B + b, p, j, 0);
 * asset i takes normal i mod 4 of block i / 4. */
static void step_normals(int d, uint32_t k0, uint32_t k1, int k, uint32_t p,
                         uint32_t j, uint32_t slot, double *z)
{
    int nblk = (d + 3) / 4;
    for (int b = 0; b < nblk; ++b) {
        uint32_t ctr[4] = {(uint32_t)(k * nblk + b), p, j, slot};
        double blk[4];
        orc_normal_block(k0, k1, ctr, blk);
        for (int w = 0; w < 4 && 4 * b + w < d; ++w)
            z[4 * b + w] = blk[w];
    }
}

/* ------------------------------------------------------------------------- */
/* Correlation: lower Cholesky factor L with L L^T = rho.                     */

int orc_cholesky(int d, const double *rho, double *L)
{
    for (int i = 0; i < d * d; ++i) L[i] = 0.0;
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j <= i; ++j) {
            double acc = rho[i * d + j];
            for (int l = 0; l < j; ++l) acc -= L[i * d + l] * L[j * d + l];
            if (i == j) {
                if (!(acc > 0.0)) return ORC_ENOTSPD;
                L[i * d + i] = sqrt(acc);
            } else {
                L[i * d + j] = acc / L[j * d + j];
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Spec helpers.                                                              */

static double date_of(const orc_spec *s, int k)
{
    return k == 0 ? 0.0 : s->dates[k - 1];
}

static int check_spec(const orc_spec *s)
{
    if (!s || s->d < 1 || s->d > 64 || s->n_dates < 1 || s->n_dates > 65535) return ORC_EINVAL;
    if (!(s->K > 0.0) || !(s->T > 0.0)) return ORC_EINVAL;
    double prev = 0.0;
    for (int k = 0; k < s->n_dates; ++k) {
        if (!(s->dates[k] > prev)) return ORC_EINVAL;
        prev = s->dates[k];
    }
    if (fabs(prev - s->T) > 1e-12 * s->T) return ORC_EINVAL;
    for (int i = 0; i < s->d; ++i) {
        if (!(s->sigma[i] >= 0.0) || !(s->S0[i] > 0.0)) return ORC_EINVAL;
        if (fabs(s->rho[i * s->d + i] - 1.0) > 1e-12) return ORC_EINVAL;
        for (int j = 0; j < i; ++j)
            if (fabs(s->rho[i * s->d + j] - s->rho[j * s->d + i]) > 1e-12) return ORC_EINVAL;
    }
    if (s->payoff < ORC_PUT_BASKET || s->payoff > ORC_CALL_MIN) return ORC_EINVAL;
    return ORC_OK;
}

/* Payoffs of Sections 2.1-2.2 and 3.2, evaluated from S_i = exp(logS_i):
 * arithmetic basket put (K - mean S)^+, max-call (max S - K)^+,
 * geometric-average put (K - (prod S)^(1/d))^+. */
double orc_payoff(const orc_spec *s, const double *logS)
{
    int d = s->d;
    double v = 0.0;
    if (s->payoff == ORC_PUT_BASKET) {
        double mean = 0.0;
        for (int i = 0; i < d; ++i) mean += exp(logS[i]);
        mean /= d;
        v = s->K - mean;
    } else if (s->payoff == ORC_CALL_MAX) {
        double mx = exp(logS[0]);
        for (int i = 1; i < d; ++i) {
            double Si = exp(logS[i]);
            if (Si > mx) mx = Si;
        }
        v = mx - s->K;
    } else if (s->payoff == ORC_CALL_MIN) {
        double mn = exp(logS[0]);
        for (int i = 1; i < d; ++i) {
            double Si = exp(logS[i]);
            if (Si < mn) mn = Si;
        }
        v = mn - s->K;
    } else {
        double meanlog = 0.0;
        for (int i = 0; i < d; ++i) meanlog += logS[i];
        v = s->K - exp(meanlog / d);
    }
    return v > 0.0 ? v : 0.0;
}

int orc_rule_width(int method, int d)
{
    if (method == ORC_CMC) return 2 * d + 3;
    if (method == ORC_CMC_ADA) return 1 + (d + 1) + 2 * ORC_ADA_TMAX;
    int q = d - 1;
    return 1 + q + q * (q + 1) / 2;
}

/* I&Z regions (Section 2.2): the call on the maximum of d assets has d
 * exercise regions, region i where asset i is the largest, each with its own
 * boundary in the other d - 1 assets; the call on the minimum likewise with
 * region i where asset i is the smallest; the put family has one boundary in
 * assets 2..d.  A rule row holds one block of orc_rule_width(IZ, d)
 * coefficients per region. */
int orc_iz_regions(const orc_spec *s)
{
    return (s->payoff == ORC_CALL_MAX || s->payoff == ORC_CALL_MIN) ? s->d : 1;
}

int orc_rule_width_spec(const orc_spec *s, int method)
{
    if (method != ORC_IZ) return orc_rule_width(method, s->d);
    return orc_iz_regions(s) * orc_rule_width(ORC_IZ, s->d);
}

/* CMC features (reading of Section 3.2; the paper defers the classifier's
 * inputs to the Picazo reference): with u_i = ln(S_i / K) and g = Phi(S)/K,
 *   phi(S) = [1, u_1..u_d, u_1^2..u_d^2, g, g^2]. */
static void cmc_features(const orc_spec *s, const double *logS, double payoff, double *phi)
{
    int d = s->d;
    double lnK = log(s->K);
    phi[0] = 1.0;
    for (int i = 0; i < d; ++i) {
        double u = logS[i] - lnK;
        phi[1 + i] = u;
        phi[1 + d + i] = u * u;
    }
    double g = payoff / s->K;
    phi[1 + 2 * d] = g;
    phi[2 + 2 * d] = g * g;
}

/* I&Z boundary features of region r: full quadratic in v = ln(S_i/K) of the
 * assets i != r in increasing order, [1, v_1..v_q, v_a v_b for a <= b]
 * (region 0 of the put family: assets 2..d). */
static void iz_features(const orc_spec *s, const double *logS, int region, double *xi)
{
    int q = s->d - 1;
    double lnK = log(s->K);
    xi[0] = 1.0;
    for (int a = 0; a < q; ++a) xi[1 + a] = logS[a < region ? a : a + 1] - lnK;
    int f = 1 + q;
    for (int a = 0; a < q; ++a)
        for (int b = a; b < q; ++b) xi[f++] = xi[1 + a] * xi[1 + b];
}

/* AdaBoost stump features: psi = [u_1..u_d, g], u_i = ln(S_i/K), g = Phi/K. */
static void ada_features(const orc_spec *s, const double *logS, double payoff, double *psi)
{
    int d = s->d;
    double lnK = log(s->K);
    for (int i = 0; i < d; ++i) psi[i] = logS[i] - lnK;
    psi[d] = payoff / s->K;
}

/* I&Z: puts search the first asset and exercise below its boundary; the
 * calls on the maximum and the minimum search the asset of the region and
 * exercise above it. */
static int iz_direction_is_call(const orc_spec *s)
{
    return s->payoff == ORC_CALL_MAX || s->payoff == ORC_CALL_MIN;
}

static const double IZ_NEVER = 1e300;

/* Exercise test at an intermediate date (Section 3.2 stopping time for CMC;
 * crossing of the regressed boundary for I&Z).  Ties continue. */
static int exercise_now(const orc_spec *s, int method, const double *row,
                        const double *logS, double payoff)
{
    if (!(payoff > 0.0)) return 0;
    if (method == ORC_CMC) {
        double phi[2 * 64 + 3];
        cmc_features(s, logS, payoff, phi);
        int p = orc_rule_width(ORC_CMC, s->d);
        double F = 0.0;
        for (int f = 0; f < p; ++f) F += row[f] * phi[f];
        return F > 0.0;
    }
    if (method == ORC_CMC_ADA) {
        /* folded stumps: F = base + sum over features of the running sum at
         * the number of thresholds the feature reaches */
        double psi[65];
        ada_features(s, logS, payoff, psi);
        int nf = s->d + 1, at = 1 + nf;
        double F = row[0];
        for (int f = 0; f < nf; ++f) {
            int cnt = (int)row[1 + f], k = 0;
            for (int e = 0; e < cnt; ++e)
                if (psi[f] >= row[at + e]) ++k;
            if (k > 0) F += row[at + cnt + k - 1];
            at += 2 * cnt;
        }
        return F > 0.0;
    }
    double xi[1 + 63 + 63 * 64 / 2];
    int p = orc_rule_width(ORC_IZ, s->d);
    int region = 0;
    /* region of the largest (max-call) or smallest (min-call) asset, the
     * first one on ties */
    if (s->payoff == ORC_CALL_MAX)
        for (int i = 1; i < s->d; ++i)
            if (logS[i] > logS[region]) region = i;
    if (s->payoff == ORC_CALL_MIN)
        for (int i = 1; i < s->d; ++i)
            if (logS[i] < logS[region]) region = i;
    iz_features(s, logS, region, xi);
    const double *b = row + (size_t)region * p;
    double bnd = 0.0;
    for (int f = 0; f < p; ++f) bnd += b[f] * xi[f];
    if (iz_direction_is_call(s)) return logS[region] > bnd;
    return logS[0] < bnd;
}

/* ------------------------------------------------------------------------- */
/* Inner paths: the "small BA option" on [t_m, T] started at one point.       */

typedef struct {
    const orc_spec *s;
    int method;
    const double *rules;
    int width;
    int m;
    const double *L;     /* d*d */
    uint32_t k0, k1;
    uint32_t slot;       /* fourth counter word: I&Z region (0 otherwise) */
} path_ctx;

/* Runs paths p_lo..p_hi-1 of point j from log-point logx; accumulates the
 * discounted payoffs (sum, sum of squares) and executed path-steps. */
static void run_paths(const path_ctx *c, const double *logx, uint32_t j,
                      int64_t p_lo, int64_t p_hi, double *sum, double *sumsq,
                      int64_t *steps)
{
    const orc_spec *s = c->s;
    int d = s->d, NT = s->n_dates, m = c->m;
    double logS[64], z[64];
    double tm = date_of(s, m);
    for (int64_t p = p_lo; p < p_hi; ++p) {
        for (int i = 0; i < d; ++i) logS[i] = logx[i];
        for (int k = m + 1; k <= NT; ++k) {
            double dt = date_of(s, k) - date_of(s, k - 1);
            step_normals(d, c->k0, c->k1, k, (uint32_t)p, j, c->slot, z);
            for (int i = 0; i < d; ++i) {
                double corr = 0.0;
                for (int l = 0; l <= i; ++l) corr += c->L[i * d + l] * z[l];
                double drift = s->r - s->delta[i] - 0.5 * s->sigma[i] * s->sigma[i];
                logS[i] += drift * dt + s->sigma[i] * sqrt(dt) * corr;
            }
            double payoff = orc_payoff(s, logS);
            int stop = (k == NT);
            if (!stop) stop = exercise_now(s, c->method, c->rules + (size_t)k * c->width, logS, payoff);
            if (stop) {
                double pay = exp(-s->r * (date_of(s, k) - tm)) * payoff;
                *sum += pay;
                *sumsq += pay * pay;
                *steps += k - m;
                break;
            }
        }
    }
}

static int resolve_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    return 1;
}

/* Work split: items are (point, chunk of CHUNK paths).  Partial sums of each
 * chunk are merged in chunk order, so results do not depend on the thread
 * count. */
enum { CHUNK = 4096 };

typedef struct {
    const path_ctx *c;
    const double *x;
    const uint32_t *ids;
    int64_t N, n, nchunk;
    double *psum, *psq;
    int64_t *pst;
    int64_t next_item;
    pthread_mutex_t lock;
} cont_job;

static void *cont_worker(void *arg)
{
    cont_job *job = (cont_job *)arg;
    int d = job->c->s->d;
    double logx[64];
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t item = job->next_item++;
        pthread_mutex_unlock(&job->lock);
        if (item >= job->N * job->nchunk) break;
        int64_t j = item / job->nchunk, ch = item % job->nchunk;
        for (int i = 0; i < d; ++i) logx[i] = log(job->x[(size_t)i * job->N + j]);
        int64_t lo = ch * CHUNK, hi = lo + CHUNK < job->n ? lo + CHUNK : job->n;
        double sum = 0.0, sq = 0.0;
        int64_t st = 0;
        uint32_t jid = job->ids ? job->ids[j] : (uint32_t)j;
        run_paths(job->c, logx, jid, lo, hi, &sum, &sq, &st);
        job->psum[item] = sum;
        job->psq[item] = sq;
        job->pst[item] = st;
    }
    return NULL;
}

int orc_continuation(const orc_spec *s, int method, const double *rules, int m,
                     const double *x, int64_t N, const uint32_t *ids, int64_t n,
                     uint32_t seed, int stream, int nthreads, double *cont, double *se,
                     int64_t *steps, double *sum, double *sumsq)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (m < 0 || m >= s->n_dates || N < 1 || n < 2 || n > 0xFFFFFFFFll || N > 0xFFFFFFFFll)
        return ORC_EINVAL;
    int d = s->d;
    double *L = malloc(sizeof(double) * d * d);
    if (!L) return ORC_ENOMEM;
    rc = orc_cholesky(d, s->rho, L);
    if (rc) { free(L); return rc; }
    path_ctx c = {s, method, rules, orc_rule_width_spec(s, method), m, L, seed, key_hi(stream, m), 0u};
    cont_job job;
    job.c = &c; job.x = x; job.ids = ids; job.N = N; job.n = n;
    job.nchunk = (n + CHUNK - 1) / CHUNK;
    job.psum = malloc(sizeof(double) * N * job.nchunk);
    job.psq = malloc(sizeof(double) * N * job.nchunk);
    job.pst = malloc(sizeof(int64_t) * N * job.nchunk);
    job.next_item = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (!job.psum || !job.psq || !job.pst) {
        free(job.psum); free(job.psq); free(job.pst); free(L);
        return ORC_ENOMEM;
    }
    int nt = resolve_threads(nthreads);
    if (nt > N * job.nchunk) nt = (int)(N * job.nchunk);
    pthread_t *th = malloc(sizeof(pthread_t) * nt);
    for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, cont_worker, &job);
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    free(th);
    for (int64_t j = 0; j < N; ++j) {
        double a = 0.0, b = 0.0;
        int64_t st = 0;
        for (int64_t ch = 0; ch < job.nchunk; ++ch) {
            a += job.psum[j * job.nchunk + ch];
            b += job.psq[j * job.nchunk + ch];
            st += job.pst[j * job.nchunk + ch];
        }
        double mean = a / (double)n;
        double var = (b - a * a / (double)n) / (double)(n - 1);
        if (var < 0.0) var = 0.0;
        if (cont) cont[j] = mean;
        if (se) se[j] = sqrt(var / (double)n);
        if (steps) steps[j] = st;
        if (sum) sum[j] = a;
        if (sumsq) sumsq[j] = b;
    }
    pthread_mutex_destroy(&job.lock);
    free(job.psum); free(job.psq); free(job.pst); free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* CMC training points: independent Brownian components B, drawn at T and
 * bridged backward date by date (Sections 3.2-3.3):
 *   B_T = sqrt(T) Z,
 *   B_{t_m} = (t_m / t_{m+1}) B_{t_{m+1}} + sqrt(t_m (t_{m+1} - t_m) / t_{m+1}) Z,
 *   x_i = S0_i exp((r - delta_i - sigma_i^2/2) t_m + sigma_i (L B_{t_m})_i).
 * Z of point j at date m: OUTER stream, key date m, counters (b, 0, j, 0). */

static void outer_normals(int d, uint32_t seed, int date, uint32_t j, double *z)
{
    int nblk = (d + 3) / 4;
    uint32_t k1 = key_hi(ORC_STREAM_OUTER, date);
    for (int b = 0; b < nblk; ++b) {
        uint32_t ctr[4] = {(uint32_t)b, 0u, j, 0u};
        double blk[4];
        orc_normal_block(seed, k1, ctr, blk);
        for (int w = 0; w < 4 && 4 * b + w < d; ++w) z[4 * b + w] = blk[w];
    }
}

static void bridge_endpoint(const orc_spec *s, int64_t N, uint32_t seed, double *B)
{
    int d = s->d, NT = s->n_dates;
    double z[64];
    double tN = date_of(s, NT);
    for (int64_t j = 0; j < N; ++j) {
        outer_normals(d, seed, NT, (uint32_t)j, z);
        for (int i = 0; i < d; ++i) B[(size_t)i * N + j] = sqrt(tN) * z[i];
    }
}

/* B holds date m+1 on entry and date m on exit. */
static void bridge_back(const orc_spec *s, int m, int64_t N, uint32_t seed, double *B)
{
    int d = s->d;
    double z[64];
    double t0 = date_of(s, m), t1 = date_of(s, m + 1);
    double mean_f = t0 / t1;
    double sd = sqrt(t0 * (t1 - t0) / t1);
    for (int64_t j = 0; j < N; ++j) {
        outer_normals(d, seed, m, (uint32_t)j, z);
        for (int i = 0; i < d; ++i)
            B[(size_t)i * N + j] = mean_f * B[(size_t)i * N + j] + sd * z[i];
    }
}

static void points_from_bridge(const orc_spec *s, const double *L, int m, int64_t N,
                               const double *B, double *x)
{
    int d = s->d;
    double tm = date_of(s, m);
    for (int64_t j = 0; j < N; ++j) {
        for (int i = 0; i < d; ++i) {
            double w = 0.0;
            for (int l = 0; l <= i; ++l) w += L[i * d + l] * B[(size_t)l * N + j];
            double drift = s->r - s->delta[i] - 0.5 * s->sigma[i] * s->sigma[i];
            x[(size_t)i * N + j] = s->S0[i] * exp(drift * tm + s->sigma[i] * w);
        }
    }
}

int orc_points_cmc(const orc_spec *s, int m, int64_t N, uint32_t seed, double *x)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (m < 1 || m > s->n_dates || N < 1) return ORC_EINVAL;
    int d = s->d;
    double *L = malloc(sizeof(double) * d * d);
    double *B = malloc(sizeof(double) * d * N);
    if (!L || !B) { free(L); free(B); return ORC_ENOMEM; }
    rc = orc_cholesky(d, s->rho, L);
    if (!rc) {
        bridge_endpoint(s, N, seed, B);
        for (int mm = s->n_dates - 1; mm >= m; --mm) bridge_back(s, mm, N, seed, B);
        points_from_bridge(s, L, m, N, B, x);
    }
    free(L); free(B);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* I&Z lattice points [glp] (Section 2.3).  The paper takes them from SSJ or
 * quantization files; here a rank-1 Korobov lattice in the q = d-1 free
 * coordinates, u_j = frac((j g + 1/2) / J) with g = (1, a, a^2, ...) mod J,
 * whose generator a maximises the minimal toroidal distance (ties: smallest
 * a).  Coordinates map to prices through the lognormal quantile of S_{t_m}. */

int64_t orc_korobov(int64_t J, int q)
{
    if (q <= 1 || J <= 2) return 1;
    int64_t best_a = 1, best = -1;
    int64_t g[64];
    for (int64_t a = 1; a < J; ++a) {
        g[0] = 1;
        for (int i = 1; i < q; ++i) g[i] = (g[i - 1] * a) % J;
        int64_t dmin = INT64_MAX;
        for (int64_t jj = 1; jj < J && dmin > best; ++jj) {
            int64_t dist = 0;
            for (int i = 0; i < q; ++i) {
                int64_t v = (jj * g[i]) % J;
                if (J - v < v) v = J - v;
                dist += v * v;
            }
            if (dist < dmin) dmin = dist;
        }
        if (dmin > best) { best = dmin; best_a = a; }
    }
    return best_a;
}

static double norm_cdf(double x)
{
    return 0.5 * erfc(-x / sqrt(2.0));
}

/* Inverse standard normal CDF by bisection on the CDF. */
static double norm_inv(double u)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (norm_cdf(mid) < u) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

int orc_points_iz(const orc_spec *s, int m, int region, int64_t J, double *x)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (m < 1 || m > s->n_dates || J < 1 || region < 0 || region >= orc_iz_regions(s))
        return ORC_EINVAL;
    int d = s->d, q = d - 1;
    double tm = date_of(s, m);
    int64_t a = orc_korobov(J, q);
    int64_t g[64];
    if (q > 0) {
        g[0] = 1;
        for (int i = 1; i < q; ++i) g[i] = (g[i - 1] * a) % J;
    }
    for (int64_t j = 0; j < J; ++j) {
        x[(size_t)region * J + j] = s->K;
        for (int i = 0; i < q; ++i) {
            double u = ((double)((j * g[i]) % J) + 0.5) / (double)J;
            int asset = i < region ? i : i + 1;
            double drift = s->r - s->delta[asset] - 0.5 * s->sigma[asset] * s->sigma[asset];
            x[(size_t)asset * J + j] =
                s->S0[asset] * exp(drift * tm + s->sigma[asset] * sqrt(tm) * norm_inv(u));
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Small dense solver: Cholesky of (A + lambda I), then two triangular solves. */

static int spd_solve(int p, const double *A, double lambda, const double *b, double *out)
{
    double *C = malloc(sizeof(double) * p * p);
    double *y = malloc(sizeof(double) * p);
    if (!C || !y) { free(C); free(y); return ORC_ENOMEM; }
    for (int i = 0; i < p * p; ++i) C[i] = A[i];
    for (int i = 0; i < p; ++i) C[i * p + i] += lambda;
    double *L = malloc(sizeof(double) * p * p);
    if (!L) { free(C); free(y); return ORC_ENOMEM; }
    int rc = orc_cholesky(p, C, L);   /* generic factor; C need not have unit diagonal */
    if (rc) { free(C); free(y); free(L); return rc; }
    for (int i = 0; i < p; ++i) {
        double acc = b[i];
        for (int l = 0; l < i; ++l) acc -= L[i * p + l] * y[l];
        y[i] = acc / L[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
        double acc = y[i];
        for (int l = i + 1; l < p; ++l) acc -= L[l * p + i] * out[l];
        out[i] = acc / L[i * p + i];
    }
    free(C); free(y); free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* CMC classification [class] (Section 3.2, Algorithm 2).  The paper uses
 * AdaBoost or LogitBoost with parameters from the Picazo reference.  Reading:
 * LogitBoost (Friedman, Hastie, Tibshirani 2000) with a weighted
 * least-squares linear base learner on the standardised features, fitted on
 * the in-the-money training points.  Label e_j = 1 iff Phi(x_j) - C_j > 0.
 * Each round:  w = max(pi(1-pi), 1e-10),  z = clip((e - pi)/w, -4, 4),
 *   beta = (Psi^T W Psi + lambda I)^-1 Psi^T W z,  lambda = 1e-8 tr(.)/p,
 *   F += beta/2,  pi = 1/(1 + exp(-2F)).
 * The standardisation is folded into the returned weights so that
 * F(x) = sum_f w_f phi_f(x) on raw features; exercise iff Phi > 0 and F > 0. */

int orc_fit_cmc(const orc_spec *s, const double *x, const double *cont,
                int64_t N, int rounds, double *w)
{
    int rc = check_spec(s);
    if (rc) return rc;
    int d = s->d, p = orc_rule_width(ORC_CMC, d);
    for (int f = 0; f < p; ++f) w[f] = 0.0;
    double logS[64];
    /* in-the-money training points */
    int64_t nI = 0;
    double *phi = malloc(sizeof(double) * p * N);
    double *lab = malloc(sizeof(double) * N);
    if (!phi || !lab) { free(phi); free(lab); return ORC_ENOMEM; }
    for (int64_t j = 0; j < N; ++j) {
        for (int i = 0; i < d; ++i) logS[i] = log(x[(size_t)i * N + j]);
        double payoff = orc_payoff(s, logS);
        if (!(payoff > 0.0)) continue;
        cmc_features(s, logS, payoff, phi + (size_t)nI * p);
        lab[nI] = (payoff - cont[j] > 0.0) ? 1.0 : 0.0;
        ++nI;
    }
    if (nI == 0) { free(phi); free(lab); return ORC_OK; }   /* never exercise */
    /* standardise columns 1..p-1 over the fitted points */
    double *mu = calloc(p, sizeof(double)), *sd = calloc(p, sizeof(double));
    for (int f = 1; f < p; ++f) {
        double acc = 0.0;
        for (int64_t j = 0; j < nI; ++j) acc += phi[(size_t)j * p + f];
        mu[f] = acc / (double)nI;
        double v = 0.0;
        for (int64_t j = 0; j < nI; ++j) {
            double dv = phi[(size_t)j * p + f] - mu[f];
            v += dv * dv;
        }
        sd[f] = sqrt(v / (double)nI);
        if (!(sd[f] > 1e-12 * (1.0 + fabs(mu[f])))) sd[f] = 1.0;
        for (int64_t j = 0; j < nI; ++j)
            phi[(size_t)j * p + f] = (phi[(size_t)j * p + f] - mu[f]) / sd[f];
    }
    double *F = calloc(nI, sizeof(double)), *pi = malloc(sizeof(double) * nI);
    double *A = malloc(sizeof(double) * p * p), *bv = malloc(sizeof(double) * p);
    double *beta = malloc(sizeof(double) * p), *gam = calloc(p, sizeof(double));
    for (int64_t j = 0; j < nI; ++j) pi[j] = 0.5;
    rc = ORC_OK;
    for (int round = 0; round < rounds; ++round) {
        for (int f = 0; f < p * p; ++f) A[f] = 0.0;
        for (int f = 0; f < p; ++f) bv[f] = 0.0;
        for (int64_t j = 0; j < nI; ++j) {
            double wj = pi[j] * (1.0 - pi[j]);
            if (wj < 1e-10) wj = 1e-10;
            double zj = (lab[j] - pi[j]) / wj;
            if (zj > 4.0) zj = 4.0;
            if (zj < -4.0) zj = -4.0;
            const double *ps = phi + (size_t)j * p;
            for (int a = 0; a < p; ++a) {
                bv[a] += wj * zj * ps[a];
                for (int b = 0; b < p; ++b) A[a * p + b] += wj * ps[a] * ps[b];
            }
        }
        double tr = 0.0;
        for (int a = 0; a < p; ++a) tr += A[a * p + a];
        rc = spd_solve(p, A, 1e-8 * tr / p, bv, beta);
        if (rc) break;
        for (int a = 0; a < p; ++a) gam[a] += 0.5 * beta[a];
        for (int64_t j = 0; j < nI; ++j) {
            double dF = 0.0;
            for (int a = 0; a < p; ++a) dF += beta[a] * phi[(size_t)j * p + a];
            F[j] += 0.5 * dF;
            pi[j] = 1.0 / (1.0 + exp(-2.0 * F[j]));
        }
    }
    if (!rc) {
        double w0 = gam[0];
        for (int f = 1; f < p; ++f) {
            w[f] = gam[f] / sd[f];
            w0 -= gam[f] * mu[f] / sd[f];
        }
        w[0] = w0;
    }
    free(phi); free(lab); free(mu); free(sd); free(F); free(pi);
    free(A); free(bv); free(beta); free(gam);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* [class] with AdaBoost and decision stumps (Section 3.2 names AdaBoost or
 * LogitBoost; the stump form and its constants are this library's reading).
 *
 * Training set: the in-the-money points; label y_j = +1 (exercise) iff
 * Phi_j - C_j > 0, else -1; initial weight c_j = |Phi_j - C_j|, the value lost
 * by taking the wrong decision at x_j.  A stump on feature f is
 * h(x) = s for psi_f(x) in bins k..B-1 and -s below, with B = 64 uniform bins
 * between the smallest and largest psi_f over the training points; k = 0 is
 * the constant stump (taken on feature 0 only).  Each round takes the stump
 * of least weighted error, ties to the smaller (f, k) and to s = +1, with
 * weights rounded to a fixed-point grid 2^-shift (shift from the largest
 * possible total weight), so that every error is an exact integer;
 * eps = error / total, alpha = ln((1 - eps) / eps) / 2 (eps >= 1e-10), and
 * the AdaBoost update in its normalised form, w / (2 eps) for misclassified
 * points and w / (2 (1 - eps)) for the others.  Boosting stops when no stump
 * beats chance (2 error >= total) or after a perfect stump. */

static int ada_bin(double v, double lo, double hi, double inv)
{
    if (!(hi > lo)) return 0;
    double t = floor((v - lo) * inv);
    if (t < 0.0) return 0;
    if (t > ORC_ADA_BINS - 1) return ORC_ADA_BINS - 1;
    return (int)t;
}

int orc_fit_ada(const orc_spec *s, const double *x, const double *cont, int64_t N,
                int rounds, double *row, int *n_stumps, int *feat, int *bin, int *sign,
                double *eps_out, double *alpha_out, double *lo_out, double *hi_out)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (rounds < 1 || rounds > ORC_ADA_TMAX || N < 1) return ORC_EINVAL;
    const int d = s->d, nf = d + 1, B = ORC_ADA_BINS, width = orc_rule_width(ORC_CMC_ADA, d);
    for (int f = 0; f < width; ++f) row[f] = 0.0;
    if (n_stumps) *n_stumps = 0;
    double *psi = malloc(sizeof(double) * nf * N), *w = malloc(sizeof(double) * N);
    int *y = malloc(sizeof(int) * N), *bins = malloc(sizeof(int) * nf * N);
    int64_t *W = malloc(sizeof(int64_t) * N), *H = malloc(sizeof(int64_t) * nf * B * 2);
    if (!psi || !w || !y || !bins || !W || !H) {
        free(psi); free(w); free(y); free(bins); free(W); free(H);
        return ORC_ENOMEM;
    }
    double logS[64];
    int64_t nI = 0;
    double cmax = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        for (int i = 0; i < d; ++i) logS[i] = log(x[(size_t)i * N + j]);
        double payoff = orc_payoff(s, logS);
        if (!(payoff > 0.0)) continue;
        double pz[65];
        ada_features(s, logS, payoff, pz);
        for (int f = 0; f < nf; ++f) psi[(size_t)f * N + nI] = pz[f];
        double beta = payoff - cont[j];
        y[nI] = beta > 0.0 ? 1 : -1;
        w[nI] = fabs(beta);
        if (w[nI] > cmax) cmax = w[nI];
        ++nI;
    }
    double lo[65], hi[65], inv[65];
    for (int f = 0; f < nf; ++f) {
        lo[f] = hi[f] = 0.0;
        for (int64_t j = 0; j < nI; ++j) {
            double v = psi[(size_t)f * N + j];
            if (j == 0 || v < lo[f]) lo[f] = v;
            if (j == 0 || v > hi[f]) hi[f] = v;
        }
        inv[f] = hi[f] > lo[f] ? (double)B / (hi[f] - lo[f]) : 0.0;
        if (lo_out) lo_out[f] = lo[f];
        if (hi_out) hi_out[f] = hi[f];
        for (int64_t j = 0; j < nI; ++j)
            bins[(size_t)f * N + j] = ada_bin(psi[(size_t)f * N + j], lo[f], hi[f], inv[f]);
    }
    int T = 0;
    int tf[ORC_ADA_TMAX], tk[ORC_ADA_TMAX], ts[ORC_ADA_TMAX];
    double ta[ORC_ADA_TMAX];
    if (nI > 0 && cmax > 0.0) {
        int e2;
        frexp((double)nI * cmax, &e2);       /* total weight < 2^e2 */
        const int shift = 50 - e2;
        for (int t = 0; t < rounds; ++t) {
            int64_t Wp = 0, Wm = 0;
            memset(H, 0, sizeof(int64_t) * nf * B * 2);
            for (int64_t j = 0; j < nI; ++j) {
                W[j] = (int64_t)llrint(ldexp(w[j], shift));
                int c = y[j] > 0;
                if (c) Wp += W[j]; else Wm += W[j];
                for (int f = 0; f < nf; ++f) H[((size_t)f * B + bins[(size_t)f * N + j]) * 2 + c] += W[j];
            }
            const int64_t Wt = Wp + Wm;
            if (Wt == 0) break;
            int64_t best = -1;
            int bf = 0, bk = 0, bs = 1;
            for (int f = 0; f < nf; ++f) {
                int64_t Pp = 0, Pm = 0;
                for (int k = 0; k < B; ++k) {
                    if (k > 0) {
                        Pp += H[((size_t)f * B + k - 1) * 2 + 1];
                        Pm += H[((size_t)f * B + k - 1) * 2 + 0];
                    }
                    if (k == 0 && f > 0) continue;
                    const int64_t Eplus = Pp + (Wm - Pm), Eminus = Wt - Eplus;
                    if (best < 0 || Eplus < best) { best = Eplus; bf = f; bk = k; bs = 1; }
                    if (Eminus < best) { best = Eminus; bf = f; bk = k; bs = -1; }
                }
            }
            if (2 * best >= Wt) break;                    /* no stump beats chance */
            const double eps = (double)best / (double)Wt;
            const double ea = eps > 1e-10 ? eps : 1e-10;
            tf[T] = bf; tk[T] = bk; ts[T] = bs;
            ta[T] = 0.5 * log((1.0 - ea) / ea);
            if (feat) feat[T] = bf;
            if (bin) bin[T] = bk;
            if (sign) sign[T] = bs;
            if (eps_out) eps_out[T] = eps;
            if (alpha_out) alpha_out[T] = ta[T];
            ++T;
            if (best == 0) break;                         /* perfect stump */
            const double up = 2.0 * eps, dn = 2.0 * (1.0 - eps);
            for (int64_t j = 0; j < nI; ++j) {
                int h = bins[(size_t)bf * N + j] >= bk ? bs : -bs;
                w[j] = h != y[j] ? w[j] / up : w[j] / dn;
            }
        }
    }
    /* fold: F(x) = base + sum over features of the step function
     * G_f(psi_f) = sum of delta = 2 alpha s over the stumps of f whose
     * threshold psi_f reaches.  Row: base, per-feature counts, then per
     * feature its thresholds in ascending order (ties in round order) and the
     * running sums of their deltas in that order. */
    double base = 0.0;
    for (int t = 0; t < T; ++t) base -= ta[t] * ts[t];
    row[0] = base;
    int at = 1 + nf;
    for (int f = 0; f < nf; ++f) {
        double th[ORC_ADA_TMAX], de[ORC_ADA_TMAX];
        int cnt = 0;
        const double step = (hi[f] - lo[f]) / (double)B;
        for (int t = 0; t < T; ++t) {
            if (tf[t] != f) continue;
            double v = tk[t] == 0 ? -1e300 : lo[f] + (double)tk[t] * step;
            double dl = 2.0 * ta[t] * ts[t];
            int q = cnt++;
            while (q > 0 && th[q - 1] > v) {   /* stable insertion by threshold */
                th[q] = th[q - 1];
                de[q] = de[q - 1];
                --q;
            }
            th[q] = v;
            de[q] = dl;
        }
        double run = 0.0;
        for (int e = 0; e < cnt; ++e) {
            run += de[e];
            row[at + e] = th[e];
            row[at + cnt + e] = run;
        }
        at += 2 * cnt;
        row[1 + f] = (double)cnt;
    }
    if (n_stumps) *n_stumps = T;
    free(psi); free(w); free(y); free(bins); free(W); free(H);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* I&Z boundary-point search (Section 2.1 eq. (1), Section 2.4): start the
 * searched coordinate at K and iterate s <- Phi^{-1}(C(s)) with the same
 * inner paths each time (common random numbers), until |s' - s| < eps.
 * The searched coordinate is asset 1 for the put family and the asset of the
 * region for the calls; Phi^{-1}(c) is its price whose payoff equals c:
 *   geometric put      (K - c)^d / prod_{i>=2} x_i,
 *   arithmetic put     d (K - c) - sum_{i>=2} x_i,
 *   max- and min-call  K + c.
 * A non-positive inverse drops the point; so does a fixed point outside the
 * region (a max-call point not above every other asset, a min-call point not
 * below every other asset).
 *
 * Secant mode (the paper speaks of Newton iterations): with r(s) = G(s) - s,
 * G the plain map, the first step is the plain one and each later step goes
 * to s - r(s) (s - s_prev) / (r(s) - r(s_prev)), limited to 20 |r(s)|; a zero
 * denominator, a non-finite or a non-positive result takes the plain step.
 * Both modes stop at the first evaluated s with |r(s)| < eps and return G(s). */

static double iz_invert(const orc_spec *s, const double *x_other, double c)
{
    int d = s->d;
    if (s->payoff == ORC_CALL_MAX || s->payoff == ORC_CALL_MIN) return s->K + c;
    if (!(s->K - c > 0.0)) return -1.0;
    if (s->payoff == ORC_PUT_GEO || d == 1) {
        double prod = 1.0;
        for (int i = 1; i < d; ++i) prod *= x_other[i];
        return pow(s->K - c, (double)d) / prod;
    }
    double rest = 0.0;
    for (int i = 1; i < d; ++i) rest += x_other[i];
    return (double)d * (s->K - c) - rest;
}

typedef struct {
    const path_ctx *c;
    const double *x;
    int region;
    int64_t J, n;
    double eps;
    int max_iter, mode;
    double *s_out;
    int32_t *iters;
    int64_t *steps;
    int64_t next;
    pthread_mutex_t lock;
} iz_job;

static void *iz_worker(void *arg)
{
    iz_job *job = (iz_job *)arg;
    const orc_spec *s = job->c->s;
    int d = s->d;
    double xo[64], logx[64];
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t j = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (j >= job->J) break;
        int r = job->region;
        double others_max = 0.0, others_min = INFINITY;
        for (int i = 0; i < d; ++i) {
            xo[i] = job->x[(size_t)i * job->J + j];
            if (i != r && xo[i] > others_max) others_max = xo[i];
            if (i != r && xo[i] < others_min) others_min = xo[i];
        }
        double sv = s->K, result = -1.0, s_prev = 0.0, r_prev = 0.0;
        int it = 0, have_prev = 0;
        int64_t st = 0;
        while (it < job->max_iter) {
            for (int i = 0; i < d; ++i) logx[i] = i == r ? log(sv) : log(xo[i]);
            double sum = 0.0, sq = 0.0;
            run_paths(job->c, logx, (uint32_t)j, 0, job->n, &sum, &sq, &st);
            double cval = sum / (double)job->n;
            double snew = iz_invert(s, xo, cval);
            ++it;
            if (!(snew > 0.0) || !isfinite(snew)) break;
            double res = snew - sv;
            if (fabs(res) < job->eps) {
                int outside = (s->payoff == ORC_CALL_MAX && snew <= others_max) ||
                              (s->payoff == ORC_CALL_MIN && snew >= others_min);
                if (!outside) result = snew;
                break;
            }
            double next = snew;
            if (job->mode == ORC_SEARCH_SECANT && have_prev) {
                double den = res - r_prev;
                if (den != 0.0) {
                    double step = -res * (sv - s_prev) / den;
                    double lim = 20.0 * fabs(res);
                    if (step > lim) step = lim;
                    if (step < -lim) step = -lim;
                    if (isfinite(step) && sv + step > 0.0) next = sv + step;
                }
            }
            s_prev = sv;
            r_prev = res;
            have_prev = 1;
            sv = next;
        }
        job->s_out[j] = result;
        job->iters[j] = it;
        job->steps[j] = st;
    }
    return NULL;
}

int orc_iz_search(const orc_spec *s, const double *rules, int m, int region,
                  const double *x, int64_t J, int64_t n, uint32_t seed, double eps,
                  int max_iter, int mode, int nthreads, double *s_out, int32_t *iters,
                  int64_t *steps_total)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (m < 1 || m >= s->n_dates || J < 1 || n < 2 || max_iter < 1 || !(eps > 0.0) ||
        region < 0 || region >= orc_iz_regions(s) ||
        (mode != ORC_SEARCH_PLAIN && mode != ORC_SEARCH_SECANT))
        return ORC_EINVAL;
    int d = s->d;
    double *L = malloc(sizeof(double) * d * d);
    int64_t *st = calloc(J, sizeof(int64_t));
    if (!L || !st) { free(L); free(st); return ORC_ENOMEM; }
    rc = orc_cholesky(d, s->rho, L);
    if (rc) { free(L); free(st); return rc; }
    path_ctx c = {s, ORC_IZ, rules, orc_rule_width_spec(s, ORC_IZ), m, L, seed,
                  key_hi(ORC_STREAM_INNER, m), (uint32_t)region};
    iz_job job = {&c, x, region, J, n, eps, max_iter, mode, s_out, iters, st, 0};
    pthread_mutex_init(&job.lock, NULL);
    int nt = resolve_threads(nthreads);
    if (nt > J) nt = (int)J;
    pthread_t *th = malloc(sizeof(pthread_t) * nt);
    for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, iz_worker, &job);
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    free(th);
    int64_t tot = 0;
    for (int64_t j = 0; j < J; ++j) tot += st[j];
    if (steps_total) *steps_total = tot;
    pthread_mutex_destroy(&job.lock);
    free(L); free(st);
    return ORC_OK;
}

/* [reg] (Section 2.3): least squares of ln s*_j on the full quadratic in the
 * log-moneyness of the other assets (those of the region's boundary), over the
 * converged points, through the normal equations with a ridge of 1e-10 tr/p.
 * No converged point: never exercise. */
int orc_fit_iz(const orc_spec *s, int region, const double *x, const double *sstar,
               int64_t J, double *b)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (region < 0 || region >= orc_iz_regions(s) || J < 1) return ORC_EINVAL;
    int d = s->d, p = orc_rule_width(ORC_IZ, d);
    double *A = calloc((size_t)p * p, sizeof(double)), *bv = calloc(p, sizeof(double));
    double xi[1 + 63 + 63 * 64 / 2], logS[64];
    int64_t cnt = 0;
    for (int64_t j = 0; j < J; ++j) {
        if (!(sstar[j] > 0.0)) continue;
        for (int i = 0; i < d; ++i) logS[i] = log(x[(size_t)i * J + j]);
        iz_features(s, logS, region, xi);
        double y = log(sstar[j]);
        for (int a = 0; a < p; ++a) {
            bv[a] += xi[a] * y;
            for (int c = 0; c < p; ++c) A[a * p + c] += xi[a] * xi[c];
        }
        ++cnt;
    }
    for (int f = 0; f < p; ++f) b[f] = 0.0;
    if (cnt == 0) {
        b[0] = iz_direction_is_call(s) ? IZ_NEVER : -IZ_NEVER;
    } else {
        double tr = 0.0;
        for (int a = 0; a < p; ++a) tr += A[a * p + a];
        rc = spd_solve(p, A, 1e-10 * tr / p, bv, b);
    }
    free(A); free(bv);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Whole pricer: backward sweep over the dates, then final pricing with an
 * independent stream; price, sample variance, standard error and the 95%
 * half-width 1.96 se (the reading under which the CI column of Table 4 is
 * consistent). */

int orc_price(const orc_spec *s, int method, int64_t N, int64_t n, int64_t n_final,
              uint32_t seed, int rounds, double eps, int max_iter, int search_mode,
              int nthreads, double *rules_out, double *result)
{
    int rc = check_spec(s);
    if (rc) return rc;
    if (N < 2 || n < 2 || n_final < 2 ||
        (method != ORC_CMC && method != ORC_IZ && method != ORC_CMC_ADA))
        return ORC_EINVAL;
    if (method == ORC_CMC_ADA && (rounds < 1 || rounds > ORC_ADA_TMAX)) return ORC_EINVAL;
    int d = s->d, NT = s->n_dates, width = orc_rule_width_spec(s, method);
    int regions = method == ORC_IZ ? orc_iz_regions(s) : 1, pw = width / regions;
    double *rules = calloc((size_t)(NT + 1) * width, sizeof(double));
    double *L = malloc(sizeof(double) * d * d);
    double *x = malloc(sizeof(double) * d * N);
    double *B = malloc(sizeof(double) * d * N);
    double *cont = malloc(sizeof(double) * N);
    int64_t *steps = malloc(sizeof(int64_t) * N);
    int32_t *iters = malloc(sizeof(int32_t) * N);
    if (!rules || !L || !x || !B || !cont || !steps || !iters) { rc = ORC_ENOMEM; goto done; }
    rc = orc_cholesky(d, s->rho, L);
    if (rc) goto done;
    int64_t inner = 0, unconv = 0, iz_it = 0;
    if (method != ORC_IZ) {
        bridge_endpoint(s, N, seed, B);
        for (int m = NT - 1; m >= 1; --m) {
            bridge_back(s, m, N, seed, B);
            points_from_bridge(s, L, m, N, B, x);
            rc = orc_continuation(s, method, rules, m, x, N, NULL, n, seed, ORC_STREAM_INNER,
                                  nthreads, cont, NULL, steps, NULL, NULL);
            if (rc) goto done;
            for (int64_t j = 0; j < N; ++j) inner += steps[j];
            if (method == ORC_CMC)
                rc = orc_fit_cmc(s, x, cont, N, rounds, rules + (size_t)m * width);
            else
                rc = orc_fit_ada(s, x, cont, N, rounds, rules + (size_t)m * width, NULL, NULL, NULL,
                                 NULL, NULL, NULL, NULL, NULL);
            if (rc) goto done;
        }
    } else {
        for (int m = NT - 1; m >= 1; --m) {
            /* Algorithm 1: one search and one regression per region; every
             * region's search at date m sees the rules of dates > m only. */
            for (int r = 0; r < regions; ++r) {
                rc = orc_points_iz(s, m, r, N, x);
                if (rc) goto done;
                int64_t st = 0;
                rc = orc_iz_search(s, rules, m, r, x, N, n, seed, eps, max_iter, search_mode,
                                   nthreads, cont, iters, &st);
                if (rc) goto done;
                inner += st;
                for (int64_t j = 0; j < N; ++j) {
                    iz_it += iters[j];
                    if (!(cont[j] > 0.0)) ++unconv;
                }
                rc = orc_fit_iz(s, r, x, cont, N, rules + (size_t)m * width + (size_t)r * pw);
                if (rc) goto done;
            }
        }
    }
    {
        double sum = 0.0, sq = 0.0;
        int64_t fsteps = 0;
        rc = orc_continuation(s, method, rules, 0, s->S0, 1, NULL, n_final, seed,
                              ORC_STREAM_FINAL, nthreads, NULL, NULL, &fsteps, &sum, &sq);
        if (rc) goto done;
        double price = sum / (double)n_final;
        double var = (sq - sum * sum / (double)n_final) / (double)(n_final - 1);
        if (var < 0.0) var = 0.0;
        double se = sqrt(var / (double)n_final);
        result[0] = price;
        result[1] = var;
        result[2] = se;
        result[3] = 1.96 * se;
        result[4] = (double)inner;
        result[5] = (double)fsteps;
        result[6] = (double)unconv;
        result[7] = (double)iz_it;
    }
    if (rules_out) memcpy(rules_out, rules, sizeof(double) * (NT + 1) * width);
done:
    free(rules); free(L); free(x); free(B); free(cont); free(steps); free(iters);
    return rc;
}
