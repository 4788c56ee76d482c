// CMC classification [class] by AdaBoost with decision stumps (Section 3.2
// names AdaBoost or LogitBoost).  Training set: the in-the-money points of a
// date; label y = +1 (exercise) iff Phi - C > 0, else -1; initial weight
// |Phi - C|, the value lost by the wrong decision.  Features
// psi = [u_1..u_d, g], u_i = ln(S_i/K), g = Phi/K.  A stump on feature f
// predicts s in bins k..B-1 and -s below, with B uniform bins between the
// feature's extremes over the training points (k = 0, the constant stump, on
// feature 0 only).
//
// Every round runs on the device without host round trips:
//   k_ada_hist    weights rounded to a fixed-point grid 2^-shift and summed
//                 per (feature, bin, label) with 64-bit integer atomics, so
//                 the sums are exact and independent of the order;
//   k_ada_pick    one thread per feature scans its bins for the stump of
//                 least error (ties: smaller bin, then s = +1), thread 0 takes
//                 the best feature (ties: smaller feature), eps = error/total,
//                 alpha = ln((1 - eps)/eps)/2 (eps >= 1e-10); stops when no
//                 stump beats chance, or after a perfect stump;
//   k_ada_update  the normalised AdaBoost step w/(2 eps) for misclassified
//                 points, w/(2 (1 - eps)) for the others (correctly rounded
//                 divisions, no exponentials).
// k_ada_fold then writes the rule row [base, count_0..count_d, then per
// feature its thresholds theta in ascending order (ties in round order) and
// the running sums of the increments delta = 2 alpha s in that order]:
// F(x) = base + per feature the running sum at the number of thresholds psi
// reaches; exercise iff Phi > 0 and F > 0.
#include <climits>

#include "fit_common.hpp"
#include "internal.hpp"

namespace bmc {

namespace {

constexpr int NFMAX = D_MAX + 1;
// Training sets up to this size are fitted by one workgroup.
constexpr int64_t ADA_BLOCK_N = 1 << 16;

struct AdaState {
    int32_t n_itm, shift, T, stop;
    int32_t f[ADA_TMAX], k[ADA_TMAX], s[ADA_TMAX];
    double alpha[ADA_TMAX], eps[ADA_TMAX];
    double lo[NFMAX], hi[NFMAX], inv[NFMAX];
};

__device__ inline int ada_bin(double v, double lo, double hi, double inv)
{
    if (!(hi > lo)) return 0;
    const double t = floor((v - lo) * inv);
    if (t < 0.0) return 0;
    if (t > (double)(ADA_BINS - 1)) return ADA_BINS - 1;
    return (int)t;
}

// Payoff of point j in the arithmetic of the classifier's definition: price
// by price from the log-prices, the basket mean divided by d, the largest of
// the prices for the max-call (the weights are exact only up to the rounding
// of the fixed-point grid, so the costs |Phi - C| follow the definition).
__device__ inline double ada_payoff(const SpecT<double>& S, const double* __restrict__ x, int64_t N, int64_t j)
{
#pragma clang fp contract(off)
    const int d = S.d;
    double v;
    if (S.payoff == CALL_MAX) {
        double mx = exp(log(x[j]));
        for (int i = 1; i < d; ++i) mx = fmax(mx, exp(log(x[i * N + j])));
        v = mx - S.K;
    } else if (S.payoff == CALL_MIN) {
        double mn = exp(log(x[j]));
        for (int i = 1; i < d; ++i) mn = fmin(mn, exp(log(x[i * N + j])));
        v = mn - S.K;
    } else if (S.payoff == PUT_GEO) {
        double sl = 0.0;
        for (int i = 0; i < d; ++i) sl += log(x[i * N + j]);
        v = S.K - exp(sl / (double)d);
    } else {
        double sm = 0.0;
        for (int i = 0; i < d; ++i) sm += exp(log(x[i * N + j]));
        v = S.K - sm / (double)d;
    }
    return v > 0.0 ? v : 0.0;
}

// Per point: features, label, initial weight; per block: feature extremes,
// largest weight and count over the in-the-money points.
__global__ void __launch_bounds__(256) k_ada_prep(const DevSpec* __restrict__ s, const double* __restrict__ x,
                                                  const double* __restrict__ cont, int64_t N, double* psi, double* w,
                                                  int8_t* y, double* part)
{
    const SpecT<double>& S = s->f64;
    const int d = S.d, nf = d + 1;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool itm = false;
    if (j < N) {
        const double pay = ada_payoff(S, x, N, j);
        itm = pay > 0.0;
        if (itm) {
            for (int i = 0; i < d; ++i) psi[i * N + j] = log(x[i * N + j]) - S.lnK;
            psi[d * N + j] = pay / S.K;
            const double beta = pay - cont[j];
            y[j] = beta > 0.0 ? 1 : -1;
            w[j] = fabs(beta);
        } else {
            y[j] = 0;
            w[j] = 0.0;
        }
    }
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* out = part + (size_t)blockIdx.x * (2 * nf + 2);
    for (int f = 0; f < nf + 1; ++f) {
        // f < nf: extremes of feature f; f == nf: largest weight and count
        double a, b;
        if (f < nf) {
            a = itm ? psi[(int64_t)f * N + j] : INFINITY;
            b = itm ? psi[(int64_t)f * N + j] : -INFINITY;
        } else {
            a = itm ? w[j] : 0.0;
            b = itm ? 1.0 : 0.0;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ao = __shfl_xor(a, off), bo = __shfl_xor(b, off);
            if (f < nf) {
                a = fmin(a, ao);
                b = fmax(b, bo);
            } else {
                a = fmax(a, ao);
                b += bo;
            }
        }
        if (lane == 0) {
            red[0][wv] = a;
            red[1][wv] = b;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ra = red[0][0], rb = red[1][0];
            for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
                if (f < nf) {
                    ra = fmin(ra, red[0][q]);
                    rb = fmax(rb, red[1][q]);
                } else {
                    ra = fmax(ra, red[0][q]);
                    rb += red[1][q];
                }
            }
            out[2 * f] = ra;
            out[2 * f + 1] = rb;
        }
        __syncthreads();
    }
}

// Ranges, fixed-point shift, cleared histograms and stump list.
__global__ void k_ada_setup(int nf, int nblocks, const double* __restrict__ part, AdaState* st, int64_t* H)
{
    const int t = threadIdx.x;
    for (int f = t; f < nf; f += blockDim.x) {
        double lo = INFINITY, hi = -INFINITY;
        for (int b = 0; b < nblocks; ++b) {
            lo = fmin(lo, part[(size_t)b * (2 * nf + 2) + 2 * f]);
            hi = fmax(hi, part[(size_t)b * (2 * nf + 2) + 2 * f + 1]);
        }
        st->lo[f] = lo;
        st->hi[f] = hi;
        st->inv[f] = hi > lo ? (double)ADA_BINS / (hi - lo) : 0.0;
    }
    for (int e = t; e < 2 * nf * ADA_BINS * 2; e += blockDim.x) H[e] = 0;
    if (t == 0) {
        double cmax = 0.0, cnt = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            cmax = fmax(cmax, part[(size_t)b * (2 * nf + 2) + 2 * nf]);
            cnt += part[(size_t)b * (2 * nf + 2) + 2 * nf + 1];
        }
        const int nI = (int)cnt;
        int e2 = 0;
        frexp((double)nI * cmax, &e2);          // total weight < 2^e2
        st->n_itm = nI;
        st->shift = 50 - e2;
        st->T = 0;
        st->stop = (nI == 0 || !(cmax > 0.0)) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(256) k_ada_bins(const double* __restrict__ psi, const int8_t* __restrict__ y,
                                                  int64_t N, int nf, const AdaState* __restrict__ st,
                                                  uint8_t* bins)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N || y[j] == 0) return;
    for (int f = 0; f < nf; ++f)
        bins[(int64_t)f * N + j] = (uint8_t)ada_bin(psi[(int64_t)f * N + j], st->lo[f], st->hi[f], st->inv[f]);
}

__device__ inline int64_t ada_fixed(double w, int shift)
{
    return (int64_t)llrint(ldexp(w, shift));
}

// Round histogram: H[(f*B + bin)*2 + (y > 0)] += fixed-point weight.
__global__ void __launch_bounds__(256) k_ada_hist(const double* __restrict__ w, const int8_t* __restrict__ y,
                                                  const uint8_t* __restrict__ bins, int64_t N, int nf,
                                                  const AdaState* __restrict__ st, int64_t* H)
{
    if (st->stop) return;
    extern __shared__ unsigned long long hs[];
    const int nh = nf * ADA_BINS * 2;
    for (int e = threadIdx.x; e < nh; e += blockDim.x) hs[e] = 0ull;
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N && y[j] != 0) {
        const unsigned long long W = (unsigned long long)ada_fixed(w[j], st->shift);
        const int c = y[j] > 0;
        if (W)
            for (int f = 0; f < nf; ++f) atomicAdd(&hs[((int)bins[(int64_t)f * N + j] + f * ADA_BINS) * 2 + c], W);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nh; e += blockDim.x)
        if (hs[e]) atomicAdd(reinterpret_cast<unsigned long long*>(H) + e, hs[e]);
}

// Best stump of round t from the histogram Hc; clears the other histogram.
__global__ void k_ada_pick(int t, int nf, const int64_t* __restrict__ Hc, int64_t* Hn, AdaState* st)
{
    __shared__ long long best_e[NFMAX];
    __shared__ int best_k[NFMAX], best_s[NFMAX];
    __shared__ long long totals[2];
    if (st->stop) return;
    const int f = threadIdx.x;
    if (f < nf) {
        const int64_t* h = Hc + (size_t)f * ADA_BINS * 2;
        long long Wp = 0, Wm = 0;
        for (int b = 0; b < ADA_BINS; ++b) {
            Wm += h[2 * b];
            Wp += h[2 * b + 1];
        }
        const long long Wt = Wp + Wm;
        long long Pp = 0, Pm = 0, be = -1;
        int bk = 0, bs = 1;
        for (int k = 0; k < ADA_BINS; ++k) {
            if (k > 0) {
                Pm += h[2 * (k - 1)];
                Pp += h[2 * (k - 1) + 1];
            }
            if (k == 0 && f > 0) continue;
            const long long Eplus = Pp + (Wm - Pm), Eminus = Wt - Eplus;
            if (be < 0 || Eplus < be) {
                be = Eplus;
                bk = k;
                bs = 1;
            }
            if (Eminus < be) {
                be = Eminus;
                bk = k;
                bs = -1;
            }
        }
        best_e[f] = be;
        best_k[f] = bk;
        best_s[f] = bs;
        if (f == 0) {
            totals[0] = Wt;
            totals[1] = 0;
        }
    }
    for (int e = threadIdx.x; e < nf * ADA_BINS * 2; e += blockDim.x) Hn[e] = 0;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const long long Wt = totals[0];
    long long be = best_e[0];
    int bf = 0;
    for (int g = 1; g < nf; ++g)
        if (best_e[g] < be) {
            be = best_e[g];
            bf = g;
        }
    if (Wt == 0 || 2 * be >= Wt) {   // no stump beats chance
        st->stop = 1;
        return;
    }
    const double eps = (double)be / (double)Wt;
    const double ea = eps > 1e-10 ? eps : 1e-10;
    st->f[t] = bf;
    st->k[t] = best_k[bf];
    st->s[t] = best_s[bf];
    st->eps[t] = eps;
    st->alpha[t] = 0.5 * log((1.0 - ea) / ea);
    st->T = t + 1;
    if (be == 0) st->stop = 1;   // perfect stump: nothing left to reweight
}

__global__ void __launch_bounds__(256) k_ada_update(int t, double* w, const int8_t* __restrict__ y,
                                                    const uint8_t* __restrict__ bins, int64_t N,
                                                    const AdaState* __restrict__ st)
{
    if (st->stop || st->T != t + 1) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N || y[j] == 0) return;
    const int f = st->f[t], k = st->k[t], s = st->s[t];
    const double eps = st->eps[t];
    const int h = (int)bins[(int64_t)f * N + j] >= k ? s : -s;
    w[j] = h != y[j] ? w[j] / (2.0 * eps) : w[j] / (2.0 * (1.0 - eps));
}

// Folded rule row (FP64 and its FP32 copy), zero-padded to width.
__global__ void k_ada_fold(int nf, int width, const AdaState* __restrict__ st, double* row64, float* row32)
{
#pragma clang fp contract(off)
    // the state in LDS first, the row built in LDS, then written out: the
    // insertion below reads back what it wrote, which in global memory would
    // cost a round trip per step
    __shared__ double alpha_s[ADA_TMAX], lo_s[NFMAX], hi_s[NFMAX];
    __shared__ int f_s[ADA_TMAX], k_s[ADA_TMAX], s_s[ADA_TMAX];
    __shared__ double out[1 + NFMAX + 2 * ADA_TMAX];
    __shared__ int used;
    const int T = st->T;
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        alpha_s[t] = st->alpha[t];
        f_s[t] = st->f[t];
        k_s[t] = st->k[t];
        s_s[t] = st->s[t];
    }
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
        lo_s[f] = st->lo[f];
        hi_s[f] = st->hi[f];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double base = 0.0;
        for (int t = 0; t < T; ++t) base -= alpha_s[t] * (double)s_s[t];
        out[0] = base;
        int at = 1 + nf;
        for (int f = 0; f < nf; ++f) {
            // the feature's stumps inserted by threshold, stable (round order
            // on ties): thresholds at at.., increments after the last stump of
            // the feature, summed once the count is known
            int cnt = 0;
            for (int t = 0; t < T; ++t) cnt += f_s[t] == f;
            double* th = out + at;
            double* de = out + at + cnt;
            int c = 0;
            const double step = (hi_s[f] - lo_s[f]) / (double)ADA_BINS;
            for (int t = 0; t < T; ++t) {
                if (f_s[t] != f) continue;
                const double v = k_s[t] == 0 ? -1e300 : lo_s[f] + (double)k_s[t] * step;
                const double dl = 2.0 * alpha_s[t] * (double)s_s[t];
                int q = c++;
                for (; q > 0 && th[q - 1] > v; --q) {
                    th[q] = th[q - 1];
                    de[q] = de[q - 1];
                }
                th[q] = v;
                de[q] = dl;
            }
            double run = 0.0;
            for (int e = 0; e < cnt; ++e) {
                run += de[e];
                de[e] = run;
            }
            at += 2 * cnt;
            out[1 + f] = (double)cnt;
        }
        used = at;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < width; e += blockDim.x) {
        const double v = e < used ? out[e] : 0.0;
        row64[e] = v;
        row32[e] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// The whole fit of a date in one workgroup (N up to ADA_BLOCK_N points): the
// same steps and arithmetic as the multi-kernel sequence, with the histogram
// in LDS and block barriers instead of launches.

constexpr int ADA_BT = 1024;

// Block-wide min and max (f < nf) or max and sum (the weight statistics).
__device__ inline void ada_block_reduce(double& a, double& b, bool minmax, double (*red)[ADA_BT / 64])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        const double ao = __shfl_xor(a, off), bo = __shfl_xor(b, off);
        a = minmax ? fmin(a, ao) : fmax(a, ao);
        b = minmax ? fmax(b, bo) : b + bo;
    }
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    a = red[0][0];
    b = red[1][0];
    for (int q = 1; q < ADA_BT / 64; ++q) {
        a = minmax ? fmin(a, red[0][q]) : fmax(a, red[0][q]);
        b = minmax ? fmax(b, red[1][q]) : b + red[1][q];
    }
    __syncthreads();
}

// Best stump of feature f from its histogram h[(f*B + bin)*2 + (y > 0)], by
// one wavefront, lane k = split before bin k: prefix sums by shuffles, then
// the least error in the scan order (k ascending, s = +1 before -1) by a
// lexicographic (error, k) minimum; lane 0 writes the feature's result (and
// the total weight, for feature 0).
__device__ inline void ada_pick_wave(const unsigned long long* h, int f, long long* best_e, int* best_k,
                                     int* best_s, long long* total)
{
    static_assert(ADA_BINS == 64, "one lane per bin");
    const int k = threadIdx.x & 63;
    const long long m0 = (long long)h[(f * ADA_BINS + k) * 2], p0 = (long long)h[(f * ADA_BINS + k) * 2 + 1];
    long long Pm = m0, Pp = p0;   // inclusive prefix over bins <= k
    for (int off = 1; off < 64; off <<= 1) {
        const long long um = __shfl_up(Pm, off), up = __shfl_up(Pp, off);
        if (k >= off) {
            Pm += um;
            Pp += up;
        }
    }
    // lane 63's totals through the scalar unit
    auto lane63 = [](long long v) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)v >> 32), 63);
        return (long long)(((unsigned long long)hi << 32) | lo);
    };
    const long long Wm = lane63(Pm), Wp = lane63(Pp), Wt = Wm + Wp;
    Pm -= m0;   // bins below k
    Pp -= p0;
    const long long Eplus = Pp + (Wm - Pm), Eminus = Wt - Eplus;
    const long long e = Eplus <= Eminus ? Eplus : Eminus;
    // one key per lane ordered as (error, k, s = +1 first): errors stay below
    // 2^50 (the fixed-point total does), so the key fits 57 bits
    long long key = (e << 7) | ((long long)k << 1) | (Eplus <= Eminus ? 0 : 1);
    if (k == 0 && f > 0) key = LLONG_MAX;   // the constant stump lives on feature 0
    for (int off = 32; off > 0; off >>= 1) {
        const long long ko = __shfl_xor(key, off);
        key = ko < key ? ko : key;
    }
    if (k == 0) {
        best_e[f] = key >> 7;
        best_k[f] = (int)((key >> 1) & 63);
        best_s[f] = (key & 1) ? -1 : 1;
        if (f == 0) *total = Wt;
    }
}

__global__ void __launch_bounds__(ADA_BT) k_ada_fit_block(const DevSpec* __restrict__ s, const double* __restrict__ x,
                                                         const double* __restrict__ cont, int64_t N, int rounds,
                                                         double* psi, double* w, int8_t* y, uint8_t* bins,
                                                         AdaState* st, double* row64, float* row32, int width)
{
    extern __shared__ unsigned long long hs[];   // [nf][B][2]
    __shared__ double red[2][ADA_BT / 64];
    __shared__ long long best_e[NFMAX];
    __shared__ int best_k[NFMAX], best_s[NFMAX], flag;
    __shared__ long long total;
    const SpecT<double>& S = s->f64;
    const int d = S.d, nf = d + 1, nh = nf * ADA_BINS * 2, tid = threadIdx.x;
    // training set
    for (int64_t j = tid; j < N; j += ADA_BT) {
        const double pay = ada_payoff(S, x, N, j);
        if (pay > 0.0) {
            for (int i = 0; i < d; ++i) psi[i * N + j] = log(x[i * N + j]) - S.lnK;
            psi[d * N + j] = pay / S.K;
            const double beta = pay - cont[j];
            y[j] = beta > 0.0 ? 1 : -1;
            w[j] = fabs(beta);
        } else {
            y[j] = 0;
            w[j] = 0.0;
        }
    }
    __syncthreads();
    // feature ranges, largest weight, count
    for (int f = 0; f < nf; ++f) {
        double a = INFINITY, b = -INFINITY;
        for (int64_t j = tid; j < N; j += ADA_BT)
            if (y[j] != 0) {
                a = fmin(a, psi[(int64_t)f * N + j]);
                b = fmax(b, psi[(int64_t)f * N + j]);
            }
        ada_block_reduce(a, b, true, red);
        if (tid == 0) {
            st->lo[f] = a;
            st->hi[f] = b;
            st->inv[f] = b > a ? (double)ADA_BINS / (b - a) : 0.0;
        }
    }
    {
        double a = 0.0, b = 0.0;
        for (int64_t j = tid; j < N; j += ADA_BT)
            if (y[j] != 0) {
                a = fmax(a, w[j]);
                b += 1.0;
            }
        ada_block_reduce(a, b, false, red);
        if (tid == 0) {
            const int nI = (int)b;
            int e2 = 0;
            frexp((double)nI * a, &e2);   // total weight < 2^e2
            st->n_itm = nI;
            st->shift = 50 - e2;
            st->T = 0;
            st->stop = (nI == 0 || !(a > 0.0)) ? 1 : 0;
        }
    }
    __syncthreads();
    for (int64_t j = tid; j < N; j += ADA_BT)
        if (y[j] != 0)
            for (int f = 0; f < nf; ++f)
                bins[(int64_t)f * N + j] =
                    (uint8_t)ada_bin(psi[(int64_t)f * N + j], st->lo[f], st->hi[f], st->inv[f]);
    const int shift = st->shift;
    for (int t = 0; t < rounds && !st->stop; ++t) {
        for (int e = tid; e < nh; e += ADA_BT) hs[e] = 0ull;
        __syncthreads();
        for (int64_t j = tid; j < N; j += ADA_BT) {
            if (y[j] == 0) continue;
            const unsigned long long W = (unsigned long long)ada_fixed(w[j], shift);
            const int c = y[j] > 0;
            if (W)
                for (int f = 0; f < nf; ++f)
                    atomicAdd(&hs[((int)bins[(int64_t)f * N + j] + f * ADA_BINS) * 2 + c], W);
        }
        __syncthreads();
        for (int f = tid >> 6; f < nf; f += ADA_BT / 64) ada_pick_wave(hs, f, best_e, best_k, best_s, &total);
        __syncthreads();
        if (tid == 0) {
            const long long Wt = total;
            long long be = best_e[0];
            int bf = 0;
            for (int g = 1; g < nf; ++g)
                if (best_e[g] < be) {
                    be = best_e[g];
                    bf = g;
                }
            flag = 0;
            if (Wt == 0 || 2 * be >= Wt) {
                st->stop = 1;
            } else {
                const double eps = (double)be / (double)Wt;
                const double ea = eps > 1e-10 ? eps : 1e-10;
                st->f[t] = bf;
                st->k[t] = best_k[bf];
                st->s[t] = best_s[bf];
                st->eps[t] = eps;
                st->alpha[t] = 0.5 * log((1.0 - ea) / ea);
                st->T = t + 1;
                if (be == 0) st->stop = 1;
                else flag = 1;
            }
        }
        __syncthreads();
        if (flag) {
            const int f = st->f[t], k = st->k[t], sg = st->s[t];
            const double eps = st->eps[t];
            for (int64_t j = tid; j < N; j += ADA_BT) {
                if (y[j] == 0) continue;
                const int h = (int)bins[(int64_t)f * N + j] >= k ? sg : -sg;
                w[j] = h != y[j] ? w[j] / (2.0 * eps) : w[j] / (2.0 * (1.0 - eps));
            }
        }
        __syncthreads();
    }
}

// Dynamic LDS of k_ada_fit_lds: two round histograms, then the weights,
// labels and bins of the in-the-money points.
inline size_t ada_lds_bytes(int64_t N, int nf)
{
    return 2 * sizeof(unsigned long long) * nf * ADA_BINS * 2 +
           (size_t)N * (sizeof(double) + sizeof(int32_t) + 1 + nf);
}

// The whole fit of a date in one workgroup with the training set resident in
// LDS.  k_ada_prep (one thread per point, many workgroups) has computed the
// features psi, labels y, weights w and the per-block feature extremes,
// largest weight and count; this workgroup packs the in-the-money points
// (in arrival order: every step after is independent of the order, the
// histogram sums being exact integers), merges the block extremes, and
// runs the rounds, each round's weight update adding the updated weights
// straight into the next round's histogram (two barriers a round).  Same
// stumps, weights and state as k_ada_fit_block.
__global__ void __launch_bounds__(ADA_BT) k_ada_fit_lds(int64_t N, int nf, int rounds, const double* __restrict__ psi,
                                                       const double* __restrict__ w, const int8_t* __restrict__ y,
                                                       const double* __restrict__ part, int nblocks, AdaState* st)
{
    extern __shared__ unsigned long long hs[];   // [2][nf][B][2], w [N], point [N], y [N], bins [nf][N]
    __shared__ long long best_e[NFMAX];
    __shared__ int best_k[NFMAX], best_s[NFMAX], n_pack;
    __shared__ long long total;
    __shared__ double lo_s[NFMAX], hi_s[NFMAX], inv_s[NFMAX], wmax_s, cnt_s;
    const int nh = nf * ADA_BINS * 2, tid = threadIdx.x;
    double* wl = reinterpret_cast<double*>(hs + 2 * nh);
    int32_t* jl = reinterpret_cast<int32_t*>(wl + N);
    int8_t* yl = reinterpret_cast<int8_t*>(jl + N);
    uint8_t* bl = reinterpret_cast<uint8_t*>(yl + N);
    if (tid == 0) n_pack = 0;
    __syncthreads();
    for (int64_t j = tid; j < N; j += ADA_BT) {
        const int8_t yj = y[j];
        if (yj != 0) {
            const int q = atomicAdd(&n_pack, 1);
            yl[q] = yj;
            wl[q] = w[j];
            jl[q] = (int32_t)j;
        }
    }
    // feature extremes, largest weight and count from the blocks' partials
    // (minimum, maximum and an integer count: order-free)
    const size_t ps = 2 * (size_t)nf + 2;
    for (int f = tid; f < nf; f += ADA_BT) {
        double lo = INFINITY, hi = -INFINITY;
        for (int b = 0; b < nblocks; ++b) {
            lo = fmin(lo, part[b * ps + 2 * f]);
            hi = fmax(hi, part[b * ps + 2 * f + 1]);
        }
        const double inv = hi > lo ? (double)ADA_BINS / (hi - lo) : 0.0;
        st->lo[f] = lo_s[f] = lo;
        st->hi[f] = hi_s[f] = hi;
        st->inv[f] = inv_s[f] = inv;
    }
    if (tid == ADA_BT - 1) {
        double cmax = 0.0, cnt = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            cmax = fmax(cmax, part[b * ps + 2 * nf]);
            cnt += part[b * ps + 2 * nf + 1];
        }
        wmax_s = cmax;
        cnt_s = cnt;
    }
    __syncthreads();
    const int nI = n_pack;
    const double wmax = wmax_s;
    int e2 = 0;
    frexp((double)(int)cnt_s * wmax, &e2);   // total weight < 2^e2
    const int shift = 50 - e2;
    bool stop = nI == 0 || !(wmax > 0.0);
    if (tid == 0) {
        st->n_itm = nI;
        st->shift = shift;
        st->T = 0;
        st->stop = stop ? 1 : 0;
    }
    for (int e = tid; e < nh; e += ADA_BT) hs[e] = 0ull;
    for (int q = tid; q < nI; q += ADA_BT)
        for (int f = 0; f < nf; ++f)
            bl[f * N + q] = (uint8_t)ada_bin(psi[(int64_t)f * N + jl[q]], lo_s[f], hi_s[f], inv_s[f]);
    __syncthreads();
    for (int q = tid; q < nI; q += ADA_BT) {
        const unsigned long long W = (unsigned long long)ada_fixed(wl[q], shift);
        const int c = yl[q] > 0;
        if (W)
            for (int f = 0; f < nf; ++f) atomicAdd(&hs[((int)bl[f * N + q] + f * ADA_BINS) * 2 + c], W);
    }
    __syncthreads();
    for (int t = 0; t < rounds && !stop; ++t) {
        const unsigned long long* hc = hs + (t & 1) * nh;
        unsigned long long* hn = hs + ((t + 1) & 1) * nh;
        for (int e = tid; e < nh; e += ADA_BT) hn[e] = 0ull;   // last read by the previous round's pick
        for (int f = tid >> 6; f < nf; f += ADA_BT / 64) ada_pick_wave(hc, f, best_e, best_k, best_s, &total);
        __syncthreads();
        // every thread takes the same decision from the per-feature bests
        const long long Wt = total;
        long long be = best_e[0];
        int bf = 0;
        for (int g = 1; g < nf; ++g)
            if (best_e[g] < be) {
                be = best_e[g];
                bf = g;
            }
        if (Wt == 0 || 2 * be >= Wt) {
            if (tid == 0) st->stop = 1;
            break;
        }
        const double eps = (double)be / (double)Wt;
        const double ea = eps > 1e-10 ? eps : 1e-10;
        const int k = best_k[bf], sg = best_s[bf];
        if (tid == 0) {
            st->f[t] = bf;
            st->k[t] = k;
            st->s[t] = sg;
            st->eps[t] = eps;
            st->alpha[t] = 0.5 * log((1.0 - ea) / ea);
            st->T = t + 1;
            if (be == 0) st->stop = 1;
        }
        if (be == 0) break;   // perfect stump: nothing left to reweight
        const bool next = t + 1 < rounds;
        for (int q = tid; q < nI; q += ADA_BT) {
            const int h = (int)bl[bf * N + q] >= k ? sg : -sg;
            const double w = h != yl[q] ? wl[q] / (2.0 * eps) : wl[q] / (2.0 * (1.0 - eps));
            wl[q] = w;
            const unsigned long long W = (unsigned long long)ada_fixed(w, shift);
            const int c = yl[q] > 0;
            if (next && W)
                for (int f = 0; f < nf; ++f) atomicAdd(&hn[((int)bl[f * N + q] + f * ADA_BINS) * 2 + c], W);
        }
        __syncthreads();
    }
}

}  // namespace

// Scratch (bytes): psi [nf][N], w [N], block partials, histograms [2][nf][B][2],
// state, labels [N], bins [nf][N].
size_t fit_ada_scratch_bytes(int64_t N, int d)
{
    const int nf = d + 1;
    const int64_t blocks = (N + 255) / 256;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    return al(sizeof(double) * nf * N) + al(sizeof(double) * N) + al(sizeof(double) * blocks * (2 * nf + 2)) +
           al(sizeof(int64_t) * 2 * nf * ADA_BINS * 2) + al(sizeof(AdaState)) + al(N) + al((size_t)nf * N);
}

hipError_t launch_fit_ada(const DevSpec* s, int d, const double* x, const double* cont, int64_t N, int rounds,
                          void* scratch, double* row64, float* row32, int width, hipStream_t st)
{
    const int nf = d + 1;
    const int blocks = (int)((N + 255) / 256);
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* c = (char*)scratch;
    double* psi = (double*)c;
    c += al(sizeof(double) * nf * N);
    double* w = (double*)c;
    c += al(sizeof(double) * N);
    double* part = (double*)c;
    c += al(sizeof(double) * blocks * (2 * nf + 2));
    int64_t* H = (int64_t*)c;
    c += al(sizeof(int64_t) * 2 * nf * ADA_BINS * 2);
    AdaState* state = (AdaState*)c;
    c += al(sizeof(AdaState));
    int8_t* y = (int8_t*)c;
    c += al(N);
    uint8_t* bins = (uint8_t*)c;
    const int nh = nf * ADA_BINS * 2;
    // histograms of wide rows exceed the default 64 KB of dynamic LDS
    // the resident fit's static LDS (reductions, bests, ranges) stays below 4 KB
    static const size_t lds_res = cont_lds_limit() + 1024 - 4096;
    static const bool lds_ok = [] {
        const int v = (int)(sizeof(unsigned long long) * NFMAX * ADA_BINS * 2);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ada_fit_block),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, v);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ada_hist),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, v);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ada_fit_lds),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_res);
        (void)hipGetLastError();
        return true;
    }();
    (void)lds_ok;
    if (ada_lds_bytes(N, nf) <= lds_res) {
        hipLaunchKernelGGL(k_ada_prep, dim3(blocks), dim3(256), 0, st, s, x, cont, N, psi, w, y, part);
        hipLaunchKernelGGL(k_ada_fit_lds, dim3(1), dim3(ADA_BT), ada_lds_bytes(N, nf), st, N, nf, rounds, psi, w, y,
                           part, blocks, state);
        hipLaunchKernelGGL(k_ada_fold, dim3(1), dim3(64), 0, st, nf, width, state, row64, row32);
        return hipGetLastError();
    }
    if (N <= ADA_BLOCK_N) {
        // one workgroup runs every round (no launch per step of a round)
        hipLaunchKernelGGL(k_ada_fit_block, dim3(1), dim3(ADA_BT), sizeof(unsigned long long) * nh, st, s, x, cont, N,
                           rounds, psi, w, y, bins, state, row64, row32, width);
        hipLaunchKernelGGL(k_ada_fold, dim3(1), dim3(64), 0, st, nf, width, state, row64, row32);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_ada_prep, dim3(blocks), dim3(256), 0, st, s, x, cont, N, psi, w, y, part);
    hipLaunchKernelGGL(k_ada_setup, dim3(1), dim3(256), 0, st, nf, blocks, part, state, H);
    hipLaunchKernelGGL(k_ada_bins, dim3(blocks), dim3(256), 0, st, psi, y, N, nf, state, bins);
    for (int t = 0; t < rounds; ++t) {
        int64_t* Hc = H + (size_t)(t & 1) * nh;
        int64_t* Hn = H + (size_t)((t + 1) & 1) * nh;
        hipLaunchKernelGGL(k_ada_hist, dim3(blocks), dim3(256), sizeof(unsigned long long) * nh, st, w, y, bins, N,
                           nf, state, Hc);
        hipLaunchKernelGGL(k_ada_pick, dim3(1), dim3(128), 0, st, t, nf, Hc, Hn, state);
        hipLaunchKernelGGL(k_ada_update, dim3(blocks), dim3(256), 0, st, t, w, y, bins, N, state);
    }
    hipLaunchKernelGGL(k_ada_fold, dim3(1), dim3(64), 0, st, nf, width, state, row64, row32);
    return hipGetLastError();
}

}  // namespace bmc
