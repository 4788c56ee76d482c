// I&Z boundary-point search: the step of one active point.
#pragma once

#include "internal.hpp"

namespace bmc {

// Per point: merge the chunk partials in chunk order.  The point's partials
// are contiguous; eight chunks' loads are issued before their adds, which
// keep the order of the sequential merge.
__device__ __forceinline__ void merge_serial(const double* __restrict__ part, uint32_t nchunk, int64_t j, double& s,
                                             double& q, double& c)
{
    s = 0.0;
    q = 0.0;
    c = 0.0;
    const double* o = part + (size_t)j * nchunk * 3;
    uint32_t ch = 0;
    for (; ch + 8 <= nchunk; ch += 8, o += 24) {
        double v[24];
#pragma unroll
        for (int u = 0; u < 24; ++u) v[u] = o[u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s += v[3 * u];
            q += v[3 * u + 1];
            c += v[3 * u + 2];
        }
    }
    for (; ch < nchunk; ++ch, o += 3) {
        s += o[0];
        q += o[1];
        c += o[2];
    }
}

// One search step of point (column) j after a continuation pass: merge its
// chunk partials (chunk order), c = mean payoff, s' = Phi^{-1}(c) for the
// searched coordinate (the region's own asset), then stop (converged,
// dropped, or out of iterations) or move to the next point (plain or
// secant) and append j to the next active list.
//   geometric put (K - c)^d / prod_{i>=2} x_i, arithmetic put d (K - c) -
//   sum_{i>=2} x_i, max- and min-call K + c.  Non-positive: dropped; a fixed
//   point outside the region (not above / below every other asset): dropped.
__device__ inline void iz_step_slot(const SpecT<double>& S, int d, int region0, int64_t J, int64_t Jt,
                                    const double* __restrict__ part, uint32_t nchunk, uint32_t n, int64_t j,
                                    int32_t* ids_out, int32_t* n_out, double* s_cur, double* s_prev,
                                    double* r_prev, double* x_work, double* s_out, int32_t* iters,
                                    unsigned long long* steps_acc, double eps, int max_iter, int mode, int it)
{
#pragma clang fp contract(off)
    const int region = region0 + (int)(j / J);
    double psum, psq, pst;
    merge_serial(part, nchunk, j, psum, psq, pst);
    const double c = psum / (double)n;
    steps_acc[j] += (unsigned long long)(int64_t)pst;
    double snew;
    if (S.payoff == CALL_MAX || S.payoff == CALL_MIN) {
        snew = S.K + c;
    } else if (!(S.K - c > 0.0)) {
        snew = -1.0;
    } else if (S.payoff == PUT_GEO || d == 1) {
        double prod = 1.0;
        for (int i = 1; i < d; ++i) prod *= x_work[i * Jt + j];
        snew = pow(S.K - c, (double)d) / prod;
    } else {
        double rest = 0.0;
        for (int i = 1; i < d; ++i) rest += x_work[i * Jt + j];
        snew = (double)d * (S.K - c) - rest;
    }
    const int it1 = it + 1;
    iters[j] = it1;
    if (!(snew > 0.0) || !isfinite(snew)) { s_out[j] = -1.0; return; }
    const double sv = s_cur[j], res = snew - sv;
    if (fabs(res) < eps) {
        // inside the region: above every other asset (max-call), below
        // every other asset (min-call)
        double omax = 0.0, omin = INFINITY;
        if (S.payoff == CALL_MAX || S.payoff == CALL_MIN)
            for (int i = 0; i < d; ++i)
                if (i != region) {
                    omax = fmax(omax, x_work[i * Jt + j]);
                    omin = fmin(omin, x_work[i * Jt + j]);
                }
        const bool outside = (S.payoff == CALL_MAX && snew <= omax) || (S.payoff == CALL_MIN && snew >= omin);
        s_out[j] = outside ? -1.0 : snew;
        return;
    }
    if (it1 >= max_iter) { s_out[j] = -1.0; return; }
    double next = snew;
    if (mode == SEARCH_SECANT && it > 0) {
        const double den = res - r_prev[j];
        if (den != 0.0) {
            double step = -res * (sv - s_prev[j]) / den;
            const double lim = 20.0 * fabs(res);
            if (step > lim) step = lim;
            if (step < -lim) step = -lim;
            if (isfinite(step) && sv + step > 0.0) next = sv + step;
        }
    }
    s_prev[j] = sv;
    r_prev[j] = res;
    s_cur[j] = next;
    x_work[region * Jt + j] = next;
    const int pos = atomicAdd(n_out, 1);
    ids_out[pos] = (int32_t)j;
}

}  // namespace bmc
