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
// secant).
//   geometric put (K - c)^d / prod_{i>=2} x_i, arithmetic put d (K - c) -
//   sum_{i>=2} x_i, max- and min-call K + c.  Non-positive: dropped; a fixed
//   point outside the region (not above / below every other asset): dropped.
// iz_step_compute takes the step from the point's state (sv = s, sp, rp: the
// secant's previous point and residual) and writes nothing; iz_step_apply
// stores it and appends a continuing point to the next active list.
// tau > 0 (FP32 searches): tie = 1 when a decision of the step lies within
// tau of its threshold: the stopping test (|r| against eps), the sign of
// the inverse, the region test of a call's fixed point, the secant's
// positivity test.  The pricer searches such points again in FP64 (IZ_TIE_TAU).
struct IzStepOut {
    int cont;                  // 1: the point continues at `next`
    int tie;                   // a decision of this step was a near tie
    double s_final;            // stopped: the boundary point, or -1 (dropped)
    double next, sv, res;      // continuing: next point, current point, residual
    unsigned long long pst;    // executed path-steps of the pass
};

__device__ inline IzStepOut iz_step_compute(const SpecT<double>& S, int d, int region, int64_t Jt,
                                            const double* __restrict__ part, uint32_t nchunk, uint32_t n, int64_t j,
                                            const double* __restrict__ x_work, double sv, double sp, double rp,
                                            double eps, int max_iter, int mode, int it, double tau = 0.0)
{
#pragma clang fp contract(off)
    IzStepOut o;
    o.cont = 0;
    o.tie = 0;
    o.s_final = -1.0;
    o.next = o.sv = o.res = 0.0;
    double psum, psq, pst;
    merge_serial(part, nchunk, j, psum, psq, pst);
    const double c = psum / (double)n;
    o.pst = (unsigned long long)(int64_t)pst;
    double snew;
    if (S.payoff != CALL_MAX && S.payoff != CALL_MIN && fabs(S.K - c) < tau) o.tie = 1;
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
    if (!(snew > 0.0) || !isfinite(snew)) return o;
    const double res = snew - sv;
    if (fabs(fabs(res) - eps) < tau) o.tie = 1;
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
        if ((S.payoff == CALL_MAX && fabs(snew - omax) < tau) || (S.payoff == CALL_MIN && fabs(snew - omin) < tau))
            o.tie = 1;
        o.s_final = outside ? -1.0 : snew;
        return o;
    }
    if (it + 1 >= max_iter) return o;
    double next = snew;
    if (mode == SEARCH_SECANT && it > 0) {
        const double den = res - rp;
        if (den != 0.0) {
            double step = -res * (sv - sp) / den;
            const double lim = 20.0 * fabs(res);
            if (step > lim) step = lim;
            if (step < -lim) step = -lim;
            if (isfinite(step) && fabs(sv + step) < tau) o.tie = 1;
            if (isfinite(step) && sv + step > 0.0) next = sv + step;
        }
    }
    o.cont = 1;
    o.next = next;
    o.sv = sv;
    o.res = res;
    return o;
}

__device__ inline void iz_step_apply(const IzStepOut& o, int region, int64_t Jt, int64_t j, int it,
                                     int32_t* ids_out, int32_t* n_out, double* s_cur_w, double* s_prev_w,
                                     double* r_prev_w, double* x_work, double* s_out, int32_t* iters,
                                     unsigned long long* steps_acc, int32_t* ties = nullptr)
{
    if (o.tie && ties) ties[j] = 1;
    steps_acc[j] += o.pst;
    iters[j] = it + 1;
    if (!o.cont) {
        s_out[j] = o.s_final;
        return;
    }
    s_prev_w[j] = o.sv;
    r_prev_w[j] = o.res;
    s_cur_w[j] = o.next;
    x_work[region * Jt + j] = o.next;
    const int pos = atomicAdd(n_out, 1);
    ids_out[pos] = (int32_t)j;
}

// The step of one active point by one thread: state read from the _r
// arrays (iteration it's), written to the _w arrays (iteration it + 1's).
__device__ inline void iz_step_slot(const SpecT<double>& S, int d, int region0, int64_t J, int64_t Jt,
                                    const double* __restrict__ part, uint32_t nchunk, uint32_t n, int64_t j,
                                    int32_t* ids_out, int32_t* n_out, const double* s_cur_r, const double* s_prev_r,
                                    const double* r_prev_r, double* s_cur_w, double* s_prev_w, double* r_prev_w,
                                    double* x_work, double* s_out, int32_t* iters, unsigned long long* steps_acc,
                                    double eps, int max_iter, int mode, int it, double tau, int32_t* ties)
{
    const int region = region0 + (int)(j / J);
    const IzStepOut o = iz_step_compute(S, d, region, Jt, part, nchunk, n, j, x_work, s_cur_r[j], s_prev_r[j],
                                        r_prev_r[j], eps, max_iter, mode, it, tau);
    iz_step_apply(o, region, Jt, j, it, ids_out, n_out, s_cur_w, s_prev_w, r_prev_w, x_work, s_out, iters,
                  steps_acc, ties);
}

}  // namespace bmc
