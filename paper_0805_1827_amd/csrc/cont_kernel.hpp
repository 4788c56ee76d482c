// Continuation (inner-path) kernel template; instantiated per dimension bound
// in separate translation units so that they compile in parallel.
#pragma once

#include "internal.hpp"

namespace bmc {

// ---------------------------------------------------------------------------
// Continuation kernel.  One workgroup = one (point, chunk of paths) job.  Each
// lane walks its paths with path recycling: the loop advances one exercise
// interval per iteration, and a lane whose path stops (exercise or maturity)
// starts its next path in the same iteration, so lanes of a wavefront stay
// busy whatever the stopping dates.  Per-date tables and the rule rows live
// in LDS and are read at the lane's own date.

template <class R> struct Acc;
template <> struct Acc<double> {
    double s = 0.0, q = 0.0;
    __device__ void add(double v) { s += v; q += v * v; }
    __device__ double sum() const { return s; }
    __device__ double sumsq() const { return q; }
};
// Kahan-compensated float accumulation of one lane's payoffs.
struct KahanAcc {
    float s = 0.f, cs = 0.f, q = 0.f, cq = 0.f;
    __device__ void add(double v)
    {
        const float x = (float)v;
        float y = x - cs, t = s + y;
        cs = (t - s) - y; s = t;
        y = x * x - cq; t = q + y;
        cq = (t - q) - y; q = t;
    }
    __device__ double sum() const { return (double)s - (double)cs; }
    __device__ double sumsq() const { return (double)q - (double)cq; }
};

// One (point j, chunk) job of a continuation launch, run by a whole block;
// lds: the dynamic table area, red: [3][16] wave partials.
template <int D, bool EXACT, class R, class ACC>
__device__ __forceinline__ void cont_job(const ContArgs& a, const uint32_t j, const uint32_t chunk, double* lds,
                                         double (*red)[16])
{
    const_as<SpecT<R>>& S = *as_const(&spec_of<R>(a.spec));
    const int d = EXACT ? D : S.d;
    const int NT = S.n_dates;
    const int m = a.m;
    const int W = a.width;
    double* disc = lds;
    R* lx = reinterpret_cast<R*>(disc + NT + 1);
    R* dtv = lx + D_MAX;
    R* sdtv = dtv + NT + 1;
    R* wt = sdtv + NT + 1;

    const_as<double>* t64 = as_const(a.spec)->f64.t;
    const double r64 = as_const(a.spec)->f64.r;
    const double tm = t64[m];
    for (int k = threadIdx.x; k <= NT; k += blockDim.x) {
        disc[k] = exp(-r64 * (t64[k] - tm));
        dtv[k] = S.dt[k];
        sdtv[k] = S.sdt[k];
    }
    const R* __restrict__ rules = reinterpret_cast<const R*>(a.rules);
    for (int i = (m + 1) * W + threadIdx.x; i < NT * W; i += blockDim.x) wt[i] = rules[i];
    if ((int)threadIdx.x < d) lx[threadIdx.x] = (R)log(a.x[(int64_t)threadIdx.x * a.N + j]);
    __syncthreads();

    const uint32_t lo = chunk * a.paths_per_wg;
    const uint32_t hi = min(a.n, lo + a.paths_per_wg);
    const uint32_t nb = (uint32_t)(d + 3) >> 2;
    const uint32_t k0 = a.k0, k1 = a.k1;
    const int payk = S.payoff;
    const bool call_dir = payk == CALL_MAX;
    const R K = S.K, lnK = S.lnK, invK = S.invK, inv_d = S.inv_d;

    R ls[D];
#pragma unroll
    for (int i = 0; i < D; ++i) ls[i] = (i < d) ? lx[i] : R(0);

    ACC acc;
    uint32_t steps = 0;
    uint32_t p = lo + threadIdx.x;
    int k = m + 1;
    while (p < hi) {
        const R dtk = dtv[k], sk = sdtv[k];
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (i < d) ls[i] += S.drift[i] * dtk;
        const uint32_t c0 = (uint32_t)k * nb;
#pragma unroll
        for (int b = 0; b < (D + 3) / 4; ++b) {
            if (4 * b < d) {
                const Words w = philox(k0, k1, c0 + (uint32_t)b, p, j, 0u);
                R z[4];
                box_muller(w.w[0], w.w[1], z[0], z[1]);
                if (4 * b + 2 < d) box_muller(w.w[2], w.w[3], z[2], z[3]);
                else { z[2] = R(0); z[3] = R(0); }
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int l = 4 * b + h;
                    if (l < D && l < d) {
                        const R zl = sk * z[h];
#pragma unroll
                        for (int i = l; i < D; ++i)
                            if (i < d) ls[i] += S.A[i * D_MAX + l] * zl;
                    }
                }
            }
        }
        const R phi = payoff<D, R>(payk, d, K, inv_d, ls);
        bool stop = (k == NT);
        if (!stop && phi > R(0)) {
            const R* w = wt + k * W;
            if (a.method == CMC) {
                stop = cmc_score<D, R>(d, w, lnK, phi * invK, ls) > R(0);
            } else {
                if constexpr (D <= 16) {
                    const R bnd = iz_boundary<D, R>(d, w, lnK, ls);
                    stop = call_dir ? (ls[0] > bnd) : (ls[0] < bnd);
                }
            }
        }
        if (stop) {
            acc.add((double)phi * disc[k]);
            steps += (uint32_t)(k - m);
            p += blockDim.x;
            k = m + 1;
#pragma unroll
            for (int i = 0; i < D; ++i)
                if (i < d) ls[i] = lx[i];
        } else {
            ++k;
        }
    }

    double s1 = acc.sum(), s2 = acc.sumsq(), s3 = (double)steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        s3 += __shfl_xor(s3, off);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = s1;
        red[1][wave] = s2;
        red[2][wave] = s3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            t1 += red[0][w];
            t2 += red[1][w];
            t3 += red[2][w];
        }
        double* o = a.part + ((size_t)j * a.nchunk + chunk) * 3;
        o[0] = t1;
        o[1] = t2;
        o[2] = t3;
    }
}

// One launch per (spec, date): block = one (point, chunk) job.
template <int D, bool EXACT, class R, class ACC>
__global__ void __launch_bounds__(256) k_cont(const ContArgs a)
{
    extern __shared__ double lds[];
    __shared__ double red[3][16];
    const uint32_t slot = blockIdx.x / a.nchunk;
    const uint32_t chunk = blockIdx.x - slot * a.nchunk;
    if (a.n_ids && slot >= (uint32_t)*a.n_ids) return;   // retired job (whole block)
    const uint32_t j = a.ids ? (uint32_t)a.ids[slot] : slot;
    cont_job<D, EXACT, R, ACC>(a, j, chunk, lds, red);
}

// One launch over the jobs of many tasks (options at their own dates): block
// b runs job job0 + b, mapped to (task, point, chunk) through the exclusive
// prefix sums of the tasks' job counts.  Every job writes its own partial
// sums, so results do not depend on the launch it ran in.  The task table and
// prefix sums are read through the scalar unit (uniform loads).
template <int D, bool EXACT, class R, class ACC>
__global__ void __launch_bounds__(256) k_cont_multi(const ContArgs* __restrict__ tasks,
                                                    const uint32_t* __restrict__ prefix, int ntasks, uint32_t job0)
{
    extern __shared__ double lds[];
    __shared__ double red[3][16];
    const_as<uint32_t>* pre = as_const(prefix);
    const uint32_t job = job0 + blockIdx.x;
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= job) lo = mid;
        else hi = mid;
    }
    const ContArgs a = load_const(tasks + lo);
    const uint32_t local = job - pre[lo];
    const uint32_t slot = local / a.nchunk;
    cont_job<D, EXACT, R, ACC>(a, slot, local - slot * a.nchunk, lds, red);
}

template <int D, bool EXACT>
hipError_t launch_cont_d(int prec, const ContArgs& a, int grid, int block, size_t lds,
                                hipStream_t st)
{
    if (prec == PREC_FP64)
        hipLaunchKernelGGL((k_cont<D, EXACT, double, Acc<double>>), dim3(grid), dim3(block), lds, st, a);
    else if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_cont<D, EXACT, float, Acc<double>>), dim3(grid), dim3(block), lds, st, a);
    else
        hipLaunchKernelGGL((k_cont<D, EXACT, float, KahanAcc>), dim3(grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

template <int D, bool EXACT>
hipError_t launch_cont_multi_d(int prec, const ContArgs* tasks, const uint32_t* prefix, int ntasks, uint32_t job0,
                               uint32_t jobs, int block, size_t lds, hipStream_t st)
{
    if (prec == PREC_FP64)
        hipLaunchKernelGGL((k_cont_multi<D, EXACT, double, Acc<double>>), dim3(jobs), dim3(block), lds, st, tasks,
                           prefix, ntasks, job0);
    else if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_cont_multi<D, EXACT, float, Acc<double>>), dim3(jobs), dim3(block), lds, st, tasks,
                           prefix, ntasks, job0);
    else
        hipLaunchKernelGGL((k_cont_multi<D, EXACT, float, KahanAcc>), dim3(jobs), dim3(block), lds, st, tasks,
                           prefix, ntasks, job0);
    return hipGetLastError();
}

}  // namespace bmc
