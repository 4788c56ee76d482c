// HIP kernels for gfx950: spec setup, sample points, the continuation
// (inner-path) kernel, I&Z search updates and the FP64 rule fits.
#include <math.h>

#include "internal.hpp"

namespace bmc {

// ---------------------------------------------------------------------------
// Spec setup: Cholesky of rho (FP64), A = diag(sigma) L, drifts, date tables.

__global__ void __launch_bounds__(256) k_setup(const HostSpecPack* __restrict__ in,
                                               DevSpec* __restrict__ out)
{
    __shared__ double L[D_MAX * D_MAX];
    __shared__ int bad;
    const int d = in->d, NT = in->n_dates, tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int i = tid; i < D_MAX * D_MAX; i += blockDim.x) L[i] = 0.0;
    __syncthreads();
    for (int c = 0; c < d; ++c) {
        if (tid == 0) {
            double acc = in->rho[c * d + c];
            for (int l = 0; l < c; ++l) acc -= L[c * D_MAX + l] * L[c * D_MAX + l];
            if (!(acc > 0.0)) { bad = 1; acc = 1.0; }
            L[c * D_MAX + c] = sqrt(acc);
        }
        __syncthreads();
        for (int i = c + 1 + tid; i < d; i += blockDim.x) {
            double acc = in->rho[i * d + c];
            for (int l = 0; l < c; ++l) acc -= L[i * D_MAX + l] * L[c * D_MAX + l];
            L[i * D_MAX + c] = acc / L[c * D_MAX + c];
        }
        __syncthreads();
    }
    SpecT<double>& a = out->f64;
    SpecT<float>& b = out->f32;
    if (tid == 0) {
        a.d = b.d = d;
        a.n_dates = b.n_dates = NT;
        a.payoff = b.payoff = in->payoff;
        a.K = in->K; a.lnK = log(in->K); a.invK = 1.0 / in->K; a.r = in->r; a.inv_d = 1.0 / d;
        b.K = (float)a.K; b.lnK = (float)a.lnK; b.invK = (float)a.invK; b.r = (float)a.r;
        b.inv_d = (float)a.inv_d;
        out->status = bad ? -2 : 0;
    }
    for (int i = tid; i < D_MAX; i += blockDim.x) {
        const bool on = i < d;
        const double s0 = on ? in->S0[i] : 0.0, sg = on ? in->sigma[i] : 0.0;
        const double dr = on ? in->r - in->delta[i] - 0.5 * sg * sg : 0.0;
        a.S0[i] = s0; a.sigma[i] = sg; a.drift[i] = dr;
        b.S0[i] = (float)s0; b.sigma[i] = (float)sg; b.drift[i] = (float)dr;
    }
    for (int e = tid; e < D_MAX * D_MAX; e += blockDim.x) {
        const int i = e / D_MAX, l = e % D_MAX;
        const double v = (i < d && l <= i) ? in->sigma[i] * L[e] : 0.0;
        a.A[e] = v;
        b.A[e] = (float)v;
        out->L[e] = L[e];
    }
    for (int k = tid; k <= NT_MAX; k += blockDim.x) {
        double tk = 0.0, dt = 0.0;
        if (k >= 1 && k <= NT) {
            tk = in->dates[k - 1];
            dt = tk - (k >= 2 ? in->dates[k - 2] : 0.0);
        }
        a.t[k] = tk; a.dt[k] = dt; a.sdt[k] = sqrt(dt);
        b.t[k] = (float)tk; b.dt[k] = (float)dt; b.sdt[k] = (float)sqrt(dt);
    }
}

hipError_t launch_setup(const HostSpecPack* in, DevSpec* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, in, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Continuation launch dispatch over the compiled dimension bounds.

template <int D, bool EXACT>
hipError_t launch_cont_d(int prec, const ContArgs& a, int grid, int block, size_t lds,
                         hipStream_t st);

size_t cont_lds_bytes(int prec, int n_dates, int width)
{
    const size_t rs = prec == PREC_FP64 ? sizeof(double) : sizeof(float);
    return sizeof(double) * (n_dates + 1) +
           rs * (D_MAX + 2 * (size_t)(n_dates + 1) + (size_t)(n_dates + 1) * width) + 16;
}

hipError_t launch_cont(int d, int prec, const ContArgs& a, int grid, int block, size_t lds,
                       hipStream_t st)
{
    switch (d) {
    case 1: return launch_cont_d<1, true>(prec, a, grid, block, lds, st);
    case 2: return launch_cont_d<2, true>(prec, a, grid, block, lds, st);
    case 3: return launch_cont_d<3, true>(prec, a, grid, block, lds, st);
    case 4: return launch_cont_d<4, true>(prec, a, grid, block, lds, st);
    case 5: return launch_cont_d<5, true>(prec, a, grid, block, lds, st);
    case 6: return launch_cont_d<6, true>(prec, a, grid, block, lds, st);
    case 7: return launch_cont_d<7, true>(prec, a, grid, block, lds, st);
    case 8: return launch_cont_d<8, true>(prec, a, grid, block, lds, st);
    default: break;
    }
    if (d <= 12) return launch_cont_d<12, false>(prec, a, grid, block, lds, st);
    if (d <= 16) return launch_cont_d<16, false>(prec, a, grid, block, lds, st);
    if (d <= 24) return launch_cont_d<24, false>(prec, a, grid, block, lds, st);
    if (d <= 32) return launch_cont_d<32, false>(prec, a, grid, block, lds, st);
    if (d <= 40) return launch_cont_d<40, false>(prec, a, grid, block, lds, st);
    return launch_cont_d<64, false>(prec, a, grid, block, lds, st);
}

// Per point: merge the chunk partials in chunk order into the continuation
// estimate C = sum/n and its standard error sqrt(var/n), var = (sumsq -
// sum^2/n)/(n-1).
__global__ void k_finalize(const double* __restrict__ part, uint32_t nchunk, uint32_t n, int64_t N,
                           const int32_t* __restrict__ ids, const int32_t* __restrict__ n_ids,
                           double* cont, double* se, int64_t* steps, double* sums,
                           unsigned long long* steps_total)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j = slot;
    if (ids) {
        if (slot >= *n_ids) return;
        j = ids[slot];
    } else if (slot >= N) {
        return;
    }
    double s = 0.0, q = 0.0, c = 0.0;
    for (uint32_t ch = 0; ch < nchunk; ++ch) {
        const double* o = part + ((size_t)j * nchunk + ch) * 3;
        s += o[0];
        q += o[1];
        c += o[2];
    }
    const double nn = (double)n;
    double var = (q - s * s / nn) / (nn - 1.0);
    if (var < 0.0) var = 0.0;
    if (cont) cont[j] = s / nn;
    if (se) se[j] = sqrt(var / nn);
    if (steps) steps[j] = (int64_t)c;
    if (sums) { sums[2 * j] = s; sums[2 * j + 1] = q; }
    if (steps_total) atomicAdd(steps_total, (unsigned long long)c);
}

hipError_t launch_finalize(const double* part, uint32_t nchunk, uint32_t n, int64_t N,
                           const int32_t* ids, const int32_t* n_ids, double* cont, double* se,
                           int64_t* steps, double* sums, unsigned long long* steps_total,
                           hipStream_t st)
{
    const int grid = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, st, part, nchunk, n, N, ids, n_ids,
                       cont, se, steps, sums, steps_total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CMC training points: Brownian components drawn at T and bridged backward.

__device__ __forceinline__ void outer_block(uint32_t seed, uint32_t k1, uint32_t b, uint32_t j,
                                            int d, double z[4])
{
    const Words w = philox(seed, k1, b, 0u, j, 0u);
    box_muller(w.w[0], w.w[1], z[0], z[1]);
    if (4 * (int)b + 2 < d) box_muller(w.w[2], w.w[3], z[2], z[3]);
}

__global__ void k_bridge_end(const DevSpec* __restrict__ s, int64_t N, uint32_t seed, double* B)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const SpecT<double>& S = s->f64;
    const int d = S.d, NT = S.n_dates;
    const uint32_t k1 = key_hi(STREAM_OUTER, NT);
    const double sq = sqrt(S.t[NT]);
    for (int b = 0; 4 * b < d; ++b) {
        double z[4];
        outer_block(seed, k1, (uint32_t)b, (uint32_t)j, d, z);
        for (int h = 0; h < 4 && 4 * b + h < d; ++h) B[(4 * b + h) * N + j] = sq * z[h];
    }
}

// B holds date m+1 on entry and date m on exit (bridge = 1); with bridge = 0
// B already holds date m.  x (optional) receives the points at date m.
__global__ void k_bridge_back(const DevSpec* __restrict__ s, int m, int64_t N, uint32_t seed,
                              double* B, double* x, int bridge)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const SpecT<double>& S = s->f64;
    const int d = S.d;
    const uint32_t k1 = key_hi(STREAM_OUTER, m);
    const double t0 = S.t[m];
    const double t1 = bridge ? S.t[m + 1] : t0;
    const double mf = bridge ? t0 / t1 : 1.0;
    const double sd = bridge ? sqrt(t0 * (t1 - t0) / t1) : 0.0;
    for (int b = 0; bridge && 4 * b < d; ++b) {
        double z[4];
        outer_block(seed, k1, (uint32_t)b, (uint32_t)j, d, z);
        for (int h = 0; h < 4 && 4 * b + h < d; ++h) {
            const int64_t e = (4 * b + h) * N + j;
            B[e] = mf * B[e] + sd * z[h];
        }
    }
    if (!x) return;
    for (int i = 0; i < d; ++i) {
        double w = 0.0;
        for (int l = 0; l <= i; ++l) w += s->L[i * D_MAX + l] * B[l * N + j];
        x[i * N + j] = S.S0[i] * exp(S.drift[i] * t0 + S.sigma[i] * w);
    }
}

hipError_t launch_bridge_end(const DevSpec* s, int d, int64_t N, uint32_t seed, double* B,
                             hipStream_t st)
{
    (void)d;
    hipLaunchKernelGGL(k_bridge_end, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, s, N, seed, B);
    return hipGetLastError();
}

hipError_t launch_bridge_back(const DevSpec* s, int d, int m, int64_t N, uint32_t seed, double* B,
                              double* x, int bridge, hipStream_t st)
{
    (void)d;
    hipLaunchKernelGGL(k_bridge_back, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, s, m, N,
                       seed, B, x, bridge);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// I&Z lattice: Korobov generator search (one candidate per thread; the
// packed atomic maximum keeps the largest minimal distance and, among ties,
// the smallest generator) and lognormal-quantile points.

__global__ void k_korobov(int64_t J, int q, unsigned long long* best)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (a >= J) return;
    int64_t g[16];
    g[0] = 1;
    for (int i = 1; i < q; ++i) g[i] = (g[i - 1] * a) % J;
    unsigned long long dmin = ~0ull;
    for (int64_t jj = 1; jj < J; ++jj) {
        unsigned long long dist = 0;
        for (int i = 0; i < q; ++i) {
            int64_t v = (jj * g[i]) % J;
            if (J - v < v) v = J - v;
            dist += (unsigned long long)(v * v);
        }
        if (dist < dmin) dmin = dist;
    }
    atomicMax(best, (dmin << 24) | (unsigned long long)(0xFFFFFF - a));
}

hipError_t launch_korobov(int64_t J, int q, unsigned long long* best, hipStream_t st)
{
    hipLaunchKernelGGL(k_korobov, dim3((unsigned)((J + 255) / 256)), dim3(256), 0, st, J, q, best);
    return hipGetLastError();
}

__global__ void k_lattice(const DevSpec* __restrict__ s, int m, int64_t J,
                          const unsigned long long* __restrict__ best, double* x)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    const SpecT<double>& S = s->f64;
    const int d = S.d, q = d - 1;
    const int64_t a = best ? (int64_t)(0xFFFFFF - (*best & 0xFFFFFFull)) : 1;
    const double tm = S.t[m], sq = sqrt(tm);
    x[j] = S.K;
    int64_t g = 1;
    for (int i = 0; i < q; ++i) {
        const double u = ((double)((j * g) % J) + 0.5) / (double)J;
        const int asset = i + 1;
        x[asset * J + j] = S.S0[asset] * exp(S.drift[asset] * tm + S.sigma[asset] * sq * normcdfinv(u));
        g = (g * a) % J;
    }
}

hipError_t launch_lattice(const DevSpec* s, int d, int m, int64_t J, const unsigned long long* best,
                          double* x, hipStream_t st)
{
    (void)d;
    hipLaunchKernelGGL(k_lattice, dim3((unsigned)((J + 255) / 256)), dim3(256), 0, st, s, m, J, best, x);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// I&Z boundary-point search state.  s <- Phi_1^{-1}(C(s)):
//   geometric put (K - c)^d / prod_{i>=2} x_i, arithmetic put d (K - c) -
//   sum_{i>=2} x_i, one-asset call K + c.  Non-positive: dropped.

__global__ void k_iz_init(const DevSpec* __restrict__ s, const double* __restrict__ x_in, int d,
                          int64_t J, double* x_work, double* s_cur, double* s_out, int32_t* iters,
                          int32_t* ids, int32_t* n_ids, unsigned long long* steps_acc)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    const double K = s->f64.K;
    x_work[j] = K;
    for (int i = 1; i < d; ++i) x_work[i * J + j] = x_in[i * J + j];
    s_cur[j] = K;
    s_out[j] = -1.0;
    iters[j] = 0;
    ids[j] = (int32_t)j;
    steps_acc[j] = 0;
    if (j == 0) *n_ids = (int32_t)J;
}

hipError_t launch_iz_init(const DevSpec* s, const double* x_in, int d, int64_t J, double* x_work,
                          double* s_cur, double* s_out, int32_t* iters, int32_t* ids,
                          int32_t* n_ids, unsigned long long* steps_acc, hipStream_t st)
{
    hipLaunchKernelGGL(k_iz_init, dim3((unsigned)((J + 255) / 256)), dim3(256), 0, st, s, x_in, d, J,
                       x_work, s_cur, s_out, iters, ids, n_ids, steps_acc);
    return hipGetLastError();
}

__global__ void k_iz_update(const DevSpec* __restrict__ s, int d, int64_t J,
                            const double* __restrict__ cont, const int64_t* __restrict__ steps,
                            const int32_t* __restrict__ ids_in, const int32_t* __restrict__ n_in,
                            int32_t* ids_out, int32_t* n_out, double* s_cur, double* x_work,
                            double* s_out, int32_t* iters, unsigned long long* steps_acc,
                            double eps, int max_iter, int it)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= *n_in) return;
    const int64_t j = ids_in[slot];
    const SpecT<double>& S = s->f64;
    const double c = cont[j];
    steps_acc[j] += (unsigned long long)steps[j];
    double snew;
    if (S.payoff == CALL_MAX) {
        snew = S.K + c;
    } else if (!(S.K - c > 0.0)) {
        snew = -1.0;
    } else if (S.payoff == PUT_GEO || d == 1) {
        double prod = 1.0;
        for (int i = 1; i < d; ++i) prod *= x_work[i * J + j];
        snew = pow(S.K - c, (double)d) / prod;
    } else {
        double rest = 0.0;
        for (int i = 1; i < d; ++i) rest += x_work[i * J + j];
        snew = (double)d * (S.K - c) - rest;
    }
    const int it1 = it + 1;
    iters[j] = it1;
    if (!(snew > 0.0) || !isfinite(snew)) { s_out[j] = -1.0; return; }
    if (fabs(snew - s_cur[j]) < eps) { s_out[j] = snew; return; }
    if (it1 >= max_iter) { s_out[j] = -1.0; return; }
    s_cur[j] = snew;
    x_work[j] = snew;
    const int pos = atomicAdd(n_out, 1);
    ids_out[pos] = (int32_t)j;
}

hipError_t launch_iz_update(const DevSpec* s, int d, int64_t J, const double* cont,
                            const int64_t* steps, const int32_t* ids_in, const int32_t* n_in,
                            int32_t* ids_out, int32_t* n_out, double* s_cur, double* x_work,
                            double* s_out, int32_t* iters, unsigned long long* steps_acc,
                            double eps, int max_iter, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_iz_update, dim3((unsigned)((J + 255) / 256)), dim3(256), 0, st, s, d, J,
                       cont, steps, ids_in, n_in, ids_out, n_out, s_cur, x_work, s_out, iters,
                       steps_acc, eps, max_iter, it);
    return hipGetLastError();
}

__global__ void k_narrow(const double* __restrict__ a, float* b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

hipError_t launch_rules_narrow(const double* w64, float* w32, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, w64, w32, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 rule fits.  Reductions are deterministic: a block reduces its tile
// sequentially (one thread per output quantity), and tiles are merged in tile
// order.  The small SPD systems are factorised by a block-parallel Cholesky.

__device__ __forceinline__ void pair_of(int q, int& i, int& l)
{
    i = 0;
    while (q >= i + 1) { q -= i + 1; ++i; }
    l = q;
}

__device__ __forceinline__ int tri(int i, int l) { return i * (i + 1) / 2 + l; }

// Solves (A + lam I) x = b for packed lower-triangular A (overwritten by L).
// Returns false if a pivot is not positive.  Called by a whole block.
__device__ bool block_spd_solve(int p, double* A, double lam, const double* b, double* x,
                                int* flag)
{
    const int tid = threadIdx.x;
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        if (tid == 0) {
            double acc = A[tri(c, c)] + lam;
            for (int l = 0; l < c; ++l) acc -= A[tri(c, l)] * A[tri(c, l)];
            if (!(acc > 0.0)) { *flag = 1; acc = 1.0; }
            A[tri(c, c)] = sqrt(acc);
        }
        __syncthreads();
        for (int i = c + 1 + tid; i < p; i += blockDim.x) {
            double acc = A[tri(i, c)];
            for (int l = 0; l < c; ++l) acc -= A[tri(i, l)] * A[tri(c, l)];
            A[tri(i, c)] = acc / A[tri(c, c)];
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int i = 0; i < p; ++i) {
            double acc = b[i];
            for (int l = 0; l < i; ++l) acc -= A[tri(i, l)] * x[l];
            x[i] = acc / A[tri(i, i)];
        }
        for (int i = p - 1; i >= 0; --i) {
            double acc = x[i];
            for (int l = i + 1; l < p; ++l) acc -= A[tri(l, i)] * x[l];
            x[i] = acc / A[tri(i, i)];
        }
    }
    __syncthreads();
    return *flag == 0;
}

// Payoff of point j from its log-prices (FP64, runtime d).
__device__ double point_payoff(const SpecT<double>& S, const double* __restrict__ x, int64_t N,
                               int64_t j)
{
    const int d = S.d;
    double v;
    if (S.payoff == CALL_MAX) {
        double mx = log(x[j]);
        for (int i = 1; i < d; ++i) mx = fmax(mx, log(x[i * N + j]));
        v = exp(mx) - S.K;
    } else if (S.payoff == PUT_GEO) {
        double sl = 0.0;
        for (int i = 0; i < d; ++i) sl += log(x[i * N + j]);
        v = S.K - exp(sl * S.inv_d);
    } else {
        double sm = 0.0;
        for (int i = 0; i < d; ++i) sm += exp(log(x[i * N + j]));
        v = S.K - sm * S.inv_d;
    }
    return v > 0.0 ? v : 0.0;
}

// Raw features phi = [1, u, u^2, g, g^2], labels e = [Phi - C > 0] and the
// in-the-money mask; tile sums of masked features and the count.
__global__ void k_fit_prep(const DevSpec* __restrict__ s, const double* __restrict__ x,
                           const double* __restrict__ cont, int64_t N, int p, double* phi,
                           double* lab, double* msk, double* part1)
{
    const SpecT<double>& S = s->f64;
    const int d = S.d;
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t j = j0 + threadIdx.x;
    if (j < N) {
        const double pay = point_payoff(S, x, N, j);
        const bool itm = pay > 0.0;
        msk[j] = itm ? 1.0 : 0.0;
        lab[j] = (pay - cont[j] > 0.0) ? 1.0 : 0.0;
        phi[j] = 1.0;
        for (int i = 0; i < d; ++i) {
            const double u = log(x[i * N + j]) - S.lnK;
            phi[(1 + i) * N + j] = u;
            phi[(1 + d + i) * N + j] = u * u;
        }
        const double g = pay / S.K;
        phi[(1 + 2 * d) * N + j] = g;
        phi[(2 + 2 * d) * N + j] = g * g;
    }
    __syncthreads();
    const int64_t j1 = min(N, j0 + (int64_t)blockDim.x);
    for (int f = threadIdx.x; f <= p; f += blockDim.x) {
        double acc = 0.0;
        for (int64_t jj = j0; jj < j1; ++jj) acc += (f < p) ? msk[jj] * phi[f * N + jj] : msk[jj];
        part1[(size_t)blockIdx.x * (p + 1) + f] = acc;
    }
}

// Tile sums of masked squared deviations from the means.
__global__ void k_fit_var(const double* __restrict__ phi, const double* __restrict__ msk, int64_t N,
                          int p, int ntiles, const double* __restrict__ part1, double* part2)
{
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t j1 = min(N, j0 + (int64_t)blockDim.x);
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        double sf = 0.0, cnt = 0.0;
        for (int t = 0; t < ntiles; ++t) {
            sf += part1[(size_t)t * (p + 1) + f];
            cnt += part1[(size_t)t * (p + 1) + p];
        }
        const double mu = cnt > 0.0 ? sf / cnt : 0.0;
        double acc = 0.0;
        for (int64_t jj = j0; jj < j1; ++jj) {
            const double dv = phi[f * N + jj] - mu;
            acc += msk[jj] * dv * dv;
        }
        part2[(size_t)blockIdx.x * p + f] = acc;
    }
}

// Means and standard deviations (columns 1..p-1; a constant column keeps
// scale 1), and the fitted-point count, into musd[2p + 1].
__global__ void k_fit_musd(int p, int ntiles, const double* __restrict__ part1,
                           const double* __restrict__ part2, double* musd)
{
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        double sf = 0.0, sv = 0.0, cnt = 0.0;
        for (int t = 0; t < ntiles; ++t) {
            sf += part1[(size_t)t * (p + 1) + f];
            sv += part2[(size_t)t * p + f];
            cnt += part1[(size_t)t * (p + 1) + p];
        }
        double mu = 0.0, sd = 1.0;
        if (f > 0 && cnt > 0.0) {
            mu = sf / cnt;
            sd = sqrt(sv / cnt);
            if (!(sd > 1e-12 * (1.0 + fabs(mu)))) sd = 1.0;
        }
        musd[f] = mu;
        musd[p + f] = sd;
        if (f == 0) musd[2 * p] = cnt;
    }
}

// One boosting round on a tile: apply the previous round's coefficients to
// F and pi, then accumulate this round's weighted normal equations.
__global__ void k_fit_step(const double* __restrict__ phi, const double* __restrict__ lab,
                           const double* __restrict__ msk, int64_t N, int p,
                           const double* __restrict__ musd, const double* __restrict__ beta_prev,
                           int round, int rounds, double* F, double* pi, double* partA)
{
    extern __shared__ double sh[];
    const double cnt = musd[2 * p];
    if (!(cnt > 0.0)) return;
    const int T = blockDim.x;
    double* psi = sh;              // [T][p]
    double* wz = psi + (size_t)T * p;   // [T][2]
    const int64_t j0 = (int64_t)blockIdx.x * T;
    const int64_t j = j0 + threadIdx.x;
    const int tl = threadIdx.x;
    if (j < N) {
        for (int f = 0; f < p; ++f)
            psi[tl * p + f] = f == 0 ? 1.0 : (phi[f * N + j] - musd[f]) / musd[p + f];
        double Fj, pj;
        if (round == 0) {
            Fj = 0.0;
            pj = 0.5;
        } else {
            double dF = 0.0;
            for (int f = 0; f < p; ++f) dF += beta_prev[f] * psi[tl * p + f];
            Fj = F[j] + 0.5 * dF;
            pj = 1.0 / (1.0 + exp(-2.0 * Fj));
        }
        F[j] = Fj;
        pi[j] = pj;
        double w = pj * (1.0 - pj);
        if (w < 1e-10) w = 1e-10;
        double z = (lab[j] - pj) / w;
        if (z > 4.0) z = 4.0;
        if (z < -4.0) z = -4.0;
        wz[2 * tl] = w * msk[j];
        wz[2 * tl + 1] = z;
    } else {
        for (int f = 0; f < p; ++f) psi[tl * p + f] = 0.0;
        wz[2 * tl] = 0.0;
        wz[2 * tl + 1] = 0.0;
    }
    __syncthreads();
    if (round >= rounds) return;
    const int npairs = p * (p + 1) / 2;
    const int nt = (int)min((int64_t)T, N - j0);
    for (int q = threadIdx.x; q < npairs + p; q += T) {
        double acc = 0.0;
        if (q < npairs) {
            int a, b;
            pair_of(q, a, b);
            for (int t = 0; t < nt; ++t) acc += wz[2 * t] * psi[t * p + a] * psi[t * p + b];
        } else {
            const int a = q - npairs;
            for (int t = 0; t < nt; ++t) acc += wz[2 * t] * wz[2 * t + 1] * psi[t * p + a];
        }
        partA[(size_t)blockIdx.x * (npairs + p) + q] = acc;
    }
}

// Merges the tile normal equations of one round and solves them.
__global__ void k_fit_solve(int p, int ntiles, const double* __restrict__ partA,
                            const double* __restrict__ musd, double lam_rel, double* Awork,
                            double* beta_out)
{
    __shared__ int flag;
    __shared__ double lam;
    if (!(musd[2 * p] > 0.0)) return;
    const int npairs = p * (p + 1) / 2;
    double* A = Awork;            // [npairs]
    double* b = Awork + npairs;   // [p]
    for (int q = threadIdx.x; q < npairs + p; q += blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < ntiles; ++t) acc += partA[(size_t)t * (npairs + p) + q];
        Awork[q] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < p; ++i) tr += A[tri(i, i)];
        lam = lam_rel * tr / p;
    }
    __syncthreads();
    if (!block_spd_solve(p, A, lam, b, beta_out, &flag)) {
        for (int f = threadIdx.x; f < p; f += blockDim.x) beta_out[f] = 0.0;
    }
}

// gamma = sum_r beta_r / 2, folded through the standardisation onto raw
// features: w_f = gamma_f / sd_f, w_0 = gamma_0 - sum_f gamma_f mu_f / sd_f.
__global__ void k_fit_fold(int p, int rounds, const double* __restrict__ musd,
                           const double* __restrict__ beta, double* row64, float* row32)
{
    if (threadIdx.x != 0) return;
    const bool any = musd[2 * p] > 0.0;
    double w0 = 0.0;
    for (int f = 0; f < p; ++f) {
        double g = 0.0;
        if (any)
            for (int r = 0; r < rounds; ++r) g += 0.5 * beta[r * p + f];
        if (f == 0) {
            w0 += g;
        } else {
            const double wf = g / musd[p + f];
            w0 -= g * musd[f] / musd[p + f];
            row64[f] = wf;
            row32[f] = (float)wf;
        }
    }
    row64[0] = w0;
    row32[0] = (float)w0;
}

static int fit_tile(int p)
{
    if (p <= 48) return 128;
    if (p <= 96) return 64;
    return 32;
}

size_t fit_scratch_doubles(int64_t N, int p, int rounds)
{
    const int T = fit_tile(p);
    const int64_t tiles = (N + T - 1) / T;
    const int64_t npairs = (int64_t)p * (p + 1) / 2;
    return (size_t)(p * N + 4 * N + tiles * (p + 1) + tiles * p + tiles * (npairs + p) +
                    (int64_t)rounds * p + (2 * p + 1) + (npairs + p) + 64);
}

void fit_scratch_carve(double* base, int64_t N, int p, int rounds, FitScratch* fs)
{
    const int T = fit_tile(p);
    const int64_t tiles = (N + T - 1) / T;
    const int64_t npairs = (int64_t)p * (p + 1) / 2;
    double* c = base;
    fs->phi = c; c += p * N;
    fs->lab = c; c += N;
    fs->msk = c; c += N;
    fs->F = c; c += N;
    fs->pi = c; c += N;
    fs->part1 = c; c += tiles * (p + 1);
    fs->part2 = c; c += tiles * p;
    fs->partA = c; c += tiles * (npairs + p);
    fs->beta = c; c += (int64_t)rounds * p;
    (void)c;
}

hipError_t launch_fit_cmc(const DevSpec* s, int d, const double* x, const double* cont, int64_t N,
                          int rounds, const FitScratch& fs, double* row64, float* row32,
                          hipStream_t st)
{
    const int p = rule_width(CMC, d);
    const int T = fit_tile(p);
    const int tiles = (int)((N + T - 1) / T);
    const int npairs = p * (p + 1) / 2;
    double* musd = fs.beta + (size_t)rounds * p;
    double* Awork = musd + 2 * p + 1;
    hipLaunchKernelGGL(k_fit_prep, dim3(tiles), dim3(T), 0, st, s, x, cont, N, p, fs.phi, fs.lab,
                       fs.msk, fs.part1);
    hipLaunchKernelGGL(k_fit_var, dim3(tiles), dim3(T), 0, st, fs.phi, fs.msk, N, p, tiles, fs.part1,
                       fs.part2);
    hipLaunchKernelGGL(k_fit_musd, dim3(1), dim3(256), 0, st, p, tiles, fs.part1, fs.part2, musd);
    const size_t lds = sizeof(double) * ((size_t)T * p + 2 * T);
    for (int r = 0; r < rounds; ++r) {
        const double* bprev = r > 0 ? fs.beta + (size_t)(r - 1) * p : nullptr;
        hipLaunchKernelGGL(k_fit_step, dim3(tiles), dim3(T), lds, st, fs.phi, fs.lab, fs.msk, N, p,
                           musd, bprev, r, rounds, fs.F, fs.pi, fs.partA);
        hipLaunchKernelGGL(k_fit_solve, dim3(1), dim3(256), 0, st, p, tiles, fs.partA, musd, 1e-8,
                           Awork, fs.beta + (size_t)r * p);
    }
    (void)npairs;
    hipLaunchKernelGGL(k_fit_fold, dim3(1), dim3(64), 0, st, p, rounds, musd, fs.beta, row64, row32);
    return hipGetLastError();
}

// I&Z regression: tile normal equations of ln s* on xi = [1, v, v_a v_b].
__global__ void k_fitiz_part(const DevSpec* __restrict__ s, const double* __restrict__ x, int64_t J,
                             int p, double* part)
{
    extern __shared__ double sh[];
    const SpecT<double>& S = s->f64;
    const int d = S.d, q = d - 1;
    const int T = blockDim.x;
    double* xi = sh;                     // [T][p]
    double* ym = xi + (size_t)T * p;     // [T][2]
    const int64_t j0 = (int64_t)blockIdx.x * T;
    const int64_t j = j0 + threadIdx.x;
    const int tl = threadIdx.x;
    const double sst = j < J ? x[j] : -1.0;
    if (sst > 0.0) {
        xi[tl * p] = 1.0;
        for (int a = 0; a < q; ++a) xi[tl * p + 1 + a] = log(x[(a + 1) * J + j]) - S.lnK;
        int f = 1 + q;
        for (int a = 0; a < q; ++a)
            for (int c = a; c < q; ++c) {
                xi[tl * p + f] = xi[tl * p + 1 + a] * xi[tl * p + 1 + c];
                ++f;
            }
        ym[2 * tl] = log(sst);
        ym[2 * tl + 1] = 1.0;
    } else {
        for (int f = 0; f < p; ++f) xi[tl * p + f] = 0.0;
        ym[2 * tl] = 0.0;
        ym[2 * tl + 1] = 0.0;
    }
    __syncthreads();
    const int npairs = p * (p + 1) / 2;
    const int nt = (int)min((int64_t)T, J - j0);
    for (int qq = threadIdx.x; qq <= npairs + p; qq += T) {
        double acc = 0.0;
        if (qq < npairs) {
            int a, b;
            pair_of(qq, a, b);
            for (int t = 0; t < nt; ++t) acc += xi[t * p + a] * xi[t * p + b];
        } else if (qq < npairs + p) {
            const int a = qq - npairs;
            for (int t = 0; t < nt; ++t) acc += xi[t * p + a] * ym[2 * t];
        } else {
            for (int t = 0; t < nt; ++t) acc += ym[2 * t + 1];
        }
        part[(size_t)blockIdx.x * (npairs + p + 1) + qq] = acc;
    }
}

__global__ void k_fitiz_solve(const DevSpec* __restrict__ s, int p, int ntiles,
                              const double* __restrict__ part, double* Awork, double* row64,
                              float* row32)
{
    __shared__ int flag;
    __shared__ double lam, cnt;
    // no converged point: a boundary no price crosses (puts below, the call above)
    const double dir_never = s->f64.payoff == CALL_MAX ? 1e300 : -1e300;
    const int npairs = p * (p + 1) / 2;
    double* A = Awork;
    double* b = Awork + npairs;
    double* sol = b + p;
    for (int q = threadIdx.x; q <= npairs + p; q += blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < ntiles; ++t) acc += part[(size_t)t * (npairs + p + 1) + q];
        if (q < npairs + p) Awork[q] = acc;
        else cnt = acc;
    }
    __syncthreads();
    if (!(cnt > 0.0)) {
        for (int f = threadIdx.x; f < p; f += blockDim.x) {
            const double v = f == 0 ? dir_never : 0.0;
            row64[f] = v;
            row32[f] = (float)v;
        }
        return;
    }
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < p; ++i) tr += A[tri(i, i)];
        lam = 1e-10 * tr / p;
    }
    __syncthreads();
    const bool ok = block_spd_solve(p, A, lam, b, sol, &flag);
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        const double v = ok ? sol[f] : (f == 0 ? dir_never : 0.0);
        row64[f] = v;
        row32[f] = (float)v;
    }
}

static int fitiz_tile(int p) { return p <= 48 ? 128 : 64; }

size_t fitiz_scratch_doubles(int64_t J, int p)
{
    const int T = fitiz_tile(p);
    const int64_t tiles = (J + T - 1) / T;
    const int64_t npairs = (int64_t)p * (p + 1) / 2;
    return (size_t)(tiles * (npairs + p + 1) + npairs + 2 * p + 64);
}

hipError_t launch_fit_iz(const DevSpec* s, int d, const double* x, int64_t J, double* scratch,
                         double* row64, float* row32, hipStream_t st)
{
    const int p = rule_width(IZ, d);
    const int T = fitiz_tile(p);
    const int tiles = (int)((J + T - 1) / T);
    const int npairs = p * (p + 1) / 2;
    double* part = scratch;
    double* Awork = scratch + (size_t)tiles * (npairs + p + 1);
    const size_t lds = sizeof(double) * ((size_t)T * p + 2 * T);
    hipLaunchKernelGGL(k_fitiz_part, dim3(tiles), dim3(T), lds, st, s, x, J, p, part);
    hipLaunchKernelGGL(k_fitiz_solve, dim3(1), dim3(256), 0, st, s, p, tiles, part, Awork, row64,
                       row32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Raw generator access for verification.

__global__ void k_philox(uint32_t k0, uint32_t k1, const uint32_t* __restrict__ ctr, int64_t M,
                         uint32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const Words w = philox(k0, k1, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    for (int h = 0; h < 4; ++h) out[4 * i + h] = w.w[h];
}

__global__ void k_normals(uint32_t k0, uint32_t k1, const uint32_t* __restrict__ ctr, int64_t M,
                          int prec, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const Words w = philox(k0, k1, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    if (prec == PREC_FP64) {
        double z[4];
        box_muller(w.w[0], w.w[1], z[0], z[1]);
        box_muller(w.w[2], w.w[3], z[2], z[3]);
        for (int h = 0; h < 4; ++h) out[4 * i + h] = z[h];
    } else {
        float z[4];
        box_muller(w.w[0], w.w[1], z[0], z[1]);
        box_muller(w.w[2], w.w[3], z[2], z[3]);
        for (int h = 0; h < 4; ++h) out[4 * i + h] = (double)z[h];
    }
}

hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M, uint32_t* out,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, k0, k1, ctr, M, out);
    return hipGetLastError();
}

hipError_t launch_normals(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M, int prec,
                          double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_normals, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, k0, k1, ctr, M,
                       prec, out);
    return hipGetLastError();
}

}  // namespace bmc
