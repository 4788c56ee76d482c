// FP64 rule fits: the CMC boosting classifier (multi-launch form, used when
// the one-launch form does not fit in LDS) and the I&Z quadratic
// boundary regression.
#include "fit_common.hpp"

namespace bmc {

__global__ void k_fit_prep(const DevSpec* __restrict__ s, const double* __restrict__ x,
                           const double* __restrict__ cont, int64_t N, int p, double* phi, double* lab,
                           double* msk, double* part1)
{
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x;
    fit_prep_point(s->f64, x, cont, N, j0 + threadIdx.x, phi, lab, msk);
    __syncthreads();
    fit_tile_feature_sums(phi, msk, N, p, j0, blockDim.x, part1 + (size_t)blockIdx.x * (p + 1));
}

__global__ void k_fit_var(const double* __restrict__ phi, const double* __restrict__ msk, int64_t N, int p,
                          int ntiles, const double* __restrict__ part1, double* part2)
{
    extern __shared__ double mu[];
    double cnt = 0.0;
    for (int t = 0; t < ntiles; ++t) cnt += part1[(size_t)t * (p + 1) + p];
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        double sf = 0.0;
        for (int t = 0; t < ntiles; ++t) sf += part1[(size_t)t * (p + 1) + f];
        mu[f] = cnt > 0.0 ? sf / cnt : 0.0;
    }
    __syncthreads();
    fit_tile_var_sums(phi, msk, N, p, (int64_t)blockIdx.x * blockDim.x, blockDim.x, mu,
                      part2 + (size_t)blockIdx.x * p);
}

__global__ void k_fit_musd(int p, int ntiles, const double* __restrict__ part1, const double* __restrict__ part2,
                           double* musd)
{
    double cnt = 0.0;
    for (int t = 0; t < ntiles; ++t) cnt += part1[(size_t)t * (p + 1) + p];
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        double sf = 0.0, sv = 0.0;
        for (int t = 0; t < ntiles; ++t) {
            sf += part1[(size_t)t * (p + 1) + f];
            sv += part2[(size_t)t * p + f];
        }
        fit_mu_sd(f, cnt, sf, sv, &musd[f], &musd[p + f]);
    }
    if (threadIdx.x == 0) musd[2 * p] = cnt;
}

__global__ void k_fit_step(const double* __restrict__ phi, const double* __restrict__ lab,
                           const double* __restrict__ msk, int64_t N, int p, const double* __restrict__ musd,
                           const double* __restrict__ beta_prev, double* F, double* pi, double* partA)
{
    extern __shared__ double sh[];
    if (!(musd[2 * p] > 0.0)) return;
    const int T = blockDim.x;
    double* psi = sh;
    double* wz = psi + (size_t)T * p;
    const int64_t j0 = (int64_t)blockIdx.x * T;
    fit_round_point(phi, lab, msk, N, p, musd, musd + p, beta_prev, j0 + threadIdx.x, F, pi, psi, wz);
    __syncthreads();
    const int npairs = p * (p + 1) / 2;
    fit_tile_normal_eqs(psi, wz, p, (int)min((int64_t)T, N - j0), partA + (size_t)blockIdx.x * (npairs + p));
}

__global__ void k_fit_solve(int p, int ntiles, const double* __restrict__ partA, const double* __restrict__ musd,
                            double* Awork, double* beta_out)
{
    __shared__ int flag;
    __shared__ double lam;
    if (!(musd[2 * p] > 0.0)) return;
    const int npairs = p * (p + 1) / 2;
    for (int q = threadIdx.x; q < npairs + p; q += blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < ntiles; ++t) acc += partA[(size_t)t * (npairs + p) + q];
        Awork[q] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < p; ++i) tr += Awork[tri(i, i)];
        lam = 1e-8 * tr / p;
    }
    __syncthreads();
    if (!spd_solve(p, Awork, lam, Awork + npairs, beta_out, &flag))
        for (int f = threadIdx.x; f < p; f += blockDim.x) beta_out[f] = 0.0;
}

__global__ void k_fit_fold(int p, int rounds, const double* __restrict__ musd, const double* __restrict__ beta,
                           double* row64, float* row32)
{
    fit_fold(p, rounds, musd, beta, row64, row32);
}

size_t fit_scratch_doubles(int64_t N, int p, int rounds)
{
    const int T = fit_tile(p);
    const int64_t tiles = (N + T - 1) / T;
    const int64_t npairs = (int64_t)p * (p + 1) / 2;
    return (size_t)(p * N + 4 * N + tiles * (p + 1) + tiles * p + 2 * tiles * (npairs + p) +
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
    fs->partA = c; c += 2 * tiles * (npairs + p);
    fs->beta = c; c += (int64_t)rounds * p;
    (void)c;   // then musd [2p+1] and the solve workspace [npairs + p]
}

hipError_t launch_fit_cmc(const DevSpec* s, int d, const double* x, const double* cont, int64_t N, int rounds,
                          const FitScratch& fs, double* row64, float* row32, hipStream_t st, unsigned* bar,
                          int32_t* err)
{
    const int p = rule_width(CMC, d);
    if (bar && fit_one_launch_supported(p))
        return launch_fit_cmc_grid(s, d, x, cont, N, rounds, fs, row64, row32, bar, err, st);
    const int T = fit_tile(p);
    const int tiles = (int)((N + T - 1) / T);
    const int npairs = p * (p + 1) / 2;
    double* musd = fs.beta + (size_t)rounds * p;
    double* Awork = musd + 2 * p + 1;
    hipLaunchKernelGGL(k_fit_prep, dim3(tiles), dim3(T), 0, st, s, x, cont, N, p, fs.phi, fs.lab, fs.msk,
                       fs.part1);
    hipLaunchKernelGGL(k_fit_var, dim3(tiles), dim3(T), sizeof(double) * p, st, fs.phi, fs.msk, N, p, tiles,
                       fs.part1, fs.part2);
    hipLaunchKernelGGL(k_fit_musd, dim3(1), dim3(256), 0, st, p, tiles, fs.part1, fs.part2, musd);
    const size_t lds = sizeof(double) * ((size_t)T * p + 2 * T);
    for (int r = 0; r < rounds; ++r) {
        const double* bprev = r > 0 ? fs.beta + (size_t)(r - 1) * p : nullptr;
        hipLaunchKernelGGL(k_fit_step, dim3(tiles), dim3(T), lds, st, fs.phi, fs.lab, fs.msk, N, p, musd, bprev,
                           fs.F, fs.pi, fs.partA);
        hipLaunchKernelGGL(k_fit_solve, dim3(1), dim3(256), 0, st, p, tiles, fs.partA, musd, Awork,
                           fs.beta + (size_t)r * p);
    }
    (void)npairs;
    hipLaunchKernelGGL(k_fit_fold, dim3(1), dim3(64), 0, st, p, rounds, musd, fs.beta, row64, row32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// I&Z regression of one region: tile normal equations of ln s* on
// xi = [1, v, v_a v_c] over the converged points (s*_j > 0; v over the other
// assets in increasing order), then one solve.  Regions region0 + y side by
// side (blockIdx.y = y): region y's J points are columns y J .. y J + J - 1 of
// x (rows of ld entries), its partials and solve scratch at y times the
// given strides, its boundary block at y p of the row.  s* comes from
// sstar[y J + j] when given, else from the region's own row of x.

__global__ void k_fitiz_part(const DevSpec* __restrict__ s, const double* __restrict__ x,
                             const double* __restrict__ sstar, int region0, int64_t J, int64_t ld, int p,
                             double* part, size_t part_stride)
{
    extern __shared__ double sh[];
    const SpecT<double>& S = s->f64;
    const int d = S.d, q = d - 1;
    const int T = blockDim.x;
    const int region = region0 + (int)blockIdx.y;
    x += (size_t)blockIdx.y * J;
    part += (size_t)blockIdx.y * part_stride;
    double* xi = sh;                     // [T][p]
    double* ym = xi + (size_t)T * p;     // [T][2]
    const int64_t j0 = (int64_t)blockIdx.x * T;
    const int64_t j = j0 + threadIdx.x;
    const int tl = threadIdx.x;
    const double sst = j >= J ? -1.0 : (sstar ? sstar[(size_t)blockIdx.y * J + j] : x[region * ld + j]);
    if (sst > 0.0) {
        xi[tl * p] = 1.0;
        for (int a = 0; a < q; ++a) xi[tl * p + 1 + a] = log(x[(a < region ? a : a + 1) * ld + j]) - S.lnK;
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

__global__ void k_fitiz_solve(const DevSpec* __restrict__ s, int p, int ntiles, const double* __restrict__ part,
                              size_t part_stride, double* Awork, size_t awork_stride, double* row64, float* row32)
{
    __shared__ int flag;
    __shared__ double lam, cnt;
    part += (size_t)blockIdx.x * part_stride;
    Awork += (size_t)blockIdx.x * awork_stride;
    row64 += (size_t)blockIdx.x * p;
    row32 += (size_t)blockIdx.x * p;
    // no converged point: a boundary no price crosses (puts below, the call above)
    const double never = (s->f64.payoff == CALL_MAX || s->f64.payoff == CALL_MIN) ? 1e300 : -1e300;
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
            const double v = f == 0 ? never : 0.0;
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
    const bool ok = spd_solve(p, A, lam, b, sol, &flag);
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        const double v = ok ? sol[f] : (f == 0 ? never : 0.0);
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

hipError_t launch_fit_iz(const DevSpec* s, int d, int region, const double* x, int64_t J, int64_t ld,
                         double* scratch, double* row64, float* row32, hipStream_t st, int nreg,
                         const double* sstar)
{
    const int p = rule_width(IZ, d);
    const int T = fitiz_tile(p);
    const int tiles = (int)((J + T - 1) / T);
    const int npairs = p * (p + 1) / 2;
    // per region: tile partials, then the solve's work area
    const size_t part_stride = (size_t)tiles * (npairs + p + 1);
    const size_t region_stride = fitiz_scratch_doubles(J, p);
    double* part = scratch;
    double* Awork = scratch + part_stride;
    const size_t lds = sizeof(double) * ((size_t)T * p + 2 * T);
    hipLaunchKernelGGL(k_fitiz_part, dim3(tiles, nreg), dim3(T), lds, st, s, x, sstar, region, J, ld, p, part,
                       region_stride);
    hipLaunchKernelGGL(k_fitiz_solve, dim3(nreg), dim3(256), 0, st, s, p, tiles, part, region_stride, Awork,
                       region_stride, row64, row32);
    return hipGetLastError();
}

}  // namespace bmc
