// Device arithmetic of the FP64 rule fits, shared by the one-launch (grid
// barrier) and multi-launch forms so that both give identical rules.
// Reductions are deterministic: a tile is reduced sequentially by one thread
// per output quantity; tiles are merged in tile order.
#pragma once

#include "internal.hpp"

namespace bmc {

__device__ __forceinline__ int tri(int i, int l) { return i * (i + 1) / 2 + l; }

// q-th entry of a packed lower triangle -> (row i, column l <= i): the row
// from the square root, then corrected by at most a step either way.
__device__ __forceinline__ void pair_of(int q, int& i, int& l)
{
    i = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    if (i * (i + 1) / 2 > q) --i;
    if ((i + 1) * (i + 2) / 2 <= q) ++i;
    l = q - i * (i + 1) / 2;
}

// Solves (A + lam I) x = b for the packed lower triangle A (overwritten by
// its Cholesky factor; b is overwritten too).  Whole block; false if a pivot
// is not positive.  Right-looking, column-parallel: every entry still
// subtracts its terms in increasing column order, as the sequential
// left-looking factorisation and substitutions do.
__device__ inline bool block_spd_solve(int p, double* A, double lam, double* b, double* x, int* flag)
{
    const int tid = threadIdx.x, T = blockDim.x;
    if (tid == 0) *flag = 0;
    for (int i = tid; i < p; i += T) A[tri(i, i)] += lam;
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        if (tid == 0) {
            double v = A[tri(c, c)];
            if (!(v > 0.0)) {
                *flag = 1;
                v = 1.0;
            }
            A[tri(c, c)] = sqrt(v);
        }
        __syncthreads();
        const double lcc = A[tri(c, c)];
        for (int i = c + 1 + tid; i < p; i += T) A[tri(i, c)] /= lcc;
        __syncthreads();
        // trailing update A_il -= L_ic L_lc for c < l <= i
        const int m = p - c - 1;
        for (int e = tid; e < m * (m + 1) / 2; e += T) {
            int ii, ll;
            pair_of(e, ii, ll);
            const int i = c + 1 + ii, l = c + 1 + ll;
            A[tri(i, l)] -= A[tri(i, c)] * A[tri(l, c)];
        }
        __syncthreads();
    }
    // forward substitution L y = b (y in b), then L^T x = y
    for (int c = 0; c < p; ++c) {
        if (tid == 0) b[c] /= A[tri(c, c)];
        __syncthreads();
        for (int i = c + 1 + tid; i < p; i += T) b[i] -= A[tri(i, c)] * b[c];
        __syncthreads();
    }
    for (int c = p - 1; c >= 0; --c) {
        if (tid == 0) x[c] = b[c] / A[tri(c, c)];
        __syncthreads();
        for (int i = tid; i < c; i += T) b[i] -= A[tri(c, i)] * x[c];
        __syncthreads();
    }
    return *flag == 0;
}

// Value of v in lane src (uniform src), through the scalar unit.
__device__ __forceinline__ double bcast_lane(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// The same factorisation and substitutions by one wavefront (the calling
// threads must be lanes 0..63 of one wave, all active): lane i keeps row i
// of the factor in registers and the columns travel by lane broadcasts,
// with no block barrier.  Same per-entry subtraction order as above; the
// divisions by a pivot become products with its reciprocal, which comes
// with the pivot from a refined reciprocal square root (no division).  The
// forward substitution runs inside the factorisation: column c of L is final
// once pivot c has scaled it, so y_c and the updates of the later y_i follow
// at once, in the same order as a separate pass.  Updates run on every lane:
// entries above the diagonal, and a lane's y once its own pivot has taken
// it, receive values that are never read.  Pivot lane c scales its diagonal
// like the rest of the column, dc / sqrt(dc) = L_cc.  A (packed, in LDS) is
// overwritten with the factor.
// Returns false (on every lane) if a pivot is not positive.
template <int P>
__device__ bool wave_spd_solve(int p, double* A, double lam, const double* b, double* x)
{
    const int lane = threadIdx.x & 63;
    // lane i holds row i of A + lam I; rows p..P-1 are the identity, so every
    // column runs without tests
    double row[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double v = (lane < p && k <= lane) ? A[tri(lane, k)] : 0.0;
        if (k == lane) v += lane < p ? lam : 1.0;
        row[k] = v;
    }
    bool ok = true;
    double invd = 1.0;   // lane c: 1 / L_cc
    double y = lane < p ? b[lane] : 0.0;
    double yf = 0.0;     // lane c: y_c of L y = b
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double dc = bcast_lane(row[c], c);
        if (!(dc > 0.0)) {
            ok = false;
            dc = 1.0;
        }
        // 1/sqrt(dc) from the hardware estimate and two Newton steps
        // y <- y (3 - dc y^2) / 2
        double inv = __builtin_amdgcn_rsq(dc);
        inv = inv * (1.5 - 0.5 * dc * inv * inv);
        inv = inv * (1.5 - 0.5 * dc * inv * inv);
        row[c] *= inv;
        const double yc = bcast_lane(y, c) * inv;
        if (lane == c) {
            invd = inv;
            yf = yc;
        }
        y -= row[c] * yc;
#pragma unroll
        for (int l = c + 1; l < P; ++l) {
            const double llc = bcast_lane(row[c], l);
            row[l] -= row[c] * llc;
        }
    }
    // L back into the packed triangle; each lane then reads its column, so
    // that the back substitution L^T x = y needs no per-entry broadcasts
    if (lane < p) {
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (k <= lane) A[tri(lane, k)] = row[k];
    }
    __builtin_amdgcn_wave_barrier();
    double col[P];
#pragma unroll
    for (int c = 0; c < P; ++c) col[c] = (lane < p && c >= lane && c < p) ? A[tri(c, lane)] : 0.0;
    double xv = 0.0;
    y = yf;
#pragma unroll
    for (int c = P - 1; c >= 0; --c) {
        const double xc = bcast_lane(y * invd, c);
        if (lane == c) xv = xc;
        y -= col[c] * xc;
    }
    if (lane < p) x[lane] = xv;
    return ok;
}

// Sum of the diagonal of the packed A by one wavefront, in row order (lane
// i reads A_ii; the sum runs over lane broadcasts).
template <int P>
__device__ __forceinline__ double wave_trace(int p, const double* A)
{
    const int lane = threadIdx.x & 63;
    const double v = lane < p ? A[tri(lane, lane)] : 0.0;
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) tr += bcast_lane(v, i);
    return tr;
}

// Dispatch for a whole block: one wavefront solves small systems in
// registers, larger ones use the block form.  A and b are scratch.
__device__ inline bool spd_solve(int p, double* A, double lam, double* b, double* x, int* flag);

// The same with the ridge lam = scale tr(A) / p: for p <= 32 the trace is
// summed by the solving wavefront itself (no block barrier before the solve);
// *lam_out (LDS) receives lam.
__device__ __forceinline__ bool spd_solve_ridge(int p, double* A, double scale, double* b, double* x, int* flag,
                                       double* lam_out)
{
    if (p <= 32) {
        if (threadIdx.x < 64) {
            const double lam = scale * (p <= 16 ? wave_trace<16>(p, A) : wave_trace<32>(p, A)) / p;
            if (threadIdx.x == 0) *lam_out = lam;
            bool ok;
            switch (p) {
            case 5: ok = wave_spd_solve<5>(p, A, lam, b, x); break;
            case 7: ok = wave_spd_solve<7>(p, A, lam, b, x); break;
            case 9: ok = wave_spd_solve<9>(p, A, lam, b, x); break;
            case 11: ok = wave_spd_solve<11>(p, A, lam, b, x); break;
            case 13: ok = wave_spd_solve<13>(p, A, lam, b, x); break;
            case 15: ok = wave_spd_solve<15>(p, A, lam, b, x); break;
            default: ok = p <= 16 ? wave_spd_solve<16>(p, A, lam, b, x) : wave_spd_solve<32>(p, A, lam, b, x);
            }
            if (threadIdx.x == 0) *flag = ok ? 0 : 1;
        }
        __syncthreads();
        return *flag == 0;
    }
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < p; ++i) tr += A[tri(i, i)];
        *lam_out = scale * tr / p;
    }
    __syncthreads();
    return block_spd_solve(p, A, *lam_out, b, x, flag);
}

__device__ inline bool spd_solve(int p, double* A, double lam, double* b, double* x, int* flag)
{
    if (p <= 32) {
        if (threadIdx.x < 64) {
            bool ok;
            switch (p) {   // exact widths of the CMC rules for d <= 6 (p = 2d + 3)
            case 5: ok = wave_spd_solve<5>(p, A, lam, b, x); break;
            case 7: ok = wave_spd_solve<7>(p, A, lam, b, x); break;
            case 9: ok = wave_spd_solve<9>(p, A, lam, b, x); break;
            case 11: ok = wave_spd_solve<11>(p, A, lam, b, x); break;
            case 13: ok = wave_spd_solve<13>(p, A, lam, b, x); break;
            case 15: ok = wave_spd_solve<15>(p, A, lam, b, x); break;
            default: ok = p <= 16 ? wave_spd_solve<16>(p, A, lam, b, x) : wave_spd_solve<32>(p, A, lam, b, x);
            }
            if (threadIdx.x == 0) *flag = ok ? 0 : 1;
        }
        __syncthreads();
        return *flag == 0;
    }
    return block_spd_solve(p, A, lam, b, x, flag);
}

// Intrinsic value of point j from its log-prices, before its positive part
// is taken (FP64, runtime d): negative out of the money.
__device__ inline double point_intrinsic(const SpecT<double>& S, const double* __restrict__ x, int64_t N, int64_t j)
{
    const int d = S.d;
    double v;
    if (S.payoff == CALL_MAX) {
        double mx = log(x[j]);
        for (int i = 1; i < d; ++i) mx = fmax(mx, log(x[i * N + j]));
        v = exp(mx) - S.K;
    } else if (S.payoff == CALL_MIN) {
        double mn = log(x[j]);
        for (int i = 1; i < d; ++i) mn = fmin(mn, log(x[i * N + j]));
        v = exp(mn) - S.K;
    } else if (S.payoff == PUT_GEO) {
        double sl = 0.0;
        for (int i = 0; i < d; ++i) sl += log(x[i * N + j]);
        v = S.K - exp(sl * S.inv_d);
    } else {
        double sm = 0.0;
        for (int i = 0; i < d; ++i) sm += exp(log(x[i * N + j]));
        v = S.K - sm * S.inv_d;
    }
    return v;
}

// Payoff of point j (FP64, runtime d).
__device__ inline double point_payoff(const SpecT<double>& S, const double* __restrict__ x, int64_t N, int64_t j)
{
    const double v = point_intrinsic(S, x, N, j);
    return v > 0.0 ? v : 0.0;
}

// FP32 label refinement (REFINE_KAPPA): lists in-the-money point j (payoff
// Phi) when its estimate c lies within REFINE_KAPPA standard errors se (plus
// REFINE_ETA (Phi + |c|) for rounding) of Phi.
__device__ inline void refine_point(const SpecT<double>& S, const double* __restrict__ x, int64_t N, int64_t j,
                                    double c, double se, int32_t* ids, int32_t* n_ids)
{
    const double pay = point_payoff(S, x, N, j);
    if (!(pay > 0.0)) return;   // out of the money: never in the fit
    const double tol = REFINE_KAPPA * se + REFINE_ETA * (pay + fabs(c));
    if (fabs(pay - c) <= tol) ids[atomicAdd(n_ids, 1)] = (int32_t)j;
}

// CMC training data of point j: raw features phi = [1, u, u^2, g, g^2]
// (column f at phi[f*N + j]), label e = [Phi - C > 0], in-the-money mask.
__device__ inline void fit_prep_point(const SpecT<double>& S, const double* __restrict__ x,
                                      const double* __restrict__ cont, int64_t N, int64_t j, double* phi,
                                      double* lab, double* msk)
{
    if (j >= N) return;
    const int d = S.d;
    const double pay = point_payoff(S, x, N, j);
    msk[j] = pay > 0.0 ? 1.0 : 0.0;
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

// out[f] = sum over the tile of msk * phi_f (f < p), out[p] = sum of msk.
__device__ inline void fit_tile_feature_sums(const double* phi, const double* msk, int64_t N, int p,
                                             int64_t j0, int T, double* out)
{
    const int64_t j1 = min(N, j0 + (int64_t)T);
    for (int f = threadIdx.x; f <= p; f += blockDim.x) {
        double acc = 0.0;
        for (int64_t jj = j0; jj < j1; ++jj) acc += (f < p) ? msk[jj] * phi[f * N + jj] : msk[jj];
        out[f] = acc;
    }
}

// out[f] = sum over the tile of msk * (phi_f - mu_f)^2.
__device__ inline void fit_tile_var_sums(const double* phi, const double* msk, int64_t N, int p, int64_t j0,
                                         int T, const double* mu, double* out)
{
    const int64_t j1 = min(N, j0 + (int64_t)T);
    for (int f = threadIdx.x; f < p; f += blockDim.x) {
        double acc = 0.0;
        for (int64_t jj = j0; jj < j1; ++jj) {
            const double dv = phi[f * N + jj] - mu[f];
            acc += msk[jj] * dv * dv;
        }
        out[f] = acc;
    }
}

// One tile (count c, feature sum s, squared deviations q from its own mean)
// added to the running count n, mean m and squared deviations M2.
__device__ __forceinline__ void chan_merge(double c, double s, double q, double& n, double& m, double& M2)
{
    if (!(c > 0.0)) return;
    const double mt = s / c, dm = mt - m, nn = n + c;
    m += dm * (c / nn);
    M2 += q + dm * dm * (n * c / nn);
    n = nn;
}

// Standardisation of column f from the merged count, mean and squared
// deviations; the constant column and a (numerically) constant feature keep
// scale 1.
__device__ __forceinline__ void fit_mu_sd_merged(int f, double cnt, double mean, double M2, double* mu, double* sd)
{
    double m = 0.0, s = 1.0;
    if (f > 0 && cnt > 0.0) {
        m = mean;
        s = sqrt(M2 / cnt);
        if (!(s > 1e-12 * (1.0 + fabs(m)))) s = 1.0;
    }
    *mu = m;
    *sd = s;
}

// Standardisation of column f from the merged sums; the constant column and
// a (numerically) constant feature keep scale 1.
__device__ __forceinline__ void fit_mu_sd(int f, double cnt, double sf, double sv, double* mu, double* sd)
{
    double m = 0.0, s = 1.0;
    if (f > 0 && cnt > 0.0) {
        m = sf / cnt;
        s = sqrt(sv / cnt);
        if (!(s > 1e-12 * (1.0 + fabs(m)))) s = 1.0;
    }
    *mu = m;
    *sd = s;
}

// One boosting round at point j (tile row tl = threadIdx.x): standardised
// features into psi, F += beta_prev . psi / 2 (if beta_prev), pi = 1/(1 +
// exp(-2F)), weight w = max(pi(1-pi), 1e-10) (masked) and working response
// z = clip((e - pi)/w, -4, 4) into wz.
__device__ inline void fit_round_point(const double* phi, const double* lab, const double* msk, int64_t N, int p,
                                       const double* mu, const double* sd, const double* beta_prev, int64_t j,
                                       double* F, double* pi, double* psi, double* wz)
{
    const int tl = threadIdx.x;
    if (j < N) {
        for (int f = 0; f < p; ++f) psi[tl * p + f] = f == 0 ? 1.0 : (phi[f * N + j] - mu[f]) / sd[f];
        double Fj, pj;
        if (!beta_prev) {
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
}

// Weighted normal equations of the tile: out[q] = sum w psi_a psi_b for the
// packed pair q = (a, b), then out[npairs + a] = sum w z psi_a.
__device__ inline void fit_tile_normal_eqs(const double* psi, const double* wz, int p, int nt, double* out)
{
    const int npairs = p * (p + 1) / 2;
    for (int q = threadIdx.x; q < npairs + p; q += blockDim.x) {
        double acc = 0.0;
        if (q < npairs) {
            int a, b;
            pair_of(q, a, b);
#pragma unroll 8
            for (int t = 0; t < nt; ++t) acc += wz[2 * t] * psi[t * p + a] * psi[t * p + b];
        } else {
            const int a = q - npairs;
#pragma unroll 8
            for (int t = 0; t < nt; ++t) acc += wz[2 * t] * wz[2 * t + 1] * psi[t * p + a];
        }
        out[q] = acc;
    }
}

// gamma = sum_r beta_r / 2 folded through the standardisation onto the raw
// features: w_f = gamma_f / sd_f, w_0 = gamma_0 - sum_f gamma_f mu_f / sd_f.
__device__ inline void fit_fold(int p, int rounds, const double* musd, const double* beta, double* row64,
                                float* row32)
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

// Tile reduction of nq quantities over the nt tile points, value(q, t), in
// two fixed levels: SUB runs of consecutive points per quantity, each summed
// in order by one thread, then the runs summed in order.  red: LDS [nq*SUB].
constexpr int TILE_SUB = 16;

template <class F>
__device__ inline void tile_sum2(int nq, int nt, F value, double* red, double* out)
{
    const int T = blockDim.x;
    const int run = (nt + TILE_SUB - 1) / TILE_SUB;
    for (int e = threadIdx.x; e < nq * TILE_SUB; e += T) {
        const int q = e / TILE_SUB, s = e % TILE_SUB;
        const int t0 = s * run, t1 = min(nt, t0 + run);
        double acc = 0.0;
        for (int t = t0; t < t1; ++t) acc += value(q, t);
        red[e] = acc;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += T) {
        double acc = 0.0;
        for (int s = 0; s < TILE_SUB; ++s) acc += red[q * TILE_SUB + s];
        out[q] = acc;
    }
    __syncthreads();
}

// Boosting round at point j for the matrix-core path (p <= 15): as
// fit_round_point, but the tile row has stride 16 and holds
// [psi_0..psi_{p-1}, z, 0...]; w goes to wz[2 tl].
__device__ inline void fit_round_point16(const double* phi, const double* lab, const double* msk, int64_t N,
                                         int p, const double* mu, const double* sd, const double* beta_prev,
                                         int64_t j, double* F, double* pi, double* psi16, double* wz)
{
    const int tl = threadIdx.x;
    double* row = psi16 + 16 * tl;
    if (j < N) {
        for (int f = 0; f < p; ++f) row[f] = f == 0 ? 1.0 : (phi[f * N + j] - mu[f]) / sd[f];
        double Fj, pj;
        if (!beta_prev) {
            Fj = 0.0;
            pj = 0.5;
        } else {
            double dF = 0.0;
            for (int f = 0; f < p; ++f) dF += beta_prev[f] * row[f];
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
        row[p] = z;
        for (int f = p + 1; f < 16; ++f) row[f] = 0.0;
        wz[2 * tl] = w * msk[j];
    } else {
        for (int f = 0; f < 16; ++f) row[f] = 0.0;
        wz[2 * tl] = 0.0;
    }
}

// Boosting round at point j for the wide matrix-core path (16 <= p <= 96): as
// fit_round_point16 with row stride S = 16 ceil((p+1)/16).
__device__ inline void fit_round_point_s(const double* phi, const double* lab, const double* msk, int64_t N, int p,
                                         int S, const double* mu, const double* sd, const double* beta_prev,
                                         int64_t j, double* F, double* pi, double* psis, double* wz)
{
    const int tl = threadIdx.x;
    double* row = psis + (size_t)S * tl;
    if (j < N) {
        for (int f = 0; f < p; ++f) row[f] = f == 0 ? 1.0 : (phi[f * N + j] - mu[f]) / sd[f];
        double Fj, pj;
        if (!beta_prev) {
            Fj = 0.0;
            pj = 0.5;
        } else {
            double dF = 0.0;
            for (int f = 0; f < p; ++f) dF += beta_prev[f] * row[f];
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
        row[p] = z;
        for (int f = p + 1; f < S; ++f) row[f] = 0.0;
        wz[2 * tl] = w * msk[j];
    } else {
        for (int f = 0; f < S; ++f) row[f] = 0.0;
        wz[2 * tl] = 0.0;
    }
}

// Later boosting rounds of a block that keeps its tile for the whole fit:
// the standardised features are still in row[0..p) (stride SW) and F, the
// label and the mask of its point are in registers; same arithmetic as
// fit_round_point16 / fit_round_point_s.
__device__ inline void fit_round_point_resident(int p, int SW, bool in, const double* beta_prev, double& F,
                                                double lab, double msk, double* psis, double* wz)
{
    const int tl = threadIdx.x;
    double* row = psis + (size_t)SW * tl;
    if (!in) return;   // row and weight stay zero
    double dF = 0.0;
    for (int f = 0; f < p; ++f) dF += beta_prev[f] * row[f];
    const double Fj = F + 0.5 * dF;
    const double pj = 1.0 / (1.0 + exp(-2.0 * Fj));
    F = Fj;
    double w = pj * (1.0 - pj);
    if (w < 1e-10) w = 1e-10;
    double z = (lab - pj) / w;
    if (z > 4.0) z = 4.0;
    if (z < -4.0) z = -4.0;
    row[p] = z;
    wz[2 * tl] = w * msk;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Weighted Gram matrix of a tile for 16 <= p <= 96 on the FP64 matrix cores:
// the (p+1)-wide rows r_t = [psi, z, 0..] (stride S = 16 nb) give nb(nb+1)/2
// lower 16x16 blocks G[bi][bj] = sum_t w_t r_t[16bi..] r_t[16bj..]^T; wave w
// takes blocks w, w + waves, .., each over all points of the tile (one
// 16x16x4 MFMA per four points), and writes its entries of the packed
// normal equations (A, then b_J = G[p][J]) straight to out.
__device__ inline void fit_tile_normal_eqs_mfma_wide(const double* psis, int S, const double* wz, int p, int nt,
                                                     double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int nb = S / 16, nbp = nb * (nb + 1) / 2;
    const int npairs = p * (p + 1) / 2;
    const int c = lane & 15, kq = lane >> 4;
    for (int pr = wave; pr < nbp; pr += waves) {
        int bi, bj;
        pair_of(pr, bi, bj);
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < nt; k0 += 4) {
            const int t = k0 + kq;
            const bool in = t < nt;
            const double ra = in ? psis[(size_t)S * t + 16 * bi + c] : 0.0;
            const double rb = in ? psis[(size_t)S * t + 16 * bj + c] : 0.0;
            const double w = in ? wz[2 * t] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w * ra, rb, acc, 0, 0, 0);
        }
        // D[i][j] sits in lane j + 16 (i % 4), element i / 4
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int I = 16 * bi + 4 * e + kq, J = 16 * bj + c;
            if (I < p && J <= I) out[tri(I, J)] = acc[e];
            else if (I == p && J < p) out[npairs + J] = acc[e];
        }
    }
}

// Weighted Gram matrix of the tile on the matrix cores: G = sum_t w_t
// r_t r_t^T with r_t = [psi, z, 0..] (16 wide), one 16x16x4 FP64 MFMA per
// four points; wave k covers points 64k..64k+63 and the waves' partial G are
// merged in wave order.  Writes the packed normal equations (A, then the
// right-hand side G[a][p]) like fit_tile_normal_eqs.  aux: LDS [waves*256].
__device__ inline void fit_tile_normal_eqs_mfma(const double* psi16, const double* wz, int p, int nt, double* aux,
                                                double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = wave * 64; k0 < wave * 64 + 64; k0 += 4) {
        const int t = k0 + (lane >> 4);   // point of this lane's k
        const int c = lane & 15;          // row of A / column of B
        const double r = t < nt ? psi16[16 * t + c] : 0.0;
        const double w = t < nt ? wz[2 * t] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w * r, r, acc, 0, 0, 0);
    }
    // D[i][j] sits in lane j + 16 (i % 4), element i / 4
    for (int e = 0; e < 4; ++e) aux[wave * 256 + (4 * e + (lane >> 4)) * 16 + (lane & 15)] = acc[e];
    __syncthreads();
    const int npairs = p * (p + 1) / 2;
    for (int q = threadIdx.x; q < npairs + p; q += blockDim.x) {
        int i, l;
        if (q < npairs) pair_of(q, i, l);
        else { i = q - npairs; l = p; }
        double s = 0.0;
        for (int k = 0; k < waves; ++k) s += aux[k * 256 + i * 16 + l];
        out[q] = s;
    }
}

bool fit_one_launch_supported(int p);
// bar: two device words, zero before the first launch (the launch leaves
// them so); err: a pinned host word set to 1 if a grid barrier gave up.
hipError_t launch_fit_cmc_grid(const DevSpec* s, int d, const double* x, const double* cont, int64_t N,
                               int rounds, const FitScratch& fs, double* row64, float* row32, unsigned* bar,
                               int32_t* err, hipStream_t st);

}  // namespace bmc
