// Device building blocks of the nested continuation-value Monte Carlo on
// gfx950: Philox4x32-10 counter generator, uniform-to-normal map, spec tables,
// payoffs and exercise-rule tests.  FP64 and FP32 variants share templates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmc {

constexpr int D_MAX = 64;
constexpr int NT_MAX = 512;

enum { PUT_BASKET = 0, CALL_MAX = 1, PUT_GEO = 2, CALL_MIN = 3 };
// CMC with the LogitBoost linear classifier, I&Z, CMC with AdaBoost stumps
enum { CMC = 0, IZ = 1, ADA = 2 };
// I&Z boundary-point search: plain fixed point or secant steps on its residual
enum { SEARCH_PLAIN = 0, SEARCH_SECANT = 1 };
// AdaBoost stumps: bins per feature, largest number of rounds a rule row holds
enum { ADA_BINS = 64, ADA_TMAX = 64 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP32_KAHAN = 2 };
enum { STREAM_OUTER = 1, STREAM_INNER = 2, STREAM_FINAL = 3 };

// Per-spec constants in one precision.  A = diag(sigma) L (row-major, lower),
// drift_i = r - delta_i - sigma_i^2 / 2, t[0] = 0, dt[k] = t_k - t_{k-1},
// sdt[k] = sqrt(dt[k]).
template <class R>
struct SpecT {
    int32_t d, n_dates, payoff, pad;
    R K, lnK, invK, r, inv_d;
    R S0[D_MAX], drift[D_MAX], sigma[D_MAX];
    R A[D_MAX * D_MAX];
    R t[NT_MAX + 1], dt[NT_MAX + 1], sdt[NT_MAX + 1];
};

struct DevSpec {
    SpecT<double> f64;
    SpecT<float> f32;
    double L[D_MAX * D_MAX];   // Cholesky factor of rho
    int32_t status;            // 0 or -2 (not positive definite)
};

// Read-only views in the constant address space: a kernel never writes the
// spec or its task tables, so uniform loads from them go through the scalar
// unit into SGPRs even in kernels that store to global memory in a loop.
#define BMC_CONST_AS __attribute__((address_space(4)))
template <class T> using const_as = const BMC_CONST_AS T;
template <class T> __device__ __forceinline__ const_as<T>* as_const(const T* p) { return (const_as<T>*)p; }
// Copy of a read-only struct through the scalar unit (word by word; the
// compiler merges the words into wide scalar loads when the address is uniform).
template <class T> __device__ __forceinline__ T load_const(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
    T out;
    const_as<uint32_t>* src = (const_as<uint32_t>*)p;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}

template <class R> __device__ __forceinline__ const SpecT<R>& spec_of(const DevSpec* s);
template <> __device__ __forceinline__ const SpecT<double>& spec_of<double>(const DevSpec* s) { return s->f64; }
template <> __device__ __forceinline__ const SpecT<float>& spec_of<float>(const DevSpec* s) { return s->f32; }

__host__ __device__ __forceinline__ uint32_t key_hi(int stream, int date)
{
    return ((uint32_t)stream << 16) | ((uint32_t)date & 0xFFFFu);
}

struct Words { uint32_t w[4]; };

// Philox4x32-10: ten rounds of two 32x32->64 products (multipliers
// 0xD2511F53 on counter word 0, 0xCD9E8D57 on word 2), the high halves
// xor-ed with the other words and the key, the key advanced by the Weyl
// increments 0x9E3779B9 / 0xBB67AE85 between rounds.  Key words that are
// uniform across the wavefront stay in scalar registers.
__device__ __forceinline__ Words philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                        uint32_t c2, uint32_t c3)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)0xD2511F53u * c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        // three-input xors in one instruction each (v_bitop3_b32, truth table 0x96)
        const uint32_t x0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
        const uint32_t x2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = x0;
        c2 = x2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// FP64 pieces of the uniform-to-normal map, written for its arguments
// u = (x + 1/2) 2^-32 (x a 32-bit word), within ~1.5 ulp of the exact values.
//
// ln u: x + 1/2 = m 2^e with m in [sqrt(1/2), sqrt(2)) (exact), f = m - 1,
// s = f / (2 + f), and ln m = 2 artanh s = f - s (f - R(s^2)) with the
// series R(z) = sum_k 2 z^k / (2k + 1) (|s| <= 0.1716, ten terms); then
// ln u = (e - 32) ln 2 + ln m with ln 2 split into a short high part (exact
// products) and the rest.
__device__ __forceinline__ double log_u32(uint32_t x)
{
    const double v = (double)x + 0.5;   // exact
    int e;
    double m = frexp(v, &e);            // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;           // exact
    const double den = 2.0 + f;
    // s = f / den: reciprocal estimate, two Newton steps, a residual correction
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    double sq = f * r;
    sq = fma(r, fma(-den, sq, f), sq);
    const double z = sq * sq;
    double R = 2.0 / 23;
    R = fma(R, z, 2.0 / 21);
    R = fma(R, z, 2.0 / 19);
    R = fma(R, z, 2.0 / 17);
    R = fma(R, z, 2.0 / 15);
    R = fma(R, z, 2.0 / 13);
    R = fma(R, z, 2.0 / 11);
    R = fma(R, z, 2.0 / 9);
    R = fma(R, z, 2.0 / 7);
    R = fma(R, z, 2.0 / 5);
    R = fma(R, z, 2.0 / 3);
    R *= z;
    const double t = f - sq * (f - R);
    const double E = (double)(e - 32);
    return fma(E, 0x1.62e42feep-1, t + E * 1.9082149292705877e-10);
}

// sin and cos of 2 pi u, u = (x + 1/2) 2^-32: t = 4u (exact) = q + f with q
// the nearest integer (quarter turns) and |f| <= 1/2; sin(pi f / 2) and
// cos(pi f / 2) from their Taylor series in f (coefficients (pi/2)^n / n!),
// then the quarter-turn rotation by q.
__device__ __forceinline__ void sincos_2pi_u32(uint32_t x, double& sn, double& cs)
{
    const double t = ((double)x + 0.5) * 0x1p-30;
    const double q = rint(t);
    const double f = t - q;             // exact
    const double f2 = f * f;
    double ps = 6.0669357311061955e-12;
    ps = fma(ps, f2, -6.688035109811468e-10);
    ps = fma(ps, f2, 5.692172921967927e-08);
    ps = fma(ps, f2, -3.598843235212085e-06);
    ps = fma(ps, f2, 0.00016044118478735983);
    ps = fma(ps, f2, -0.004681754135318688);
    ps = fma(ps, f2, 0.07969262624616705);
    ps = fma(ps, f2, -0.6459640975062463);
    ps = fma(ps, f2, 1.5707963267948966);
    double pc = -5.294400200734623e-13;
    pc = fma(pc, f2, 6.565963114979473e-11);
    pc = fma(pc, f2, -6.386603083791852e-09);
    pc = fma(pc, f2, 4.710874778818172e-07);
    pc = fma(pc, f2, -2.5202042373060607e-05);
    pc = fma(pc, f2, 0.0009192602748394266);
    pc = fma(pc, f2, -0.02086348076335296);
    pc = fma(pc, f2, 0.25366950790104803);
    pc = fma(pc, f2, -1.2337005501361697);
    pc = fma(pc, f2, 1.0);
    const double s0 = f * ps;
    const int qi = (int)q & 3;
    const double a = (qi & 1) ? pc : s0;    // sin: s0, c0, -s0, -c0 for q = 0..3
    const double b = (qi & 1) ? s0 : pc;    // cos: c0, -s0, -c0, s0
    sn = (qi & 2) ? -a : a;
    cs = ((qi + 1) & 2) ? -b : b;
}

// sqrt(a) for a > 0 (normal): reciprocal square root estimate, two Newton
// steps, then the product and one residual correction.
__device__ __forceinline__ double sqrt_pos(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    y = y * fma(-0.5 * a * y, y, 1.5);
    y = y * fma(-0.5 * a * y, y, 1.5);
    const double s0 = a * y;
    return fma(0.5 * y, fma(-s0, s0, a), s0);
}

// Box-Muller on one word pair: u = (x + 1/2) 2^-32 in (0, 1),
// z0 = sqrt(-2 ln u_a) cos(2 pi u_b), z1 = sqrt(-2 ln u_a) sin(2 pi u_b).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1)
{
    const double rad = sqrt_pos(-2.0 * log_u32(a));
    double s, c;
    sincos_2pi_u32(b, s, c);
    z0 = rad * c;
    z1 = rad * s;
}

// FP32 form on the hardware transcendental unit: v_log_f32 is log2,
// v_sin_f32 / v_cos_f32 take their argument in revolutions.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1)
{
    const float ua = fmaf((float)a, 0x1p-32f, 0x1p-33f);
    const float ub = fmaf((float)b, 0x1p-32f, 0x1p-33f);
    const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
    z0 = rad * __builtin_amdgcn_cosf(ub);
    z1 = rad * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// The d normals of one step: block b of step k has counter (k*nb + b, p, j, 0);
// asset i takes normal (i mod 4) of block i/4.  D is the compile-time bound,
// d the runtime dimension (d <= D).
template <int D, class R>
__device__ __forceinline__ void step_normals(int d, uint32_t k0, uint32_t k1, uint32_t c0,
                                             uint32_t p, uint32_t j, R (&z)[D])
{
    constexpr int NB = (D + 3) / 4;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (4 * b < d) {
            const Words w = philox(k0, k1, c0 + (uint32_t)b, p, j, 0u);
            R z0, z1, z2, z3;
            box_muller(w.w[0], w.w[1], z0, z1);
            if (4 * b + 0 < D) z[4 * b + 0] = z0;
            if (4 * b + 1 < D) z[4 * b + 1] = z1;
            if (4 * b + 2 < D && 4 * b + 2 < d) {
                box_muller(w.w[2], w.w[3], z2, z3);
                z[4 * b + 2] = z2;
                if (4 * b + 3 < D) z[4 * b + 3] = z3;
            }
        }
    }
}

// Payoff from log-prices.  Max-call and geometric put need one exp.
template <int D, class R>
__device__ __forceinline__ R payoff(int kind, int d, R K, R inv_d, const R (&x)[D])
{
    R v;
    if (kind == CALL_MAX) {
        R mx = x[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) mx = fmax(mx, x[i]);
        v = fexp(mx) - K;
    } else if (kind == CALL_MIN) {
        R mn = x[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) mn = fmin(mn, x[i]);
        v = fexp(mn) - K;
    } else if (kind == PUT_GEO) {
        R s = x[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) s += x[i];
        v = K - fexp(s * inv_d);
    } else {
        R s = fexp(x[0]);
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) s += fexp(x[i]);
        v = K - s * inv_d;
    }
    return v > R(0) ? v : R(0);
}

// The same payoffs in units of K from log-moneyness u_i = ln(S_i / K):
// Phi / K = (e^{max u} - 1)^+, (e^{min u} - 1)^+, (1 - e^{mean u})^+ or
// (1 - mean e^{u})^+.  The FP32 form keeps its path state in u, whose
// magnitude (|u| ~ 1 against ln S ~ 4.6) makes every rounding of the state,
// the geometric mean and the sums sixteen or more times smaller.
template <int D, class R>
__device__ __forceinline__ R payoff_moneyness(int kind, int d, R inv_d, const R (&u)[D])
{
    R v;
    if (kind == CALL_MAX || kind == CALL_MIN) {
        const bool mx = kind == CALL_MAX;
        R e = u[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) e = mx ? fmax(e, u[i]) : fmin(e, u[i]);
        v = fexp(e) - R(1);
    } else if (kind == PUT_GEO) {
        R s = u[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) s += u[i];
        v = R(1) - fexp(s * inv_d);
    } else {
        R s = fexp(u[0]);
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (i < d) s += fexp(u[i]);
        v = R(1) - s * inv_d;
    }
    return v > R(0) ? v : R(0);
}

// CMC classifier value F = w . [1, u, u^2, g, g^2] with u_i = ln S_i - ln K.
template <int D, class R>
__device__ __forceinline__ R cmc_score(int d, const R* __restrict__ w, R lnK, R g, const R (&x)[D])
{
    R F = w[0];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (i < d) {
            const R u = x[i] - lnK;
            F += (w[1 + i] + w[1 + d + i] * u) * u;
        }
    }
    F += (w[1 + 2 * d] + w[2 + 2 * d] * g) * g;
    return F;
}

// AdaBoost stump rule F = base + sum of delta over the thresholds theta that
// each feature reaches, psi = [u_1..u_d, g]; row [base, count_0..count_d,
// then per feature its count thresholds in ascending order and the running
// sums of their deltas], so each feature adds the running sum at the number
// of thresholds it reaches.  Features are visited in order.
template <int D, class R>
__device__ __forceinline__ R ada_score(int d, const R* __restrict__ w, R lnK, R g, const R (&x)[D])
{
    if constexpr (D <= 8 && sizeof(R) == 4) {   // (the FP64 kernels would lose a wave per SIMD)
        // The features' binary searches in lockstep: every feature steps
        // through h = ADA_TMAX, .., 2, 1 (a count never exceeds ADA_TMAX, so
        // the steps above a feature's largest power of two are skipped and
        // the rest are the sequential search's), and the reads of one step
        // are independent of each other.  Same k, same sum order.
        R v[D + 1];
        int cnt[D + 1], off[D + 1], k[D + 1];
        int o = 2 + d;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            v[i] = R(0);
            cnt[i] = 0;
            off[i] = 0;
            k[i] = 0;
            if (i <= d) {
                v[i] = i < d ? x[i < D ? i : 0] - lnK : g;
                cnt[i] = (int)w[1 + i];
                off[i] = o;
                o += 2 * cnt[i];
            }
        }
#pragma unroll
        for (int h = ADA_TMAX; h > 0; h >>= 1) {
#pragma unroll
            for (int i = 0; i <= D; ++i) {
                const int t = k[i] + h;
                if (i <= d && t <= cnt[i] && w[off[i] + t - 1] <= v[i]) k[i] = t;
            }
        }
        R F = w[0];
#pragma unroll
        for (int i = 0; i <= D; ++i)
            if (i <= d && k[i] > 0) F += w[off[i] + cnt[i] + k[i] - 1];
        return F;
    }
    R F = w[0];
    const R* pr = w + 2 + d;
#pragma unroll
    for (int i = 0; i <= D; ++i) {
        if (i <= d) {
            const R v = i < d ? x[i < D ? i : 0] - lnK : g;
            const int cnt = (int)w[1 + i];
            // k = number of the (ascending) thresholds pr[0..cnt-1] at or
            // below v, by binary search in powers of two; the step count
            // depends on cnt only, the same for every lane
            int k = 0;
            for (int h = cnt > 0 ? 1 << (31 - __clz(cnt)) : 0; h > 0; h >>= 1) {
                const int t = k + h;
                if (t <= cnt && pr[t - 1] <= v) k = t;
            }
            if (k > 0) F += pr[cnt + k - 1];
            pr += 2 * cnt;
        }
    }
    return F;
}

// I&Z boundary of a region, b = w . [1, v_1..v_q, v_a v_c (a <= c)], over the
// log-moneyness v = ln S_i - ln K of the assets other than the region's own
// one, in increasing order (region 0 of the put family: assets 2..d).
template <int D, class R>
__device__ __forceinline__ R iz_boundary(int d, const R* __restrict__ w, R lnK, const R (&x)[D], int region)
{
    const int q = d - 1;
    R v[D > 1 ? D - 1 : 1];
    R b = w[0];
#pragma unroll
    for (int a = 0; a + 1 < D; ++a) {
        if (a < q) {
            v[a] = (a < region ? x[a] : x[a + 1]) - lnK;
            b += w[1 + a] * v[a];
        }
    }
    int f = 1 + q;
#pragma unroll
    for (int a = 0; a + 1 < D; ++a) {
        if (a < q) {
#pragma unroll
            for (int c = a; c + 1 < D; ++c) {
                if (c < q) {
                    b += w[f] * (v[a] * v[c]);
                    ++f;
                }
            }
        }
    }
    return b;
}

__host__ __device__ __forceinline__ int rule_width(int method, int d)
{
    if (method == CMC) return 2 * d + 3;
    if (method == ADA) return 1 + (d + 1) + 2 * ADA_TMAX;
    const int q = d - 1;
    return 1 + q + q * (q + 1) / 2;
}

// I&Z exercise regions (Section 2.2): one per asset for the max-call (asset i
// the largest) and the min-call (asset i the smallest), one for the put family.
__host__ __device__ __forceinline__ int iz_regions(int payoff, int d)
{
    return (payoff == CALL_MAX || payoff == CALL_MIN) ? d : 1;
}

// Rule row width: the CMC weights, or one I&Z boundary block per region
// (region r at offset r * rule_width(IZ, d)).
__host__ __device__ __forceinline__ int rule_row_width(int method, int d, int payoff)
{
    return method != IZ ? rule_width(method, d) : iz_regions(payoff, d) * rule_width(IZ, d);
}

}  // namespace bmc
