// Continuation (inner-path) kernel template; instantiated per dimension bound
// in separate translation units so that they compile in parallel.
#pragma once

#include "internal.hpp"
#include "iz_step.hpp"

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

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Correlated increment ls += A (s z) for the FP32 buckets on the matrix cores:
// v_mfma_f32_4x4x1_16b_f32 gives element i of lane L the product
// a[4 (L/4) + i] b[L], so with b = the lane's own s z_l and a = A[4c + L%4][l]
// (lanes of a group of four hold the four rows of asset chunk c), element i
// of every lane accumulates A[4c+i][l] s z_l for its own path.  arow is A
// row-major [D][D], zero-padded; a quad of columns is one 16-byte LDS read.
// Only the lower block triangle (chunks c >= column quad t) is visited.
template <int D>
__device__ __forceinline__ void corr_mfma(const float* __restrict__ arow, const float (&zs)[D], float (&ls)[D])
{
    constexpr int NC = D / 4;
    const int r = threadIdx.x & 3;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
#pragma unroll
        for (int ch = t; ch < NC; ++ch) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(arow + (4 * ch + r) * D + 4 * t);
            f32x4 v = {ls[4 * ch], ls[4 * ch + 1], ls[4 * ch + 2], ls[4 * ch + 3]};
            v = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, zs[4 * t], v, 0, 0, 0);
            v = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, zs[4 * t + 1], v, 0, 0, 0);
            v = __builtin_amdgcn_mfma_f32_4x4x1f32(a.z, zs[4 * t + 2], v, 0, 0, 0);
            v = __builtin_amdgcn_mfma_f32_4x4x1f32(a.w, zs[4 * t + 3], v, 0, 0, 0);
            ls[4 * ch] = v.x;
            ls[4 * ch + 1] = v.y;
            ls[4 * ch + 2] = v.z;
            ls[4 * ch + 3] = v.w;
        }
    }
}

// FP32 kernels put the correlation product on the matrix cores from d = 25 on:
// below that the VALU form with the coefficients in LDS was faster when timed
// (never-exercise geometric put, N = n = 4096: by 5-17 % at d = 9..24; from
// d = 26 the matrix cores were 4-37 % ahead, d = 28 within the spread).
template <int D, class R> constexpr bool uses_mfma() { return D >= 25 && sizeof(R) == 4; }
template <int D, class R> constexpr bool uses_lds_coef() { return cont_lds_coef(D, sizeof(R)); }

// I&Z rules need their own kernels (IZK): the boundary test of d <= 16 assets
// (a full quadratic, and the region search of the max-call) would otherwise
// hold registers in every classifier kernel of those dimensions.
template <int D, bool EXACT> constexpr bool has_iz_kernel() { return EXACT && D <= 16; }

// One (point j, chunk) job of a continuation launch, run by a whole block;
// lds: the dynamic table area, red: [3][16] wave partials.  IZK: the job's
// rules are I&Z boundaries; otherwise classifier rules (CMC or AdaBoost).
template <int D, bool EXACT, class R, class ACC, bool IZK = false>
__device__ __forceinline__ void cont_job(const ContArgs& a, const uint32_t j, const uint32_t chunk, double* lds,
                                         double (*red)[16])
{
    constexpr bool MF = uses_mfma<D, R>();
    constexpr bool LC = uses_lds_coef<D, R>();
    constexpr int D4 = (D + 3) & ~3;   // matrix-core chunks of four assets
    // Bucket kernels (d < D possible) pad the path state to D entries with
    // neutral values, so that every per-asset loop runs to D without tests:
    // zero coefficients and drifts, log-prices 0 (geometric put) or -1e30
    // (max-call and arithmetic basket: no effect on a maximum or a sum of
    // exponentials), zero classifier weights.
    constexpr bool PAD = !EXACT;
    static_assert(EXACT || D % 4 == 0, "padded bounds are multiples of four");
    const_as<SpecT<R>>& S = *as_const(&spec_of<R>(a.spec));
    const int d = EXACT ? D : S.d;
    if (!EXACT) __builtin_assume(d > dim_floor(D) && d <= D);
    const int NT = S.n_dates;
    const int m = a.m;
    const int W = a.width;
    const bool padw = PAD && a.method == CMC;   // classifier rows padded to 2D+3
    const int WL = cont_rule_stride(D, W);
    double* disc = lds;
    R* lx = reinterpret_cast<R*>(disc + NT + 1);
    R* dtv = lx + D_MAX;
    R* sdtv = dtv + NT + 1;
    R* wt = sdtv + NT + 1;
    size_t coef_off = 0;
    (void)cont_lds_layout(sizeof(R), D, NT, W, &coef_off);
    const int payk = S.payoff;
    R* coef = reinterpret_cast<R*>(reinterpret_cast<char*>(lds) + coef_off);   // [D4][D4]
    R* drift = coef + D4 * D4;                                                 // [D4]

    const_as<double>* t64 = as_const(a.spec)->f64.t;
    const double r64 = as_const(a.spec)->f64.r;
    // FP32 path state: log-moneyness u = ln(S/K) (the rules' own variable);
    // FP64: the log-price, the oracle's variable
    constexpr bool UST = sizeof(R) == 4;
    const double lnshift = UST ? (double)as_const(a.spec)->f64.lnK : 0.0;
    const double tm = t64[m];
    // cancel word of a served request: read by one thread while the tables
    // load, shared through LDS by the barrier below
    __shared__ int32_t job_cancel;
    if (threadIdx.x == 0)
        job_cancel = a.cancel ? __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    for (int k = threadIdx.x; k <= NT; k += blockDim.x) {
        disc[k] = exp(-r64 * (t64[k] - tm));
        dtv[k] = S.dt[k];
        sdtv[k] = S.sdt[k];
    }
    const R* __restrict__ rules = reinterpret_cast<const R*>(a.rules);
    if (padw) {
        // [1, u_1..u_d, uu_1..uu_d, g, gg] -> [1, u_1..u_D, uu_1..uu_D, g, gg]
        for (int e = (m + 1) * WL + threadIdx.x; e < NT * WL; e += blockDim.x) {
            const int k = e / WL, f = e - k * WL;
            int src;
            if (f == 0) src = 0;
            else if (f <= D) src = f - 1 < d ? f : -1;
            else if (f <= 2 * D) src = f - 1 - D < d ? f - D + d : -1;
            else src = f - 2 * D + 2 * d;
            wt[e] = src >= 0 ? rules[k * W + src] : R(0);
        }
    } else {
        for (int i = (m + 1) * W + threadIdx.x; i < NT * W; i += blockDim.x) wt[i] = rules[i];
    }
    // Fused I&Z search step: the last thread takes the step of the previous
    // pass while the others load the tables, and sets the searched
    // coordinate of the new point; a stopped point's job ends after the
    // barrier.
    __shared__ int fz_go;
    int fz_region = -1;
    if constexpr (IZK) {
        if (a.fz.on) {
            fz_region = (int)(a.slot + (a.region_pts ? j / a.region_pts : 0u));
            if (threadIdx.x == blockDim.x - 1) {
                const double* st = a.fz.st_r;
                const IzStepOut o = iz_step_compute(a.spec->f64, d, fz_region, a.N, a.fz.part, a.nchunk, a.n, j,
                                                    a.x, st[j], st[a.N + j], st[2 * a.N + j], a.fz.eps,
                                                    a.fz.max_iter, a.fz.mode, a.fz.it, a.fz.tau);
                if (chunk == 0)
                    iz_step_apply(o, fz_region, a.N, j, a.fz.it, a.fz.ids_out, a.fz.n_out, a.fz.st_w,
                                  a.fz.st_w + a.N, a.fz.st_w + 2 * a.N, a.fz.x_work, a.fz.s_out, a.fz.iters,
                                  a.fz.steps_acc, a.fz.ties);
                fz_go = o.cont;
                if (o.cont) lx[fz_region] = (R)(log(o.next) - lnshift);
            }
        }
    }
    if ((int)threadIdx.x < D && (int)threadIdx.x != fz_region)
        lx[threadIdx.x] = (int)threadIdx.x < d ? (R)(log(a.x[(int64_t)threadIdx.x * a.N + j]) - lnshift)
                                                : (payk == PUT_GEO ? R(0) : payk == CALL_MIN ? R(1e30) : R(-1e30));
    if constexpr (LC) {
        // FP32: row-major A[i][l] (matrix-core operand rows); FP64: column-major
        // A[l][i] (consecutive rows of one column in one read).  Zero beyond d.
        for (int e = threadIdx.x; e < D4 * D4; e += blockDim.x) {
            const int i = MF ? e / D4 : e % D4, l = MF ? e % D4 : e / D4;
            coef[e] = (i < d && l <= i) ? S.A[i * D_MAX + l] : R(0);
        }
        for (int i = threadIdx.x; i < D4; i += blockDim.x) drift[i] = i < d ? S.drift[i] : R(0);
    }
    __syncthreads();
    if constexpr (IZK) {
        if (a.fz.on && !fz_go) return;
    }
    if (job_cancel) return;   // uniform: one LDS word after the barrier

    const uint32_t lo = chunk * a.paths_per_wg;
    const uint32_t hi = min(a.n, lo + a.paths_per_wg);
    const uint32_t nb = (uint32_t)(d + 3) >> 2;
    const uint32_t k0 = a.k0, k1 = a.k1;
    // counter point and fourth counter word of this job's point
    uint32_t slot = a.slot, pj = j;
    if (a.region_pts) {
        const uint32_t r = j / a.region_pts;
        slot += r;
        pj = j - r * a.region_pts;
    }
    const bool call_dir = payk == CALL_MAX || payk == CALL_MIN;
    const bool min_dir = payk == CALL_MIN;
    const int W1 = rule_width(IZ, d);   // one I&Z region's boundary block
    const R K = S.K, lnK = S.lnK, invK = S.invK, inv_d = S.inv_d;
    // the rules read u = state - lnKr; an I&Z boundary (a log-price) is
    // compared with the state after subtracting bshift
    const R lnKr = UST ? R(0) : lnK, bshift = UST ? lnK : R(0);

    // dp: the extent of the per-asset loops (D for padded buckets)
    const int dp = PAD ? D : d;
    R ls[D4];
#pragma unroll
    for (int i = 0; i < D4; ++i) ls[i] = (i < dp) ? lx[i] : R(0);

    ACC acc;
    uint32_t steps = 0;
    // Paths are handed out per wavefront: wave w owns the contiguous range
    // [wlo, whi) of the job's paths.  Each lane starts on one; whenever paths
    // stop, the lanes whose path stopped take the range's next paths in lane
    // order (ballot and lane rank), so no lane idles while its wave has paths
    // left.  The assignment depends only on the paths' lengths, so results
    // repeat bit for bit.
    const uint32_t nwave = (blockDim.x + 63) >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t cnt = hi > lo ? hi - lo : 0u;
    const uint32_t share = (cnt + nwave - 1) / nwave;
    const uint32_t wlo = lo + min(cnt, wv * share), whi = lo + min(cnt, (wv + 1) * share);
    uint32_t p = wlo + lane;
    uint32_t nxt = wlo + min(64u, blockDim.x - 64u * wv);
    int k = m + 1;
    // Matrix-core steps need every lane of the wavefront (operands come from
    // neighbouring lanes): the loop runs while any lane has a path, and lanes
    // without one step through dummy paths whose payoffs are not counted.
    auto more = [&]() { return MF ? __any(p < whi) != 0 : p < whi; };
    while (more()) {
        const bool live = MF ? p < whi : true;
        const R dtk = dtv[k], sk = sdtv[k];
        // Opaque per-iteration offset: keeps the coefficient loads inside the
        // loop instead of hoisted into registers.
        uint32_t opq = 0;
        if constexpr (LC) asm volatile("" : "+v"(opq));
        const R* cf = coef + (opq & ~3u);
        const R* dr = drift + (opq & ~3u);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (i < dp) {
                if constexpr (LC) ls[i] += dr[i] * dtk;
                else ls[i] += S.drift[i] * dtk;
            }
        }
        const uint32_t c0 = (uint32_t)k * nb;
        if constexpr (MF) {
            R zs[D4];
#pragma unroll
            for (int b = 0; b < D4 / 4; ++b) {
                R z[4] = {R(0), R(0), R(0), R(0)};
                const Words w = philox(k0, k1, c0 + (uint32_t)b, p, pj, slot);
                box_muller(w.w[0], w.w[1], z[0], z[1]);
                if (4 * b + 2 < dp) box_muller(w.w[2], w.w[3], z[2], z[3]);
#pragma unroll
                for (int h = 0; h < 4; ++h) zs[4 * b + h] = 4 * b + h < dp ? sk * z[h] : R(0);
            }
            corr_mfma<D4>(reinterpret_cast<const float*>(cf), reinterpret_cast<const float(&)[D4]>(zs),
                          reinterpret_cast<float(&)[D4]>(ls));
        } else {
#pragma unroll
            for (int b = 0; b < (D + 3) / 4; ++b) {
                if (4 * b < dp) {
                    const Words w = philox(k0, k1, c0 + (uint32_t)b, p, pj, slot);
                    R z[4];
                    box_muller(w.w[0], w.w[1], z[0], z[1]);
                    if (4 * b + 2 < dp) box_muller(w.w[2], w.w[3], z[2], z[3]);
                    else { z[2] = R(0); z[3] = R(0); }
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int l = 4 * b + h;
                        if (l < D && l < dp) {
                            const R zl = sk * z[h];
#pragma unroll
                            for (int i = l; i < D; ++i) {
                                if (i < dp) {
                                    if constexpr (LC) ls[i] += cf[l * D4 + i] * zl;
                                    else ls[i] += S.A[i * D_MAX + l] * zl;
                                }
                            }
                        }
                    }
                }
            }
        }
        R phi, g;   // payoff and payoff / K
        if constexpr (UST) {
            g = payoff_moneyness<D4, R>(payk, dp, inv_d, ls);
            phi = K * g;
        } else {
            phi = payoff<D4, R>(payk, dp, K, inv_d, ls);
            g = phi * invK;
        }
        bool stop = (k == NT);
        if (!stop && phi > R(0)) {
            const R* w = wt + k * WL;
            if constexpr (!IZK) {
                if (a.method == CMC) stop = cmc_score<D4, R>(dp, w, lnKr, g, ls) > R(0);
                else stop = ada_score<D4, R>(d, w, lnKr, g, ls) > R(0);
            } else {
                if constexpr (has_iz_kernel<D, EXACT>()) {
                    if (call_dir) {
                        // region of the largest (max-call) or smallest (min-call)
                        // asset, the first one on ties; exercise above that
                        // region's boundary
                        int reg = 0;
                        R mx = ls[0];
#pragma unroll
                        for (int i = 1; i < D; ++i)
                            if (i < d && (min_dir ? ls[i] < mx : ls[i] > mx)) {
                                mx = ls[i];
                                reg = i;
                            }
                        stop = mx > iz_boundary<D4, R>(d, w + reg * W1, lnKr, ls, reg) - bshift;
                    } else {
                        stop = ls[0] < iz_boundary<D4, R>(d, w, lnKr, ls, 0) - bshift;
                    }
                }
            }
        }
        const uint64_t ended = __ballot(stop && live);
        if (stop) {
            if (live) {
                acc.add((double)phi * disc[k]);
                steps += (uint32_t)(k - m);
                p = nxt + __builtin_amdgcn_mbcnt_hi((uint32_t)(ended >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)ended, 0u));
            }
            k = m + 1;
#pragma unroll
            for (int i = 0; i < D; ++i)
                if (i < dp) ls[i] = lx[i];
        } else {
            ++k;
        }
        nxt += (uint32_t)__popcll(ended);
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

// The job(s) of one workgroup: slot's (point, chunk) job, or (STRIDE, the
// FP64 label-refinement kernels) every slot s = slot, slot + slot_stride, ...
// below the active count.  A slot at or past the active count is a retired
// job (the whole block returns).  The loop lives in kernels of its own: in
// the one-job kernels it would cost registers (and occupancy).  A job of a
// cancelled served request (its cancel word set) stops after its table setup.
// src: where the strided loop re-reads the arguments for every job (the
// kernel's argument block, or the task's table entry).
template <int D, bool EXACT, class R, class ACC, bool IZK, bool STRIDE>
__device__ __forceinline__ void cont_slots(const ContArgs& a, uint32_t slot, const uint32_t chunk, double* lds,
                                           double (*red)[16], const ContArgs* src = nullptr)
{
    if constexpr (!STRIDE) {
        if (a.n_ids && slot >= (uint32_t)*a.n_ids) return;
        uint32_t j = a.ids ? (uint32_t)a.ids[slot] : slot;
        if (a.ord.cnt) {   // the slot-th point of the bucket lists (uniform loads)
            uint32_t rem = slot;
            int b = 0;
            for (; b < ORDER_BUCKETS - 1; ++b) {
                const uint32_t c = (uint32_t)a.ord.cnt[b];
                if (rem < c) break;
                rem -= c;
            }
            j = (uint32_t)a.ord.list[(size_t)b * (size_t)a.N + rem];
            if (j >= (uint32_t)a.N) return;   // not reached: the lists hold the N points
        }
        cont_job<D, EXACT, R, ACC, IZK>(a, j, chunk, lds, red);
    } else {
        const uint32_t lim = (uint32_t)*a.n_ids, stride = a.slot_stride;
        const int32_t* ids = a.ids;
        for (; slot < lim; slot += stride) {
            // Each job reads its arguments again through the scalar unit from a
            // location the compiler cannot see through, so that none of them
            // stays in scalar registers across the jobs: held there, they
            // crowded the path loop's scalar registers into vector lanes.
            const ContArgs* p = src;
            asm volatile("" : "+s"(p));
            const ContArgs b = load_const(p);
            cont_job<D, EXACT, R, ACC, IZK>(b, (uint32_t)ids[slot], chunk, lds, red);
            __syncthreads();   // the LDS tables and partials of the next job
        }
    }
}

// One launch per (spec, date): block = one (point, chunk) job.
template <int D, bool EXACT, class R, class ACC, bool IZK = false, bool STRIDE = false>
__global__ void __launch_bounds__(256) k_cont(const ContArgs a)
{
    extern __shared__ __align__(16) double lds[];
    __shared__ double red[3][16];
    const uint32_t slot = blockIdx.x / a.nchunk;
    const uint32_t chunk = blockIdx.x - slot * a.nchunk;
    if constexpr (IZK) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (a.fz.on) *a.fz.n_next = 0;
            // progress poll: the count of the list this launch runs over, which
            // an earlier launch completed
            if (a.fz.poll) *a.fz.poll = *a.n_ids;
        }
    }
    // the argument block starts the kernel's argument segment
    cont_slots<D, EXACT, R, ACC, IZK, STRIDE>(
        a, slot, chunk, lds, red, (const ContArgs*)__builtin_amdgcn_kernarg_segment_ptr());
}

// One launch over the jobs of many tasks (options at their own dates): block
// b runs job job0 + b, mapped to (task, point, chunk) through the exclusive
// prefix sums of the tasks' job counts.  Every job writes its own partial
// sums, so results do not depend on the launch it ran in.  The task table and
// prefix sums are read through the scalar unit (uniform loads).
template <int D, bool EXACT, class R, class ACC, bool STRIDE = false>
__global__ void __launch_bounds__(256) k_cont_multi(const ContArgs* __restrict__ tasks,
                                                    const uint32_t* __restrict__ prefix, int ntasks, uint32_t job0)
{
    extern __shared__ __align__(16) double lds[];
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
    cont_slots<D, EXACT, R, ACC, false, STRIDE>(a, slot, local - slot * a.nchunk, lds, red, tasks + lo);
}

// Lets every kernel of bound D use the device's whole LDS (done once).
template <int D, bool EXACT>
bool cont_allow_lds()
{
    const int v = (int)cont_lds_limit();
    const void* ks[] = {reinterpret_cast<const void*>(k_cont<D, EXACT, double, Acc<double>>),
                        reinterpret_cast<const void*>(k_cont<D, EXACT, float, Acc<double>>),
                        reinterpret_cast<const void*>(k_cont<D, EXACT, float, KahanAcc>),
                        reinterpret_cast<const void*>(k_cont_multi<D, EXACT, double, Acc<double>>),
                        reinterpret_cast<const void*>(k_cont_multi<D, EXACT, float, Acc<double>>),
                        reinterpret_cast<const void*>(k_cont_multi<D, EXACT, float, KahanAcc>)};
    for (const void* f : ks) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v);
    const void* kr[] = {reinterpret_cast<const void*>(k_cont<D, EXACT, double, Acc<double>, false, true>),
                        reinterpret_cast<const void*>(k_cont_multi<D, EXACT, double, Acc<double>, true>)};
    for (const void* f : kr) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v);
    if constexpr (has_iz_kernel<D, EXACT>()) {
        const void* kz[] = {reinterpret_cast<const void*>(k_cont<D, EXACT, double, Acc<double>, true>),
                            reinterpret_cast<const void*>(k_cont<D, EXACT, float, Acc<double>, true>),
                            reinterpret_cast<const void*>(k_cont<D, EXACT, float, KahanAcc, true>)};
        for (const void* f : kz) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v);
    }
    (void)hipGetLastError();   // a refused attribute must not surface at the next launch check
    return true;
}

template <int D, bool EXACT>
hipError_t launch_cont_d(int prec, const ContArgs& a, int grid, int block, size_t lds,
                                hipStream_t st)
{
    static const bool lds_ok = cont_allow_lds<D, EXACT>();
    (void)lds_ok;
    if (a.method == IZ) {
        if constexpr (has_iz_kernel<D, EXACT>()) {
            if (prec == PREC_FP64)
                hipLaunchKernelGGL((k_cont<D, EXACT, double, Acc<double>, true>), dim3(grid), dim3(block), lds, st,
                                   a);
            else if (prec == PREC_FP32)
                hipLaunchKernelGGL((k_cont<D, EXACT, float, Acc<double>, true>), dim3(grid), dim3(block), lds, st,
                                   a);
            else
                hipLaunchKernelGGL((k_cont<D, EXACT, float, KahanAcc, true>), dim3(grid), dim3(block), lds, st, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;   // I&Z rules exist for d <= 16 only
    }
    if (a.slot_stride) {   // FP64 label refinement
        if (prec != PREC_FP64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_cont<D, EXACT, double, Acc<double>, false, true>), dim3(grid), dim3(block), lds, st,
                           a);
    } else if (prec == PREC_FP64)
        hipLaunchKernelGGL((k_cont<D, EXACT, double, Acc<double>>), dim3(grid), dim3(block), lds, st, a);
    else if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_cont<D, EXACT, float, Acc<double>>), dim3(grid), dim3(block), lds, st, a);
    else
        hipLaunchKernelGGL((k_cont<D, EXACT, float, KahanAcc>), dim3(grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

template <int D, bool EXACT>
hipError_t launch_cont_multi_d(int prec, const ContArgs* tasks, const uint32_t* prefix, int ntasks, uint32_t job0,
                               uint32_t jobs, int block, size_t lds, hipStream_t st, bool stride)
{
    static const bool lds_ok = cont_allow_lds<D, EXACT>();
    (void)lds_ok;
    if (stride) {   // FP64 label refinement
        if (prec != PREC_FP64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_cont_multi<D, EXACT, double, Acc<double>, true>), dim3(jobs), dim3(block), lds, st,
                           tasks, prefix, ntasks, job0);
    } else if (prec == PREC_FP64)
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
