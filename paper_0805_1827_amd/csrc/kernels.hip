// HIP kernels for gfx950: spec setup, sample points, the continuation
// (inner-path) kernel, I&Z search updates and the FP64 rule fits.
#include <math.h>

#include "fit_common.hpp"
#include "iz_step.hpp"

namespace bmc {

// ---------------------------------------------------------------------------
// Spec setup: Cholesky of rho (FP64), A = diag(sigma) L, drifts, date tables.

__global__ void __launch_bounds__(256) k_setup(const HostSpecPack* __restrict__ in,
                                               DevSpec* __restrict__ out, const uint32_t* __restrict__ slots,
                                               int32_t* status_host)
{
    __shared__ double L[D_MAX * D_MAX];
    __shared__ int bad;
    in += blockIdx.x;   // one block per spec, written to its slot
    out += slots ? slots[blockIdx.x] : blockIdx.x;
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
        if (status_host) *status_host = out->status;   // single-spec setups: straight to pinned memory
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

hipError_t launch_setup(const HostSpecPack* in, DevSpec* out, int count, hipStream_t st, const uint32_t* slots,
                        int32_t* status_host)
{
    hipLaunchKernelGGL(k_setup, dim3(count), dim3(256), 0, st, in, out, slots, status_host);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Continuation launch dispatch over the compiled dimension bounds.

template <int D, bool EXACT>
hipError_t launch_cont_d(int prec, const ContArgs& a, int grid, int block, size_t lds,
                         hipStream_t st);

int cont_bucket(int d)
{
    if (d <= 32) return d;
    if (d <= 40) return (d + 3) / 4 * 4;
    return (d + 7) / 8 * 8;
}

size_t cont_lds_bytes(int prec, int d, int n_dates, int width)
{
    const size_t rs = prec == PREC_FP64 ? sizeof(double) : sizeof(float);
    return cont_lds_layout(rs, cont_bucket(d), n_dates, width, nullptr);
}

size_t cont_lds_limit()
{
    static size_t limit = 0;
    if (limit == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        limit = (size_t)v - 1024;   // the kernels' static LDS (wave partials) stays below 1 KB
    }
    return limit;
}

#define BMC_BUCKETS(X)  \
    X(1, true) X(2, true) X(3, true) X(4, true) X(5, true) X(6, true) X(7, true) X(8, true) \
     X(9, true) X(10, true) X(11, true) X(12, true) X(13, true) X(14, true) X(15, true) X(16, true) \
     X(17, true) X(18, true) X(19, true) X(20, true) X(21, true) X(22, true) X(23, true) X(24, true) \
     X(25, true) X(26, true) X(27, true) X(28, true) X(29, true) X(30, true) X(31, true) X(32, true) \
     X(36, false) X(40, false) X(48, false) X(56, false) X(64, false)

hipError_t launch_cont(int d, int prec, const ContArgs& a, int grid, int block, size_t lds,
                       hipStream_t st)
{
#define BMC_ONE(DD, EX) \
    case DD: return launch_cont_d<DD, EX>(prec, a, grid, block, lds, st);
    switch (cont_bucket(d)) {
        BMC_BUCKETS(BMC_ONE)
    default: return hipErrorInvalidValue;
    }
#undef BMC_ONE
}

template <int D, bool EXACT>
hipError_t launch_cont_multi_d(int prec, const ContArgs* tasks, const uint32_t* prefix, int ntasks, uint32_t job0,
                               uint32_t jobs, int block, size_t lds, hipStream_t st, bool stride);

hipError_t launch_cont_multi(int bucket, int prec, const ContArgs* tasks, const uint32_t* prefix, int ntasks,
                             uint32_t job0, uint32_t jobs, int block, size_t lds, hipStream_t st, bool stride)
{
#define BMC_ONE(DD, EX) \
    case DD: return launch_cont_multi_d<DD, EX>(prec, tasks, prefix, ntasks, job0, jobs, block, lds, st, stride);
    switch (bucket) {
        BMC_BUCKETS(BMC_ONE)
    default: return hipErrorInvalidValue;
    }
#undef BMC_ONE
}

// Continuation estimate C = sum/n and its standard error sqrt(var/n), with
// var = (sumsq - sum^2/n)/(n-1), from a point's merged sums.
__device__ __forceinline__ void finalize_point(int64_t j, double s, double q, double c, uint32_t n, double* cont,
                                               double* se, int64_t* steps, double* sums,
                                               unsigned long long* steps_total, const RefineSel& sel = {},
                                               int64_t N = 0)
{
    const double nn = (double)n;
    double var = (q - s * s / nn) / (nn - 1.0);
    if (var < 0.0) var = 0.0;
    if (cont) cont[j] = s / nn;
    if (se) se[j] = sqrt(var / nn);
    if (sel.s) refine_point(sel.s->f64, sel.x, N, j, s / nn, sqrt(var / nn), sel.ids, sel.n_ids);
    if (steps) steps[j] = (int64_t)c;
    if (sums) {
        sums[2 * j] = s;
        sums[2 * j + 1] = q;
    }
    if (steps_total) atomicAdd(steps_total, (unsigned long long)c);
}

// Same merge for points with many chunks (final pricing), by a 256-thread
// block: each thread merges a contiguous run of chunks in order, then a
// fixed-shape tree over the threads; the result is valid in thread 0.
__device__ __forceinline__ void merge_wide(const double* __restrict__ part, uint32_t nchunk, int64_t j,
                                           double (*red)[256], double& s, double& q, double& c)
{
    const uint32_t T = blockDim.x, t = threadIdx.x;
    const uint32_t lo = (uint32_t)(((uint64_t)nchunk * t) / T), hi = (uint32_t)(((uint64_t)nchunk * (t + 1)) / T);
    double s_ = 0.0, q_ = 0.0, c_ = 0.0;
    for (uint32_t ch = lo; ch < hi; ++ch) {
        const double* o = part + ((size_t)j * nchunk + ch) * 3;
        s_ += o[0];
        q_ += o[1];
        c_ += o[2];
    }
    red[0][t] = s_;
    red[1][t] = q_;
    red[2][t] = c_;
    __syncthreads();
    for (uint32_t w = T / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] += red[2][t + w];
        }
        __syncthreads();
    }
    s = red[0][0];
    q = red[1][0];
    c = red[2][0];
}

__global__ void k_finalize(const double* __restrict__ part, uint32_t nchunk, uint32_t n, int64_t N,
                           const int32_t* __restrict__ ids, const int32_t* __restrict__ n_ids,
                           double* cont, double* se, int64_t* steps, double* sums,
                           unsigned long long* steps_total, const RefineSel sel)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j = slot;
    if (ids) {
        if (slot >= *n_ids) return;
        j = ids[slot];
    } else if (slot >= N) {
        return;
    }
    double s, q, c;
    merge_serial(part, nchunk, j, s, q, c);
    finalize_point(j, s, q, c, n, cont, se, steps, sums, steps_total, sel, N);
}

__global__ void __launch_bounds__(256) k_finalize_wide(const double* __restrict__ part, uint32_t nchunk,
                                                       uint32_t n, int64_t N, double* cont, double* se,
                                                       int64_t* steps, double* sums, unsigned long long* steps_total,
                                                       const RefineSel sel)
{
    __shared__ double red[3][256];
    const int64_t j = blockIdx.x;
    double s, q, c;
    merge_wide(part, nchunk, j, red, s, q, c);
    if (threadIdx.x == 0) finalize_point(j, s, q, c, n, cont, se, steps, sums, steps_total, sel, N);
}

// Finalize of many tasks in one launch: a wide task has one block per point,
// a narrow one a block per 256 points.
__global__ void __launch_bounds__(256) k_finalize_multi(const FinTask* __restrict__ tasks,
                                                        const uint32_t* __restrict__ prefix, int ntasks)
{
    __shared__ double red[3][256];
    const int ti = task_of_block(prefix, ntasks, blockIdx.x);
    const FinTask& f = tasks[ti];
    const uint32_t local = blockIdx.x - prefix[ti];
    double s, q, c;
    if (f.wide) {
        merge_wide(f.part, f.nchunk, local, red, s, q, c);
        if (threadIdx.x == 0)
            finalize_point(local, s, q, c, f.n, f.cont, f.se, f.steps, f.sums, f.steps_total, f.sel, f.N);
    } else {
        const int64_t slot = (int64_t)local * blockDim.x + threadIdx.x;
        int64_t j = slot;
        if (f.ids) {
            if (slot >= *f.n_ids) return;
            j = f.ids[slot];
        } else if (slot >= f.N) {
            return;
        }
        merge_serial(f.part, f.nchunk, j, s, q, c);
        finalize_point(j, s, q, c, f.n, f.cont, f.se, f.steps, f.sums, f.steps_total, f.sel, f.N);
    }
}

bool finalize_is_wide(uint32_t nchunk, int64_t N, bool has_ids) { return !has_ids && nchunk >= 64 && N <= 4096; }

hipError_t launch_finalize_multi(const FinTask* tasks, const uint32_t* prefix, int ntasks, uint32_t blocks,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize_multi, dim3(blocks), dim3(256), 0, st, tasks, prefix, ntasks);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* part, uint32_t nchunk, uint32_t n, int64_t N,
                           const int32_t* ids, const int32_t* n_ids, double* cont, double* se,
                           int64_t* steps, double* sums, unsigned long long* steps_total,
                           hipStream_t st, const RefineSel* sel)
{
    const RefineSel sl = sel ? *sel : RefineSel{};
    if (finalize_is_wide(nchunk, N, ids != nullptr)) {
        hipLaunchKernelGGL(k_finalize_wide, dim3((unsigned)N), dim3(256), 0, st, part, nchunk, n, N, cont, se, steps,
                           sums, steps_total, sl);
        return hipGetLastError();
    }
    const int grid = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, st, part, nchunk, n, N, ids, n_ids,
                       cont, se, steps, sums, steps_total, sl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Start order of a date's continuation jobs.  The inner paths of a point far
// out of the money mostly run to maturity and those of a point deep in the
// money stop at once, so a launch that starts its jobs by increasing
// intrinsic value of the point runs the long jobs first and ends on short
// ones (in point order the last jobs to start left much of the device idle
// for their whole length).  Only the schedule depends on the order: every
// job writes its own partial sums.  The bridge step that draws the date's
// points appends each one to one of ORDER_BUCKETS lists by a squashed
// intrinsic value; the continuation launch walks the lists in bucket order.

// Intrinsic value of point j in single precision (an ordering key only).
__device__ __forceinline__ float order_key(const SpecT<double>& S, const double* __restrict__ x, int64_t N, int64_t j)
{
    const int d = S.d;
    const int pay = S.payoff;
    const float K = (float)S.K;
    float acc = pay == PUT_GEO || pay == PUT_BASKET ? 0.f : logf((float)x[j]);
    for (int i = (pay == PUT_GEO || pay == PUT_BASKET) ? 0 : 1; i < d; ++i) {
        const float v = (float)x[i * N + j];
        if (pay == CALL_MAX) acc = fmaxf(acc, logf(v));
        else if (pay == CALL_MIN) acc = fminf(acc, logf(v));
        else if (pay == PUT_GEO) acc += logf(v);
        else acc += v;
    }
    if (pay == PUT_GEO) return K - expf(acc * (float)S.inv_d);
    if (pay == PUT_BASKET) return K - acc * (float)S.inv_d;
    return expf(acc) - K;
}

__device__ __forceinline__ int order_bucket_of(float k, float K)
{
    const float t = (float)ORDER_BUCKETS * (0.5f + 0.5f * tanhf(4.f * k / K));   // NaN -> bucket 0
    return t > 0.f ? (t < (float)(ORDER_BUCKETS - 1) ? (int)t : ORDER_BUCKETS - 1) : 0;
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

__device__ __forceinline__ void bridge_end_point(const DevSpec* __restrict__ s, int64_t N, uint32_t seed, double* B,
                                                 int64_t j)
{
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
__device__ __forceinline__ void bridge_back_point(const DevSpec* __restrict__ s, int m, int64_t N, uint32_t seed,
                                                  double* B, double* x, int bridge, int64_t j)
{
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

__global__ void k_bridge_end(const DevSpec* __restrict__ s, int64_t N, uint32_t seed, double* B,
                             unsigned long long* zero_u64, int32_t* zero_words, int nwords)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (zero_u64 && j == 0) *zero_u64 = 0;
    if (zero_words && j < nwords) zero_words[j] = 0;
    if (j < N) bridge_end_point(s, N, seed, B, j);
}

__global__ void k_bridge_back(const DevSpec* __restrict__ s, int m, int64_t N, uint32_t seed,
                              double* B, double* x, int bridge, int32_t* zero_count, int32_t* ord_cnt,
                              int32_t* ord_list, int32_t* ord_clear)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (zero_count && j == 0) *zero_count = 0;
    if (ord_clear && j < ORDER_BUCKETS) ord_clear[j] = 0;
    if (!ord_cnt) {
        if (j < N) bridge_back_point(s, m, N, seed, B, x, bridge, j);
        return;
    }
    // bucket appends: ranks inside the block, then one range per bucket
    __shared__ int lcnt[ORDER_BUCKETS], lbase[ORDER_BUCKETS];
    if (threadIdx.x < ORDER_BUCKETS) lcnt[threadIdx.x] = 0;
    __syncthreads();
    int b = -1, r = 0;
    if (j < N) {
        bridge_back_point(s, m, N, seed, B, x, bridge, j);
        b = order_bucket_of(order_key(s->f64, x, N, j), (float)s->f64.K);
        r = atomicAdd(&lcnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < ORDER_BUCKETS) {
        const int c = lcnt[threadIdx.x];
        lbase[threadIdx.x] = c ? atomicAdd(&ord_cnt[threadIdx.x], c) : 0;
    }
    __syncthreads();
    if (b >= 0) ord_list[(size_t)b * (size_t)N + (size_t)(lbase[b] + r)] = (int32_t)j;
}

// Bridge steps of many options in one launch (256 points per block).
__global__ void k_bridge_multi(const BridgeTask* __restrict__ tasks, const uint32_t* __restrict__ prefix, int ntasks,
                               int end)
{
    const int ti = task_of_block(prefix, ntasks, blockIdx.x);
    const BridgeTask& t = tasks[ti];
    const int64_t j = (int64_t)(blockIdx.x - prefix[ti]) * blockDim.x + threadIdx.x;
    if (!end && t.zero_count && j == 0) *t.zero_count = 0;
    if (j >= t.N) return;
    if (end) bridge_end_point(t.s, t.N, t.seed, t.B, j);
    else bridge_back_point(t.s, t.m, t.N, t.seed, t.B, t.x, 1, j);
}

hipError_t launch_bridge_end(const DevSpec* s, int d, int64_t N, uint32_t seed, double* B,
                             hipStream_t st, unsigned long long* zero_u64, int32_t* zero_words, int nwords)
{
    (void)d;
    if (nwords < 0 || (zero_words && nwords > 256)) return hipErrorInvalidValue;   // block 0 clears them
    hipLaunchKernelGGL(k_bridge_end, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, s, N, seed, B,
                       zero_u64, zero_words, nwords);
    return hipGetLastError();
}

hipError_t launch_bridge_back(const DevSpec* s, int d, int m, int64_t N, uint32_t seed, double* B,
                              double* x, int bridge, hipStream_t st, int32_t* zero_count, int32_t* ord_cnt,
                              int32_t* ord_list, int32_t* ord_clear)
{
    (void)d;
    if (ord_cnt && (!x || !ord_list || N > ORDER_MAX_N)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bridge_back, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, s, m, N,
                       seed, B, x, bridge, zero_count, ord_cnt, ord_list, ord_clear);
    return hipGetLastError();
}

hipError_t launch_bridge_multi(const BridgeTask* tasks, const uint32_t* prefix, int ntasks, uint32_t blocks,
                               int end, hipStream_t st)
{
    hipLaunchKernelGGL(k_bridge_multi, dim3(blocks), dim3(256), 0, st, tasks, prefix, ntasks, end);
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

// Lattice of a region's boundary (region region0 + blockIdx.y in the
// column block blockIdx.y; rows of gridDim.y J entries): coordinate i maps to
// the i-th asset other than the region's own one, whose row is set to K.
__global__ void k_lattice(const DevSpec* __restrict__ s, int m, int region0, int64_t J,
                          const unsigned long long* __restrict__ best, double* x_all)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    const int region = region0 + (int)blockIdx.y;
    const int64_t ld = (int64_t)gridDim.y * J;
    double* x = x_all + (int64_t)blockIdx.y * J;
    const SpecT<double>& S = s->f64;
    const int d = S.d, q = d - 1;
    const int64_t a = best ? (int64_t)(0xFFFFFF - (*best & 0xFFFFFFull)) : 1;
    const double tm = S.t[m], sq = sqrt(tm);
    x[region * ld + j] = S.K;
    int64_t g = 1;
    for (int i = 0; i < q; ++i) {
        const double u = ((double)((j * g) % J) + 0.5) / (double)J;
        const int asset = i < region ? i : i + 1;
        x[asset * ld + j] = S.S0[asset] * exp(S.drift[asset] * tm + S.sigma[asset] * sq * normcdfinv(u));
        g = (g * a) % J;
    }
}

hipError_t launch_lattice(const DevSpec* s, int d, int m, int region0, int nreg, int64_t J,
                          const unsigned long long* best, double* x, hipStream_t st)
{
    (void)d;
    hipLaunchKernelGGL(k_lattice, dim3((unsigned)((J + 255) / 256), (unsigned)nreg), dim3(256), 0, st, s, m,
                       region0, J, best, x);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// I&Z boundary-point search state (the step itself: iz_step.hpp).

// Columns j of nreg regions side by side (J each, rows of Jt = nreg J).
// n_ids: the three rotating active counts; the first starts at every column,
// the other two at zero.
// ties: null, or [Jt] near-tie flags.  subset = 0: every column starts
// (its flag cleared); subset = 1: only the flagged columns start again (a
// search of them in another precision), listed in ids by an atomic count
// that the caller clears beforehand; the others keep their results.
__global__ void k_iz_init(const DevSpec* __restrict__ s, const double* __restrict__ x_in, int d, int region0,
                          int64_t J, int64_t Jt, double* x_work, double* s_cur, double* s_out, int32_t* iters,
                          int32_t* ids, int32_t* n_ids, unsigned long long* steps_acc, int32_t* ties, int subset)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Jt) return;
    if (subset && !ties[j]) return;
    const int region = region0 + (int)(j / J);
    const double K = s->f64.K;
    for (int i = 0; i < d; ++i) x_work[i * Jt + j] = i == region ? K : x_in[i * Jt + j];
    s_cur[j] = K;
    s_out[j] = -1.0;
    iters[j] = 0;
    steps_acc[j] = 0;
    if (subset) {
        ids[atomicAdd(&n_ids[0], 1)] = (int32_t)j;
        return;
    }
    if (ties) ties[j] = 0;
    ids[j] = (int32_t)j;
    if (j == 0) {
        n_ids[0] = (int32_t)Jt;
        n_ids[1] = 0;
        n_ids[2] = 0;
    }
}

hipError_t launch_iz_init(const DevSpec* s, const double* x_in, int d, int region0, int nreg, int64_t J,
                          double* x_work, double* s_cur, double* s_out, int32_t* iters, int32_t* ids,
                          int32_t* n_ids, unsigned long long* steps_acc, hipStream_t st, int32_t* ties, int subset)
{
    const int64_t Jt = (int64_t)nreg * J;
    hipLaunchKernelGGL(k_iz_init, dim3((unsigned)((Jt + 255) / 256)), dim3(256), 0, st, s, x_in, d, region0, J, Jt,
                       x_work, s_cur, s_out, iters, ids, n_ids, steps_acc, ties, subset);
    return hipGetLastError();
}

// One search step per active point (iz_step_slot), one thread per slot:
// state read from st_r, written to st_w ([3][Jt] each: point, previous
// point, previous residual).  Also clears n_next, the active count of the
// iteration after next.
__global__ void k_iz_update(const DevSpec* __restrict__ s, int d, int region0, int64_t J, int64_t Jt,
                            const double* __restrict__ part, uint32_t nchunk, uint32_t n,
                            const int32_t* __restrict__ ids_in, const int32_t* __restrict__ n_in,
                            int32_t* ids_out, int32_t* n_out, int32_t* n_next, const double* st_r, double* st_w,
                            double* x_work, double* s_out, int32_t* iters, unsigned long long* steps_acc,
                            double eps, int max_iter, int mode, int it, double tau, int32_t* ties)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot == 0) *n_next = 0;
    if (slot >= *n_in) return;
    iz_step_slot(s->f64, d, region0, J, Jt, part, nchunk, n, ids_in[slot], ids_out, n_out, st_r, st_r + Jt,
                 st_r + 2 * Jt, st_w, st_w + Jt, st_w + 2 * Jt, x_work, s_out, iters, steps_acc, eps, max_iter,
                 mode, it, tau, ties);
}

hipError_t launch_iz_update(const DevSpec* s, int d, int region0, int nreg, int64_t J, const double* part,
                            uint32_t nchunk, uint32_t n, const int32_t* ids_in, const int32_t* n_in,
                            int32_t* ids_out, int32_t* n_out, int32_t* n_next, const double* st_r, double* st_w,
                            double* x_work, double* s_out, int32_t* iters, unsigned long long* steps_acc,
                            double eps, int max_iter, int mode, int it, hipStream_t st, double tau, int32_t* ties)
{
    const int64_t Jt = (int64_t)nreg * J;
    hipLaunchKernelGGL(k_iz_update, dim3((unsigned)((Jt + 255) / 256)), dim3(256), 0, st, s, d, region0, J, Jt,
                       part, nchunk, n, ids_in, n_in, ids_out, n_out, n_next, st_r, st_w, x_work, s_out, iters,
                       steps_acc, eps, max_iter, mode, it, tau, ties);
    return hipGetLastError();
}

// Search totals of a date: per block sums, then one 64-bit atomic add per
// total (integer sums: the result does not depend on the order).
__global__ void __launch_bounds__(256) k_iz_tally(const unsigned long long* __restrict__ steps_acc,
                                                  const double* __restrict__ s_out, const int32_t* __restrict__ iters,
                                                  int64_t count, unsigned long long* tally)
{
    __shared__ unsigned long long red[3][4];
    unsigned long long a = 0, b = 0, c = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
         j += (int64_t)gridDim.x * blockDim.x) {
        a += steps_acc[j];
        b += s_out[j] > 0.0 ? 0ull : 1ull;
        c += (unsigned long long)iters[j];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
        red[2][wv] = c;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int w = 0; w < 4; ++w) v += red[threadIdx.x][w];
        atomicAdd(&tally[threadIdx.x], v);
    }
}

hipError_t launch_iz_tally(const unsigned long long* steps_acc, const double* s_out, const int32_t* iters,
                           int64_t count, unsigned long long* tally, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 256);
    hipLaunchKernelGGL(k_iz_tally, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, steps_acc,
                       s_out, iters, count, tally);
    return hipGetLastError();
}

__global__ void k_narrow(const double* __restrict__ a, float* b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Never-exercise rows: value nv in column 0 of every row, zeros elsewhere.
__global__ void k_rules_fill(double* w64, float* w32, int rows, int width, double nv)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * width) return;
    const double v = e % width == 0 ? nv : 0.0;
    w64[e] = v;
    w32[e] = (float)v;
}

hipError_t launch_rules_fill(double* w64, float* w32, int rows, int width, double nv, hipStream_t st)
{
    hipLaunchKernelGGL(k_rules_fill, dim3((unsigned)((rows * width + 255) / 256)), dim3(256), 0, st, w64, w32, rows,
                       width, nv);
    return hipGetLastError();
}

hipError_t launch_rules_narrow(const double* w64, float* w32, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, w64, w32, count);
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
