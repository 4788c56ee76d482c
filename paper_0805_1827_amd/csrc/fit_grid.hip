// One-launch CMC boosting fit: the tiles of training points are spread over
// the blocks (at most one per CU); each boosting round ends with one grid
// barrier, after which every block merges the tile partials (in tile order)
// and solves the small system itself, so the coefficients never leave the
// block between rounds.  Used while the block's LDS layout fits the
// device's per-workgroup LDS (every p up to d = 64 on gfx950's 160 KB); the
// multi-launch form in fit.hip is the fallback for smaller LDS.  For p <= 15 the tile's weighted normal
// equations run on the FP64 matrix cores.
#include "fit_common.hpp"

namespace bmc {

// Normal-equation path by rule width: 1 = one 16x16 MFMA block (p <= 15),
// 2 = 16x16 MFMA blocks (p <= 96, tiles of 64+ points), 0 = scalar.
__host__ __device__ inline int coop_mode(int p) { return p <= 15 ? 1 : (p <= 96 ? 2 : 0); }
__host__ __device__ inline int coop_psi_width(int p)
{
    const int m = coop_mode(p);
    return m == 1 ? 16 : (m == 2 ? 16 * ((p + 16) / 16) : p);
}
__host__ __device__ inline int coop_aux(int p, int T)
{
    const int a = TILE_SUB * (p + 1), b = coop_mode(p) == 1 ? (T / 64) * 256 : 0;
    return a > b ? a : b;
}

// Sum over tiles, in tile order, of the Q columns of a [ntiles][Q] array
// into out[Q] (LDS): thread q reads its column straight from memory (the
// threads of a tile row read consecutive words), sixteen (then eight) tiles'
// loads in flight before their adds, which keep the order of a sequential
// merge from zero.
__device__ void merge_tiles(const double* __restrict__ part, int ntiles, int Q, double* out)
{
    const int T = blockDim.x, tid = threadIdx.x;
    __syncthreads();
    for (int q = tid; q < Q; q += T) {
        double acc = 0.0;
        int t = 0;
        for (; t + 16 <= ntiles; t += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = part[(size_t)(t + u) * Q + q];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u];
        }
        for (; t + 8 <= ntiles; t += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(t + u) * Q + q];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; t < ntiles; ++t) acc += part[(size_t)t * Q + q];
        out[q] = acc;
    }
    __syncthreads();
}

// Raw features and mask of tile points j0.. into LDS: stage[f*T + t], m[t].
__device__ void stage_tile(const double* __restrict__ phi, const double* __restrict__ msk, int64_t N, int p,
                           int64_t j0, double* stage, double* m)
{
    const int T = blockDim.x, tid = threadIdx.x;
    const int64_t j = j0 + tid;
    for (int f = 0; f < p; ++f) stage[f * T + tid] = j < N ? phi[f * N + j] : 0.0;
    m[tid] = j < N ? msk[j] : 0.0;
    __syncthreads();
}

// The fit runs on a group of blocks: the whole grid of its launch, or one
// block (many options fitted side by side, one per block).  Tile t belongs
// to group member t mod size; every member merges all tiles in tile order,
// so the result does not depend on the group size.
//
// The grid barrier of the one-launch fit.  The launch has at most one block
// per CU, so on a device that is not full every block is resident at once.
// bar[0] counts arrivals and bar[1] is the generation; bar[0] returns to zero
// at every barrier, so the words are zeroed once, before the first launch.
// Thread 0 of each block reads the generation, then arrives with an
// acquire-release add at device scope; the last arrival clears the count and
// publishes the next generation with a release store, the others poll the
// generation and take an acquire fence once it moved.  The block barriers
// before and after order the other threads' tile partials and reads.  A
// wait longer than FIT_BARRIER_SPINS polls (about a second) sets *err and
// gives up, so a launch whose blocks cannot all be resident ends with an
// error instead of waiting for ever.
constexpr uint32_t FIT_BARRIER_SPINS = 1u << 20;

struct GridGroup {
    unsigned* bar;
    int32_t* err;   // pinned host word
    __device__ int rank() const { return blockIdx.x; }
    __device__ int size() const { return gridDim.x; }
    __device__ void sync()
    {
        __syncthreads();
        if (gridDim.x == 1) return;   // one block: the block barrier is the grid barrier
        if (threadIdx.x == 0) {
            const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == gridDim.x - 1) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                uint32_t spins = 0;
                while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    if (++spins > FIT_BARRIER_SPINS) {
                        *err = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        __syncthreads();
    }
};
struct BlockGroup {
    __device__ int rank() const { return 0; }
    __device__ int size() const { return 1; }
    __device__ void sync() { __syncthreads(); }
};

template <class G>
__device__ void fit_cmc_body(const FitTask& a, G grp)
{
    extern __shared__ double sh[];
    __shared__ int flag;
    __shared__ double lam, cnt_s;
    const int p = a.p, T = blockDim.x, npairs = p * (p + 1) / 2, Q = npairs + p;
    const int tid = threadIdx.x;
    const int mode = coop_mode(p);
    const int SW = coop_psi_width(p);
    double* psi = sh;                                   // [T][psi width]; also the staging area
    double* wz = psi + (size_t)T * coop_psi_width(p);  // [T][2]
    double* aux = wz + 2 * T;                           // two-level sums / per-wave Gram matrices
    double* A = aux + coop_aux(p, T);                   // [npairs] packed lower triangle, then bv
    double* bv = A + npairs;                            // [p]
    double* beta = bv + p;                              // [p]
    double* mu = beta + p;                              // [p]
    double* sd = mu + p;                                // [p]
    const SpecT<double>& S = a.s->f64;
    const FitScratch& fs = a.fs;
    const int64_t N = a.N;

    // features, labels, in-the-money mask; per tile the count, the feature
    // sums and the squared deviations from the tile's own means
    for (int t = grp.rank(); t < a.ntiles; t += grp.size()) {
        const int64_t j0 = (int64_t)t * T;
        fit_prep_point(S, a.x, a.cont, N, j0 + tid, fs.phi, fs.lab, fs.msk);
        __syncthreads();
        stage_tile(fs.phi, fs.msk, N, p, j0, psi, wz);
        const int nt = (int)min((int64_t)T, N - j0);
        tile_sum2(p + 1, nt, [&](int f, int q) { return f < p ? wz[q] * psi[f * T + q] : wz[q]; }, aux, A);
        for (int f = tid; f <= p; f += T) fs.part1[(size_t)t * (p + 1) + f] = A[f];
        for (int f = tid; f < p; f += T) mu[f] = A[p] > 0.0 ? A[f] / A[p] : 0.0;   // the tile's means
        __syncthreads();
        tile_sum2(p, nt,
                  [&](int f, int q) {
                      const double dv = psi[f * T + q] - mu[f];
                      return wz[q] * dv * dv;
                  },
                  aux, fs.part2 + (size_t)t * p);
    }
    grp.sync();
    // every block: the tiles combined in tile order by the pairwise update of
    // count, mean and sum of squared deviations (Chan, Golub and LeVeque)
    for (int f = tid; f < p; f += T) {
        double n = 0.0, m = 0.0, M2 = 0.0;
        int t = 0;
        for (; t + 8 <= a.ntiles; t += 8) {
            double c8[8], s8[8], q8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                c8[u] = fs.part1[(size_t)(t + u) * (p + 1) + p];
                s8[u] = fs.part1[(size_t)(t + u) * (p + 1) + f];
                q8[u] = fs.part2[(size_t)(t + u) * p + f];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) chan_merge(c8[u], s8[u], q8[u], n, m, M2);
        }
        for (; t < a.ntiles; ++t)
            chan_merge(fs.part1[(size_t)t * (p + 1) + p], fs.part1[(size_t)t * (p + 1) + f],
                       fs.part2[(size_t)t * p + f], n, m, M2);
        if (f == 0) cnt_s = n;
        fit_mu_sd_merged(f, n, m, M2, &mu[f], &sd[f]);
        if (grp.rank() == 0) {
            a.musd[f] = mu[f];
            a.musd[p + f] = sd[f];
        }
    }
    __syncthreads();
    const double cnt = cnt_s;
    if (grp.rank() == 0 && tid == 0) a.musd[2 * p] = cnt;
    if (!(cnt > 0.0)) {   // no in-the-money point: never exercise (same in every block)
        if (grp.rank() == 0)
            for (int f = tid; f < p; f += T) { a.row64[f] = 0.0; a.row32[f] = 0.0f; }
        return;
    }
    // Round r's tile partials go to buffer r % 2: a block writes round r+2's
    // partials only after the barrier of round r+1, which every block passes
    // after reading round r's, so one barrier per round suffices.
    const size_t part_stride = (size_t)a.ntiles * Q;
    // A block with (at most) one tile keeps it for the whole fit: its rows
    // stay in psi, F, the label and the mask in registers.
    const bool resident = mode != 0 && a.ntiles <= grp.size();
    double F_reg = 0.0, lab_reg = 0.0, msk_reg = 0.0;
    const int64_t j_own = (int64_t)grp.rank() * T + tid;
    const bool own_in = grp.rank() < a.ntiles && j_own < N;
    if (resident && own_in) {
        lab_reg = fs.lab[j_own];
        msk_reg = fs.msk[j_own];
    }
    for (int r = 0; r < a.rounds; ++r) {
        double* partA = fs.partA + (size_t)(r & 1) * part_stride;
        for (int t = grp.rank(); t < a.ntiles; t += grp.size()) {
            const int64_t j0 = (int64_t)t * T;
            const int nt = (int)min((int64_t)T, N - j0);
            if (resident && r > 0) {
                fit_round_point_resident(p, SW, own_in, beta, F_reg, lab_reg, msk_reg, psi, wz);
                __syncthreads();
                if (mode == 1) fit_tile_normal_eqs_mfma(psi, wz, p, nt, aux, partA + (size_t)t * Q);
                else fit_tile_normal_eqs_mfma_wide(psi, SW, wz, p, nt, partA + (size_t)t * Q);
            } else if (mode == 1) {
                fit_round_point16(fs.phi, fs.lab, fs.msk, N, p, mu, sd, r > 0 ? beta : nullptr, j0 + tid, fs.F,
                                  fs.pi, psi, wz);
                __syncthreads();
                fit_tile_normal_eqs_mfma(psi, wz, p, nt, aux, partA + (size_t)t * Q);
            } else if (mode == 2) {
                fit_round_point_s(fs.phi, fs.lab, fs.msk, N, p, SW, mu, sd, r > 0 ? beta : nullptr, j0 + tid, fs.F,
                                  fs.pi, psi, wz);
                __syncthreads();
                fit_tile_normal_eqs_mfma_wide(psi, SW, wz, p, nt, partA + (size_t)t * Q);
            } else {
                fit_round_point(fs.phi, fs.lab, fs.msk, N, p, mu, sd, r > 0 ? beta : nullptr, j0 + tid, fs.F,
                                fs.pi, psi, wz);
                __syncthreads();
                fit_tile_normal_eqs(psi, wz, p, nt, partA + (size_t)t * Q);
            }
            __syncthreads();
        }
        if (resident && r == 0 && own_in) F_reg = fs.F[j_own];   // round 0 wrote it
        grp.sync();
        merge_tiles(partA, a.ntiles, Q, A);   // A then bv
        // ridge 1e-8 tr / p, the trace summed inside the solver's wavefront
        if (!spd_solve_ridge(p, A, 1e-8, bv, beta, &flag, &lam))
            for (int f = tid; f < p; f += T) beta[f] = 0.0;
        __syncthreads();
        if (grp.rank() == 0)
            for (int f = tid; f < p; f += T) fs.beta[(size_t)r * p + f] = beta[f];
    }
    if (grp.rank() == 0) {
        __syncthreads();
        fit_fold(p, a.rounds, a.musd, fs.beta, a.row64, a.row32);
    }
}

__global__ void __launch_bounds__(256) k_fit_cmc_grid(FitTask a, unsigned* bar, int32_t* err)
{
    fit_cmc_body(a, GridGroup{bar, err});
}

// One option per block.
__global__ void __launch_bounds__(256) k_fit_cmc_multi(const FitTask* __restrict__ tasks)
{
    const FitTask a = tasks[blockIdx.x];
    fit_cmc_body(a, BlockGroup{});
}

size_t fit_task_lds(int p)
{
    const int T = fit_tile(p), npairs = p * (p + 1) / 2;
    return sizeof(double) * ((size_t)T * coop_psi_width(p) + 2 * T + coop_aux(p, T) + npairs + 4 * p);
}

// Dynamic LDS the fit kernels may use on the current device: the
// per-workgroup maximum (160 KB on gfx950) less their static LDS.  Falls
// back to 64 KB if the runtime refuses the larger size.
static size_t fit_lds_limit()
{
    static size_t limit = 0;
    if (limit == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        size_t lim = (size_t)v;
        for (const void* f : {reinterpret_cast<const void*>(k_fit_cmc_grid),
                              reinterpret_cast<const void*>(k_fit_cmc_multi)}) {
            hipFuncAttributes fa;
            size_t dyn = 64 * 1024 - 256;
            if (hipFuncGetAttributes(&fa, f) == hipSuccess && fa.sharedSizeBytes < (size_t)v) {
                const size_t want = (size_t)v - fa.sharedSizeBytes;
                if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) == hipSuccess)
                    dyn = want;
            }
            lim = std::min(lim, dyn);
        }
        (void)hipGetLastError();   // a refused attribute must not surface at the next launch check
        limit = lim;
    }
    return limit;
}

bool fit_one_launch_supported(int p) { return fit_task_lds(p) <= fit_lds_limit(); }

FitTask fit_task_make(const DevSpec* s, int d, const double* x, const double* cont, int64_t N, int rounds,
                      const FitScratch& fs, double* row64, float* row32)
{
    FitTask a;
    a.s = s;
    a.x = x;
    a.cont = cont;
    a.N = N;
    a.p = rule_width(CMC, d);
    a.rounds = rounds;
    const int T = fit_tile(a.p);
    a.ntiles = (int)((N + T - 1) / T);
    a.fs = fs;
    a.musd = fs.beta + (size_t)rounds * a.p;
    a.row64 = row64;
    a.row32 = row32;
    return a;
}

hipError_t launch_fit_cmc_grid(const DevSpec* s, int d, const double* x, const double* cont, int64_t N,
                               int rounds, const FitScratch& fs, double* row64, float* row32, unsigned* bar,
                               int32_t* err, hipStream_t st)
{
    FitTask a = fit_task_make(s, d, x, cont, N, rounds, fs, row64, row32);
    const int T = fit_tile(a.p);
    const size_t lds = fit_task_lds(a.p);
    int dev = 0, cus = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev))) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))) return e;
    const int grid = (int)std::min<int64_t>(a.ntiles, cus);   // at most one block per CU
    hipLaunchKernelGGL(k_fit_cmc_grid, dim3(grid), dim3(T), lds, st, a, bar, err);
    return hipGetLastError();
}

hipError_t launch_fit_cmc_multi(const FitTask* tasks, int ntasks, int T, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL(k_fit_cmc_multi, dim3(ntasks), dim3(T), lds, st, tasks);
    return hipGetLastError();
}

}  // namespace bmc
