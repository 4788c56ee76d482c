// Internal launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cont_args.hpp"
#include "device.hpp"

namespace bmc {

// Spec as uploaded from the host, before the device-side setup kernel derives
// the Cholesky factor and the per-precision tables.
struct HostSpecPack {
    int32_t d, n_dates, payoff, pad;
    double K, r, T;
    double S0[D_MAX], delta[D_MAX], sigma[D_MAX];
    double rho[D_MAX * D_MAX];
    double dates[NT_MAX];
};

// Task of a multi-task launch whose blocks are numbered through the
// exclusive prefix sums of the tasks' block counts.
__device__ __forceinline__ int task_of_block(const uint32_t* __restrict__ prefix, int ntasks, uint32_t b)
{
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// FP32 label refinement: a training point whose FP32 continuation estimate
// C lies within REFINE_KAPPA standard errors (plus REFINE_ETA of |Phi| + |C|
// for rounding) of its in-the-money exercise value Phi is re-estimated in
// FP64 before the fit.  A label can differ from the FP64 form's only where
// Phi lies between the two estimates, so |Phi - C| <= |C - C_FP64|; the
// largest |C - C_FP64| measured over every point and date of the 256-option
// uneven workload is 0.61 standard errors, a third of REFINE_KAPPA.  The
// finalize of the FP32 estimates lists the points (RefineSel); the FP64
// re-estimates run REFINE_PPT paths per lane (the fastest measured shape at
// N = n = 4096 and on the uneven batch), REFINE_SLOTS (or N, if
// fewer) points at a time.
constexpr double REFINE_KAPPA = 2.0;
// I&Z searches of the FP32 forms flag every point with a decision within
// IZ_TIE_TAU K of its threshold (iz_step_compute: stopping test, sign of the
// inverse, region test); the pricer searches those points again in FP64.
// The FP32 map's own error at a given point is a few 10^-8 K (rounding of
// the payoff sums; median 4e-6 at K = 100 on the 5-asset geometric put),
// well inside the band.
constexpr double IZ_TIE_TAU = 1e-6;
// The FP64 search of the flagged points runs one path per lane (a few points
// per date, so its launches are latency-bound and shorter chunks finish
// sooner: 4.0 against 4.6 ms per Table 1 price with the FP64 form's shape).
constexpr int IZ_RESEARCH_PPT = 1;
constexpr double REFINE_ETA = 1e-5;
constexpr uint32_t REFINE_SLOTS = 256;
constexpr int REFINE_PPT = 2;
// Selection made by a finalize: s == null selects nothing.  The list ids
// (count *n_ids, cleared beforehand) receives the points to refine.
struct RefineSel {
    const DevSpec* s;
    const double* x;
    int32_t* ids;
    int32_t* n_ids;
};

// Finalize of one task inside a multi-task launch (see launch_finalize).
// ids/n_ids: merge only the listed points (narrow tasks).
struct FinTask {
    const double* part;
    double* cont;
    double* se;
    int64_t* steps;
    double* sums;
    unsigned long long* steps_total;
    const int32_t* ids;
    const int32_t* n_ids;
    RefineSel sel;
    int64_t N;
    uint32_t nchunk, n;
    int32_t wide;
    int32_t pad;
};

// Bridge step of one option inside a multi-task launch; zero_count (or
// null): a counter the bridge-back step clears for the launches after it.
struct BridgeTask {
    const DevSpec* s;
    double* B;
    double* x;
    int32_t* zero_count;
    int64_t N;
    uint32_t seed;
    int32_t m;
};

struct LaunchCfg {
    int block = 256;          // threads per workgroup
    int ppt = 4;              // paths per thread per chunk
};

// Kernels (kernels.hip).  All enqueue on `st` and return hipError_t.
// Spec setup of count packs; pack i goes to out[slots ? slots[i] : i].
// status_host (count = 1): device address of a pinned host word that also
// receives the setup status (0, or -2 if rho is not positive definite).
hipError_t launch_setup(const HostSpecPack* in, DevSpec* out, int count, hipStream_t st,
                        const uint32_t* slots = nullptr, int32_t* status_host = nullptr);
hipError_t launch_cont(int d, int prec, const ContArgs& a, int grid, int block, size_t lds,
                       hipStream_t st);
// One launch over jobs job0 .. job0+jobs-1 of many tasks of one bucket;
// prefix[t] is the first job of task t, prefix[ntasks] the total.  stride:
// the tasks run their slots with a slot stride (FP64 label refinement).
hipError_t launch_cont_multi(int bucket, int prec, const ContArgs* tasks, const uint32_t* prefix, int ntasks,
                             uint32_t job0, uint32_t jobs, int block, size_t lds, hipStream_t st,
                             bool stride = false);
bool finalize_is_wide(uint32_t nchunk, int64_t N, bool has_ids);
// prefix: first block of each task (wide: N blocks, else ceil(N/256)).
hipError_t launch_finalize_multi(const FinTask* tasks, const uint32_t* prefix, int ntasks, uint32_t blocks,
                                 hipStream_t st);
// end = 1: draw B at maturity; end = 0: bridge back to date m and write x.
// prefix: first block of each task (ceil(N/256) blocks each).
hipError_t launch_bridge_multi(const BridgeTask* tasks, const uint32_t* prefix, int ntasks, uint32_t blocks,
                               int end, hipStream_t st);
hipError_t launch_finalize(const double* part, uint32_t nchunk, uint32_t n, int64_t N,
                           const int32_t* ids, const int32_t* n_ids, double* cont, double* se,
                           int64_t* steps, double* sums, unsigned long long* steps_total,
                           hipStream_t st, const RefineSel* sel = nullptr);
// zero_u64 and zero_words[0 .. nwords) (each or null; nwords <= 256) are
// cleared by the launch, before any later launch on the stream reads them.
hipError_t launch_bridge_end(const DevSpec* s, int d, int64_t N, uint32_t seed, double* B,
                             hipStream_t st, unsigned long long* zero_u64 = nullptr,
                             int32_t* zero_words = nullptr, int nwords = 0);
// zero_count (or null) is cleared by the launch.  ord_cnt (or null, with
// x): the launch appends every point to the bucket list of its intrinsic
// value (ord_cnt[ORDER_BUCKETS] counts, zero beforehand; ord_list
// [ORDER_BUCKETS][N]) and clears ord_clear[ORDER_BUCKETS], the other date
// parity's counts.
hipError_t launch_bridge_back(const DevSpec* s, int d, int m, int64_t N, uint32_t seed, double* B,
                              double* x, int bridge, hipStream_t st, int32_t* zero_count = nullptr,
                              int32_t* ord_cnt = nullptr, int32_t* ord_list = nullptr, int32_t* ord_clear = nullptr);
// Largest N whose date launches are given a job order (bucket lists of
// ORDER_BUCKETS N entries).
constexpr int64_t ORDER_MAX_N = 65536;
hipError_t launch_korobov(int64_t J, int q, unsigned long long* best, hipStream_t st);
// I&Z regions region0 .. region0 + nreg - 1 side by side: J points each,
// region region0 + r in columns r J .. r J + J - 1 of rows of nreg J entries.
// Lattice: over the other assets, the region's own asset set to K.  Search
// state: the region's own asset is the searched coordinate.
hipError_t launch_lattice(const DevSpec* s, int d, int m, int region0, int nreg, int64_t J,
                          const unsigned long long* best, double* x, hipStream_t st);
// ties (or null): near-tie flags [nreg J], cleared; with subset = 1 only the
// flagged columns start again, appended to ids by the count n_ids[0] (cleared
// by the caller), and the other columns keep their results.
hipError_t launch_iz_init(const DevSpec* s, const double* x_in, int d, int region0, int nreg, int64_t J,
                          double* x_work, double* s_cur, double* s_out, int32_t* iters, int32_t* ids,
                          int32_t* n_ids, unsigned long long* steps_acc, hipStream_t st, int32_t* ties = nullptr,
                          int subset = 0);
// One search step: merges the continuation partials (part, nchunk chunks of
// n paths in all) of the active points and updates them; mode SEARCH_PLAIN or
// SEARCH_SECANT; search state [3][nreg * J] (point, the secant's previous
// point and residual per column) read from st_r and written to st_w; clears
// *n_next.
hipError_t launch_iz_update(const DevSpec* s, int d, int region0, int nreg, int64_t J, const double* part,
                            uint32_t nchunk, uint32_t n, const int32_t* ids_in, const int32_t* n_in,
                            int32_t* ids_out, int32_t* n_out, int32_t* n_next, const double* st_r, double* st_w,
                            double* x_work, double* s_out, int32_t* iters, unsigned long long* steps_acc,
                            double eps, int max_iter, int mode, int it, hipStream_t st, double tau = 0.0,
                            int32_t* ties = nullptr);
// tally[0] += sum of steps_acc, tally[1] += number of s_out <= 0 (or NaN),
// tally[2] += sum of iters, over count points.
hipError_t launch_iz_tally(const unsigned long long* steps_acc, const double* s_out, const int32_t* iters,
                           int64_t count, unsigned long long* tally, hipStream_t st);
hipError_t launch_rules_fill(double* w64, float* w32, int rows, int width, double nv, hipStream_t st);
hipError_t launch_rules_narrow(const double* w64, float* w32, int64_t count, hipStream_t st);

// CMC boosting fit (FP64) of rule row m.
struct FitScratch {
    double* phi;     // [p][N] raw features
    double* lab;     // [N]
    double* msk;     // [N]
    double* F;       // [N]
    double* pi;      // [N]
    double* part1;   // [tiles][p+1]
    double* part2;   // [tiles][p]
    double* partA;   // [2][tiles][npairs + p]
    double* beta;    // [rounds][p]
};
// Points per tile (= threads per block) of the fits.
__host__ __device__ __forceinline__ int fit_tile(int p)
{
    if (p <= 15) return 256;
    if (p <= 48) return 128;
    if (p <= 96) return 64;
    return 32;
}

// One CMC fit as run by the one-launch grid or by one block of a
// multi-option launch.
struct FitTask {
    const DevSpec* s;
    const double* x;
    const double* cont;
    int64_t N;
    int p, rounds, ntiles;
    FitScratch fs;
    double* musd;
    double* row64;
    float* row32;
};
FitTask fit_task_make(const DevSpec* s, int d, const double* x, const double* cont, int64_t N, int rounds,
                      const FitScratch& fs, double* row64, float* row32);
size_t fit_task_lds(int p);
bool fit_one_launch_supported(int p);
// One block per task; all tasks share the tile size T = fit_tile(p).
hipError_t launch_fit_cmc_multi(const FitTask* tasks, int ntasks, int T, size_t lds, hipStream_t st);
size_t fit_scratch_doubles(int64_t N, int p, int rounds);
void fit_scratch_carve(double* base, int64_t N, int p, int rounds, FitScratch* fs);
// bar/err: the one-launch form's barrier words and error flag (null: the
// multi-launch form).
hipError_t launch_fit_cmc(const DevSpec* s, int d, const double* x, const double* cont, int64_t N,
                          int rounds, const FitScratch& fs, double* row64, float* row32,
                          hipStream_t st, unsigned* bar = nullptr, int32_t* err = nullptr);
// I&Z quadratic regression of rule row m; x[0*J + j] = s*_j.
size_t fitiz_scratch_doubles(int64_t J, int p);
// AdaBoost-stump fit of one date (rounds <= ADA_TMAX) into a rule row of width
// entries; scratch of fit_ada_scratch_bytes(N, d) bytes.
size_t fit_ada_scratch_bytes(int64_t N, int d);
hipError_t launch_fit_ada(const DevSpec* s, int d, const double* x, const double* cont, int64_t N, int rounds,
                          void* scratch, double* row64, float* row32, int width, hipStream_t st);
// Boundary blocks of regions region .. region + nreg - 1 (row64/row32 point
// at the first one; the others follow every p entries) from nreg sets of J
// points side by side in rows of ld entries (region r's in columns r J ..);
// s* from sstar[r J + j] when given, else from each region's own row of x.
// Scratch: nreg fitiz_scratch_doubles(J, p).
hipError_t launch_fit_iz(const DevSpec* s, int d, int region, const double* x, int64_t J, int64_t ld,
                         double* scratch, double* row64, float* row32, hipStream_t st, int nreg = 1,
                         const double* sstar = nullptr);

hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M, uint32_t* out,
                         hipStream_t st);
hipError_t launch_normals(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t M, int prec,
                          double* out, hipStream_t st);

}  // namespace bmc
