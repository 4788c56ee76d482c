// Interface of the continuation kernel: its launch arguments, the dimension
// buckets and the LDS layout of a job (shared by the kernel and its callers).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"

namespace bmc {

// I&Z search launches (I&Z rules only): before its pass, a job takes the
// search step of the previous pass for its point (merge of that pass's
// partials, next point or stop) and starts from the new point; a stopped
// point's jobs return at once.  The job of chunk 0 stores the step.
struct IzFuse {
    int32_t on;                 // 0: a plain pass from x
    int32_t it;                 // iteration of the step taken
    int32_t max_iter, mode;     // iteration limit, SEARCH_PLAIN / SEARCH_SECANT
    double eps;                 // convergence tolerance
    const double* part;         // previous pass's partials [N * nchunk * 3]
    const double* st_r;         // search state read [3][N]: point, previous point, previous residual
    double* st_w;               // search state written [3][N]
    double* x_work;             // the points [d][N] (a.x), searched coordinate updated
    double* s_out;              // [N] boundary point of a stopped column, -1: dropped
    int32_t* iters;             // [N] steps taken
    unsigned long long* steps_acc;   // [N] executed path-steps
    int32_t* ids_out;           // columns that continue (appended)
    int32_t* n_out;             // their count
    int32_t* n_next;            // count of the iteration after, cleared here
    int32_t* ties;              // [N] near-tie flags of an FP32 search (or null)
    double tau;                 // near-tie width (0: no flags)
    int32_t* poll;              // pinned host word that receives the count of the launch's list (or null;
                                // also read when on = 0)
    int32_t pad_;
};

// One continuation launch: points (ids or 0..N-1) x chunks of paths.
// Job order of a launch over all N points (cnt null: point order): the
// points listed bucket by bucket, cnt[b] points of bucket b at list[b N ..].
constexpr int ORDER_BUCKETS = 16;
struct JobOrder {
    const int32_t* cnt;    // [ORDER_BUCKETS]
    const int32_t* list;   // [ORDER_BUCKETS][N]
};

struct ContArgs {
    const DevSpec* spec;
    const void* rules;        // R[(NT+1) * width], row k = date k
    const double* x;          // SoA points [d][N]
    int64_t N;                // row stride of x
    const int32_t* ids;       // active point ids, or null for 0..N-1
    const int32_t* n_ids;     // device count of ids, or null
    uint32_t n;               // paths per point
    int32_t m;                // start date
    int32_t method;           // CMC / IZ / ADA
    int32_t width;            // rule row width
    uint32_t paths_per_wg;    // paths of one workgroup (a chunk)
    uint32_t nchunk;          // chunks per point
    uint32_t k0, k1;          // Philox key
    uint32_t slot;            // fourth Philox counter word (I&Z region, else 0)
    uint32_t region_pts;      // > 0: points of several I&Z regions side by side, region_pts
                              // each; point j counts as point j % region_pts of
                              // region slot + j / region_pts in the counters
    double* part;             // [N * nchunk * 3]: sum, sum of squares, steps
    uint32_t slot_stride;     // > 0: a workgroup runs the jobs of slots s, s + slot_stride, ...
                              // below *n_ids (chunk as its block gives); 0: one job
    uint32_t pad_;
    IzFuse fz;                // fused search step (on = 0 otherwise)
    JobOrder ord;             // start order of the jobs (ids null)
    const int32_t* cancel;    // (or null) device word: nonzero = the jobs stop after their setup
};

// Dimension buckets: every d <= 32 has its own instantiation (bucket_exact);
// larger d share a bound D with dim_floor(D) < d <= D (36, 40, then
// multiples of 8) and pad the path state to D.  For d >= 9 the correlation
// coefficients live in LDS and, in FP32, the correlation runs on the matrix
// cores in chunks of four assets.
__host__ __device__ constexpr bool bucket_exact(int D) { return D <= 32; }
__host__ __device__ constexpr int dim_floor(int D) { return bucket_exact(D) ? D - 1 : (D <= 40 ? D - 4 : D - 8); }
int cont_bucket(int d);

// Row stride of the rule rows in LDS: padded buckets widen classifier rows
// to 2D+3 (zero weights for the padded assets).
__host__ __device__ inline int cont_rule_stride(int D, int width)
{
    return !bucket_exact(D) && width < 2 * D + 3 ? 2 * D + 3 : width;
}

// Whether a continuation kernel of bound D reads the correlation coefficients
// and drifts from LDS (rsize: bytes of its stepping precision) rather than
// from scalar registers: from D = 9 on, and in FP64 from D = 2 on, where the
// coefficients' register pairs would not fit beside the generator's keys and
// the compiler would keep them in vector-register lanes instead.
__host__ __device__ constexpr bool cont_lds_coef(int D, size_t rsize) { return D >= 9 || (rsize == 8 && D >= 2); }

// LDS bytes of a continuation job: discount table (double), then in the
// stepping precision: log-point [D_MAX], dt and sqrt(dt) [NT+1], rule rows
// [(NT+1) stride], and where cont_lds_coef holds the correlation
// coefficients [D4][D4] (D4 = D rounded up to a multiple of 4; 16-byte
// aligned, at *coef_off) and the drifts [D4].
__host__ __device__ inline size_t cont_lds_layout(size_t rsize, int D, int n_dates, int width, size_t* coef_off)
{
    size_t off = sizeof(double) * (n_dates + 1) +
                 rsize * (D_MAX + 2 * (size_t)(n_dates + 1) + (size_t)(n_dates + 1) * cont_rule_stride(D, width));
    off = (off + 15) & ~(size_t)15;
    if (coef_off) *coef_off = off;
    const size_t D4 = (size_t)((D + 3) & ~3);
    if (cont_lds_coef(D, rsize)) off += rsize * (D4 * D4 + D4);
    return off + 16;
}
size_t cont_lds_bytes(int prec, int d, int n_dates, int width);
// Dynamic LDS a continuation workgroup may use on the current device.
size_t cont_lds_limit();
}  // namespace bmc
