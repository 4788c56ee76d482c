// Host-side runtime structures shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "bmc.h"

namespace bmc {
struct IzFuse;
struct RefineSel;

struct HostSpecPack;

constexpr int IZ_D_MAX = 16;

// Grow-only device allocation.
struct DBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n);
    void release();
};

// Launch shape of the continuation kernel (0 = automatic).
struct Tuning {
    int block = 0;
    int ppt = 0;
};

bmc_status fail(bmc_status st, const char* fmt, ...);
bmc_status hip_fail(hipError_t e, const char* where);
bmc_status validate_spec(const bmc_spec* s);

}  // namespace bmc

struct bmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bmc::HostSpecPack* pack_host = nullptr;   // pinned staging
    void* host_io = nullptr;                  // pinned 4 KB for small results
    void* host_io_dev = nullptr;              // its device address (kernels write progress polls there)
    bmc::DBuf spec, spec2, pack_dev, part, B, x, x2, cont, se, steps, fit, iz, counters, korobov;
    bmc::DBuf rf;   // FP32 label refinement: [count (256 B)][ids N]
    bmc::DBuf order;   // job order of the pricer's date launches: [count (256 B)][ids N]
    bmc::DBuf gbar;   // the one-launch fit's grid-barrier words (zeroed once; host_io + 136: its error flag)
    // batched pricing: device specs, per-option arena, task tables; pinned staging
    bmc::DBuf bspec, barena, btab;
    void* bhost = nullptr;
    size_t bhost_bytes = 0;
    // continuation launch shapes (paths per lane per job) by (dimension
    // bucket, precision, log2 n class); 0 fields are wildcards
    std::map<uint64_t, int> ppt_table;
    // batched date sweeps as a HIP graph: the last captured launch sequence,
    // replayed while the signature (launch shapes and buffers) is unchanged
    std::vector<hipEvent_t> ev_pool;   // reusable timing events
    hipEvent_t poll_ev[2] = {nullptr, nullptr};   // I&Z search progress polls (host_io + 128)
    // (J, q) whose Korobov generator the korobov buffer holds (-1: none)
    int64_t korobov_J = -1;
    int korobov_q = -1;
    bmc::DBuf srules;                  // rule table of bmc_price when the caller keeps none
    bool graphs = false;
    std::string graph_sig;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t graph_stream = nullptr;
    int64_t graph_captures = 0, graph_replays = 0;
    ~bmc_ctx();
};

struct bmc_rules {
    bmc_ctx* ctx = nullptr;
    int method = 0, d = 0, n_dates = 0, width = 0, payoff = 0;
    double* w64 = nullptr;   // device [(n_dates+1) * width]
    float* w32 = nullptr;    // device, same rows in float
};

namespace bmc {

// Takes the device address of the no-allocation entry point's scratch array
// on `device` (the current device) once; bmc_ctx_create calls it.
bmc_status noalloc_setup(int device);
bmc_status upload_spec(bmc_ctx* ctx, const bmc_spec* s, DBuf& slot);
// As upload_spec without waiting: the setup status (0 or -2) is copied to
// *status_host (pinned) on the stream; the caller checks it after a sync.
bmc_status upload_spec_async(bmc_ctx* ctx, const bmc_spec* s, DBuf& slot, int32_t* status_host);
// Rule table in context scratch (rows of never-exercise values), for callers
// that do not keep the rules; valid until the next call on the context.
bmc_status scratch_rules(bmc_ctx* ctx, const bmc_spec* spec, int method, bmc_rules* out);
void pack_spec(const bmc_spec* s, HostSpecPack* p);
const double* dev_S0(const void* devspec);
// Error flag of the one-launch fit's grid barrier (a pinned host word; the
// device address for the kernel), and its check after a synchronization:
// BMC_EDEVICE (and the flag and barrier words reset) if a barrier gave up.
int32_t* fit_barrier_flag_dev(bmc_ctx* ctx);
bmc_status check_fit_barrier(bmc_ctx* ctx);
uint32_t choose_ppt(const bmc_ctx* ctx, int d, int prec, int64_t points, int64_t n, const Tuning* tune);
uint64_t ppt_key(int bucket, int prec_plus1, int nclass);
int n_class(int64_t n);
bmc_status run_cont(bmc_ctx* ctx, const void* devspec, int d, int n_dates, int method, int width,
                    const void* rules64, const void* rules32, int prec, int m, const double* x,
                    int64_t N, const int32_t* ids, const int32_t* n_ids, uint32_t n, uint32_t k0,
                    uint32_t k1, double* cont, double* se, int64_t* steps, double* sums,
                    unsigned long long* steps_total, const Tuning* tune, uint32_t slot = 0,
                    uint32_t region_pts = 0, uint32_t* nchunk_out = nullptr, double* part = nullptr,
                    const IzFuse* fz = nullptr, const RefineSel* sel = nullptr, const JobOrder* ord = nullptr,
                    int64_t max_active = 0);
// region: the I&Z region whose boundary row block is fitted (0 for CMC), from
// N points in rows of ld entries (0: N).
bmc_status fit_rule_impl(bmc_ctx* ctx, const void* devspec, int d, bmc_rules* rules, int date,
                         const double* x, const double* values, int64_t N, int rounds, int region = 0,
                         int64_t ld = 0);
// I&Z: regions region .. region + nreg - 1 side by side (N points each, rows
// of nreg N entries).
bmc_status sample_points_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec, int method,
                              int date, int64_t N, uint32_t seed, double* x, double* Bbuf, int region = 0,
                              int nreg = 1);
// Searches regions region .. region + nreg - 1 together: x, s_out and iters
// hold nreg J points side by side, as sample_points_impl lays them out.
// ties (FP32 searches of the pricer): near-tie flags [nreg J] written by the
// search (IZ_TIE_TAU); again = 1 searches only the flagged points again, in
// precision prec, keeping every other point's results.
// tally (device, optional): adds the executed path-steps, the points left
// without a boundary point and the iterations to tally[0..2] on the stream,
// so that a caller sweeping dates reads them once at the end.
bmc_status iz_search_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec,
                          const bmc_rules* rules, int date, int region, int nreg, const double* x, int64_t J,
                          uint32_t n, uint32_t seed, int prec, double eps, int max_iter, int mode,
                          double* s_out, int32_t* iters, int64_t* steps_out, const Tuning* tune,
                          unsigned long long* tally = nullptr, int32_t* ties = nullptr, int again = 0);
// FP32 label refinement of the CMC pricers: whether a
// pricing refines (an FP32 form whose FP64 rule tables fit the LDS), and
// the FP64 re-estimates of the points the FP32 finalize listed at date m
// (ids, count *n_ids; same draws, REFINE_PPT paths per lane), written over cont.
bool refine_supported(int prec, int d, int n_dates, int width);
bmc_status refine_labels(bmc_ctx* ctx, const void* devspec, int d, int n_dates, const bmc_rules* rules, int m,
                         const double* x, int64_t N, uint32_t n, uint32_t seed, double* cont, const int32_t* ids,
                         const int32_t* n_ids);
bmc_status final_price_impl(bmc_ctx* ctx, const void* devspec, const bmc_spec* spec,
                            const bmc_rules* rules, int64_t n_final, uint32_t seed, int prec,
                            double* host_sums, const Tuning* tune, bool sync = true);
// With sync = false the sums land in the context's pinned area at the next
// stream sync; read_final_sums then unpacks them.
void read_final_sums(const bmc_ctx* ctx, double* host_sums);

}  // namespace bmc

// Whole CMC / I&Z pricer (pricer.hip); tune forces a launch shape (or NULL).
bmc_status bmc_price_impl(bmc_ctx* ctx, const bmc_spec* spec, const bmc_opts* opts, bmc_rules** rules_out,
                          bmc_result* out, const bmc::Tuning* tune);

namespace bmc {
void fill_price(const double* sums, int64_t n_final, bmc_result* out);

}  // namespace bmc
