// Whole-pricer driver (Algorithm 1 for I&Z, Algorithm 2 for CMC): backward
// sweep over the exercise dates on the device, then the final pricing pass.
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

using namespace bmc;

namespace {

// Phase timers on the context stream, summed after the closing sync; the
// events come from the context's pool and go back to it.
struct PhaseTimer {
    bmc_ctx* ctx;
    std::vector<hipEvent_t> evs;
    std::vector<int> phase;
    explicit PhaseTimer(bmc_ctx* c) : ctx(c) {}
    ~PhaseTimer()
    {
        for (hipEvent_t e : evs) ctx->ev_pool.push_back(e);
    }
    void mark(int ph)
    {
        hipEvent_t e;
        if (!ctx->ev_pool.empty()) {
            e = ctx->ev_pool.back();
            ctx->ev_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return;
        }
        (void)hipEventRecord(e, ctx->stream);
        evs.push_back(e);
        phase.push_back(ph);
    }
    // Time from each mark to the next, credited to the earlier mark's phase.
    void totals(double* sec) const
    {
        for (size_t i = 0; i + 1 < evs.size(); ++i) {
            float ms = 0.f;
            if (phase[i] >= 0 && hipEventElapsedTime(&ms, evs[i], evs[i + 1]) == hipSuccess)
                sec[phase[i]] += ms * 1e-3;
        }
    }
};

enum { PH_CALC = 0, PH_FIT = 1, PH_FINAL = 2, PH_REFINE = 3 };

}  // namespace

bmc_status bmc_price_impl(bmc_ctx* ctx, const bmc_spec* spec, const bmc_opts* opts, bmc_rules** rules_out,
                          bmc_result* out, const Tuning* tune)
{
    auto t_start = std::chrono::steady_clock::now();
    if (!ctx || !opts || !out) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    const int method = opts->method, prec = opts->precision;
    if (method != BMC_CMC && method != BMC_IZ && method != BMC_CMC_ADA)
        return fail(BMC_EINVAL, "unknown method %d", method);
    if (prec < BMC_FP64 || prec > BMC_FP32_KAHAN) return fail(BMC_EINVAL, "unknown precision %d", prec);
    if (opts->N < 2 || opts->N > 0x7FFFFFFF || opts->n < 2 || opts->n > 0x7FFFFFFF || opts->n_final < 2 ||
        opts->n_final > 0x7FFFFFFF)
        return fail(BMC_EINVAL, "N, n and n_final must be in 2..2^31-1");
    if (opts->seed > 0xFFFFFFFFull) return fail(BMC_EINVAL, "seed must fit in 32 bits");
    const int rounds = opts->cls_rounds > 0 ? opts->cls_rounds : (method == BMC_CMC_ADA ? ADA_TMAX : 8);
    const int max_iter = opts->iz_max_iter > 0 ? opts->iz_max_iter : 100;
    const double eps = opts->iz_eps > 0.0 ? opts->iz_eps : 0.01;
    const int search = opts->iz_search;
    if (search != BMC_SEARCH_PLAIN && search != BMC_SEARCH_SECANT)
        return fail(BMC_EINVAL, "unknown I&Z search mode %d", search);
    if (rounds > 64) return fail(BMC_EINVAL, "cls_rounds must be <= 64");
    if (method == BMC_IZ && opts->N > 65536) return fail(BMC_EUNSUPPORTED, "I&Z supports N <= 65536 lattice points");
    // spec setup status and the step total come back with the final sums (one sync)
    int32_t* status_host = (int32_t*)((char*)ctx->host_io + 72);
    bmc_status st = upload_spec_async(ctx, spec, ctx->spec, status_host);
    if (st) return st;
    bmc_rules scratch;
    bmc_rules* rules = nullptr;
    if (rules_out) {
        if ((st = bmc_rules_create(ctx, spec, method, &rules))) return st;
    } else {
        if ((st = scratch_rules(ctx, spec, method, &scratch))) return st;
        rules = &scratch;
    }
    auto release = [&]() {
        if (rules != &scratch) bmc_rules_destroy(rules);
    };

    const int d = spec->d, NT = spec->n_dates;
    const int64_t N = opts->N;
    const uint32_t n = (uint32_t)opts->n, seed = (uint32_t)opts->seed;
    const void* ds = ctx->spec.ptr;
    hipError_t e;
    PhaseTimer timer(ctx);
    int64_t unconv = 0, iz_iters = 0, iz_steps = 0;
    // I&Z: the points of every region side by side
    const int64_t NR = method == BMC_IZ ? N * iz_regions(spec->payoff, d) : N;
    if ((e = ctx->counters.ensure(64)) || (e = ctx->x.ensure(sizeof(double) * d * NR)) ||
        (e = ctx->cont.ensure(sizeof(double) * NR)) || (e = ctx->B.ensure(sizeof(double) * d * N)) ||
        (e = ctx->steps.ensure(sizeof(int64_t) * N + sizeof(int32_t) * NR))) {
        release();
        return fail(BMC_ENOMEM, "device buffers: %s", hipGetErrorString(e));
    }
    unsigned long long* steps_total = (unsigned long long*)ctx->counters.ptr;
    double* x = (double*)ctx->x.ptr;
    double* cont = (double*)ctx->cont.ptr;
    double* B = (double*)ctx->B.ptr;
    // the CMC forms clear the step total (and the job-order counts) in their
    // first bridge launch
    if (method == BMC_IZ && (e = hipMemsetAsync(steps_total, 0, sizeof(unsigned long long), ctx->stream))) {
        release();
        return hip_fail(e, "counter reset");
    }

    if (method != BMC_IZ) {
        // FP32 forms: the finalize of each date's estimates lists the
        // near-tie training points, re-estimated in FP64 before the fit
        const bool refine = refine_supported(prec, d, NT, rules->width);
        RefineSel sel{};
        if (refine) {
            if ((e = ctx->rf.ensure(256 + sizeof(int32_t) * (size_t)N))) {
                release();
                return fail(BMC_ENOMEM, "device buffers: %s", hipGetErrorString(e));
            }
            sel = RefineSel{(const DevSpec*)ds, x, (int32_t*)((char*)ctx->rf.ptr + 256), (int32_t*)ctx->rf.ptr};
        }
        // each date's jobs start in order of increasing intrinsic value: the
        // bridge step of date m fills count set m % 2 and the lists, and
        // clears the other set for the next date
        int32_t *ord_cnt = nullptr, *ord_list = nullptr;
        if (N <= ORDER_MAX_N) {
            if ((e = ctx->order.ensure(256 + sizeof(int32_t) * ORDER_BUCKETS * (size_t)N))) {
                release();
                return fail(BMC_ENOMEM, "device buffers: %s", hipGetErrorString(e));
            }
            ord_cnt = (int32_t*)ctx->order.ptr;
            ord_list = (int32_t*)((char*)ctx->order.ptr + 256);
        }
        if ((e = launch_bridge_end((const DevSpec*)ds, d, N, seed, B, ctx->stream, steps_total, ord_cnt,
                                   ord_cnt ? 64 : 0)))   // both count sets (256 B)
            st = hip_fail(e, "bridge");
        for (int m = NT - 1; m >= 1 && !st; --m) {
            int32_t* cnt_m = ord_cnt ? ord_cnt + ORDER_BUCKETS * (m & 1) : nullptr;
            int32_t* cnt_clear = ord_cnt ? ord_cnt + ORDER_BUCKETS * ((m & 1) ^ 1) : nullptr;
            if ((e = launch_bridge_back((const DevSpec*)ds, d, m, N, seed, B, x, 1, ctx->stream, sel.n_ids, cnt_m,
                                        ord_list, cnt_clear))) {
                st = hip_fail(e, "bridge");
                break;
            }
            timer.mark(PH_CALC);
            const JobOrder ord{cnt_m, ord_list};
            st = run_cont(ctx, ds, d, NT, method, rules->width, rules->w64, rules->w32, prec, m, x, N, nullptr,
                          nullptr, n, seed, key_hi(BMC_STREAM_INNER, m), cont, nullptr, nullptr, nullptr,
                          steps_total, tune, 0, 0, nullptr, nullptr, nullptr, refine ? &sel : nullptr,
                          cnt_m ? &ord : nullptr);
            if (!st && refine) {
                timer.mark(PH_REFINE);
                st = refine_labels(ctx, ds, d, NT, rules, m, x, N, n, seed, cont, sel.ids, sel.n_ids);
            }
            if (st) break;
            timer.mark(PH_FIT);
            st = fit_rule_impl(ctx, ds, d, rules, m, x, cont, N, rounds);
            timer.mark(-1);
        }
    } else {
        double* s_out = cont;
        int32_t* iters = (int32_t*)((char*)ctx->steps.ptr + sizeof(int64_t) * N);
        const int regions = iz_regions(spec->payoff, d);
        // search totals (path-steps, points without a boundary point,
        // iterations) summed on the device date by date, read with the price
        unsigned long long* tally = (unsigned long long*)((char*)ctx->counters.ptr + 64);
        if ((e = hipMemsetAsync(tally, 0, 3 * sizeof(unsigned long long), ctx->stream)))
            st = hip_fail(e, "counter reset");
        // Algorithm 1: per date, the boundary points of every region, then one
        // regression per region.  The regions' searches are independent (each
        // uses the rules of later dates only), so they run side by side in the
        // same launches: region r in columns r N .. r N + N - 1.
        // FP32 forms: points whose search met a near tie are searched again in FP64
        int32_t* ties = nullptr;
        if (prec != BMC_FP64) {
            if ((e = ctx->rf.ensure(sizeof(int32_t) * (size_t)NR))) st = hip_fail(e, "search flags");
            ties = (int32_t*)ctx->rf.ptr;
        }
        for (int m = NT - 1; m >= 1 && !st; --m) {
            if ((st = sample_points_impl(ctx, ds, spec, BMC_IZ, m, N, seed, x, B, 0, regions))) break;
            timer.mark(PH_CALC);
            st = iz_search_impl(ctx, ds, spec, rules, m, 0, regions, x, N, n, seed, prec, eps, max_iter, search,
                                s_out, iters, nullptr, tune, ties ? nullptr : tally, ties);
            if (!st && ties) timer.mark(PH_REFINE);
            if (!st && ties)
                st = iz_search_impl(ctx, ds, spec, rules, m, 0, regions, x, N, n, seed, BMC_FP64, eps, max_iter,
                                    search, s_out, iters, nullptr, tune, tally, ties, 1);
            if (st) break;
            timer.mark(PH_FIT);
            // every region's regression in one launch pair, s* read from the
            // search output (region r's points in columns r N ..)
            {
                const int p = rule_width(BMC_IZ, d);
                if ((e = ctx->fit.ensure(sizeof(double) * fitiz_scratch_doubles(N, p) * regions)))
                    st = hip_fail(e, "fit scratch");
                else if ((e = launch_fit_iz((const DevSpec*)ds, d, 0, x, N, NR, (double*)ctx->fit.ptr,
                                            rules->w64 + (size_t)m * rules->width,
                                            rules->w32 + (size_t)m * rules->width, ctx->stream, regions, s_out)))
                    st = hip_fail(e, "fit launch");
            }
            if (st) break;
            timer.mark(-1);
        }
        if (!st && (e = hipMemcpyAsync((char*)ctx->host_io + 80, tally, 3 * sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, ctx->stream)))
            st = hip_fail(e, "search results");
    }
    double sums[3] = {0, 0, 0};
    unsigned long long* inner_host = (unsigned long long*)((char*)ctx->host_io + 64);
    if (!st && (e = hipMemcpyAsync(inner_host, steps_total, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                   ctx->stream)))
        st = hip_fail(e, "result read");
    if (!st) {
        timer.mark(PH_FINAL);
        st = final_price_impl(ctx, ds, spec, rules, opts->n_final, seed, prec, sums, tune, false);
        timer.mark(-1);   // before the sync, so that every timing event has completed after it
        if (!st && (e = hipStreamSynchronize(ctx->stream))) st = hip_fail(e, "result read");
        if (!st) read_final_sums(ctx, sums);
        if (!st && method == BMC_IZ) {
            unsigned long long t[3];
            std::memcpy(t, (const char*)ctx->host_io + 80, sizeof(t));
            iz_steps = (int64_t)t[0];
            unconv = (int64_t)t[1];
            iz_iters = (int64_t)t[2];
        }
    }
    if (!st && *status_host != 0) st = fail(BMC_ENOTSPD, "correlation matrix is not positive definite");
    if (method != BMC_IZ) {
        const bmc_status fb = check_fit_barrier(ctx);
        if (!st) st = fb;
    }
    const unsigned long long inner = st ? 0 : *inner_host;
    if (st) {
        release();
        return st;
    }
    bmc_result r;
    std::memset(&r, 0, sizeof(r));
    fill_price(sums, opts->n_final, &r);
    r.inner_path_steps = method != BMC_IZ ? (int64_t)inner : iz_steps;
    r.iz_unconverged = unconv;
    r.iz_iterations = iz_iters;
    double sec[4] = {0, 0, 0, 0};
    timer.totals(sec);
    r.calc_seconds = sec[PH_CALC];
    r.fit_seconds = sec[PH_FIT];
    r.final_seconds = sec[PH_FINAL];
    r.refine_seconds = sec[PH_REFINE];
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    *out = r;
    if (rules_out) *rules_out = rules;
    else release();
    return BMC_OK;
}

extern "C" bmc_status bmc_price(bmc_ctx* ctx, const bmc_spec* spec, const bmc_opts* opts, bmc_rules** rules_out,
                                bmc_result* out)
{
    return bmc_price_impl(ctx, spec, opts, rules_out, out, nullptr);
}
