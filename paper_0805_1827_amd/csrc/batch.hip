// Batched CMC pricing (Algorithm 2) of many options of uneven dimension,
// date count and path counts, through the round engine: round r handles
// date N_T - 1 - r of every option that still has one, and an option's
// final pricing joins the round after its last date.  The whole launch
// sequence is planned on the host first; the task tables go to the device
// in one copy.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"

using namespace bmc;

static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Launch signature of a planned sweep: every launch's shape and table
// offsets and the buffers they address.  Spec values, seeds and task-table
// contents are device data, so a sweep with the same signature replays.
static std::string sweep_signature(const std::vector<Step>& steps, const char* dtab, const char* base,
                                   const DevSpec* dspec, size_t tab_bytes)
{
    std::string s;
    auto add = [&](const void* p, size_t n) { s.append((const char*)p, n); };
    add(&dtab, sizeof(dtab));
    add(&base, sizeof(base));
    add(&dspec, sizeof(dspec));
    add(&tab_bytes, sizeof(tab_bytes));
    for (const Step& st : steps) {
        if (st.kind == K_MARK) continue;
        const int64_t v[] = {st.kind, st.bucket, st.prec, st.ntasks, st.T, st.blocks, (int64_t)st.tasks,
                             (int64_t)st.prefix, (int64_t)st.lds, st.date, st.stride};
        add(v, sizeof(v));
        if (st.kind == K_FIT_SINGLE) {
            add(&st.single_dev, sizeof(st.single_dev));
            const int64_t q[] = {st.single_q.d, st.single_q.N, st.single_q.rounds};
            add(q, sizeof(q));
        }
    }
    return s;
}

// Runs the sweep as a HIP graph on the context's graph stream, ordered
// after and before the work on st: captured when the signature is new,
// replayed otherwise.  *ran = false (and no error) when the runtime cannot
// capture the sweep: the caller then launches it directly.  evs receives a
// start and an end event (one calc phase).
static bmc_status run_graph(bmc_ctx* ctx, const std::vector<Step>& steps, const char* dtab, const char* base,
                            const DevSpec* dspec, size_t tab_bytes, hipStream_t st, std::vector<hipEvent_t>& evs,
                            std::vector<int>& ev_phase, bool* ran)
{
    hipError_t e;
    *ran = false;
    if (!ctx->graph_stream && (e = hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking)))
        return hip_fail(e, "graph stream");
    hipStream_t gs = ctx->graph_stream;
    const std::string sig = sweep_signature(steps, dtab, base, dspec, tab_bytes);
    if (!ctx->graph_exec || sig != ctx->graph_sig) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
        ctx->graph_sig.clear();
        if ((e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal))) {
            (void)hipGetLastError();
            return BMC_OK;
        }
        const hipError_t el = run_steps(steps, dtab, gs, [](int) {});
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(gs, &g);
        hipGraphExec_t x = nullptr;
        const hipError_t ei = (el || ec || !g) ? hipErrorUnknown : hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (el || ec || ei || !x) {
            (void)hipGetLastError();
            return BMC_OK;
        }
        ctx->graph_exec = x;
        ctx->graph_sig = sig;
        ++ctx->graph_captures;
    } else {
        ++ctx->graph_replays;
    }
    hipEvent_t before, t0, t1;
    if ((e = hipEventCreate(&before)) || (e = hipEventCreate(&t0)) || (e = hipEventCreate(&t1)))
        return hip_fail(e, "graph events");
    evs.push_back(t0);
    ev_phase.push_back(PH_CALC);
    evs.push_back(t1);
    ev_phase.push_back(-1);
    if ((e = hipEventRecord(before, st)) || (e = hipStreamWaitEvent(gs, before, 0)) || (e = hipEventRecord(t0, gs)) ||
        (e = hipGraphLaunch(ctx->graph_exec, gs)) || (e = hipEventRecord(t1, gs)) ||
        (e = hipStreamWaitEvent(st, t1, 0))) {
        (void)hipEventDestroy(before);
        return hip_fail(e, "graph launch");
    }
    (void)hipEventDestroy(before);
    *ran = true;
    return BMC_OK;
}

extern "C" bmc_status bmc_price_batch(bmc_ctx* ctx, int32_t count, const bmc_spec* specs, const bmc_opts* opts,
                                      bmc_rules** rules_out, bmc_result* results)
{
    auto t_start = std::chrono::steady_clock::now();
    if (!ctx || !specs || !opts || !results) return fail(BMC_EINVAL, "NULL argument");
    if (count < 1 || count > 65536) return fail(BMC_EINVAL, "count = %d outside 1..65536", count);
    (void)hipSetDevice(ctx->device);
    bmc_status st;
    hipError_t e;

    // ---- plan every option as bmc_price would run it
    std::vector<OptPlan> P(count);
    // arena: all counters first (one read-back copy), then the option regions
    size_t arena = (sizeof(uint64_t) * 4 * (size_t)count + 255) & ~(size_t)255;
    std::vector<size_t> base_off(count);
    int max_rounds = 0;
    for (int i = 0; i < count; ++i) {
        if ((st = plan_option(ctx, &specs[i], &opts[i], i, &P[i]))) return st;
        base_off[i] = arena;
        arena += P[i].bytes;
        max_rounds = std::max(max_rounds, P[i].NT);   // N_T - 1 dates + final
    }
    if ((e = ctx->barena.ensure(std::max<size_t>(arena, 256))) ||
        (e = ctx->bspec.ensure(sizeof(DevSpec) * (size_t)count)) ||
        (e = ctx->pack_dev.ensure(sizeof(HostSpecPack) * (size_t)count)))
        return fail(BMC_ENOMEM, "batch buffers (%zu bytes): %s", arena, hipGetErrorString(e));
    char* base = (char*)ctx->barena.ptr;
    DevSpec* dspec = (DevSpec*)ctx->bspec.ptr;
    std::vector<OptDev> V(count);
    uint64_t* cnt = (uint64_t*)base;
    for (int i = 0; i < count; ++i) {
        V[i] = carve_option(P[i], dspec + i, base + base_off[i]);
        V[i].cnt = cnt + 4 * (size_t)i;
    }

    // ---- the launch sequence and its task tables
    Table tab;
    std::vector<Step> steps;
    for (int r = 0; r < max_rounds; ++r) {
        std::vector<RoundItem> items;
        for (int i = 0; i < count; ++i) {
            if (r < P[i].NT - 1) items.push_back({&P[i], &V[i], P[i].NT - 1 - r});
            else if (r == P[i].NT - 1) items.push_back({&P[i], &V[i], 0});
        }
        if ((st = plan_round(items, tab, steps))) return st;
    }

    // ---- pinned staging: spec packs, task tables, read-back area
    const size_t packs_bytes = align_up(sizeof(HostSpecPack) * (size_t)count);
    const size_t tab_bytes = align_up(tab.bytes.size());
    const size_t status_off = packs_bytes + tab_bytes;
    const size_t readback_off = status_off + align_up(sizeof(int32_t) * (size_t)count);
    const size_t host_bytes = readback_off + sizeof(uint64_t) * 4 * (size_t)count;
    if ((e = hipStreamSynchronize(ctx->stream))) return hip_fail(e, "stream sync");
    if (ctx->bhost_bytes < host_bytes) {
        if (ctx->bhost) (void)hipHostFree(ctx->bhost);
        ctx->bhost = nullptr;
        ctx->bhost_bytes = 0;
        if ((e = hipHostMalloc(&ctx->bhost, host_bytes, 0)))
            return fail(BMC_ENOMEM, "pinned staging (%zu bytes): %s", host_bytes, hipGetErrorString(e));
        ctx->bhost_bytes = host_bytes;
    }
    if ((e = ctx->btab.ensure(std::max<size_t>(tab_bytes, 256))))
        return fail(BMC_ENOMEM, "task tables: %s", hipGetErrorString(e));
    char* hb = (char*)ctx->bhost;
    HostSpecPack* packs = (HostSpecPack*)hb;
    for (int i = 0; i < count; ++i) pack_spec(&specs[i], &packs[i]);
    std::memcpy(hb + packs_bytes, tab.bytes.data(), tab.bytes.size());
    char* dtab = (char*)ctx->btab.ptr;
    hipStream_t sm = ctx->stream;
    if ((e = hipMemcpyAsync(ctx->pack_dev.ptr, packs, sizeof(HostSpecPack) * (size_t)count, hipMemcpyHostToDevice,
                            sm)) ||
        (e = launch_setup((const HostSpecPack*)ctx->pack_dev.ptr, dspec, count, sm)) ||
        (e = hipMemcpy2DAsync(hb + status_off, sizeof(int32_t), (const char*)dspec + offsetof(DevSpec, status),
                              sizeof(DevSpec), sizeof(int32_t), (size_t)count, hipMemcpyDeviceToHost, sm)) ||
        (e = hipMemcpyAsync(dtab, hb + packs_bytes, tab.bytes.size(), hipMemcpyHostToDevice, sm)) ||
        (e = hipMemsetAsync(base, 0, arena, sm)) ||
        (e = hipStreamSynchronize(sm)))
        return hip_fail(e, "batch setup");
    for (int i = 0; i < count; ++i)
        if (((const int32_t*)(hb + status_off))[i] != 0)
            return fail(BMC_ENOTSPD, "option %d: correlation matrix is not positive definite", i);

    // ---- run: direct launches with phase marks, or the captured graph
    std::vector<hipEvent_t> evs;
    std::vector<int> ev_phase;
    auto mark = [&](int phase) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return;
        (void)hipEventRecord(ev, sm);
        evs.push_back(ev);
        ev_phase.push_back(phase);
    };
    st = BMC_OK;
    bool ran = false;
    if (ctx->graphs) {
        if ((st = run_graph(ctx, steps, dtab, base, dspec, tab.bytes.size(), sm, evs, ev_phase, &ran))) return st;
    }
    if (!ran && (e = run_steps(steps, dtab, sm, mark))) st = hip_fail(e, "batch launch");
    // per-option counters [steps, sum, sum of squares, final steps]
    if (!st && (e = hipMemcpyAsync(hb + readback_off, cnt, 32 * (size_t)count, hipMemcpyDeviceToHost, sm)))
        st = hip_fail(e, "batch results");
    if (!st && (e = hipStreamSynchronize(sm))) st = hip_fail(e, "batch results");
    double sec[3] = {0, 0, 0};
    for (size_t k = 0; k + 1 < evs.size(); ++k) {
        float ms = 0.f;
        if (!st && ev_phase[k] >= 0 && hipEventElapsedTime(&ms, evs[k], evs[k + 1]) == hipSuccess)
            sec[ev_phase[k]] += ms * 1e-3;
    }
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    if (st) return st;

    // ---- optional rule tables, then the results
    std::vector<bmc_rules*> made;
    if (rules_out) {
        for (int i = 0; i < count && !st; ++i) {
            bmc_rules* rl = nullptr;
            if ((st = bmc_rules_create(ctx, &specs[i], BMC_CMC, &rl))) break;
            made.push_back(rl);
            const size_t rows = (size_t)(P[i].NT + 1) * P[i].p;
            if ((e = hipMemcpyAsync(rl->w64, V[i].w64, sizeof(double) * rows, hipMemcpyDeviceToDevice, sm)) ||
                (e = hipMemcpyAsync(rl->w32, V[i].w32, sizeof(float) * rows, hipMemcpyDeviceToDevice, sm)))
                st = hip_fail(e, "rule copy");
        }
        if (!st && (e = hipStreamSynchronize(sm))) st = hip_fail(e, "rule copy");
        if (st) {
            for (bmc_rules* rl : made) bmc_rules_destroy(rl);
            return st;
        }
    }
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    const uint64_t* rb = (const uint64_t*)(hb + readback_off);
    for (int i = 0; i < count; ++i) {
        double sums[3];
        std::memcpy(&sums[0], &rb[4 * i + 1], sizeof(double));
        std::memcpy(&sums[1], &rb[4 * i + 2], sizeof(double));
        int64_t fsteps;
        std::memcpy(&fsteps, &rb[4 * i + 3], sizeof(int64_t));
        sums[2] = (double)fsteps;
        bmc_result res;
        std::memset(&res, 0, sizeof(res));
        fill_price(sums, P[i].n_final, &res);
        res.inner_path_steps = (int64_t)rb[4 * i];
        res.seconds = wall;
        res.calc_seconds = sec[PH_CALC];
        res.fit_seconds = sec[PH_FIT];
        res.final_seconds = sec[PH_FINAL];
        results[i] = res;
        if (rules_out) rules_out[i] = made[i];
    }
    return BMC_OK;
}
