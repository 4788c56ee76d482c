// Batched CMC pricing (Algorithm 2) of many options of uneven dimension,
// date count and path counts.  The options advance together in rounds: round
// r handles date N_T - 1 - r of every option that still has one, and an
// option's final pricing joins the round after its last date.  A round is a
// few launches shared by all its options: one bridge step, one persistent
// continuation launch per template bucket and precision (jobs of many options
// at their own dates, one workgroup per job), one finalize and the
// boosting fits, one block per option.  Every option keeps the chunking, tile
// order and merge order of bmc_price, so its price and rules are
// bit-identical to a standalone run.  The whole launch sequence is planned on
// the host first; the task tables go to the device in one copy.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

using namespace bmc;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Workgroups per continuation launch (larger job ranges are split).
constexpr uint32_t MAX_GRID = 1u << 22;

struct OptPlan {
    int d, NT, p, prec, rounds, bucket;
    int64_t N;
    uint32_t n, n_final, seed;
    uint32_t nchunk, per_wg, fnchunk, fper_wg;
    size_t lds;                                   // continuation LDS bytes
    size_t oB, ox, ocont, opart, ofit;            // arena offsets (bytes)
    size_t ow64, ow32;                            // rule tables
};

enum Kind { K_BRIDGE_END, K_BRIDGE_BACK, K_CONT, K_FIN, K_FIT, K_FIT_SINGLE, K_MARK };

struct Step {
    int kind = K_MARK;
    int bucket = 0, prec = 0, ntasks = 0, T = 0, phase = -1;
    uint32_t blocks = 0;             // grid (K_CONT: total jobs)
    size_t tasks = 0, prefix = 0;    // table offsets
    size_t lds = 0;
    int opt = -1, date = 0;          // K_FIT_SINGLE
};

// Host image of the task tables.
struct Table {
    std::vector<char> bytes;
    template <class T>
    size_t put(const std::vector<T>& v)
    {
        const size_t off = align_up(bytes.size());
        bytes.resize(off + sizeof(T) * v.size());
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), sizeof(T) * v.size());
        return off;
    }
};

enum { PH_CALC = 0, PH_FIT = 1, PH_FINAL = 2 };

bmc_status check_opts(const bmc_opts* o, int i)
{
    if (o->method != BMC_CMC)
        return fail(BMC_EUNSUPPORTED, "option %d: batched pricing runs the CMC method only", i);
    if (o->precision < BMC_FP64 || o->precision > BMC_FP32_KAHAN)
        return fail(BMC_EINVAL, "option %d: unknown precision %d", i, o->precision);
    if (o->N < 2 || o->N > 0x7FFFFFFF || o->n < 2 || o->n > 0x7FFFFFFF || o->n_final < 2 ||
        o->n_final > 0x7FFFFFFF)
        return fail(BMC_EINVAL, "option %d: N, n and n_final must be in 2..2^31-1", i);
    if (o->seed > 0xFFFFFFFFull) return fail(BMC_EINVAL, "option %d: seed must fit in 32 bits", i);
    if (o->cls_rounds > 64) return fail(BMC_EINVAL, "option %d: cls_rounds must be <= 64", i);
    return BMC_OK;
}

}  // namespace

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
    size_t arena = 0;
    auto take = [&](size_t bytes) {
        const size_t off = arena;
        arena += align_up(bytes);
        return off;
    };
    size_t rules64_bytes = 0, rules32_bytes = 0;
    for (int i = 0; i < count; ++i) {
        if ((st = validate_spec(&specs[i])) || (st = check_opts(&opts[i], i))) return st;
        OptPlan& q = P[i];
        q.d = specs[i].d;
        q.NT = specs[i].n_dates;
        q.p = rule_width(BMC_CMC, q.d);
        q.prec = opts[i].precision;
        q.rounds = opts[i].cls_rounds > 0 ? opts[i].cls_rounds : 8;
        q.bucket = cont_bucket(q.d);
        q.N = opts[i].N;
        q.n = (uint32_t)opts[i].n;
        q.n_final = (uint32_t)opts[i].n_final;
        q.seed = (uint32_t)opts[i].seed;
        q.per_wg = 256u * choose_ppt(ctx, q.d, q.prec, q.N, q.n, nullptr);
        q.nchunk = (q.n + q.per_wg - 1) / q.per_wg;
        q.fper_wg = 256u * choose_ppt(ctx, q.d, q.prec, 1, q.n_final, nullptr);
        q.fnchunk = (q.n_final + q.fper_wg - 1) / q.fper_wg;
        q.lds = cont_lds_bytes(q.prec, q.d, q.NT, q.p);
        if (q.lds > cont_lds_limit()) return fail(BMC_EUNSUPPORTED, "option %d: rule table too large for LDS", i);
        if ((uint64_t)q.N * q.nchunk > 0x7FFFFFFFull) return fail(BMC_EINVAL, "option %d: too many jobs", i);
        q.ow64 = rules64_bytes;
        rules64_bytes += align_up(sizeof(double) * (size_t)(q.NT + 1) * q.p);
        q.ow32 = rules32_bytes;
        rules32_bytes += align_up(sizeof(float) * (size_t)(q.NT + 1) * q.p);
    }
    // arena: [rules64][rules32][counters: 4 words per option][per-option buffers]
    const size_t o_rules64 = take(rules64_bytes);
    const size_t o_rules32 = take(rules32_bytes);
    int max_rounds = 0;
    for (const OptPlan& q : P) max_rounds = std::max(max_rounds, q.NT);   // N_T - 1 dates + final
    const size_t o_counters = take(sizeof(uint64_t) * 4 * (size_t)count);
    const size_t counters_bytes = arena - o_counters;
    for (OptPlan& q : P) {
        q.oB = take(sizeof(double) * q.d * q.N);
        q.ox = take(sizeof(double) * q.d * q.N);
        q.ocont = take(sizeof(double) * q.N);
        q.opart = take(sizeof(double) * 3 * std::max<size_t>((size_t)q.N * q.nchunk, q.fnchunk));
        q.ofit = take(sizeof(double) * fit_scratch_doubles(q.N, q.p, q.rounds));
    }
    if ((e = ctx->barena.ensure(arena)) || (e = ctx->bspec.ensure(sizeof(DevSpec) * (size_t)count)) ||
        (e = ctx->pack_dev.ensure(sizeof(HostSpecPack) * (size_t)count)))
        return fail(BMC_ENOMEM, "batch buffers (%zu bytes): %s", arena, hipGetErrorString(e));
    char* base = (char*)ctx->barena.ptr;
    DevSpec* dspec = (DevSpec*)ctx->bspec.ptr;
    uint64_t* cnt = (uint64_t*)(base + o_counters);
    auto w64_of = [&](int i) { return (double*)(base + o_rules64 + P[i].ow64); };
    auto w32_of = [&](int i) { return (float*)(base + o_rules32 + P[i].ow32); };

    // ---- the launch sequence and its task tables
    Table tab;
    std::vector<Step> steps;
    {   // draws at maturity for every option with at least one date to learn
        std::vector<BridgeTask> bt;
        std::vector<uint32_t> pre{0};
        for (int i = 0; i < count; ++i) {
            if (P[i].NT < 2) continue;
            bt.push_back({dspec + i, (double*)(base + P[i].oB), nullptr, P[i].N, P[i].seed, P[i].NT});
            pre.push_back(pre.back() + (uint32_t)((P[i].N + 255) / 256));
        }
        if (!bt.empty()) {
            Step s;
            s.kind = K_BRIDGE_END;
            s.ntasks = (int)bt.size();
            s.blocks = pre.back();
            s.tasks = tab.put(bt);
            s.prefix = tab.put(pre);
            steps.push_back(s);
        }
    }
    for (int r = 0; r < max_rounds; ++r) {
        std::vector<int> train, fin;
        for (int i = 0; i < count; ++i) {
            if (r < P[i].NT - 1) train.push_back(i);
            else if (r == P[i].NT - 1) fin.push_back(i);
        }
        if (train.empty() && fin.empty()) continue;
        // bridge back to each training option's date
        if (!train.empty()) {
            std::vector<BridgeTask> bt;
            std::vector<uint32_t> pre{0};
            for (int i : train) {
                const OptPlan& q = P[i];
                bt.push_back({dspec + i, (double*)(base + q.oB), (double*)(base + q.ox), q.N, q.seed,
                              q.NT - 1 - r});
                pre.push_back(pre.back() + (uint32_t)((q.N + 255) / 256));
            }
            Step s;
            s.kind = K_BRIDGE_BACK;
            s.ntasks = (int)bt.size();
            s.blocks = pre.back();
            s.tasks = tab.put(bt);
            s.prefix = tab.put(pre);
            steps.push_back(s);
        }
        // continuation jobs, grouped by (bucket, precision); longest jobs first
        struct Job { int opt; bool final; double cost; };
        std::map<std::pair<int, int>, std::vector<Job>> groups;
        for (int i : train) {
            const OptPlan& q = P[i];
            const int m = q.NT - 1 - r;
            groups[{q.bucket, q.prec}].push_back({i, false, (double)q.per_wg * (q.NT - m) * (q.d + 4)});
        }
        for (int i : fin) {
            const OptPlan& q = P[i];
            groups[{q.bucket, q.prec}].push_back({i, true, (double)q.fper_wg * q.NT * (q.d + 4)});
        }
        Step mark;
        mark.phase = train.empty() ? PH_FINAL : PH_CALC;
        steps.push_back(mark);
        std::vector<FinTask> ft;
        std::vector<uint32_t> fpre{0};
        for (auto& g : groups) {
            std::vector<Job>& jobs = g.second;
            std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) { return a.cost > b.cost; });
            std::vector<ContArgs> ca;
            std::vector<uint32_t> pre{0};
            size_t lds = 0;
            uint64_t total = 0;
            for (const Job& jb : jobs) {
                const int i = jb.opt;
                const OptPlan& q = P[i];
                ContArgs a;
                std::memset(&a, 0, sizeof(a));
                a.spec = dspec + i;
                a.rules = q.prec == BMC_FP64 ? (const void*)w64_of(i) : (const void*)w32_of(i);
                a.ids = nullptr;
                a.n_ids = nullptr;
                a.method = BMC_CMC;
                a.width = q.p;
                a.k0 = q.seed;
                a.part = (double*)(base + q.opart);
                FinTask f;
                std::memset(&f, 0, sizeof(f));
                f.part = a.part;
                if (!jb.final) {
                    const int m = q.NT - 1 - r;
                    a.x = (const double*)(base + q.ox);
                    a.N = q.N;
                    a.n = q.n;
                    a.m = m;
                    a.paths_per_wg = q.per_wg;
                    a.nchunk = q.nchunk;
                    a.k1 = key_hi(BMC_STREAM_INNER, m);
                    f.cont = (double*)(base + q.ocont);
                    f.steps_total = (unsigned long long*)&cnt[4 * i];
                } else {
                    a.x = dev_S0(dspec + i);
                    a.N = 1;
                    a.n = q.n_final;
                    a.m = 0;
                    a.paths_per_wg = q.fper_wg;
                    a.nchunk = q.fnchunk;
                    a.k1 = key_hi(BMC_STREAM_FINAL, 0);
                    f.sums = (double*)&cnt[4 * i + 1];
                    f.steps = (int64_t*)&cnt[4 * i + 3];
                }
                f.N = a.N;
                f.nchunk = a.nchunk;
                f.n = a.n;
                f.wide = finalize_is_wide(a.nchunk, a.N, false) ? 1 : 0;
                total += (uint64_t)a.N * a.nchunk;
                pre.push_back((uint32_t)total);
                ca.push_back(a);
                lds = std::max(lds, q.lds);
                ft.push_back(f);
                fpre.push_back(fpre.back() + (f.wide ? (uint32_t)f.N : (uint32_t)((f.N + 255) / 256)));
            }
            if (total > 0xFFFFFFFFull) return fail(BMC_EINVAL, "too many continuation jobs in one round");
            Step s;
            s.kind = K_CONT;
            s.bucket = g.first.first;
            s.prec = g.first.second;
            s.ntasks = (int)ca.size();
            s.blocks = (uint32_t)total;
            s.tasks = tab.put(ca);
            s.prefix = tab.put(pre);
            s.lds = lds;
            steps.push_back(s);
        }
        {
            Step s;
            s.kind = K_FIN;
            s.ntasks = (int)ft.size();
            s.blocks = fpre.back();
            s.tasks = tab.put(ft);
            s.prefix = tab.put(fpre);
            steps.push_back(s);
        }
        if (train.empty()) continue;
        Step fmark;
        fmark.phase = PH_FIT;
        steps.push_back(fmark);
        // boosting fits: one block per option, grouped by tile size
        std::map<int, std::vector<int>> by_tile;
        for (int i : train) {
            if (fit_coop_supported(P[i].p)) {
                by_tile[fit_tile(P[i].p)].push_back(i);
            } else {
                Step s;
                s.kind = K_FIT_SINGLE;
                s.opt = i;
                s.date = P[i].NT - 1 - r;
                steps.push_back(s);
            }
        }
        for (auto& g : by_tile) {
            std::vector<FitTask> fts;
            size_t lds = 0;
            for (int i : g.second) {
                const OptPlan& q = P[i];
                const int m = q.NT - 1 - r;
                FitScratch fs;
                fit_scratch_carve((double*)(base + q.ofit), q.N, q.p, q.rounds, &fs);
                fts.push_back(fit_task_make(dspec + i, q.d, (const double*)(base + q.ox),
                                            (const double*)(base + q.ocont), q.N, q.rounds, fs,
                                            w64_of(i) + (size_t)m * q.p, w32_of(i) + (size_t)m * q.p));
                lds = std::max(lds, fit_task_lds(q.p));
            }
            Step s;
            s.kind = K_FIT;
            s.T = g.first;
            s.ntasks = (int)fts.size();
            s.tasks = tab.put(fts);
            s.lds = lds;
            steps.push_back(s);
        }
    }
    Step endmark;
    endmark.phase = -1;
    steps.push_back(endmark);

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
        (e = hipMemsetAsync(base + o_rules64, 0, o_counters + counters_bytes - o_rules64, sm)) ||
        (e = hipStreamSynchronize(sm)))
        return hip_fail(e, "batch setup");
    for (int i = 0; i < count; ++i)
        if (((const int32_t*)(hb + status_off))[i] != 0)
            return fail(BMC_ENOTSPD, "option %d: correlation matrix is not positive definite", i);

    // ---- run
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
    for (const Step& s : steps) {
        const void* tasks = dtab + s.tasks;
        const uint32_t* pre = (const uint32_t*)(dtab + s.prefix);
        switch (s.kind) {
        case K_MARK: mark(s.phase); break;
        case K_BRIDGE_END:
        case K_BRIDGE_BACK:
            e = launch_bridge_multi((const BridgeTask*)tasks, pre, s.ntasks, s.blocks, s.kind == K_BRIDGE_END, sm);
            break;
        case K_CONT:
            for (uint32_t j0 = 0; j0 < s.blocks && !e; j0 += MAX_GRID)
                e = launch_cont_multi(s.bucket, s.prec, (const ContArgs*)tasks, pre, s.ntasks, j0,
                                      std::min(MAX_GRID, s.blocks - j0), 256, s.lds, sm);
            break;
        case K_FIN: e = launch_finalize_multi((const FinTask*)tasks, pre, s.ntasks, s.blocks, sm); break;
        case K_FIT: e = launch_fit_cmc_multi((const FitTask*)tasks, s.ntasks, s.T, s.lds, sm); break;
        case K_FIT_SINGLE: {
            const OptPlan& q = P[s.opt];
            FitScratch fs;
            fit_scratch_carve((double*)(base + q.ofit), q.N, q.p, q.rounds, &fs);
            e = launch_fit_cmc(dspec + s.opt, q.d, (const double*)(base + q.ox), (const double*)(base + q.ocont), q.N,
                               q.rounds, fs, w64_of(s.opt) + (size_t)s.date * q.p, w32_of(s.opt) + (size_t)s.date * q.p,
                               sm);
            break;
        }
        }
        if (s.kind != K_MARK && e) {
            st = hip_fail(e, "batch launch");
            break;
        }
    }
    if (!st) {
        if ((e = hipMemcpyAsync(hb + readback_off, cnt, sizeof(uint64_t) * 4 * (size_t)count, hipMemcpyDeviceToHost,
                                sm)) ||
            (e = hipStreamSynchronize(sm)))
            st = hip_fail(e, "batch results");
    }
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
            if ((e = hipMemcpyAsync(rl->w64, w64_of(i), sizeof(double) * rows, hipMemcpyDeviceToDevice, sm)) ||
                (e = hipMemcpyAsync(rl->w32, w32_of(i), sizeof(float) * rows, hipMemcpyDeviceToDevice, sm)))
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
