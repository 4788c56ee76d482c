// Round engine: per-pricing plans and one round's shared launches.
#include <algorithm>
#include <map>

#include "engine.hpp"

namespace bmc {

namespace {

// Workgroups per continuation launch (larger job ranges are split).
constexpr uint32_t MAX_GRID = 1u << 22;

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

bmc_status plan_option(const bmc_ctx* ctx, const bmc_spec* spec, const bmc_opts* o, int i, OptPlan* q)
{
    bmc_status st = validate_spec(spec);
    if (st) return st;
    if (o->method != BMC_CMC)
        return fail(BMC_EUNSUPPORTED, "option %d: batched and served pricing run the CMC method only", i);
    if (o->precision < BMC_FP64 || o->precision > BMC_FP32_KAHAN)
        return fail(BMC_EINVAL, "option %d: unknown precision %d", i, o->precision);
    if (o->N < 2 || o->N > 0x7FFFFFFF || o->n < 2 || o->n > 0x7FFFFFFF || o->n_final < 2 ||
        o->n_final > 0x7FFFFFFF)
        return fail(BMC_EINVAL, "option %d: N, n and n_final must be in 2..2^31-1", i);
    if (o->seed > 0xFFFFFFFFull) return fail(BMC_EINVAL, "option %d: seed must fit in 32 bits", i);
    if (o->cls_rounds > 64) return fail(BMC_EINVAL, "option %d: cls_rounds must be <= 64", i);
    q->d = spec->d;
    q->NT = spec->n_dates;
    q->p = rule_width(BMC_CMC, q->d);
    q->prec = o->precision;
    q->rounds = o->cls_rounds > 0 ? o->cls_rounds : 8;
    q->bucket = cont_bucket(q->d);
    q->N = o->N;
    q->n = (uint32_t)o->n;
    q->n_final = (uint32_t)o->n_final;
    q->seed = (uint32_t)o->seed;
    q->per_wg = 256u * choose_ppt(ctx, q->d, q->prec, q->N, q->n, nullptr);
    q->nchunk = (q->n + q->per_wg - 1) / q->per_wg;
    q->fper_wg = 256u * choose_ppt(ctx, q->d, q->prec, 1, q->n_final, nullptr);
    q->fnchunk = (q->n_final + q->fper_wg - 1) / q->fper_wg;
    q->lds = cont_lds_bytes(q->prec, q->d, q->NT, q->p);
    if (q->lds > cont_lds_limit()) return fail(BMC_EUNSUPPORTED, "option %d: rule table too large for LDS", i);
    q->lds64 = cont_lds_bytes(BMC_FP64, q->d, q->NT, q->p);
    q->refine = refine_supported(q->prec, q->d, q->NT, q->p);
    q->rper_wg = 256u * REFINE_PPT;
    q->rnchunk = (q->n + q->rper_wg - 1) / q->rper_wg;
    if ((uint64_t)q->N * q->nchunk > 0x7FFFFFFFull) return fail(BMC_EINVAL, "option %d: too many jobs", i);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off += align256(b);
        return at;
    };
    const size_t rows = (size_t)(q->NT + 1) * q->p;
    q->ow64 = take(sizeof(double) * rows);
    q->ow32 = take(sizeof(float) * rows);
    q->ocnt = take(sizeof(uint64_t) * 4);   // a 256-byte block: results in the first 32 bytes, a served
                                            // request's cancel word at byte 64
    q->zero_bytes = off;
    q->oB = take(sizeof(double) * q->d * q->N);
    q->ox = take(sizeof(double) * q->d * q->N);
    q->ocont = take(sizeof(double) * q->N);
    size_t parts = std::max<size_t>((size_t)q->N * q->nchunk, q->fnchunk);
    if (q->refine) parts = std::max<size_t>(parts, (size_t)q->N * q->rnchunk);
    q->opart = take(sizeof(double) * 3 * parts);
    q->ofit = take(sizeof(double) * fit_scratch_doubles(q->N, q->p, q->rounds));
    q->oids = q->refine ? take(256 + sizeof(int32_t) * q->N) : 0;
    q->bytes = off;
    return BMC_OK;
}

OptDev carve_option(const OptPlan& q, const DevSpec* spec, char* base)
{
    OptDev v;
    v.spec = spec;
    v.w64 = (double*)(base + q.ow64);
    v.w32 = (float*)(base + q.ow32);
    v.cnt = (uint64_t*)(base + q.ocnt);
    v.B = (double*)(base + q.oB);
    v.x = (double*)(base + q.ox);
    v.cont = (double*)(base + q.ocont);
    v.part = (double*)(base + q.opart);
    v.fit = (double*)(base + q.ofit);
    v.n_ids = q.refine ? (int32_t*)(base + q.oids) : nullptr;
    v.ids = q.refine ? (int32_t*)(base + q.oids + 256) : nullptr;
    v.cancel = nullptr;
    return v;
}

bmc_status plan_round(const std::vector<RoundItem>& items, Table& tab, std::vector<Step>& steps)
{
    std::vector<const RoundItem*> train, fin;
    for (const RoundItem& it : items) (it.stage >= 1 ? train : fin).push_back(&it);
    if (train.empty() && fin.empty()) return BMC_OK;
    // Brownian end points of pricings starting to learn, then the bridge back
    auto bridge = [&](bool end) {
        std::vector<BridgeTask> bt;
        std::vector<uint32_t> pre{0};
        for (const RoundItem* it : train) {
            const OptPlan& q = *it->q;
            if (end && it->stage != q.NT - 1) continue;
            bt.push_back({it->dev->spec, it->dev->B, end ? nullptr : it->dev->x, end ? nullptr : it->dev->n_ids, q.N,
                          q.seed, it->stage});
            pre.push_back(pre.back() + (uint32_t)((q.N + 255) / 256));
        }
        if (bt.empty()) return;
        Step s;
        s.kind = end ? K_BRIDGE_END : K_BRIDGE_BACK;
        s.ntasks = (int)bt.size();
        s.blocks = pre.back();
        s.tasks = tab.put(bt);
        s.prefix = tab.put(pre);
        steps.push_back(s);
    };
    bridge(true);
    bridge(false);

    // continuation jobs grouped by (bucket, precision), longest jobs first
    struct Job { const RoundItem* it; double cost; };
    std::map<std::pair<int, int>, std::vector<Job>> groups;
    for (const RoundItem* it : train) {
        const OptPlan& q = *it->q;
        groups[{q.bucket, q.prec}].push_back({it, (double)q.per_wg * (q.NT - it->stage) * (q.d + 4)});
    }
    for (const RoundItem* it : fin) {
        const OptPlan& q = *it->q;
        groups[{q.bucket, q.prec}].push_back({it, (double)q.fper_wg * q.NT * (q.d + 4)});
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
            const OptPlan& q = *jb.it->q;
            const OptDev& v = *jb.it->dev;
            const int m = jb.it->stage;
            ContArgs a{};
            std::memset(&a, 0, sizeof(a));
            a.spec = v.spec;
            a.rules = q.prec == BMC_FP64 ? (const void*)v.w64 : (const void*)v.w32;
            a.method = BMC_CMC;
            a.width = q.p;
            a.k0 = q.seed;
            a.part = v.part;
            a.cancel = v.cancel;
            FinTask f;
            std::memset(&f, 0, sizeof(f));
            f.part = a.part;
            if (m >= 1) {
                a.x = v.x;
                a.N = q.N;
                a.n = q.n;
                a.m = m;
                a.paths_per_wg = q.per_wg;
                a.nchunk = q.nchunk;
                a.k1 = key_hi(BMC_STREAM_INNER, m);
                f.cont = v.cont;
                f.steps_total = (unsigned long long*)&v.cnt[0];
                if (q.refine) f.sel = RefineSel{v.spec, v.x, v.ids, v.n_ids};
            } else {
                a.x = dev_S0(v.spec);
                a.N = 1;
                a.n = q.n_final;
                a.m = 0;
                a.paths_per_wg = q.fper_wg;
                a.nchunk = q.fnchunk;
                a.k1 = key_hi(BMC_STREAM_FINAL, 0);
                f.sums = (double*)&v.cnt[1];
                f.steps = (int64_t*)&v.cnt[3];
            }
            f.N = a.N;
            f.nchunk = a.nchunk;
            f.n = a.n;
            f.wide = finalize_is_wide(a.nchunk, a.N, false) ? 1 : 0;
            total += (uint64_t)a.N * a.nchunk;
            if (total > 0xFFFFFFFFull) return fail(BMC_EINVAL, "too many continuation jobs in one round");
            pre.push_back((uint32_t)total);
            ca.push_back(a);
            lds = std::max(lds, q.lds);
            ft.push_back(f);
            fpre.push_back(fpre.back() + (f.wide ? (uint32_t)f.N : (uint32_t)((f.N + 255) / 256)));
        }
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
    // FP32 label refinement: the finalize above listed the near-tie points;
    // their FP64 re-estimates and the finalize of those
    std::map<int, std::vector<const RoundItem*>> by_bucket;
    for (const RoundItem* it : train)
        if (it->q->refine) by_bucket[it->q->bucket].push_back(it);
    if (!by_bucket.empty()) {
        std::vector<FinTask> rft;
        std::vector<uint32_t> rfpre{0};
        for (auto& g : by_bucket) {
            std::vector<ContArgs> ca;
            std::vector<uint32_t> pre{0};
            size_t lds = 0;
            for (const RoundItem* it : g.second) {
                const OptPlan& q = *it->q;
                const OptDev& v = *it->dev;
                const int m = it->stage;
                ContArgs a;
                std::memset(&a, 0, sizeof(a));
                a.spec = v.spec;
                a.rules = v.w64;
                a.method = BMC_CMC;
                a.width = q.p;
                a.k0 = q.seed;
                a.k1 = key_hi(BMC_STREAM_INNER, m);
                a.part = v.part;
                a.x = v.x;
                a.N = q.N;
                a.ids = v.ids;
                a.n_ids = v.n_ids;
                a.n = q.n;
                a.m = m;
                a.paths_per_wg = q.rper_wg;
                a.nchunk = q.rnchunk;
                a.slot_stride = (uint32_t)std::min<int64_t>(q.N, REFINE_SLOTS);
                a.cancel = v.cancel;
                pre.push_back(pre.back() + a.slot_stride * a.nchunk);
                ca.push_back(a);
                lds = std::max(lds, q.lds64);
                FinTask f;
                std::memset(&f, 0, sizeof(f));
                f.part = v.part;
                f.cont = v.cont;
                f.ids = v.ids;
                f.n_ids = v.n_ids;
                f.N = q.N;
                f.nchunk = q.rnchunk;
                f.n = q.n;
                rft.push_back(f);
                rfpre.push_back(rfpre.back() + (uint32_t)((q.N + 255) / 256));
            }
            Step s;
            s.kind = K_CONT;
            s.bucket = g.first;
            s.prec = BMC_FP64;
            s.stride = true;
            s.ntasks = (int)ca.size();
            s.blocks = pre.back();
            s.tasks = tab.put(ca);
            s.prefix = tab.put(pre);
            s.lds = lds;
            steps.push_back(s);
        }
        Step s;
        s.kind = K_FIN;
        s.ntasks = (int)rft.size();
        s.blocks = rfpre.back();
        s.tasks = tab.put(rft);
        s.prefix = tab.put(rfpre);
        steps.push_back(s);
    }
    if (train.empty()) {
        Step end;
        end.phase = -1;
        steps.push_back(end);
        return BMC_OK;
    }
    Step fmark;
    fmark.phase = PH_FIT;
    steps.push_back(fmark);
    // boosting fits: one block per pricing, grouped by tile size
    std::map<int, std::vector<const RoundItem*>> by_tile;
    for (const RoundItem* it : train) {
        if (fit_one_launch_supported(it->q->p)) {
            by_tile[fit_tile(it->q->p)].push_back(it);
        } else {
            Step s;
            s.kind = K_FIT_SINGLE;
            s.single_q = *it->q;
            s.single_dev = *it->dev;
            s.date = it->stage;
            steps.push_back(s);
        }
    }
    for (auto& g : by_tile) {
        std::vector<FitTask> fts;
        size_t lds = 0;
        for (const RoundItem* it : g.second) {
            const OptPlan& q = *it->q;
            const OptDev& v = *it->dev;
            const int m = it->stage;
            FitScratch fs;
            fit_scratch_carve(v.fit, q.N, q.p, q.rounds, &fs);
            fts.push_back(fit_task_make(v.spec, q.d, v.x, v.cont, q.N, q.rounds, fs, v.w64 + (size_t)m * q.p,
                                        v.w32 + (size_t)m * q.p));
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
    Step end;
    end.phase = -1;
    steps.push_back(end);
    return BMC_OK;
}

hipError_t run_step(const Step& s, const char* dtab, hipStream_t st)
{
    const void* tasks = dtab + s.tasks;
    const uint32_t* pre = (const uint32_t*)(dtab + s.prefix);
    hipError_t e = hipSuccess;
    switch (s.kind) {
    case K_BRIDGE_END:
    case K_BRIDGE_BACK:
        return launch_bridge_multi((const BridgeTask*)tasks, pre, s.ntasks, s.blocks, s.kind == K_BRIDGE_END, st);
    case K_CONT:
        for (uint32_t j0 = 0; j0 < s.blocks && !e; j0 += MAX_GRID)
            e = launch_cont_multi(s.bucket, s.prec, (const ContArgs*)tasks, pre, s.ntasks, j0,
                                  std::min(MAX_GRID, s.blocks - j0), 256, s.lds, st, s.stride);
        return e;
    case K_FIN: return launch_finalize_multi((const FinTask*)tasks, pre, s.ntasks, s.blocks, st);
    case K_FIT: return launch_fit_cmc_multi((const FitTask*)tasks, s.ntasks, s.T, s.lds, st);
    case K_FIT_SINGLE: {
        const OptPlan& q = s.single_q;
        const OptDev& v = s.single_dev;
        FitScratch fs;
        fit_scratch_carve(v.fit, q.N, q.p, q.rounds, &fs);
        return launch_fit_cmc(v.spec, q.d, v.x, v.cont, q.N, q.rounds, fs, v.w64 + (size_t)s.date * q.p,
                              v.w32 + (size_t)s.date * q.p, st);
    }
    default: return hipSuccess;
    }
}

}  // namespace bmc
