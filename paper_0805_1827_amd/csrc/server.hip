// Serving loop: continuous batching of CMC pricing requests on one device.
//
// A server thread runs rounds of the round engine.  Between rounds it admits
// queued requests (first come, first served) while their device footprint
// fits the server's HBM arena and an in-flight slot is free; admitted
// requests join the next round, so requests of different sizes that arrive
// while others are on the device share their launches.  A request whose
// (spec, options, launch shape) matches a learned rule table in the on-device
// cache skips learning and runs only the final pricing.  Each result is
// bit-identical to bmc_price on the same context.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.hpp"
#include "engine.hpp"

using namespace bmc;

namespace {

using clk = std::chrono::steady_clock;

// Byte offset of a request's cancel word in its counters block (the block's
// first 32 bytes hold the pricing's results).
constexpr size_t CANCEL_WORD_OFFSET = 64;

// Sets a cancel word with an agent-scope store (read by the jobs of launches
// already running on the server's other stream).
__global__ void k_cancel_set(int32_t* w) { __hip_atomic_store(w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

struct Request {
    uint64_t ticket = 0;
    HostSpecPack pack;
    OptPlan q;
    std::string key;
    clk::time_point submitted, admitted, done;
    size_t off = 0;
    uint32_t slot = 0;
    OptDev dev;
    int stage = 0;          // next stage (see RoundItem); -1 when finished
    bool hit = false, fresh = false;
    bool cancel = false;    // cancelled while on the device: dropped at the end of the round
    int32_t* cancel_word = nullptr;   // device word read by its continuation jobs (zeroed with its counters)
    bmc_status status = BMC_OK;
    bmc_result result;
};

}  // namespace

struct bmc_server {
    bmc_ctx* ctx = nullptr;
    bmc_ctx view;             // tuning table snapshot (shapes fixed for the server's lifetime)
    hipStream_t stream = nullptr;
    int max_inflight = 256, cache_cap = 256;
    char* dev_arena = nullptr;
    DevSpec* specs = nullptr;
    Arena arena;
    std::vector<uint32_t> free_slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::unordered_map<uint64_t, Request*> all;     // by ticket, until polled
    RuleCache cache;
    std::list<std::string> lru;                       // front = most recent
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    bmc_server_stats st{};
    void* host = nullptr;     // pinned staging
    size_t host_bytes = 0;
    hipStream_t ctrl = nullptr;   // cancel-word stores, beside the rounds on `stream`
    bmc::DBuf dtab;
    bmc::DBuf dpack;
    double busy = 0.0;

    bmc_status ensure_host(size_t bytes)
    {
        if (host_bytes >= bytes) return BMC_OK;
        if (host) (void)hipHostFree(host);
        host = nullptr;
        host_bytes = 0;
        hipError_t e = hipHostMalloc(&host, bytes, 0);
        if (e) return hip_fail(e, "pinned staging");
        host_bytes = bytes;
        return BMC_OK;
    }
    void loop();
    bmc_status round(std::vector<Request*>& fresh);
    void finish(Request* r, bmc_status s);
    bool evict_one() { return cache_evict_one(cache, lru, arena); }   // caller holds mu
};

namespace {

// Cache key: the packed spec and every option that shapes the learned rules.
std::string rule_key(const HostSpecPack& pk, const OptPlan& q)
{
    std::string k;
    auto add = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    add(&pk.d, sizeof(int32_t) * 3);
    add(&pk.K, sizeof(double) * 3);
    add(pk.S0, sizeof(double) * pk.d);
    add(pk.delta, sizeof(double) * pk.d);
    add(pk.sigma, sizeof(double) * pk.d);
    add(pk.rho, sizeof(double) * (size_t)pk.d * pk.d);
    add(pk.dates, sizeof(double) * pk.n_dates);
    const int64_t v[] = {q.prec, q.rounds, q.N, q.n, q.seed, q.per_wg, q.nchunk};
    add(v, sizeof(v));
    return k;
}

}  // namespace

void bmc_server::finish(Request* r, bmc_status s)
{
    r->status = s;
    r->stage = -1;
    r->done = clk::now();
    r->result.seconds = std::chrono::duration<double>(r->done - r->submitted).count();
    r->result.calc_seconds = std::chrono::duration<double>(r->admitted - r->submitted).count();
    if (s == BMC_OK) ++st.completed;
    else if (s == BMC_ECANCELED) ++st.canceled;
    else ++st.failed;
}

// One round for the active requests (fresh: admitted since the last round).
bmc_status bmc_server::round(std::vector<Request*>& fresh)
{
    hipError_t e;
    bmc_status s;
    const size_t pack_bytes = (sizeof(HostSpecPack) * fresh.size() + 255) & ~(size_t)255;
    // ---- new requests: spec setup into their slots, zeroed rules and counters,
    // cached rules for hits
    if (!fresh.empty()) {
        const size_t slots_off = pack_bytes;
        const size_t status_off = slots_off + ((sizeof(uint32_t) * fresh.size() + 255) & ~(size_t)255);
        if ((s = ensure_host(status_off + sizeof(int32_t) * fresh.size()))) return s;
        if ((e = dpack.ensure(status_off))) return hip_fail(e, "spec staging");
        char* hb = (char*)host;
        for (size_t i = 0; i < fresh.size(); ++i) {
            std::memcpy(hb + sizeof(HostSpecPack) * i, &fresh[i]->pack, sizeof(HostSpecPack));
            ((uint32_t*)(hb + slots_off))[i] = fresh[i]->slot;
        }
        if ((e = hipMemcpyAsync(dpack.ptr, hb, status_off, hipMemcpyHostToDevice, stream)) ||
            (e = launch_setup((const HostSpecPack*)dpack.ptr, specs, (int)fresh.size(), stream,
                              (const uint32_t*)((char*)dpack.ptr + slots_off))))
            return hip_fail(e, "request setup");
        for (size_t i = 0; i < fresh.size(); ++i) {
            Request* r = fresh[i];
            if ((e = hipMemcpyAsync(hb + status_off + sizeof(int32_t) * i, (char*)(specs + r->slot) + offsetof(DevSpec, status),
                                    sizeof(int32_t), hipMemcpyDeviceToHost, stream)) ||
                (e = hipMemsetAsync(dev_arena + r->off, 0, r->q.zero_bytes, stream)))
                return hip_fail(e, "request setup");
            if (r->hit) {
                const CacheEntry& c = cache.at(r->key);
                if ((e = hipMemcpyAsync(r->dev.w64, dev_arena + c.off, sizeof(double) * c.rows, hipMemcpyDeviceToDevice,
                                        stream)) ||
                    (e = hipMemcpyAsync(r->dev.w32, dev_arena + c.off + sizeof(double) * c.rows,
                                        sizeof(float) * c.rows, hipMemcpyDeviceToDevice, stream)))
                    return hip_fail(e, "cached rules");
            }
        }
        if ((e = hipStreamSynchronize(stream))) return hip_fail(e, "request setup");
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = 0; i < fresh.size(); ++i) {
            Request* r = fresh[i];
            if (r->hit) --cache.at(r->key).users;
            if (((const int32_t*)(hb + status_off))[i] != 0) {
                arena.release(r->off, r->q.bytes);
                free_slots.push_back(r->slot);
                active.erase(std::find(active.begin(), active.end(), r));
                finish(r, BMC_ENOTSPD);
            }
        }
        cv_done.notify_all();
    }
    if (active.empty()) return BMC_OK;
    // ---- one engine round for every active request
    std::vector<RoundItem> items;
    items.reserve(active.size());
    for (Request* r : active) items.push_back({&r->q, &r->dev, r->stage});
    Table tab;
    std::vector<Step> steps;
    if ((s = plan_round(items, tab, steps))) return s;
    std::vector<Request*> ending;
    for (Request* r : active)
        if (r->stage == 0) ending.push_back(r);
    const size_t rb_off = (tab.bytes.size() + 255) & ~(size_t)255;
    if ((s = ensure_host(rb_off + 32 * ending.size() + 256))) return s;
    if ((e = dtab.ensure(std::max<size_t>(tab.bytes.size(), 256)))) return hip_fail(e, "task tables");
    char* hb = (char*)host;
    std::memcpy(hb, tab.bytes.data(), tab.bytes.size());
    if ((e = hipMemcpyAsync(dtab.ptr, hb, tab.bytes.size(), hipMemcpyHostToDevice, stream)))
        return hip_fail(e, "task tables");
    if ((e = run_steps(steps, (const char*)dtab.ptr, stream, [](int) {}))) return hip_fail(e, "round launch");
    for (size_t i = 0; i < ending.size(); ++i)
        if ((e = hipMemcpyAsync(hb + rb_off + 32 * i, ending[i]->dev.cnt, 32, hipMemcpyDeviceToHost, stream)))
            return hip_fail(e, "results");
    // rules of requests that have just learned their last date go to the cache
    std::vector<Request*> learned;
    for (Request* r : active)
        if (r->stage == 1 && cache_cap > 0) learned.push_back(r);
    {
        std::lock_guard<std::mutex> g(mu);
        for (Request* r : learned) {
            if (r->cancel || cache.count(r->key)) continue;   // a cancelled request's jobs may have been skipped
            while ((int)cache.size() >= cache_cap && evict_one()) {
            }
            if ((int)cache.size() >= cache_cap) continue;
            const int rows = (r->q.NT + 1) * r->q.p;
            const size_t bytes = (sizeof(double) + sizeof(float)) * (size_t)rows;
            size_t off;
            if (!arena.alloc(bytes, &off)) continue;   // no room: not cached
            if ((e = hipMemcpyAsync(dev_arena + off, r->dev.w64, sizeof(double) * rows, hipMemcpyDeviceToDevice,
                                    stream)) ||
                (e = hipMemcpyAsync(dev_arena + off + sizeof(double) * rows, r->dev.w32, sizeof(float) * rows,
                                    hipMemcpyDeviceToDevice, stream))) {
                arena.release(off, bytes);
                return hip_fail(e, "rule cache");
            }
            CacheEntry c;
            c.key = r->key;
            c.off = off;
            c.bytes = bytes;
            c.rows = rows;
            cache_insert(cache, lru, std::move(c));
        }
    }
    if ((e = hipStreamSynchronize(stream))) return hip_fail(e, "round");
    // ---- advance
    std::lock_guard<std::mutex> g(mu);
    ++st.rounds;
    for (size_t i = 0; i < ending.size(); ++i) {
        Request* r = ending[i];
        if (r->cancel) continue;
        const uint64_t* rb = (const uint64_t*)(hb + rb_off + 32 * i);
        double sums[3];
        std::memcpy(&sums[0], &rb[1], sizeof(double));
        std::memcpy(&sums[1], &rb[2], sizeof(double));
        int64_t fsteps;
        std::memcpy(&fsteps, &rb[3], sizeof(int64_t));
        sums[2] = (double)fsteps;
        std::memset(&r->result, 0, sizeof(r->result));
        fill_price(sums, r->q.n_final, &r->result);
        r->result.inner_path_steps = r->hit ? 0 : (int64_t)rb[0];
        st.inner_path_steps += r->result.inner_path_steps;
        st.final_path_steps += fsteps;
        arena.release(r->off, r->q.bytes);
        free_slots.push_back(r->slot);
        finish(r, BMC_OK);
    }
    bool any_cancel = false;
    for (Request* r : active) any_cancel |= r->cancel && r->stage >= 0;
    // a cancel-word store still queued must land before the memory is reused
    if (any_cancel && (e = hipStreamSynchronize(ctrl))) return hip_fail(e, "cancel");
    for (Request* r : active)
        if (r->cancel && r->stage >= 0) {
            arena.release(r->off, r->q.bytes);
            free_slots.push_back(r->slot);
            finish(r, BMC_ECANCELED);
        }
    for (Request* r : active)
        if (r->stage >= 1) --r->stage;
    active.erase(std::remove_if(active.begin(), active.end(), [](Request* r) { return r->stage < 0; }),
                 active.end());
    cv_done.notify_all();
    return BMC_OK;
}

void bmc_server::loop()
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Request*> fresh;
        {
            std::unique_lock<std::mutex> g(mu);
            cv_work.wait(g, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop && queue.empty() && active.empty()) break;
            // admission: first come, first served, by footprint and slots; a
            // request whose rule table is being learned by an earlier one
            // waits for it (and then runs from the cache)
            std::unordered_map<std::string, int> learning;
            if (cache_cap > 0)
                for (Request* a : active)
                    if (!a->hit && a->stage >= 1) ++learning[a->key];
            auto key_of = [](Request* r) -> const std::string& { return r->key; };
            auto bytes_of = [](Request* r) { return r->q.bytes; };
            auto inflight = [&] { return (int)active.size(); };
            auto on_admit = [&](Request* r, size_t off, uint32_t slot, bool hit) {
                r->hit = hit;
                r->off = off;
                r->slot = slot;
                r->dev = carve_option(r->q, specs + r->slot, dev_arena + off);
                // the cancel word sits in the counters block, which the
                // request's setup zeroes before its first launch
                r->cancel_word = (int32_t*)((char*)r->dev.cnt + CANCEL_WORD_OFFSET);
                r->dev.cancel = r->cancel_word;
                r->stage = r->hit ? 0 : r->q.NT - 1;
                r->admitted = clk::now();
                if (r->hit) {
                    ++st.cache_hits;
                    CacheEntry& c = cache.at(r->key);
                    ++c.users;
                    cache_touch(lru, c);
                } else {
                    ++st.cache_misses;
                }
                active.push_back(r);
                fresh.push_back(r);
            };
            admit_pass(queue, arena, cache, lru, free_slots, max_inflight, learning, cache_cap > 0, key_of, bytes_of,
                       inflight, on_admit);
        }
        const auto t0 = clk::now();
        const bmc_status s = round(fresh);
        std::lock_guard<std::mutex> g(mu);
        busy += std::chrono::duration<double>(clk::now() - t0).count();
        if (s) {   // device failure: fail every request on the device
            for (Request* r : active) {
                arena.release(r->off, r->q.bytes);
                free_slots.push_back(r->slot);
                finish(r, s);
            }
            active.clear();
            cv_done.notify_all();
        }
    }
}

extern "C" bmc_status bmc_server_create(bmc_ctx* ctx, const bmc_server_opts* opts, bmc_server** out)
{
    if (!ctx || !out) return fail(BMC_EINVAL, "NULL argument");
    (void)hipSetDevice(ctx->device);
    const int64_t budget = opts && opts->hbm_budget > 0 ? opts->hbm_budget : (int64_t)4 << 30;
    const int inflight = opts && opts->max_inflight > 0 ? opts->max_inflight : 256;
    const int cache_cap = opts ? (opts->rule_cache < 0 ? 0 : (opts->rule_cache > 0 ? opts->rule_cache : 256)) : 256;
    if (inflight > 65536) return fail(BMC_EINVAL, "max_inflight must be <= 65536");
    bmc_server* s = new bmc_server();
    s->ctx = ctx;
    s->view.device = ctx->device;
    s->view.ppt_table = ctx->ppt_table;
    s->max_inflight = inflight;
    s->cache_cap = cache_cap;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) ||
        (e = hipStreamCreateWithFlags(&s->ctrl, hipStreamNonBlocking)) ||
        (e = hipMalloc((void**)&s->dev_arena, (size_t)budget)) ||
        (e = hipMalloc((void**)&s->specs, sizeof(DevSpec) * (size_t)inflight))) {
        if (s->specs) (void)hipFree(s->specs);
        if (s->dev_arena) (void)hipFree(s->dev_arena);
        if (s->ctrl) (void)hipStreamDestroy(s->ctrl);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(BMC_ENOMEM, "server device memory (%lld bytes): %s", (long long)budget, hipGetErrorString(e));
    }
    s->arena.init((size_t)budget);
    for (int i = inflight - 1; i >= 0; --i) s->free_slots.push_back((uint32_t)i);
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return BMC_OK;
}

extern "C" void bmc_server_destroy(bmc_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) delete kv.second;
    if (s->dev_arena) (void)hipFree(s->dev_arena);
    if (s->specs) (void)hipFree(s->specs);
    s->dtab.release();
    s->dpack.release();
    if (s->host) (void)hipHostFree(s->host);
    if (s->ctrl) {
        (void)hipStreamSynchronize(s->ctrl);
        (void)hipStreamDestroy(s->ctrl);
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

extern "C" bmc_status bmc_server_submit(bmc_server* s, const bmc_spec* spec, const bmc_opts* opts, uint64_t* ticket)
{
    if (!s || !spec || !opts || !ticket) return fail(BMC_EINVAL, "NULL argument");
    Request* r = new Request();
    bmc_status st = plan_option(&s->view, spec, opts, 0, &r->q);
    if (st) {
        delete r;
        return st;
    }
    if (!s->arena.could_ever_hold(r->q.bytes)) {
        const size_t need = r->q.bytes;
        delete r;
        std::lock_guard<std::mutex> g(s->mu);
        ++s->st.rejected;
        return fail(BMC_ENOMEM, "request needs %zu bytes of device memory, the server has %zu", need,
                    s->arena.size());
    }
    std::memset(&r->pack, 0, sizeof(r->pack));
    pack_spec(spec, &r->pack);
    r->key = rule_key(r->pack, r->q);
    r->submitted = clk::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
        ++s->st.submitted;
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return BMC_OK;
}

static bmc_status take_result(bmc_server* s, std::unordered_map<uint64_t, Request*>::iterator it, bmc_result* out)
{
    Request* r = it->second;
    const bmc_status st = r->status;
    if (st == BMC_OK && out) *out = r->result;
    s->all.erase(it);
    delete r;
    if (st == BMC_ENOTSPD) return fail(st, "correlation matrix is not positive definite");
    if (st == BMC_ECANCELED) return fail(st, "request cancelled");
    if (st) return fail(st, "request failed on the device");
    return BMC_OK;
}

extern "C" bmc_status bmc_server_poll(bmc_server* s, uint64_t ticket, bmc_result* out)
{
    if (!s) return fail(BMC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(BMC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->stage >= 0 || it->second->done.time_since_epoch().count() == 0) return BMC_EBUSY;
    return take_result(s, it, out);
}

extern "C" bmc_status bmc_server_wait(bmc_server* s, uint64_t ticket, double timeout_s, bmc_result* out)
{
    if (!s) return fail(BMC_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(BMC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    auto ready = [&] { return r->stage < 0 && r->done.time_since_epoch().count() != 0; };
    if (timeout_s < 0) s->cv_done.wait(g, ready);
    else if (!s->cv_done.wait_for(g, std::chrono::duration<double>(timeout_s), ready)) return BMC_EBUSY;
    return take_result(s, s->all.find(ticket), out);
}

extern "C" bmc_status bmc_server_cancel(bmc_server* s, uint64_t ticket)
{
    if (!s) return fail(BMC_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(BMC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        Request* r = it->second;
        if (r->stage < 0 && r->done.time_since_epoch().count() != 0)
            return fail(BMC_EINVAL, "request %llu has already finished", (unsigned long long)ticket);
        auto q = std::find(s->queue.begin(), s->queue.end(), r);
        if (q != s->queue.end()) {   // not admitted yet
            s->queue.erase(q);
            s->finish(r, BMC_ECANCELED);
        } else if (!r->cancel) {     // on the device: its jobs see the word, the round end drops it
            r->cancel = true;
            (void)hipSetDevice(s->ctx->device);
            hipLaunchKernelGGL(k_cancel_set, dim3(1), dim3(1), 0, s->ctrl, r->cancel_word);
            (void)hipGetLastError();   // a refused store only delays the cancel to the round end
        }
    }
    s->cv_done.notify_all();
    s->cv_work.notify_one();
    return BMC_OK;
}

extern "C" bmc_status bmc_server_stats_get(bmc_server* s, bmc_server_stats* out)
{
    if (!s || !out) return fail(BMC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->inflight = (int64_t)s->active.size();
    out->hbm_in_use = (int64_t)s->arena.used();
    out->hbm_peak = (int64_t)s->arena.peak();
    out->cached_rules = (int64_t)s->cache.size();
    out->busy_seconds = s->busy;
    return BMC_OK;
}
