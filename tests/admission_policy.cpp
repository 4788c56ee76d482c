// CPU driver of the serving loop's host-side policy (admission.hpp): the
// first-fit arena against a brute-force model of 256-byte units, and the
// admission pass with fake requests — order, in-flight and slot limits,
// waiting on memory, same-table deduplication, cache hits and evictions —
// plus the submission-time footprint check.  Prints one line per check and
// exits nonzero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "admission.hpp"

using namespace bmc;

static int checks = 0;
#define CHECK(cond)                                                                   \
    do {                                                                              \
        ++checks;                                                                     \
        if (!(cond)) {                                                                \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);               \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

// ---- arena against a unit bitmap ------------------------------------------

static void arena_against_model()
{
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 20; ++trial) {
        const size_t units = 64 + rng() % 200;
        Arena a;
        a.init(units * 256 + (rng() % 256));   // a ragged size rounds down to whole units
        CHECK(a.size() == units * 256);
        std::vector<int> owner(units, -1);     // model: which allocation holds each unit
        struct Live { size_t off, bytes; int id; };
        std::vector<Live> live;
        size_t used = 0, peak = 0;
        for (int step = 0; step < 2000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t bytes = 1 + rng() % (16 * 256);
                const size_t need = (bytes + 255) / 256;
                // first fit in the model: the lowest run of `need` free units
                size_t want = SIZE_MAX;
                for (size_t u = 0, run = 0; u < units; ++u) {
                    run = owner[u] < 0 ? run + 1 : 0;
                    if (run == need) {
                        want = (u + 1 - need) * 256;
                        break;
                    }
                }
                size_t off = 0;
                const bool ok = a.alloc(bytes, &off);
                CHECK(ok == (want != SIZE_MAX));
                if (ok) {
                    CHECK(off == want);
                    for (size_t u = off / 256; u < off / 256 + need; ++u) owner[u] = step;
                    live.push_back({off, bytes, step});
                    used += need * 256;
                    peak = std::max(peak, used);
                }
            } else {
                const size_t k = rng() % live.size();
                const Live l = live[k];
                live.erase(live.begin() + (long)k);
                a.release(l.off, l.bytes);
                for (size_t u = l.off / 256; u < l.off / 256 + (l.bytes + 255) / 256; ++u) owner[u] = -1;
                used -= (l.bytes + 255) / 256 * 256;
            }
            CHECK(a.used() == used);
            CHECK(a.peak() == peak);
            // the free map is exactly the model's maximal free runs
            std::map<size_t, size_t> runs;
            for (size_t u = 0; u < units;) {
                if (owner[u] >= 0) {
                    ++u;
                    continue;
                }
                size_t v = u;
                while (v < units && owner[v] < 0) ++v;
                runs[u * 256] = (v - u) * 256;
                u = v;
            }
            CHECK(a.free_blocks() == runs);
        }
    }
    std::printf("ok arena: first fit, coalescing, used and peak against the unit model\n");
}

// ---- admission --------------------------------------------------------------

struct FakeReq {
    int id;
    std::string key;
    size_t bytes;
};

struct Server {
    Arena arena;
    RuleCache cache;
    std::list<std::string> lru;
    std::vector<uint32_t> free_slots;
    std::deque<FakeReq*> queue;
    std::vector<FakeReq*> active;
    std::vector<std::pair<int, bool>> admitted;   // (id, hit) in admission order
    std::unordered_map<std::string, int> learning;
    int max_inflight = 8;
    bool caching = true;

    Server(size_t arena_bytes, int slots, int inflight) : max_inflight(inflight)
    {
        arena.init(arena_bytes);
        for (int i = slots - 1; i >= 0; --i) free_slots.push_back((uint32_t)i);
    }
    void cache_table(const std::string& key, size_t bytes, int users = 0)
    {
        size_t off = 0;
        CHECK(arena.alloc(bytes, &off));
        CacheEntry c;
        c.key = key;
        c.off = off;
        c.bytes = bytes;
        c.users = users;
        cache_insert(cache, lru, c);
    }
    void pass()
    {
        learning.clear();
        admit_pass(queue, arena, cache, lru, free_slots, max_inflight, learning, caching,
                   [](FakeReq* r) -> const std::string& { return r->key; }, [](FakeReq* r) { return r->bytes; },
                   [&] { return (int)active.size(); },
                   [&](FakeReq* r, size_t, uint32_t, bool hit) {
                       active.push_back(r);
                       admitted.push_back({r->id, hit});
                       if (hit) {
                           CacheEntry& c = cache.at(r->key);
                           ++c.users;
                           cache_touch(lru, c);
                       }
                   });
    }
    std::vector<int> queued_ids() const
    {
        std::vector<int> v;
        for (FakeReq* r : queue) v.push_back(r->id);
        return v;
    }
};

static void admission_cases()
{
    const size_t U = 256;
    std::vector<FakeReq> reqs;
    auto make = [&](int n, size_t bytes, const char* key_prefix, bool same_key = false) {
        reqs.clear();
        reqs.reserve((size_t)n);
        for (int i = 0; i < n; ++i)
            reqs.push_back({i, same_key ? std::string(key_prefix) : std::string(key_prefix) + std::to_string(i),
                            bytes});
    };
    {   // everything fits: first come, first served, every miss marks its key
        Server s(64 * U, 16, 16);
        make(5, 4 * U, "k");
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 5 && s.queue.empty());
        for (int i = 0; i < 5; ++i) CHECK(s.admitted[(size_t)i].first == i && !s.admitted[(size_t)i].second);
        CHECK(s.learning.size() == 5);
        CHECK(s.arena.used() == 20 * U && s.free_slots.size() == 11);
        std::printf("ok admission: first come, first served\n");
    }
    {   // in-flight limit: the rest wait in order
        Server s(64 * U, 16, 3);
        make(6, U, "k");
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 3);
        CHECK((s.queued_ids() == std::vector<int>{3, 4, 5}));
        std::printf("ok admission: the in-flight limit holds the rest back in order\n");
    }
    {   // device slots run out before the in-flight limit
        Server s(64 * U, 2, 10);
        make(4, U, "k");
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 2 && s.free_slots.empty());
        std::printf("ok admission: no request without a free device slot\n");
    }
    {   // memory: the first request that does not fit stops the pass, and the
        // smaller ones behind it wait too
        Server s(10 * U, 16, 16);
        reqs = {{0, "a", 6 * U}, {1, "b", 6 * U}, {2, "c", U}};
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 1 && s.admitted[0].first == 0);
        CHECK((s.queued_ids() == std::vector<int>{1, 2}));
        // once the first one's memory is back, the next two go in order
        s.arena.release(0, 6 * U);
        s.active.clear();
        s.admitted.clear();
        s.pass();
        CHECK(s.admitted.size() == 2 && s.admitted[0].first == 1 && s.admitted[1].first == 2);
        std::printf("ok admission: waiting on memory keeps the queue order\n");
    }
    {   // a table being learned: later requests for it wait, other keys pass them
        Server s(64 * U, 16, 16);
        reqs = {{0, "x", U}, {1, "x", U}, {2, "y", U}, {3, "x", U}};
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 2 && s.admitted[0].first == 0 && s.admitted[1].first == 2);
        CHECK((s.queued_ids() == std::vector<int>{1, 3}));
        CHECK(s.learning.at("x") == 1 && s.learning.at("y") == 1);
        // without the cache there is no waiting
        Server t(64 * U, 16, 16);
        t.caching = false;
        for (auto& r : reqs) t.queue.push_back(&r);
        t.pass();
        CHECK(t.admitted.size() == 4 && t.learning.empty());
        std::printf("ok admission: one learner per rule table, other tables overtake\n");
    }
    {   // cached tables: hits do not learn, several may share the entry
        Server s(64 * U, 16, 16);
        s.cache_table("x", 2 * U);
        reqs = {{0, "x", U}, {1, "x", U}, {2, "z", U}};
        for (auto& r : reqs) s.queue.push_back(&r);
        s.pass();
        CHECK(s.admitted.size() == 3);
        CHECK(s.admitted[0].second && s.admitted[1].second && !s.admitted[2].second);
        CHECK(s.cache.at("x").users == 2);
        CHECK(!s.learning.count("x") && s.learning.count("z"));
        std::printf("ok admission: cache hits share their table and learn nothing\n");
    }
    {   // eviction: least recently used first, never an entry in use; a hit
        // whose own entry had to go runs as a miss
        Server s(8 * U, 16, 16);
        s.cache_table("old", 3 * U);
        s.cache_table("busy", 2 * U, 1);   // read by a request on the device
        s.cache_table("new", 3 * U);       // most recently used
        reqs = {{0, "q", 3 * U}};
        s.queue.push_back(&reqs[0]);
        s.pass();
        CHECK(s.admitted.size() == 1 && !s.admitted[0].second);
        CHECK(!s.cache.count("old") && s.cache.count("busy") && s.cache.count("new"));
        // the arena is full again: the next request evicts "new", not "busy"
        FakeReq r1{1, "new", 3 * U};
        s.queue.push_back(&r1);
        s.pass();
        CHECK(s.admitted.size() == 2 && s.admitted[1].first == 1 && !s.admitted[1].second);
        CHECK(!s.cache.count("new") && s.cache.count("busy"));
        // nothing left to evict: the next one waits
        FakeReq r2{2, "w", U};
        s.queue.push_back(&r2);
        s.pass();
        CHECK(s.admitted.size() == 2 && s.queue.size() == 1);
        std::printf("ok admission: eviction spares tables in use and frees room least recently used first\n");
    }
    {   // submission: a footprint above the whole arena is refused up front
        Arena a;
        a.init(1000 * U);
        CHECK(a.could_ever_hold(1000 * U) && !a.could_ever_hold(1000 * U + 1));
        std::printf("ok submission: requests larger than the arena are refused (BMC_ENOMEM)\n");
    }
}

int main()
{
    arena_against_model();
    admission_cases();
    std::printf("all %d checks passed\n", checks);
    return 0;
}
