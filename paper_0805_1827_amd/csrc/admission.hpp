// Host-side state and policy of the serving loop that make no device call:
// the first-fit arena over the server's one device allocation, the
// least-recently-used index of the rule-table cache that lives in it, and the
// admission pass the server thread runs between rounds.  Plain C++ (no HIP),
// so that a CPU test drives the policy with requests of its own.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <list>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace bmc {

// First-fit allocator over one device allocation (offsets, 256-byte units):
// the lowest free block that holds the request is split; a released block
// merges with free neighbours, so the free map never holds two adjacent blocks.
class Arena {
public:
    void init(size_t bytes)
    {
        size_ = bytes & ~(size_t)255;
        used_ = peak_ = 0;
        free_.clear();
        if (size_) free_[0] = size_;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    // A request larger than the whole arena can never run (the server
    // refuses it at submission with BMC_ENOMEM).
    bool could_ever_hold(size_t bytes) const { return bytes <= size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }
    const std::map<size_t, size_t>& free_blocks() const { return free_; }   // offset -> bytes

private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// A learned rule table kept in the arena, keyed by everything that shapes it.
struct CacheEntry {
    std::string key;
    size_t off = 0, bytes = 0;   // [w64 rows][w32 rows] in the arena
    int rows = 0;                // (N_T + 1) * p
    int users = 0;               // requests copying from it this round
    std::list<std::string>::iterator lru;
};
using RuleCache = std::unordered_map<std::string, CacheEntry>;

// Marks an entry most recently used (front of lru).
inline void cache_touch(std::list<std::string>& lru, CacheEntry& c)
{
    lru.erase(c.lru);
    lru.push_front(c.key);
    c.lru = lru.begin();
}

// Adds an entry as the most recently used one.
inline void cache_insert(RuleCache& cache, std::list<std::string>& lru, CacheEntry c)
{
    lru.push_front(c.key);
    c.lru = lru.begin();
    const std::string key = c.key;
    cache.emplace(key, std::move(c));
}

// Drops the least recently used entry that no request is reading and returns
// its bytes to the arena; false if every entry is in use (or none exists).
inline bool cache_evict_one(RuleCache& cache, std::list<std::string>& lru, Arena& arena)
{
    for (auto it = lru.rbegin(); it != lru.rend(); ++it) {
        auto c = cache.find(*it);
        if (c != cache.end() && c->second.users == 0) {
            arena.release(c->second.off, c->second.bytes);
            lru.erase(std::next(it).base());
            cache.erase(c);
            return true;
        }
    }
    return false;
}

// One admission pass, first come, first served.  A queued request is admitted
// while fewer than max_inflight requests are in flight (inflight()) and a
// device slot is free, once its footprint (bytes_of) has a place in the arena,
// after evicting unused cache entries (least recently used first) if needed;
// the first request that still finds no place ends the pass, so the requests
// behind it wait too (no overtaking on memory).  A request whose rule table is
// not cached while an admitted request is learning the same table
// (learning[key] > 0) is passed over and stays queued, to run from the cache
// later; a request admitted to learn marks its key when caching is on.
// on_admit(r, offset, slot, hit) takes each admitted request (hit: its table
// is cached, looked up after the evictions) before the next is considered.
template <class R, class Key, class Bytes, class Inflight, class OnAdmit>
void admit_pass(std::deque<R*>& queue, Arena& arena, RuleCache& cache, std::list<std::string>& lru,
                std::vector<uint32_t>& free_slots, int max_inflight, std::unordered_map<std::string, int>& learning,
                bool caching, Key key_of, Bytes bytes_of, Inflight inflight, OnAdmit on_admit)
{
    for (auto qi = queue.begin(); qi != queue.end() && inflight() < max_inflight && !free_slots.empty();) {
        R* r = *qi;
        const std::string& key = key_of(r);
        if (!cache.count(key) && learning.count(key)) {
            ++qi;
            continue;
        }
        size_t off = 0;
        bool ok = arena.alloc(bytes_of(r), &off);
        while (!ok && cache_evict_one(cache, lru, arena)) ok = arena.alloc(bytes_of(r), &off);
        if (!ok) break;   // wait for memory to free up
        const bool hit = cache.count(key) != 0;
        qi = queue.erase(qi);
        if (!hit && caching) ++learning[key];
        const uint32_t slot = free_slots.back();
        free_slots.pop_back();
        on_admit(r, off, slot, hit);
    }
}

}  // namespace bmc
