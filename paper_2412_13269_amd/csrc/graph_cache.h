// Cache of captured op lists (HIP graphs), host logic only.
//
// A captured graph bakes in device addresses: of the registers, plaintexts and
// keys it was captured with, and of the per-stream scratch it wrote.  Replaying
// it is only valid while every one of those allocations is the one it was
// captured against.  So an entry is keyed on object identities, never on
// addresses:
//   * every context, ciphertext / plaintext and switching key carries a uid
//     from next_uid(), never reused, so a new object that happens to get a
//     freed object's address has a different key;
//   * every entry lists the uids it depends on; destroying any of those
//     objects drops the entry (drop_uid);
//   * scratch regions (per-stream workspaces, batched-key-switch and repacking
//     regions) carry no uid; instead a process-wide epoch moves whenever any of
//     them is freed or moved, and an entry captured in an older epoch is
//     dropped instead of replayed;
//   * the cache holds at most `cap` entries and drops the least recently used.
// Dropping an entry hands its executable to the destroy callback (which waits
// for the entry's last replay before freeing it).  All members lock one mutex;
// `launch` runs the caller's replay under it, so no other thread can drop the
// entry between the lookup and the launch.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace pfx {

// Identity of a library object: 1, 2, 3, ... in creation order, process-wide.
inline uint64_t next_uid() {
    static std::atomic<uint64_t> n{0};
    return ++n;
}

// Epoch of the scratch regions: moves whenever one is freed or reallocated.
inline std::atomic<uint64_t> &scratch_epoch() {
    static std::atomic<uint64_t> e{1};
    return e;
}
inline void bump_scratch_epoch() { scratch_epoch().fetch_add(1); }

template <class Exec>
class GraphCache {
public:
    using Meta = std::vector<std::pair<uint32_t, double>>;   // per register: (n_limbs | degree << 16, scale)
    using Destroy = std::function<void(Exec &)>;

    GraphCache(size_t cap, Destroy destroy) : cap_(cap), destroy_(std::move(destroy)) {}
    ~GraphCache() { clear(); }
    GraphCache(const GraphCache &) = delete;
    GraphCache &operator=(const GraphCache &) = delete;

    // If `key` holds an entry captured in `epoch`, call replay(exec, meta)
    // under the lock and return true.  An entry of an older epoch is dropped.
    bool launch(const std::string &key, uint64_t epoch, const std::function<void(Exec &, const Meta &)> &replay) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = map_.find(key);
        if (it == map_.end()) return false;
        if (it->second.epoch != epoch) {
            erase(it);
            return false;
        }
        lru_.splice(lru_.begin(), lru_, it->second.pos);
        replay(it->second.exec, it->second.meta);
        return true;
    }

    // Add an entry (replacing one with the same key) and replay it under the
    // lock; the least recently used entries beyond the capacity are dropped.
    void insert_and_launch(const std::string &key, uint64_t epoch, Exec exec, std::vector<uint64_t> uids, Meta meta,
                           const std::function<void(Exec &, const Meta &)> &replay) {
        std::lock_guard<std::mutex> g(mu_);
        auto old = map_.find(key);
        if (old != map_.end()) erase(old);
        lru_.push_front(key);
        Entry &e = map_[key];
        e.exec = exec;
        std::sort(uids.begin(), uids.end());
        uids.erase(std::unique(uids.begin(), uids.end()), uids.end());
        e.uids = std::move(uids);
        e.epoch = epoch;
        e.meta = std::move(meta);
        e.pos = lru_.begin();
        ++captures_;
        replay(e.exec, e.meta);
        while (map_.size() > cap_) erase(map_.find(lru_.back()));
    }

    // Drop every entry that depends on object `uid`.
    void drop_uid(uint64_t uid) {
        std::lock_guard<std::mutex> g(mu_);
        for (auto it = map_.begin(); it != map_.end();) {
            auto nx = std::next(it);
            if (std::binary_search(it->second.uids.begin(), it->second.uids.end(), uid)) erase(it);
            it = nx;
        }
    }

    void clear() {
        std::lock_guard<std::mutex> g(mu_);
        while (!map_.empty()) erase(map_.begin());
    }

    size_t size() {
        std::lock_guard<std::mutex> g(mu_);
        return map_.size();
    }
    uint64_t captures() {
        std::lock_guard<std::mutex> g(mu_);
        return captures_;
    }

private:
    struct Entry {
        Exec exec{};
        std::vector<uint64_t> uids;   // sorted
        uint64_t epoch = 0;
        Meta meta;
        std::list<std::string>::iterator pos;
    };
    void erase(typename std::map<std::string, Entry>::iterator it) {
        destroy_(it->second.exec);
        lru_.erase(it->second.pos);
        map_.erase(it);
    }

    size_t cap_;
    Destroy destroy_;
    std::mutex mu_;
    std::map<std::string, Entry> map_;
    std::list<std::string> lru_;   // most recently used first
    uint64_t captures_ = 0;
};

}  // namespace pfx
