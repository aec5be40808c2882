// Host-only checks of the HIP-graph cache (paper_2412_13269_amd/csrc/graph_cache.h),
// built with g++ under AddressSanitizer + UndefinedBehaviorSanitizer (and, with
// -DPFX_THREADS, ThreadSanitizer) by tests/test_graph_cache.py.  The
// executable type is an int; "destroying" one records it.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "graph_cache.h"

using pfx::GraphCache;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

// The key of a register set as the library builds it: identity and capacity of
// each register, never its address.
static std::string reg_key(const std::vector<std::pair<uint64_t, uint32_t>> &regs) {
    std::string k = "ops";
    for (auto &r : regs) {
        k.append((const char *)&r.first, sizeof r.first);
        k.append((const char *)&r.second, sizeof r.second);
    }
    return k;
}

int main() {
    std::vector<int> destroyed;
    auto cache = new GraphCache<int>(3, [&](int &x) { destroyed.push_back(x); });
    int replayed = -1;
    auto rep = [&](int &x, const GraphCache<int>::Meta &) { replayed = x; };
    const uint64_t ep = pfx::scratch_epoch().load();

    // uids are never reused
    std::set<uint64_t> seen;
    for (int i = 0; i < 1000; ++i) CHECK(seen.insert(pfx::next_uid()).second);

    // a register destroyed and recreated (same address in a real run, new uid,
    // other capacity) never finds the old graph
    const uint64_t r1 = pfx::next_uid(), key1 = pfx::next_uid();
    const std::string kA = reg_key({{r1, 24}, {key1, 0}});
    cache->insert_and_launch(kA, ep, 10, {r1, key1}, {{24, 1.0}}, rep);
    CHECK(replayed == 10);
    replayed = -1;
    CHECK(cache->launch(kA, ep, rep) && replayed == 10);
    cache->drop_uid(r1);                              // pfx_ct_destroy of the register
    CHECK(destroyed.size() == 1 && destroyed[0] == 10);
    CHECK(!cache->launch(kA, ep, rep));
    const uint64_t r2 = pfx::next_uid();
    const std::string kB = reg_key({{r2, 12}, {key1, 0}});
    CHECK(kB != kA);
    CHECK(!cache->launch(kB, ep, rep));               // must be captured afresh
    cache->insert_and_launch(kB, ep, 11, {r2, key1}, {{12, 1.0}}, rep);
    CHECK(cache->captures() == 2);

    // dropping a key used by several graphs drops them all, and only them
    const uint64_t r3 = pfx::next_uid();
    const std::string kC = reg_key({{r3, 24}});
    cache->insert_and_launch(kC, ep, 12, {r3}, {}, rep);
    cache->drop_uid(key1);
    CHECK(destroyed.size() == 2 && destroyed[1] == 11);
    CHECK(cache->size() == 1 && cache->launch(kC, ep, rep) && replayed == 12);

    // a scratch region freed or moved: the epoch moves and older graphs are
    // captured again, never replayed
    pfx::bump_scratch_epoch();
    const uint64_t ep2 = pfx::scratch_epoch().load();
    CHECK(ep2 != ep);
    CHECK(!cache->launch(kC, ep2, rep));
    CHECK(destroyed.size() == 3 && destroyed[2] == 12 && cache->size() == 0);

    // the same key captured again replaces (and destroys) the old entry
    cache->insert_and_launch(kC, ep2, 13, {r3}, {}, rep);
    cache->insert_and_launch(kC, ep2, 14, {r3}, {}, rep);
    CHECK(destroyed.back() == 13 && cache->size() == 1);

    // bounded: the least recently used entry goes first
    cache->insert_and_launch("k1", ep2, 21, {}, {}, rep);
    cache->insert_and_launch("k2", ep2, 22, {}, {}, rep);   // {kC, k1, k2} full
    CHECK(cache->launch(kC, ep2, rep));                      // kC most recent
    cache->insert_and_launch("k3", ep2, 23, {}, {}, rep);   // evicts k1
    CHECK(destroyed.back() == 21 && cache->size() == 3);
    CHECK(!cache->launch("k1", ep2, rep) && cache->launch("k2", ep2, rep) && cache->launch(kC, ep2, rep));

    delete cache;                                            // destroys what is left
    CHECK(destroyed.size() == 8);

#ifdef PFX_THREADS
    // concurrent lookups, inserts and drops (ThreadSanitizer build)
    std::atomic<int> live{0};
    GraphCache<int> shared(8, [&](int &) { live.fetch_sub(1); });
    std::vector<std::thread> ts;
    for (int t = 0; t < 4; ++t)
        ts.emplace_back([&, t]() {
            for (int i = 0; i < 2000; ++i) {
                const std::string k = "t" + std::to_string((t * 7 + i) % 13);
                const uint64_t u = (uint64_t)((t + i) % 5 + 1);
                auto r = [](int &, const GraphCache<int>::Meta &) {};
                if (!shared.launch(k, 1, r)) {
                    live.fetch_add(1);
                    shared.insert_and_launch(k, 1, i, {u}, {}, r);
                }
                if (i % 17 == 0) shared.drop_uid(u);
            }
        });
    for (auto &th : ts) th.join();
    shared.clear();
    CHECK(live.load() == 0);
#endif
    if (failures) return 1;
    std::puts("graph cache ok");
    return 0;
}
