// Host-only check of the plan cache's bookkeeping (plan_cache.hpp): pins of
// calls in progress, the `captured` mark, eviction order and shutdown.
// Built and run by tests/test_plan_cache.py with the host C++ compiler; no
// GPU and no HIP are involved.  Prints one line per failed check and exits
// non-zero if any failed.
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <vector>

#include "plan_cache.hpp"

namespace {

struct Entry {
    int pins = 0;
    bool captured = false;
    size_t bytes = 0;
    int key = 0;
};

int g_failed = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);        \
            ++g_failed;                                               \
        }                                                             \
    } while (0)

struct Cache {
    std::mutex m;
    mck::PlanList<Entry> l;
    std::mutex& mutex() { return m; }
    mck::PlanList<Entry>& list() { return l; }
};

Entry make(int key, size_t bytes)
{
    Entry e;
    e.key = key;
    e.bytes = bytes;
    return e;
}

// a "call": looks the key up pinned (inserting it if absent), then leaves
// through one of several exits; the hold must be released on each
int call(Cache& c, int key, int exit_path, std::vector<int>* freed)
{
    mck::PinnedPlan<Cache, Entry> hold(c);
    {
        std::lock_guard<std::mutex> lock(c.mutex());
        Entry* e = c.list().find([&](const Entry& q) { return q.key == key; }, true);
        if (e == nullptr) {
            c.list().make_room(100, 4, 1000, [&](Entry& q) { freed->push_back(q.key); });
            e = c.list().insert(make(key, 100), true);
        }
        hold.adopt(e);
    }
    if (exit_path == 0)
        return 0;              // normal return
    if (exit_path == 1)
        return -1;             // an error status after the lookup
    if (exit_path == 2)
        throw std::runtime_error("unwinding");
    hold.release();            // explicit early release
    return 1;
}

}  // namespace

int main()
{
    // eviction: least recently used first, pinned and captured entries kept
    {
        mck::PlanList<Entry> l;
        std::vector<int> freed;
        auto rel = [&](Entry& e) { freed.push_back(e.key); };
        for (int k = 0; k < 4; ++k)
            l.insert(make(k, 100), false);          // MRU order: 3 2 1 0
        Entry* e1 = l.find([](const Entry& q) { return q.key == 1; }, true);  // 1 3 2 0, 1 pinned
        CHECK(e1 != nullptr && e1->pins == 1);
        Entry* e0 = l.find([](const Entry& q) { return q.key == 0; }, false);  // 0 1 3 2
        e0->captured = true;
        l.make_room(100, 4, 1000, rel);             // 4 entries at the limit: one must go
        CHECK(freed.size() == 1 && freed[0] == 2);  // the LRU one that is free to go
        l.make_room(100, 1, 1000, rel);             // room for one: every free entry goes
        CHECK(freed.size() == 2 && freed[1] == 3);
        CHECK(l.size() == 2);                       // pinned 1 and captured 0 stay
        l.make_room(950, 10, 1000, rel);            // byte limit: nothing more can go
        CHECK(l.size() == 2 && l.total_bytes() == 200);
        CHECK(l.pinned() == 1);
        l.unpin(e1);
        CHECK(l.pinned() == 0);
        l.make_room(100, 1, 1000, rel);             // 1 is free now; 0 stays (captured)
        CHECK(freed.size() == 3 && freed[2] == 1 && l.size() == 1);
        l.clear_unpinned(rel);                      // shutdown frees captured entries too
        CHECK(l.size() == 0 && freed.size() == 4 && freed[3] == 0);
    }
    // shutdown keeps entries that a call or a graph holds
    {
        mck::PlanList<Entry> l;
        std::vector<int> freed;
        l.insert(make(7, 10), true);
        l.insert(make(8, 10), false);
        l.clear_unpinned([&](Entry& e) { freed.push_back(e.key); });
        CHECK(l.size() == 1 && freed.size() == 1 && freed[0] == 8);
    }
    // every exit path of a call releases its pin exactly once
    {
        Cache c;
        std::vector<int> freed;
        for (int path = 0; path < 4; ++path) {
            try {
                call(c, 40 + path, path, &freed);
            } catch (const std::runtime_error&) {
            }
            std::lock_guard<std::mutex> lock(c.mutex());
            CHECK(c.list().pinned() == 0);
        }
        // repeated calls on one key: still no pin left, no entry duplicated
        for (int r = 0; r < 3; ++r)
            call(c, 40, 0, &freed);
        std::lock_guard<std::mutex> lock(c.mutex());
        CHECK(c.list().pinned() == 0 && c.list().size() == 4);
    }
    // a held entry survives a burst of other calls that would evict it
    {
        Cache c;
        std::vector<int> freed;
        mck::PinnedPlan<Cache, Entry> held(c);
        {
            std::lock_guard<std::mutex> lock(c.mutex());
            held.adopt(c.list().insert(make(99, 100), true));
        }
        for (int k = 0; k < 20; ++k)
            call(c, k, 0, &freed);
        bool evicted = false;
        for (int k : freed)
            evicted = evicted || k == 99;
        CHECK(!evicted);
        CHECK(held->key == 99 && held->pins == 1);
        held.release();
        CHECK(held.get() == nullptr);
        call(c, 1000, 0, &freed);
        call(c, 1001, 0, &freed);
        call(c, 1002, 0, &freed);
        call(c, 1003, 0, &freed);
        evicted = false;
        for (int k : freed)
            evicted = evicted || k == 99;
        CHECK(evicted);  // once released it is an ordinary LRU entry
    }
    if (g_failed == 0)
        std::printf("plan cache checks passed\n");
    return g_failed == 0 ? 0 : 1;
}
