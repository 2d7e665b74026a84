// plan_cache.hpp -- bookkeeping of the parameter-plan cache: entries in
// most-recently-used order, the pins of calls in progress and of recorded
// graphs, the `captured` mark of plans that a graph captured from a stream
// reads at every replay, and the choice of entries to free.  No HIP here:
// the runtime supplies the key test, the release of an entry's device
// memory and the mutex, so that this logic also builds and runs in a plain
// host test.
#pragma once

#include <cstddef>
#include <list>
#include <mutex>
#include <utility>

namespace mck {

// P must have the members `int pins`, `bool captured` and `size_t bytes`.
// The caller holds the cache's mutex around every call.
template <class P>
class PlanList {
public:
    // The entry `match` accepts, moved to the front (most recently used) and
    // pinned once more when `pin`; null when there is none.
    template <class Match>
    P* find(Match match, bool pin)
    {
        for (auto it = items_.begin(); it != items_.end(); ++it) {
            if (match(*it)) {
                items_.splice(items_.begin(), items_, it);
                if (pin)
                    ++items_.front().pins;
                return &items_.front();
            }
        }
        return nullptr;
    }

    // Frees least recently used entries, skipping pinned and captured ones,
    // until an entry of `bytes` more fits under max_items and max_bytes (or
    // nothing more can be freed).
    template <class Release>
    void make_room(size_t bytes, size_t max_items, size_t max_bytes, Release release)
    {
        size_t used = total_bytes();
        for (auto it = items_.end(); it != items_.begin() && (items_.size() >= max_items || used + bytes > max_bytes);) {
            --it;
            if (it->pins > 0 || it->captured)
                continue;
            used -= it->bytes;
            release(*it);
            it = items_.erase(it);
        }
    }

    // Adds a new entry at the front, pinned once when `pin`.
    P* insert(P&& p, bool pin)
    {
        items_.push_front(std::move(p));
        if (pin)
            ++items_.front().pins;
        return &items_.front();
    }

    void unpin(P* p) { --p->pins; }

    // mck_shutdown: frees every entry no call or recorded graph holds
    // (captured ones included: the graphs that read them must be gone).
    template <class Release>
    void clear_unpinned(Release release)
    {
        for (auto it = items_.begin(); it != items_.end();) {
            if (it->pins > 0) {
                ++it;
                continue;
            }
            release(*it);
            it = items_.erase(it);
        }
    }

    size_t size() const { return items_.size(); }

    size_t total_bytes() const
    {
        size_t b = 0;
        for (const P& p : items_)
            b += p.bytes;
        return b;
    }

    int pinned() const
    {
        int k = 0;
        for (const P& p : items_)
            k += p.pins > 0 ? 1 : 0;
        return k;
    }

private:
    std::list<P> items_;
};

// One call's hold on an entry: taken by `acquire` (the entry comes back
// pinned), released exactly once, on every exit path, by `release` or the
// destructor.  Cache provides `std::mutex& mutex()` and a PlanList
// `list()`.
template <class Cache, class P>
class PinnedPlan {
public:
    explicit PinnedPlan(Cache& c) : cache_(c) {}
    PinnedPlan(const PinnedPlan&) = delete;
    PinnedPlan& operator=(const PinnedPlan&) = delete;
    ~PinnedPlan() { release(); }

    // adopts an entry that the cache has already pinned for this call
    void adopt(P* p)
    {
        release();
        p_ = p;
    }
    P* get() const { return p_; }
    P* operator->() const { return p_; }
    void release()
    {
        if (p_ != nullptr) {
            std::lock_guard<std::mutex> lock(cache_.mutex());
            cache_.list().unpin(p_);
            p_ = nullptr;
        }
    }

private:
    Cache& cache_;
    P* p_ = nullptr;
};

}  // namespace mck
