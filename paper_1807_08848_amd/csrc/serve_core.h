// Host-only core of the request server: a first-fit arena for request slots
// (device HBM and pinned host staging alike) and the admission / batch
// former.  No HIP types: the same header is compiled into the library and
// into a CPU unit test.
#pragma once

#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace msrs {
namespace serve {

// First-fit allocator over [0, capacity) with kAlign-byte granularity.  Free
// blocks are kept by offset and merged with both neighbours on release, so
// releasing everything restores one block of the whole capacity.
class Arena {
public:
    static constexpr int64_t kAlign = 256;

    explicit Arena(int64_t capacity = 0) { reset(capacity); }

    void reset(int64_t capacity) {
        cap_ = capacity / kAlign * kAlign;
        used_ = 0;
        free_.clear();
        if (cap_ > 0) free_[0] = cap_;
    }

    static int64_t round(int64_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // Offset of a block of at least `bytes`, or -1 if no free block is large enough.
    int64_t alloc(int64_t bytes) {
        const int64_t need = round(bytes > 0 ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const int64_t off = it->first, rest = it->second - need;
            free_.erase(it);
            if (rest > 0) free_[off + need] = rest;
            used_ += need;
            return off;
        }
        return -1;
    }

    // Give back a block returned by alloc(bytes).
    void release(int64_t off, int64_t bytes) {
        int64_t size = round(bytes > 0 ? bytes : 1);
        used_ -= size;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }

    int64_t capacity() const { return cap_; }
    int64_t used() const { return used_; }
    int64_t largest_free() const {
        int64_t m = 0;
        for (auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

    // Free blocks are disjoint, inside the capacity, not adjacent (merged),
    // and free + used bytes equal the capacity.
    bool consistent() const {
        int64_t end = -1, tot = 0;
        for (auto& kv : free_) {
            if (kv.second <= 0 || kv.first < 0 || kv.first + kv.second > cap_) return false;
            if (kv.first <= end) return false;   // overlap or unmerged neighbour
            end = kv.first + kv.second;
            tot += kv.second;
        }
        return tot + used_ == cap_;
    }

private:
    int64_t cap_ = 0, used_ = 0;
    std::map<int64_t, int64_t> free_;
};

// Admission and batch forming over request ids.  Requests wait in arrival
// order until their slot fits (strict FIFO: a large request at the head is
// not overtaken, so no request starves); admitted requests queue per model,
// and a batch takes up to max_batch admitted requests of the model whose
// oldest admitted request arrived first.
class Scheduler {
public:
    struct Item { int64_t id; int model; int64_t bytes; uint64_t seq; };

    explicit Scheduler(int n_models = 0) : ready_(n_models) {}

    void push(int64_t id, int model, int64_t bytes) { waiting_.push_back({id, model, bytes, seq_++}); }

    // Admit waiting requests in order while `fit(item)` succeeds; returns the
    // admitted items in order.
    template <class Fit>
    std::vector<Item> admit(Fit&& fit) {
        std::vector<Item> out;
        while (!waiting_.empty()) {
            const Item& it = waiting_.front();
            if (!fit(it)) break;
            ready_[it.model].push_back(it);
            out.push_back(it);
            waiting_.pop_front();
        }
        return out;
    }

    // Next batch (one model, arrival order), empty if nothing is admitted.
    std::vector<Item> form(int max_batch) {
        int best = -1;
        for (int m = 0; m < (int)ready_.size(); ++m)
            if (!ready_[m].empty() && (best < 0 || ready_[m].front().seq < ready_[best].front().seq)) best = m;
        std::vector<Item> out;
        if (best < 0) return out;
        auto& q = ready_[best];
        while (!q.empty() && (int)out.size() < max_batch) {
            out.push_back(q.front());
            q.pop_front();
        }
        return out;
    }

    // Remove every queued (waiting or admitted, not launched) request.
    std::vector<Item> drop_all() {
        std::vector<Item> out(waiting_.begin(), waiting_.end());
        waiting_.clear();
        for (auto& q : ready_) {
            out.insert(out.end(), q.begin(), q.end());
            q.clear();
        }
        return out;
    }

    size_t waiting() const { return waiting_.size(); }
    size_t ready() const {
        size_t n = 0;
        for (auto& q : ready_) n += q.size();
        return n;
    }

private:
    std::deque<Item> waiting_;
    std::vector<std::deque<Item>> ready_;
    uint64_t seq_ = 0;
};

}  // namespace serve
}  // namespace msrs
