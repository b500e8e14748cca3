// serve_host.h -- host-only parts of the serving engine (no HIP): the device-arena allocator
// and the choice of the requests merged into one call.  Kept free of HIP so that they can be
// compiled and tested with a plain C++ compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace ctp {

// Allocator over [0, size) in 256-byte units with two ends: `alloc` places a block first-fit
// from the bottom, `alloc_high` last-fit from the top (at the end of the highest free block
// that holds it).  The serving engine keeps long-lived outputs at the bottom and the scratch of
// running calls at the top, so freed scratch always rejoins the free space above the outputs
// instead of leaving holes between them.  Offsets only: the caller adds them to the base of its
// device arena.  Free blocks are coalesced with their neighbours.
class Arena {
public:
    static constexpr size_t kAlign = 256;
    static constexpr size_t kFail = SIZE_MAX;

    void reset(size_t bytes)
    {
        size_ = bytes & ~(kAlign - 1);
        free_.clear();
        used_.clear();
        in_use_ = peak_ = 0;
        if (size_ > 0)
            free_[0] = size_;
    }

    static size_t round_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

    // Lowest-address free block that holds `bytes` (rounded up to 256); kFail if none.
    // Zero bytes are allocated as one 256-byte unit so that every allocation has an address.
    size_t alloc(size_t bytes)
    {
        const size_t n = round_up(bytes == 0 ? 1 : bytes);
        if (n < bytes)
            return kFail;   // overflow
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            const size_t off = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest > 0)
                free_[off + n] = rest;
            used_[off] = n;
            in_use_ += n;
            if (in_use_ > peak_)
                peak_ = in_use_;
            return off;
        }
        return kFail;
    }

    // Highest-address placement: the top end of the highest free block that holds `bytes`.
    size_t alloc_high(size_t bytes)
    {
        const size_t n = round_up(bytes == 0 ? 1 : bytes);
        if (n < bytes)
            return kFail;   // overflow
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second < n)
                continue;
            const size_t start = it->first, rest = it->second - n;
            const size_t off = start + rest;
            if (rest > 0)
                it->second = rest;
            else
                free_.erase(std::next(it).base());
            used_[off] = n;
            in_use_ += n;
            if (in_use_ > peak_)
                peak_ = in_use_;
            return off;
        }
        return kFail;
    }

    // Returns false for an offset that is not a live allocation.
    bool release(size_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end())
            return false;
        size_t start = off, n = u->second;
        used_.erase(u);
        in_use_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + n) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                n += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = n;
        return true;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &f : free_)
            m = f.second > m ? f.second : m;
        return m;
    }
    size_t n_free_blocks() const { return free_.size(); }

private:
    size_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
    std::map<size_t, size_t> used_;   // offset -> bytes
};

// Requests that may share one call: same plan, direction and storage types.
struct BatchKey {
    const void *plan;
    int dir, in_dtype, out_dtype;
    bool operator==(const BatchKey &o) const
    {
        return plan == o.plan && dir == o.dir && in_dtype == o.in_dtype && out_dtype == o.out_dtype;
    }
};

// Positions in `queue` (oldest first) of the requests merged into a call headed by
// queue[head]: the head, then, in arrival order, the other queued requests with the same key,
// at most max_batch in all.  `key_of` maps a queue element to its BatchKey.
template <typename T, typename KeyOf>
std::vector<size_t> batch_candidates(const std::deque<T> &queue, size_t head, int max_batch,
                                     KeyOf key_of)
{
    std::vector<size_t> pos;
    if (head >= queue.size() || max_batch < 1)
        return pos;
    const BatchKey hk = key_of(queue[head]);
    pos.push_back(head);
    for (size_t i = 0; i < queue.size() && (int)pos.size() < max_batch; ++i)
        if (i != head && key_of(queue[i]) == hk)
            pos.push_back(i);
    return pos;
}

// Order in which queued requests are tried as the head of the next call.  Requests that have
// waited at least age_cap_ns ("aged") come first, oldest first; the others follow cheapest first
// (smallest predicted work), ties in arrival order, so that short requests are not held behind
// long ones while no request waits longer than the cap before it is next in line.  With
// age_cap_ns <= 0 every request counts as aged: strict first come, first served.  `info` maps a
// queue element to {work, submit time}.  *n_aged receives the number of aged requests (they
// are the first *n_aged positions).
template <typename T, typename Info>
std::vector<size_t> head_order(const std::deque<T> &queue, int64_t now_ns, int64_t age_cap_ns,
                               Info info, size_t *n_aged)
{
    std::vector<size_t> aged, young;
    for (size_t i = 0; i < queue.size(); ++i) {
        const auto wi = info(queue[i]);
        if (age_cap_ns <= 0 || now_ns - wi.second >= age_cap_ns)
            aged.push_back(i);
        else
            young.push_back(i);
    }
    std::stable_sort(young.begin(), young.end(), [&](size_t a, size_t b) {
        return info(queue[a]).first < info(queue[b]).first;
    });
    if (n_aged)
        *n_aged = aged.size();
    aged.insert(aged.end(), young.begin(), young.end());
    return aged;
}

}  // namespace ctp
