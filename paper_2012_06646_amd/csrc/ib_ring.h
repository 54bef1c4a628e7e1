// Device-arena regions for batches, handed out and returned in FIFO order (batches retire
// in launch order): a ring over [0, cap).  Host-only, no HIP dependency.
#pragma once

#include <stddef.h>

#include <deque>
#include <utility>

namespace ibk {

struct Ring {
    size_t cap = 0;
    std::deque<std::pair<size_t, size_t>> live;  // (offset, size) of live regions, oldest first

    // Where a region of sz bytes would go now (false if it does not fit).
    bool place(size_t sz, size_t* off) const
    {
        if (sz == 0 || sz > cap) return false;
        if (live.empty()) {
            *off = 0;
            return true;
        }
        const size_t first = live.front().first;
        const size_t end = live.back().first + live.back().second;
        if (end > first) {  // not wrapped: free space is [end, cap) and [0, first)
            if (cap - end >= sz) {
                *off = end;
                return true;
            }
            if (first >= sz) {
                *off = 0;
                return true;
            }
            return false;
        }
        if (first - end >= sz) {  // wrapped: free space is [end, first)
            *off = end;
            return true;
        }
        return false;
    }

    void push(size_t off, size_t sz) { live.emplace_back(off, sz); }
    void pop() { live.pop_front(); }
};

}  // namespace ibk
