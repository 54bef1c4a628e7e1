// Host test of the batch arena ring: random FIFO allocate/free sequences never hand out
// overlapping or out-of-range regions, and a region is refused only when neither free gap
// that keeps FIFO order can hold it.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "ib_ring.h"

static int fail(const char* what, int it)
{
    std::printf("FAIL %s at iteration %d\n", what, it);
    return 1;
}

int main()
{
    std::mt19937_64 rng(12345);
    for (size_t cap : {size_t(1000), size_t(4096), size_t(1) << 20}) {
        ibk::Ring r;
        r.cap = cap;
        for (int it = 0; it < 200000; ++it) {
            const bool alloc = r.live.empty() || (rng() % 100) < 55;
            if (alloc) {
                const size_t sz = 1 + rng() % (cap / 3);
                size_t off = 0;
                const bool ok = r.place(sz, &off);
                // the gaps a FIFO ring may use
                size_t g1 = cap, g2 = 0;
                if (!r.live.empty()) {
                    const size_t first = r.live.front().first;
                    const size_t end = r.live.back().first + r.live.back().second;
                    if (end > first) { g1 = cap - end; g2 = first; }
                    else { g1 = first - end; g2 = 0; }
                }
                if (!ok) {
                    if (g1 >= sz || g2 >= sz) return fail("refused a fitting region", it);
                    continue;
                }
                if (off + sz > cap) return fail("out of range", it);
                for (auto& L : r.live)
                    if (off < L.first + L.second && L.first < off + sz) return fail("overlap", it);
                r.push(off, sz);
            } else {
                r.pop();
            }
        }
        // exact fits
        ibk::Ring e;
        e.cap = cap;
        size_t off = 7;
        if (!e.place(cap, &off) || off != 0) return fail("whole arena", 0);
        e.push(0, cap);
        if (e.place(1, &off)) return fail("full arena", 0);
        e.pop();
        if (e.place(cap + 1, &off)) return fail("oversize", 0);
    }
    std::printf("ok\n");
    return 0;
}
