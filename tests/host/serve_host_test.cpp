// Unit test of the serving engine's host logic (paper_2503_16741_amd/csrc/serve_host.h):
// the device-arena allocator against a unit-by-unit model, and the choice of merged requests.
// Prints "ok" and exits 0 on success.
#include "../../paper_2503_16741_amd/csrc/serve_host.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "%s:%d: CHECK(%s) failed\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

using ctp::Arena;

static void allocator_model_test(unsigned seed)
{
    const size_t units = 257;                 // arena of 257 units (+ a ragged tail)
    Arena a;
    a.reset(units * Arena::kAlign + 100);
    CHECK(a.size() == units * Arena::kAlign);
    std::vector<int> owner(units, -1);        // model: which allocation holds each unit
    struct Live { size_t off, n; };
    std::vector<Live> live;
    std::mt19937 rng(seed);
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 100 < 55) {
            const size_t bytes = rng() % 9 == 0 ? 0 : 1 + rng() % (Arena::kAlign * 20);
            const size_t n = bytes == 0 ? 1 : (bytes + Arena::kAlign - 1) / Arena::kAlign;
            const bool high = rng() % 2 == 0;
            size_t want = Arena::kFail;
            if (!high) {
                // first fit in the model
                for (size_t u = 0; u + n <= units && want == Arena::kFail; ++u) {
                    bool fr = true;
                    for (size_t k = 0; k < n && fr; ++k)
                        fr = owner[u + k] < 0;
                    if (fr)
                        want = u * Arena::kAlign;
                }
            } else {
                // the top end of the highest free run that holds n units
                size_t end = units;
                while (end > 0 && want == Arena::kFail) {
                    while (end > 0 && owner[end - 1] >= 0)
                        --end;
                    size_t beg = end;
                    while (beg > 0 && owner[beg - 1] < 0)
                        --beg;
                    if (end - beg >= n)
                        want = (end - n) * Arena::kAlign;
                    end = beg;
                }
            }
            const size_t off = high ? a.alloc_high(bytes) : a.alloc(bytes);
            CHECK(off == want);
            if (off != Arena::kFail) {
                CHECK(off % Arena::kAlign == 0);
                for (size_t k = 0; k < n; ++k)
                    owner[off / Arena::kAlign + k] = (int)live.size();
                live.push_back({off, n});
            }
        } else {
            const size_t i = rng() % live.size();
            CHECK(a.release(live[i].off));
            CHECK(!a.release(live[i].off));   // double free is refused
            for (size_t k = 0; k < live[i].n; ++k)
                owner[live[i].off / Arena::kAlign + k] = -1;
            live[i] = live.back();
            live.pop_back();
            for (size_t u = 0; u < units; ++u)  // re-label owners after the swap
                if (owner[u] >= 0)
                    owner[u] = -1;
            for (size_t j = 0; j < live.size(); ++j)
                for (size_t k = 0; k < live[j].n; ++k)
                    owner[live[j].off / Arena::kAlign + k] = (int)j;
        }
        size_t used = 0;
        for (const Live &l : live)
            used += l.n * Arena::kAlign;
        CHECK(a.in_use() == used);
        CHECK(a.peak() >= used);
        // free blocks are maximal: their count equals the number of free runs of the model
        size_t runs = 0;
        for (size_t u = 0; u < units; ++u)
            if (owner[u] < 0 && (u == 0 || owner[u - 1] >= 0))
                ++runs;
        CHECK(a.n_free_blocks() == runs);
    }
    for (const Live &l : live)
        CHECK(a.release(l.off));
    CHECK(a.in_use() == 0);
    CHECK(a.n_free_blocks() == 1);
    CHECK(a.largest_free() == a.size());
}

struct Q { const void *plan; int dir, in_dt, out_dt; };

static void batch_candidates_test()
{
    int p1, p2;
    auto key = [](const Q &q) { return ctp::BatchKey{q.plan, q.dir, q.in_dt, q.out_dt}; };
    std::deque<Q> q;
    CHECK(ctp::batch_candidates(q, 0, 4, key).empty());
    q = {{&p1, 0, 0, 0}, {&p2, 0, 0, 0}, {&p1, 0, 0, 0}, {&p1, 1, 0, 0}, {&p1, 0, 0, 1},
         {&p1, 0, 0, 0}, {&p1, 0, 0, 0}};
    auto c = ctp::batch_candidates(q, 0, 8, key);
    CHECK((c == std::vector<size_t>{0, 2, 5, 6}));       // same plan, direction and dtypes
    c = ctp::batch_candidates(q, 0, 2, key);
    CHECK((c == std::vector<size_t>{0, 2}));             // at most max_batch, oldest first
    c = ctp::batch_candidates(q, 0, 0, key);
    CHECK(c.empty());
    c = ctp::batch_candidates(q, 5, 3, key);
    CHECK((c == std::vector<size_t>{5, 0, 2}));          // head first, then arrival order
    c = ctp::batch_candidates(q, 1, 8, key);
    CHECK((c == std::vector<size_t>{1}));                // a lone head is served alone
    CHECK(ctp::batch_candidates(q, 7, 8, key).empty());  // past the end
}

struct W { double work; int64_t t; };

static void head_order_test()
{
    auto info = [](const W &w) { return std::make_pair(w.work, w.t); };
    std::deque<W> q = {{5.0, 0}, {1.0, 10}, {3.0, 20}, {1.0, 30}, {9.0, 40}};
    size_t n_aged = 99;
    // no cap: arrival order, everything counts as aged
    auto o = ctp::head_order(q, 100, 0, info, &n_aged);
    CHECK((o == std::vector<size_t>{0, 1, 2, 3, 4}) && n_aged == 5);
    // cap 1000 at time 100: nothing aged, cheapest first, ties in arrival order
    o = ctp::head_order(q, 100, 1000, info, &n_aged);
    CHECK((o == std::vector<size_t>{1, 3, 2, 0, 4}) && n_aged == 0);
    // cap 85 at time 100: requests submitted at 0 and 10 are aged and lead, oldest first
    o = ctp::head_order(q, 100, 85, info, &n_aged);
    CHECK((o == std::vector<size_t>{0, 1, 3, 2, 4}) && n_aged == 2);
    std::deque<W> e;
    CHECK(ctp::head_order(e, 0, 10, info, &n_aged).empty() && n_aged == 0);
}

int main()
{
    for (unsigned s = 1; s <= 4; ++s)
        allocator_model_test(s);
    Arena a;
    a.reset(0);
    CHECK(a.alloc(1) == Arena::kFail);
    a.reset(1024);
    CHECK(a.alloc(SIZE_MAX - 10) == Arena::kFail);       // size overflow
    CHECK(a.alloc(1024) == 0 && a.alloc(1) == Arena::kFail);
    a.reset(4096);
    CHECK(a.alloc_high(300) == 4096 - 512 && a.alloc(1) == 0 && a.alloc_high(256) == 4096 - 768);
    CHECK(a.alloc_high(SIZE_MAX - 10) == Arena::kFail);
    batch_candidates_test();
    head_order_test();
    std::printf("ok\n");
    return 0;
}
