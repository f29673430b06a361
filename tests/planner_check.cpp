// CPU check of the recursion planner (csrc/planner.hpp): built with g++ and
// the host sanitizers by tests/test_planner.py, no GPU involved.
//
// split_task turns one finished task's bucket bounds into base-case bins and
// next-level subproblems.  Every bin of one sort is sorted at the same time
// as every other, so the bins must be pairwise disjoint; each must lie inside
// the task whose buckets it packs; each bucket of 2..cap elements that is not
// an equality bucket must lie in exactly one bin; nothing of a bucket larger
// than cap may lie in a bin.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1705_02257_amd/csrc/planner.hpp"

using namespace ips4o;

static uint64_t rs = 0x2545F4914F6CDD1Dull;
static uint64_t rnd() {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL line %d: ", __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            return 1;                                     \
        }                                                 \
    } while (0)

struct Range {
    uint64_t lo, hi;
};

// bins pairwise disjoint
static bool disjoint(std::vector<SegD> bins) {
    std::sort(bins.begin(), bins.end(), [](const SegD& a, const SegD& b) { return a.off < b.off; });
    for (size_t i = 1; i < bins.size(); ++i)
        if (bins[i - 1].off + bins[i - 1].len > bins[i].off) return false;
    return true;
}

// The case that once produced overlapping bins: two tasks of a level with a
// bucket of the previous level between them that already has its own bin.
static int regression_gap_between_tasks() {
    const uint64_t cap = 1000, bin_cap = 1000;
    std::vector<SegD> bins;
    std::vector<Seg> next;
    uint64_t eb = 0;
    // level 0: [0, 9000) -> [0, 5000) large, [5000, 5200) small, [5200, 9000) large
    const uint64_t b0[] = {0, 5000, 5200, 9000};
    CHECK(split_task(0, 9000, 0, 3, false, b0, cap, bin_cap, bins, next, &eb), "level 0");
    CHECK(bins.size() == 1 && bins[0].off == 5000 && bins[0].len == 200, "the small bucket's bin");
    CHECK(next.size() == 2, "two subproblems");
    // level 1: the first task ends with a 100-element bucket, the second
    // starts with one; together with the gap they span 400 <= bin_cap
    const uint64_t b1[] = {0, 2000, 4900, 5000};
    const uint64_t b2[] = {0, 100, 3800};
    std::vector<Seg> next2;
    CHECK(split_task(next[0].off, next[0].m, 0, 3, false, b1, cap, bin_cap, bins, next2, &eb), "task 1");
    CHECK(split_task(next[1].off, next[1].m, 0, 2, false, b2, cap, bin_cap, bins, next2, &eb), "task 2");
    CHECK(disjoint(bins), "bins overlap across a task boundary");
    CHECK(bins.size() == 3, "one bin per task's small bucket plus the earlier one (got %zu)", bins.size());
    CHECK(eb == 400, "elements sent to the base case (got %llu)", (unsigned long long)eb);
    return 0;
}

// Bins merge inside a task across final buckets (equality buckets, sizes
// 0 and 1) and stop at the bin capacity and at large buckets.
static int merging_inside_a_task() {
    std::vector<SegD> bins;
    std::vector<Seg> next;
    uint64_t eb = 0;
    // bucket sizes 10 | 50 | 20 | 0 | 1 | 300 | 2000 | 30, task at offset 100
    const uint64_t bd[] = {0, 10, 60, 80, 80, 81, 381, 2381, 2411};
    // with equality buckets (the odd ones: 50, 0, 300, 30 are final):
    // 10 and 20 share a bin [100, 180) across the equality bucket, the
    // single element is final, 2000 is recursed
    CHECK(split_task(100, 2411, 7, 8, true, bd, 1000, 400, bins, next, &eb), "split");
    CHECK(bins.size() == 1, "bins %zu", bins.size());
    CHECK(bins[0].off == 100 && bins[0].len == 80, "bin %llu+%u", (unsigned long long)bins[0].off, bins[0].len);
    CHECK(next.size() == 1 && next[0].off == 481 && next[0].m == 2000 && next[0].grp == 7, "large bucket");
    CHECK(eb == 30, "elements to the base case %llu", (unsigned long long)eb);
    // without equality buckets: 10, 50, 20 and (across the single element)
    // 300 share [100, 481) (381 <= 400); 30 after the recursed bucket gets
    // a bin of its own
    bins.clear();
    next.clear();
    eb = 0;
    CHECK(split_task(100, 2411, 7, 8, false, bd, 1000, 400, bins, next, &eb), "split");
    CHECK(next.size() == 1 && next[0].off == 481 && next[0].m == 2000, "large bucket");
    CHECK(bins.size() == 2, "bins %zu", bins.size());
    CHECK(bins[0].off == 100 && bins[0].len == 381, "bin 0: %llu+%u", (unsigned long long)bins[0].off, bins[0].len);
    CHECK(bins[1].off == 2481 && bins[1].len == 30, "bin 1");
    CHECK(eb == 410, "elements to the base case %llu", (unsigned long long)eb);
    // a tighter bin capacity splits where the span would exceed it
    bins.clear();
    next.clear();
    eb = 0;
    CHECK(split_task(100, 2411, 7, 8, false, bd, 1000, 80, bins, next, &eb), "split");
    CHECK(bins.size() == 3 && bins[0].len == 80 && bins[1].off == 181 && bins[1].len == 300, "bin capacity");
    return 0;
}

static int inconsistent_bounds() {
    std::vector<SegD> bins;
    std::vector<Seg> next;
    uint64_t eb = 0;
    const uint64_t dec[] = {0, 50, 40, 100};
    CHECK(!split_task(0, 100, 0, 3, false, dec, 10, 10, bins, next, &eb), "decreasing bounds accepted");
    const uint64_t short_end[] = {0, 50, 99};
    CHECK(!split_task(0, 100, 0, 2, false, short_end, 10, 10, bins, next, &eb), "bounds[K] != m accepted");
    const uint64_t late_start[] = {1, 50, 100};
    CHECK(!split_task(0, 100, 0, 2, false, late_start, 10, 10, bins, next, &eb), "bounds[0] != 0 accepted");
    return 0;
}

// Buckets flagged as one key value (the strictly in-place hand-off finds
// them by their two ends) are final whatever their size: neither recursed
// into nor binned.
static int one_key_buckets() {
    std::vector<SegD> bins;
    std::vector<Seg> next;
    uint64_t eb = 0;
    const uint64_t bd[] = {0, 50, 2050, 2100, 4100};
    const uint8_t one[] = {0, 1, 0, 0};
    CHECK(split_task(0, 4100, 0, 4, false, bd, 1000, 400, bins, next, &eb, nullptr, 0, one), "split");
    CHECK(next.size() == 1 && next[0].off == 2100 && next[0].m == 2000, "only the unflagged large bucket recurses");
    CHECK(bins.size() == 2 && bins[0].off == 0 && bins[0].len == 50 && bins[1].off == 2050 && bins[1].len == 50,
          "bins %zu", bins.size());
    CHECK(eb == 100, "elements to the base case %llu", (unsigned long long)eb);
    std::vector<SegD> bins2;
    std::vector<Seg> next2;
    uint64_t eb2 = 0;
    const uint8_t small_one[] = {1, 0, 1, 0};
    CHECK(split_task(0, 4100, 0, 4, false, bd, 1000, 400, bins2, next2, &eb2, nullptr, 0, small_one), "split");
    CHECK(bins2.empty() && eb2 == 0 && next2.size() == 2, "flagged small buckets are not binned");
    return 0;
}

// Random recursions over random segment lists: every property above.
static int random_recursions() {
    for (int trial = 0; trial < 400; ++trial) {
        const uint64_t cap = 16 + rnd() % 600;
        const uint64_t bin_cap = std::max<uint64_t>(2, cap / (1 + rnd() % 3));
        std::vector<Seg> cur;
        uint64_t at = rnd() % 50;
        const uint32_t nseg = 1 + rnd() % 5;
        std::vector<Range> segs;
        for (uint32_t g = 0; g < nseg; ++g) {
            const uint64_t m = rnd() % (30 * cap);
            if (m > cap) cur.push_back(Seg{at, m, g});
            segs.push_back(Range{at, at + m});
            at += m + rnd() % 3;
        }
        std::vector<SegD> bins;
        std::vector<Range> owner;          // task range of each bin
        std::vector<Range> must_bin;       // buckets of 2..cap elements, not equality buckets
        std::vector<Range> large;          // buckets recursed into
        std::vector<int> large_level, bin_level;
        uint64_t eb_total = 0, must_total = 0;
        for (int level = 0; !cur.empty() && level < 64; ++level) {
            std::vector<Seg> next;
            for (const Seg& t : cur) {
                // random bounds: K buckets, sizes drawn to mix empty, single,
                // small and large ones (the partition always makes progress)
                const uint32_t K = 2 + rnd() % 40;
                const bool eq = (rnd() % 3) == 0;
                std::vector<uint64_t> cuts(K - 1);
                for (auto& x : cuts) {
                    const uint64_t r = rnd() % 10;
                    x = r < 6 ? rnd() % t.m : (r < 8 ? cuts.empty() ? 0 : t.m / 2 : rnd() % (t.m / 2 + 1));
                }
                std::sort(cuts.begin(), cuts.end());
                std::vector<uint64_t> bd(K + 1);
                bd[0] = 0;
                for (uint32_t i = 0; i + 1 < K; ++i) bd[i + 1] = cuts[i];
                bd[K] = t.m;
                // guarantee progress: no bucket keeps the whole task
                bool whole = false;
                for (uint32_t i = 0; i < K; ++i) whole |= bd[i + 1] - bd[i] == t.m;
                if (whole) bd[1] = t.m / 2;
                for (uint32_t i = 0; i < K; ++i) {
                    const uint64_t sz = bd[i + 1] - bd[i];
                    if (sz > 1 && !(eq && (i & 1))) {
                        if (sz <= cap) {
                            must_bin.push_back(Range{t.off + bd[i], t.off + bd[i + 1]});
                            must_total += sz;
                        } else {
                            large.push_back(Range{t.off + bd[i], t.off + bd[i + 1]});
                            large_level.push_back(level);
                        }
                    }
                }
                const size_t before = bins.size();
                uint64_t eb = 0;
                std::vector<BinSrc> srcs;
                const uint32_t task_id = (uint32_t)(rnd() % 1000);
                CHECK(split_task(t.off, t.m, t.grp, K, eq, bd.data(), cap, bin_cap, bins, next, &eb, &srcs, task_id),
                      "trial %d: consistent bounds refused", trial);
                eb_total += eb;
                CHECK(srcs.size() == bins.size() - before, "trial %d: %zu bin sources for %zu bins", trial,
                      srcs.size(), bins.size() - before);
                for (size_t i = before; i < bins.size(); ++i) {
                    owner.push_back(Range{t.off, t.off + t.m});
                    bin_level.push_back(level);
                    // the bin spans exactly buckets j0 .. j1, none of them recursed into
                    const BinSrc& bs = srcs[i - before];
                    CHECK(bs.task == task_id && bs.j0 <= bs.j1 && bs.j1 < K, "trial %d: bad bin source", trial);
                    CHECK(bins[i].off == t.off + bd[bs.j0] && bins[i].off + bins[i].len == t.off + bd[bs.j1 + 1],
                          "trial %d: bin and its buckets differ", trial);
                    for (uint32_t j = bs.j0; j <= bs.j1; ++j)
                        CHECK(bd[j + 1] - bd[j] <= cap || (eq && (j & 1)),
                              "trial %d: a bin spans a recursed bucket", trial);
                }
            }
            for (const Seg& s : next) CHECK(s.m > cap, "trial %d: a subproblem within the capacity", trial);
            cur.swap(next);
        }
        CHECK(cur.empty(), "trial %d: recursion did not end", trial);
        CHECK(disjoint(bins), "trial %d: bins overlap", trial);
        CHECK(eb_total == must_total, "trial %d: base-case elements %llu, expected %llu", trial,
              (unsigned long long)eb_total, (unsigned long long)must_total);
        for (size_t i = 0; i < bins.size(); ++i) {
            CHECK(bins[i].len <= std::max(bin_cap, cap), "trial %d: bin larger than allowed", trial);
            CHECK(bins[i].off >= owner[i].lo && bins[i].off + bins[i].len <= owner[i].hi,
                  "trial %d: bin %zu leaves its task", trial, i);
        }
        // each bucket that needs the base case lies in exactly one bin; a bin
        // made on some level meets no bucket recursed into on that level or
        // deeper (the deeper ones lie inside that level's recursed buckets;
        // the bins made inside them come from deeper levels)
        auto covering = [&](const Range& r) {
            int c = 0;
            for (const SegD& b : bins)
                if (b.off <= r.lo && r.hi <= b.off + b.len) ++c;
            return c;
        };
        for (const Range& r : must_bin) CHECK(covering(r) == 1, "trial %d: a small bucket in %d bins", trial, covering(r));
        for (size_t q = 0; q < large.size(); ++q)
            for (size_t i = 0; i < bins.size(); ++i)
                if (bin_level[i] <= large_level[q])
                    CHECK(bins[i].off + bins[i].len <= large[q].lo || large[q].hi <= bins[i].off,
                          "trial %d: a bin meets a recursed bucket", trial);
        std::vector<SegD> sorted_bins = bins;
        // every bin lies inside one caller segment
        for (const SegD& b : sorted_bins) {
            int in = 0;
            for (const Range& s : segs) in += (s.lo <= b.off && b.off + b.len <= s.hi) ? 1 : 0;
            CHECK(in == 1, "trial %d: a bin outside the caller's segments", trial);
        }
    }
    return 0;
}

int main() {
    if (regression_gap_between_tasks()) return 1;
    if (merging_inside_a_task()) return 1;
    if (inconsistent_bounds()) return 1;
    if (one_key_buckets()) return 1;
    if (random_recursions()) return 1;
    std::printf("planner ok\n");
    return 0;
}
