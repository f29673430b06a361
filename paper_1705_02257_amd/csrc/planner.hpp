// Host-side recursion planning that needs no GPU: how one finished level's
// bucket bounds turn into base-case bins and the next level's subproblems.
// Plain C++ (no HIP types), so that it is compiled into the library and,
// unchanged, into a CPU-only test program.
//
// Recursion (Section 4, first paragraph; "Implementation Details"): a bucket
// larger than the base-case capacity is partitioned again, a bucket of at
// most the capacity is sorted by the base case, and an equality bucket
// (Section 4, "The Case of Many Identical Keys") holds one key value and is
// final, like a bucket of at most one element.
#pragma once
#include <cstdint>
#include <vector>

namespace ips4o {

// A base-case bin as the base-case kernels read it: elements [off, off+len)
// of the array.
struct SegD {
    uint64_t off;
    uint32_t len;
    uint32_t pad;
};

// The buckets a bin spans: buckets j0 .. j1 of task `task` of the level that
// made it (every bucket in between included: equality buckets and buckets
// of at most one element lie inside the span too).
struct BinSrc {
    uint32_t task, j0, j1, pad;
};

// A subproblem: elements [off, off+m); grp is the caller's segment it lies in;
// dup: the task it came from used equality buckets (its keys repeat, so its
// own sample likely repeats splitters too).
struct Seg {
    uint64_t off, m;
    uint32_t grp;
    uint32_t dup;
};

// The buckets of one finished task (a subproblem [off, off+m) of the level
// just partitioned into K buckets, bounds[0..K] relative to off).
//
// Buckets of at most `cap` elements go to the base case.  Consecutive ones
// share a bin while the bin spans at most `bin_cap` elements: a bin spans
// whole buckets of this task, and whatever lies between two of them inside
// the task is already final (an equality bucket, a bucket of at most one
// element) or a bucket larger than cap >= bin_cap, which no bin can span; the
// buckets of a partition hold disjoint key ranges in ascending order, so
// sorting the span sorts each bucket in place exactly as sorting them one by
// one would.  A bin never reaches beyond its task: between two tasks of a
// level may lie buckets of an earlier level that already have bins of their
// own, and two bins sorted at once must not overlap.
// Larger buckets are appended to `next` (grp inherited, dup = eq).  Returns false when
// the bounds are inconsistent (bounds[0] != 0, bounds[K] != m, decreasing).
// With `srcs`, every bin made here also gets its BinSrc (task `task`),
// appended in the order of the bins.  With `one`, a bucket i with one[i]
// set is known to hold one key value and is final like an equality bucket.
inline bool split_task(uint64_t off, uint64_t m, uint32_t grp, uint32_t K, bool eq, const uint64_t* bounds,
                       uint64_t cap, uint64_t bin_cap, std::vector<SegD>& bins, std::vector<Seg>& next,
                       uint64_t* elements_base, std::vector<BinSrc>* srcs = nullptr, uint32_t task = 0,
                       const uint8_t* one = nullptr) {
    if (K == 0 || bounds[0] != 0 || bounds[K] != m) return false;
    for (uint32_t i = 0; i < K; ++i)
        if (bounds[i + 1] < bounds[i]) return false;
    const size_t task_first = bins.size();   // bins before this index belong to other tasks
    for (uint32_t i = 0; i < K; ++i) {
        const uint64_t sz = bounds[i + 1] - bounds[i];
        if (sz <= 1) continue;
        if (eq && (i & 1)) continue;             // equality bucket: one key value
        if (one && one[i]) continue;             // found to hold one key value
        const uint64_t at = off + bounds[i];
        if (sz > cap) {
            next.push_back(Seg{at, sz, grp, eq ? 1u : 0u});
            continue;
        }
        *elements_base += sz;
        if (bins.size() > task_first) {
            SegD& cur = bins.back();
            if (at + sz - cur.off <= bin_cap) {
                cur.len = (uint32_t)(at + sz - cur.off);
                if (srcs) srcs->back().j1 = i;
                continue;
            }
        }
        bins.push_back(SegD{at, (uint32_t)sz, 0});
        if (srcs) srcs->push_back(BinSrc{task, i, i, 0});
    }
    return true;
}

}  // namespace ips4o
