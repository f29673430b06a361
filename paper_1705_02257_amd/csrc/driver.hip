// Host side of the gfx950 samplesort: the C ABI declared in include/ips4o.h,
// argument validation, workspace management and the recursion planner.
//
// Recursion (Section 4, first paragraph: large subproblems are partitioned
// by all threads together, the remaining ones are handed out to be sorted
// independently): here every level partitions all current subproblems at
// once, as tasks of one set of launches; subproblems no larger than the
// base-case capacity are collected and sorted by one base-case launch at the
// end; equality buckets are never recursed into (Section 4, many identical
// keys).  The host reads the bucket boundaries back after each level to plan
// the next one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "../../include/ips4o.h"
#include "kernels.hpp"

using namespace ips4o;

namespace {

constexpr uint32_t kDefaultK = 256;
constexpr uint32_t kDefaultKSmall = 128;       // the default below kSmallTopN elements
constexpr uint64_t kSmallTopN = uint64_t(1) << 27;
constexpr size_t kStatsOffset = 1024;        // misc: error word at 0, level counters here
constexpr uint32_t kStatLevels = 16;         // levels with counters of their own (deeper ones share the last)
constexpr size_t kStatsBytes = 32 * 64;      // one level's counters (STAT_SPREAD cache lines)
constexpr uint32_t kDefaultBlockBytes = 2048;
constexpr uint32_t kMaxBlockBytes = 8192;
constexpr uint64_t kDefaultSeed = 0x1705022570ull;
constexpr uint32_t kDefaultSpin = 1u << 16;      // waits last microseconds; this is about 0.1 s
constexpr uint32_t kMaxLevels = 48;
constexpr uint64_t kStripeBlocksMax = 256 * 1024 - 2048;   // blocks per classification stripe
constexpr uint32_t kLevelStripes = 512;      // classification workgroups per level
constexpr uint32_t kMinStripes = 128;         // stripes a task may take whatever its size (see plan_level)
constexpr int kSmallSample = 2048;           // sample capacity of the small sampling instance
constexpr uint32_t kTinyBin = 512;           // u64/f64 base-case bins sorted by one wave
constexpr size_t kExactOrder = 4096;         // stripes sorted exactly by cost for the launch order
constexpr uint32_t kDefaultWorkers = 8192;   // permutation wavefronts per level
constexpr uint32_t kBaseGrid = 1024;
constexpr uint64_t kMaxElements = 1ull << 40;  // n (and a segmented call's total) must stay below
constexpr uint64_t kBufBudgetDiv = 8;        // stripe buffers: at most 1/8 of the elements sorted

size_t elem_size(int dt) {
    switch (dt) {
    case DT_U64: case DT_F64: return 8;
    case DT_PAIR: return 16;
    case DT_QUARTET: return 32;
    case DT_BYTES100: return 100;
    }
    return 0;
}
size_t elem_align(int dt) { return dt == DT_BYTES100 ? 4 : 8; }

uint32_t next_pow2(uint64_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Arena {  // grow-only device buffer
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need) {
        if (need <= bytes) return IPS4O_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        size_t want = need + need / 4;
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return IPS4O_ERR_OUT_OF_MEMORY;
        }
        bytes = want;
        return IPS4O_OK;
    }
    // grow to exactly `need` bytes (no slack), for the large regions
    int ensure_exact(size_t need) {
        if (need <= bytes) return IPS4O_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, need) != hipSuccess) {
            p = nullptr;
            return IPS4O_ERR_OUT_OF_MEMORY;
        }
        bytes = need;
        return IPS4O_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct HostArena {  // grow-only pinned host buffer (fast, asynchronous copies)
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need) {
        if (need <= bytes) return IPS4O_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        size_t want = need + need / 4;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return IPS4O_ERR_OUT_OF_MEMORY;
        }
        bytes = want;
        return IPS4O_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct Carve {  // sequential sub-allocation with 256-byte alignment
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* r = (T*)(base + off);
        off += count * sizeof(T);
        return r;
    }
    static size_t size_of(size_t off, size_t bytes) { return ((off + 255) & ~(size_t)255) + bytes; }
};

}  // namespace

enum { KK_SAMPLE = 0, KK_CLASSIFY, KK_SCAN, KK_FIX, KK_PERMUTE, KK_CLEANUP, KK_BASE, KK_MARK, KK_N };

struct ips4o_handle {
    int device = 0;
    int num_cus = 256;
    void* small = nullptr;    // this device's address of the file-scope array `scratch`
    ips4o_params dflt[5]{};   // per element type: parameters for the fields a call leaves 0
    Arena work;       // per-level descriptors and bucket state (even levels)
    Arena work2;      // the same for odd levels (planned while the previous level runs)
    Arena bufs;       // stripe buffers: partial buffers and side areas, shared by all levels
    Arena misc;       // error word, per-level counters
    Arena segs;       // base-case segment list
    Arena rscratch;   // base-case record scratch
    HostArena hbounds;    // pinned copy of a level's error word, task state and bounds (even levels)
    HostArena hbounds2;   // the same for odd levels
    HostArena hdesc;      // pinned staging of a level's descriptors (even levels)
    HostArena hdesc2;     // the same for odd levels
    hipEvent_t scanned[2] = {nullptr, nullptr};   // a level's bounds have reached the host
    HostArena hsegs;      // pinned staging of the base-case bin list
    hipEvent_t staged = nullptr;   // recorded after the copies out of hsegs of a launch not waited for
    bool staged_pending = false;   // such a launch may still read hsegs and segs
    HostArena hfused;     // pinned staging of a level's fused-cleanup bucket flags
    HostArena hstage;     // pinned copies of caller arrays given in device memory
    ips4o_stats last{};
    ips4o_kernel_stat kstats[KK_N]{};
    std::vector<ips4o_pass_stat> pstats;   // per distribution level, then the base case
    std::vector<hipEvent_t> events;   // pool for IPS4O_FLAG_TIMING
    hipError_t last_hip = hipSuccess;
};

namespace {

// HIP events around every launch of one call (only with IPS4O_FLAG_TIMING).
struct Timer {
    ips4o_handle* h;
    hipStream_t st;
    bool on;
    struct Rec {
        int kind;
        uint32_t pass;
        size_t e0;
        double bytes;
    };
    std::vector<Rec> recs;
    size_t used = 0;
    uint32_t pass = 0;                 // distribution level of the launches recorded now
    std::vector<uint64_t> pass_elems;  // elements partitioned / sorted per pass
    Timer(ips4o_handle* hh, hipStream_t s, bool enabled) : h(hh), st(s), on(enabled) {}
    void set_pass(uint32_t p, uint64_t elements) {
        pass = p;
        if (pass_elems.size() <= p) pass_elems.resize(p + 1, 0);
        pass_elems[p] += elements;
    }
    hipEvent_t ev(size_t i) {
        while (h->events.size() <= i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            h->events.push_back(e);
        }
        return h->events[i];
    }
    int begin(int kind) {
        if (!on) return -1;
        hipEvent_t e = ev(used);
        if (!e || !ev(used + 1)) { on = false; return -1; }
        (void)hipEventRecord(e, st);
        recs.push_back(Rec{kind, pass, used, 0.0});
        used += 2;
        return (int)recs.size() - 1;
    }
    void end(int idx, double bytes) {
        if (!on || idx < 0) return;
        (void)hipEventRecord(h->events[recs[idx].e0 + 1], st);
        recs[idx].bytes = bytes;
    }
    void set_bytes(int idx, double bytes) {
        if (on && idx >= 0) recs[idx].bytes = bytes;
    }
    void add_bytes(int idx, double bytes) {
        if (on && idx >= 0) recs[idx].bytes += bytes;
    }
    void move_to_pass(int idx, uint32_t p) {
        if (on && idx >= 0) recs[idx].pass = p;
    }
    // after the stream has been synchronized
    void finish() {
        for (auto& k : h->kstats) k = ips4o_kernel_stat{};
        h->pstats.clear();
        if (!on) return;
        h->pstats.resize(pass_elems.size());
        for (size_t p = 0; p < pass_elems.size(); ++p) h->pstats[p].elements = pass_elems[p];
        for (const Rec& r : recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h->events[r.e0], h->events[r.e0 + 1]) != hipSuccess) ms = 0.f;
            ips4o_kernel_stat& k = h->kstats[r.kind];
            k.launches += 1;
            k.ms += ms;
            k.alg_bytes += r.bytes;
            if (r.pass < h->pstats.size()) {
                ips4o_pass_stat& ps = h->pstats[r.pass];
                ps.launches += 1;
                ps.ms += ms;
                ps.alg_bytes += r.bytes;
                ps.base_case = r.kind == KK_BASE ? 1u : 0u;
            }
        }
    }
};

}  // namespace

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) {                        \
            h->last_hip = e_;                          \
            return IPS4O_ERR_HIP;                      \
        }                                              \
    } while (0)

namespace {

struct Resolved {
    uint32_t k, b, cap, alpha_x100, stripes, workers, flags, spin;
    uint64_t seed;
    bool k_default;     // the caller left k at 0
};

// The first level's bucket count for an array of m elements when the caller
// leaves k at 0: 256 as in the paper, but 128 below 2^27 elements, where a
// first level of 256 buckets leaves most of its elements in partial buffers
// (u64, best 128 / 256 ms: 2^20 0.245 / 0.273, 2^24 0.86 / 1.00, 2^27
// 4.83 / 4.16).
uint32_t top_k(uint64_t m, const Resolved& R) {
    return R.k_default && m < kSmallTopN ? kDefaultKSmall : R.k;
}

template <int DT>
int resolve(const ips4o_params* p, Resolved* r) {
    const size_t s = sizeof(typename Traits<DT>::Elem);
    ips4o_params d{};
    if (p) d = *p;
    r->k = d.k ? d.k : kDefaultK;
    r->k_default = d.k == 0;
    if (r->k < 2 || r->k > (uint32_t)KT_MAX || (r->k & (r->k - 1))) return IPS4O_ERR_INVALID_ARG;
    // the strict hand-off reads a partition into one bucket as one key
    // value, which needs at least three buckets
    if ((d.flags & IPS4O_FLAG_STRICT) && r->k < 4) return IPS4O_ERR_INVALID_ARG;
    uint32_t bb = d.block_bytes ? d.block_bytes : kDefaultBlockBytes;
    if (bb < s || bb > kMaxBlockBytes) return IPS4O_ERR_INVALID_ARG;
    // b = max(1, 2^floor(log2(block_bytes / s))) (Section 4, Implementation Details)
    uint32_t q = (uint32_t)(bb / s), b = 1;
    while (b * 2 <= q) b *= 2;
    r->b = b;
    uint32_t cap = d.base_cap ? d.base_cap : (uint32_t)Traits<DT>::kBaseCap;
    if (cap < 2 || cap > (uint32_t)Traits<DT>::kBaseCap) return IPS4O_ERR_INVALID_ARG;
    r->cap = cap;
    r->alpha_x100 = d.alpha_x100;
    r->stripes = d.stripes;
    if (d.stripes > STRIPES_PER_TASK_MAX) return IPS4O_ERR_INVALID_ARG;
    // every worker of a task may count as a reader of one bucket at once
    if (d.workers > (WR_MAX_READERS & ~3u)) return IPS4O_ERR_INVALID_ARG;
    r->workers = d.workers ? ((d.workers + 3) & ~3u) : kDefaultWorkers;
    r->flags = d.flags;
    r->spin = d.spin_limit ? d.spin_limit : kDefaultSpin;
    r->seed = d.seed ? d.seed : kDefaultSeed;
    return IPS4O_OK;
}

// The budget of a level's stripe buffers never falls below what one stripe
// per CU needs with buffers for k buckets (Theorem 2: O(k b) per thread), so
// that mid-size sorts keep a classification workgroup per CU.
uint64_t budget_floor(const ips4o_handle* h, const Resolved& R) {
    return 2ull * R.k * R.b * (uint64_t)(h ? h->num_cus : 256);
}

// Blocks of one subproblem must stay below WR_MAX_BLOCKS (the permutation's
// packed pointer word): for a subproblem of m elements the block doubles
// until they do, up to the largest block a permutation wave holds in its
// registers (2048 words).  Returns false if even that block is too small.
template <int DT>
bool scale_block(Resolved* R, uint64_t m) {
    using TR = Traits<DT>;
    constexpr uint64_t wpe = sizeof(typename TR::Elem) / sizeof(typename TR::Word);
    while ((m + R->b - 1) / R->b >= WR_MAX_BLOCKS) {
        if ((uint64_t)R->b * 2 * wpe > 2048) return false;
        R->b *= 2;
    }
    return true;
}

// IPS4O_CLASSIFY_TREE=1: classification by the implicit search tree
// (Section 3) instead of the lookup table, for 8-byte keys (an A/B switch).
// IPS4O_FUSE=1: every call cleans base-case buckets inside the base case
// (as IPS4O_FLAG_FUSE; comparison timing)
bool fuse_on() {
    static int on = -1;
    if (on < 0) {
        const char* e = std::getenv("IPS4O_FUSE");
        on = (e && e[0] == '1') ? 1 : 0;
    }
    return on == 1;
}

bool tree_cls_on() {
    static int on = -1;
    if (on < 0) {
        const char* e = std::getenv("IPS4O_CLASSIFY_TREE");
        on = (e && e[0] == '1') ? 1 : 0;
    }
    return on == 1;
}

// The caller's parameters with every zero field (flags aside) taken from the
// handle's defaults for the element type (ips4o_set_default_params).
const ips4o_params* merged_params(const ips4o_handle* h, int dt, const ips4o_params* p, ips4o_params* tmp) {
    if (!h || dt < 0 || dt > 4) return p;
    const ips4o_params& d = h->dflt[dt];
    *tmp = p ? *p : ips4o_params{};
    if (!tmp->k) tmp->k = d.k;
    if (!tmp->block_bytes) tmp->block_bytes = d.block_bytes;
    if (!tmp->base_cap) tmp->base_cap = d.base_cap;
    if (!tmp->alpha_x100) tmp->alpha_x100 = d.alpha_x100;
    if (!tmp->stripes) tmp->stripes = d.stripes;
    if (!tmp->workers) tmp->workers = d.workers;
    if (!tmp->seed) tmp->seed = d.seed;
    if (!tmp->spin_limit) tmp->spin_limit = d.spin_limit;
    return tmp;
}

bool log_enabled() {
    static int on = -1;
    if (on < 0) {
        const char* e = std::getenv("IPS4O_LOG");
        on = (e && e[0] == '1') ? 1 : 0;
    }
    return on == 1;
}

// Oversampling factor: the paper's 0.2 log2 n (at least 1), raised to the
// LDS sample capacity (at most 32 per bucket).  Every level ends in the base
// case, whose capacity is fixed: the relative spread of bucket sizes falls
// as 1/sqrt(alpha), a bucket just above the capacity costs a whole further
// level, and sampling costs little on the GPU.  An explicit alpha applies
// to every level as given.
template <int DT>
uint32_t alpha_for(uint64_t m, const Resolved& R, uint32_t k) {
    const uint32_t smax = (uint32_t)sample_max<typename Traits<DT>::Key>();
    uint32_t a;
    if (R.alpha_x100) a = std::max(1u, R.alpha_x100 / 100);
    else {
        a = std::max<uint32_t>(1u, (uint32_t)std::floor(0.2 * std::log2((double)std::max<uint64_t>(m, 2))));
        a = std::max(a, std::min(32u, smax / k));
    }
    while (a > 1 && (uint64_t)a * k > (uint64_t)smax) --a;
    return a;
}

// splitmix64 finaliser, used to derive per-task sampling streams
uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Host copy of the per-task splitter state for caller-given splitters.
template <int DT>
struct HostTree {
    using Key = typename Traits<DT>::Key;
    std::vector<Key> tree, spl;
    TaskS ts{};
};

template <int DT>
int build_host_tree(const void* h_split, uint32_t m, int eq, uint64_t nseg, uint32_t b,
                    HostTree<DT>* out) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    using Elem = typename TR::Elem;
    if (m < 1 || m > (uint32_t)KGIVEN_MAX || !h_split) return IPS4O_ERR_INVALID_ARG;
    std::vector<Key> keys(m);
    const char* src = (const char*)h_split;
    for (uint32_t i = 0; i < m; ++i) {
        Elem e;
        std::memcpy(&e, src + (size_t)i * sizeof(Elem), sizeof(Elem));
        keys[i] = TR::key(e);
        if (i > 0 && keys[i] < keys[i - 1]) return IPS4O_ERR_INVALID_ARG;
    }
    std::vector<Key> u;
    if (eq) {
        for (uint32_t i = 0; i < m; ++i)
            if (u.empty() || !(u.back() == keys[i])) u.push_back(keys[i]);
    } else {
        u = keys;
    }
    const uint32_t nu = (uint32_t)u.size();
    uint32_t kt = next_pow2((uint64_t)nu + 1);
    if (kt < 2) kt = 2;
    out->spl.assign(kt, u.back());
    for (uint32_t i = 0; i < nu; ++i) out->spl[i] = u[i];
    out->tree.assign(kt, u.back());
    for (uint32_t i = 1; i < kt; ++i) {
        uint32_t l = 31u - (uint32_t)__builtin_clz(i), p = i - (1u << l);
        uint32_t idx = ((2 * p + 1) * kt) >> (l + 1);
        out->tree[i] = out->spl[idx - 1];
    }
    TaskS& s = out->ts;
    s.K = eq ? 2 * nu + 1 : nu + 1;
    s.kt = kt;
    s.eq = eq ? 1 : 0;
    s.nuniq = nu;
    s.nblocks = (uint32_t)((nseg + b - 1) / b);
    s.ovf_bucket = NO_BUCKET;
    return IPS4O_OK;
}

// One level: device pointers carved from the workspace, host plan.
template <int DT>
struct Level {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    using Elem = typename TR::Elem;
    std::vector<TaskD> tasks;
    std::vector<StripeD> stripes;
    std::vector<uint32_t> order;     // classification launch order
    uint32_t total_slots = 0, total_tree = 0, total_workers = 0;
    uint64_t total_buf = 0, total_cnt = 0;
    Ctx<DT> c{};
    uint8_t* fused_flags = nullptr;  // [total_slots]: set in c.fused when the base case cleans buckets
};

// Bucket count for a subproblem of m elements: enough leaves that the
// average bucket is half the base-case capacity.  Above the capacity this
// gives k >= 4, so at least three splitters: a subproblem of one or two
// distinct keys then always repeats a splitter, equality buckets switch on
// and the level makes progress (with a single splitter all keys could stay
// in one bucket, level after level).
// Below the first level k is at most kDeepK: the stripe buffers of a level
// grow with k, and on the second level of 2^30 keys k = 1024 needed either
// twice the buffers or half the stripes (its classification then took
// 2.4 ms longer); with at most 512 buckets a small third level now and then
// costs about 0.1 ms.
// A subproblem that kDeepK buckets would leave at more than 3/4 of the
// capacity on average takes 2 kDeepK instead: otherwise most of its buckets
// overflow into a third level (2^31 u64 keys, level-2 subproblems of 8 M:
// 68.8 ms with 512, most of it a large third level).
constexpr uint32_t kDeepK = 512;
static_assert(2 * kDeepK <= (uint32_t)KT_MAX, "deep bucket counts fit the tree");
uint32_t adaptive_k(uint64_t m, const Resolved& R) {
    const uint64_t want = (2 * m + R.cap - 1) / R.cap;
    if (want > (uint64_t)kDeepK * 3 / 2) return 2 * kDeepK;
    return std::min<uint32_t>(kDeepK, std::max<uint32_t>(2u, next_pow2(want)));
}

// `first`: the top level of one array, whose k is the caller's (or the
// default); `segmented`: the top level of many segments, each with the
// adaptive k but at most the caller's.
// `kbuf_given`: the bucket count of caller-given splitters (else a task's
// buffers hold k buckets: sampling keeps K <= k).
template <int DT>
void plan_level(Level<DT>& L, const std::vector<Seg>& segs, const Resolved& R, uint32_t level,
                bool first, uint32_t k_given, bool segmented = false, uint32_t kbuf_given = 0,
                uint64_t buf_budget = 0) {
    const uint32_t b = R.b;
    uint64_t total_m = 0, total_blocks = 0;
    for (const Seg& s : segs) {
        total_m += s.m;
        total_blocks += (s.m + b - 1) / b;
    }
    L.tasks.clear();
    L.stripes.clear();
    L.tasks.reserve(segs.size());
    L.stripes.reserve(segs.size() + kLevelStripes);
    // Stripes per task: kLevelStripes shared out in proportion to the task
    // sizes (largest remainders, at least one each), so that a level that
    // fits in one round of workgroups per CU leaves no partial last round.
    std::vector<uint64_t> share(segs.size(), 1);
    if (segs.size() < kLevelStripes) {
        std::vector<std::pair<double, size_t>> rem;
        uint64_t given = 0;
        for (size_t i = 0; i < segs.size(); ++i) {
            const double q = (double)kLevelStripes * (double)segs[i].m / (double)total_m;
            share[i] = std::max<uint64_t>(1, (uint64_t)q);
            given += share[i];
            rem.push_back({q - std::floor(q), i});
        }
        // the largest remainders get one more (only as many as are left)
        const size_t extra = std::min<size_t>(rem.size(), given < kLevelStripes ? kLevelStripes - given : 0);
        if (extra)
            std::partial_sort(rem.begin(), rem.begin() + extra, rem.end(),
                              [](const auto& a, const auto& b) { return a.first > b.first; });
        for (size_t r = 0; r < extra; ++r) share[rem[r].second] += 1;
    }
    // Permutation workers per task, in groups of four (one workgroup):
    // R.workers / 4 groups shared out in proportion to the task's blocks
    // (largest remainders, at least one group each, no more groups than it
    // takes to give every block a worker), so that a level's workers fit the one round of workgroups
    // that R.workers is sized for; a task whose workers wait for a second
    // round only starts once the first round has drained.
    std::vector<uint64_t> wgroups(segs.size(), 1);
    {
        const uint64_t G = std::max<uint32_t>(1u, R.workers / 4);
        std::vector<std::pair<double, size_t>> rem;
        uint64_t given = 0;
        for (size_t i = 0; i < segs.size(); ++i) {
            const uint64_t nb = (segs[i].m + b - 1) / b;
            const uint64_t gmax = std::max<uint64_t>(1, (nb + 3) / 4);
            const double q = (double)G * (double)nb / (double)std::max<uint64_t>(1, total_blocks);
            wgroups[i] = std::min<uint64_t>(gmax, std::max<uint64_t>(1, (uint64_t)q));
            given += wgroups[i];
            if (wgroups[i] < gmax) rem.push_back({q - std::floor(q), i});
        }
        // the largest remainders get one more group (only as many as are
        // left: with more tasks than groups, none)
        const size_t extra = std::min<size_t>(rem.size(), given < G ? G - given : 0);
        if (extra)
            std::partial_sort(rem.begin(), rem.begin() + extra, rem.end(),
                              [](const auto& a, const auto& b) { return a.first > b.first; });
        for (size_t r = 0; r < extra; ++r) wgroups[rem[r].second] += 1;
    }
    // bucket count, buffer count and stripes of every task
    const size_t T = segs.size();
    std::vector<uint32_t> kk(T), kb(T);
    std::vector<uint64_t> nss(T), nsmin(T);
    for (size_t i = 0; i < T; ++i) {
        const Seg& s = segs[i];
        uint32_t k;
        if (k_given) k = k_given;
        else if (segmented) k = std::min(R.k, adaptive_k(s.m, R));
        else if (first) k = top_k(s.m, R);
        else k = adaptive_k(s.m, R);
        kk[i] = k;
        // buffers for k buckets; for 2k (up to KMAX) at the top level and
        // where the keys are known to repeat, so that the sample's equality
        // buckets (2u + 1 of them) need no thinning
        kb[i] = kbuf_given ? kbuf_given
                           : ((first || s.dup) ? std::min<uint32_t>(2 * k, (uint32_t)KMAX) : k);
        const uint64_t nb = (s.m + b - 1) / b;
        // stripes: the task's share, but enough blocks per stripe to keep
        // the partial buffers small (at least 8 buffer sets of k blocks
        // each) -- except that a task may take up to kMinStripes stripes of
        // 32 blocks or more: below about 2^26 keys the first rule leaves
        // the GPU idle (2^20 u64 keys: 2 stripes, 0.71 ms; 128 stripes,
        // 0.27 ms; 2^24: 32 stripes 1.49 ms, 128 stripes 1.27 ms), while the
        // partial buffers of such small tasks cost little
        uint64_t by_size = std::max<uint64_t>(nb / (8ull * k), std::min<uint64_t>(kMinStripes, nb / 32));
        uint64_t ns = std::max<uint64_t>(1, std::min(by_size, share[i]));
        if (first && !segmented && R.stripes) ns = R.stripes;
        // the classification's block lists fit its LDS for stripes of up
        // to kStripeBlocksMax blocks
        nsmin[i] = std::min<uint64_t>((nb + kStripeBlocksMax - 1) / kStripeBlocksMax,
                                      std::min<uint64_t>(nb, STRIPES_PER_TASK_MAX));
        ns = std::max<uint64_t>(ns, nsmin[i]);
        nss[i] = std::min<uint64_t>(ns, std::min<uint64_t>(nb, STRIPES_PER_TASK_MAX));
        nsmin[i] = std::max<uint64_t>(1, nsmin[i]);
    }
    // memory budget of the stripe buffers (Theorem 2: O(k b) per
    // workgroup): at most buf_budget elements, or what one stripe per task
    // needs.  Over budget, first the top level's tasks go back to k buffers,
    // then the tasks with the largest buffers per stripe get fewer stripes,
    // then repeating-key tasks go back to k buffers (their sample then thins
    // its equality buckets).
    if (buf_budget) {
        auto total = [&]() {
            uint64_t t = 0;
            for (size_t i = 0; i < T; ++i) t += nss[i] * 2 * kb[i] * (uint64_t)b;
            return t;
        };
        uint64_t tot = total();
        if (tot > buf_budget) {
            // tasks by buffer count, largest first, ties in task order (a
            // counting sort: kb is a power of two up to KMAX, and a level
            // may hold tens of thousands of tasks)
            std::vector<size_t> idx(T);
            {
                constexpr int NC = 12;                          // log2 of kb: 0 .. 11
                size_t start[NC + 1] = {0};
                auto cls = [&](size_t i) { return NC - 1 - std::min(NC - 1, 31 - __builtin_clz(std::max(1u, kb[i]))); };
                for (size_t i = 0; i < T; ++i) ++start[cls(i) + 1];
                for (int c = 0; c < NC; ++c) start[c + 1] += start[c];
                for (size_t i = 0; i < T; ++i) idx[start[cls(i)]++] = i;
            }
            auto cut_kbuf = [&](bool dup) {
                for (size_t i : idx) {
                    if (tot <= buf_budget) break;
                    if (kb[i] > kk[i] && !kbuf_given && (segs[i].dup != 0) == dup) {
                        tot -= nss[i] * 2 * (uint64_t)(kb[i] - kk[i]) * b;
                        kb[i] = kk[i];
                    }
                }
            };
            // one stripe at a time from the task whose stripes are shortest,
            // so that stripe lengths stay balanced (cutting the first tasks
            // in turn left a segmented sort's largest segments with a few
            // huge stripes: 40 segments of 2^10..2^26 keys spent 33 ms in
            // the classification)
            auto cut_stripes = [&]() {
                using Ent = std::pair<double, size_t>;         // (blocks per stripe, task)
                std::priority_queue<Ent, std::vector<Ent>, std::greater<Ent>> q;
                for (size_t i = 0; i < T; ++i)
                    if (nss[i] > nsmin[i]) q.push({(double)((segs[i].m + b - 1) / b) / (double)nss[i], i});
                while (tot > buf_budget && !q.empty()) {
                    const size_t i = q.top().second;
                    q.pop();
                    nss[i] -= 1;
                    tot -= 2 * kb[i] * (uint64_t)b;
                    if (nss[i] > nsmin[i]) q.push({(double)((segs[i].m + b - 1) / b) / (double)nss[i], i});
                }
            };
            // the top level's 2k buffers are insurance against repeated
            // keys: they go first (2^27 u64 Uniform 4.57 -> 4.42 ms); a
            // subproblem whose keys are known to repeat keeps them longer
            // than its stripes (2^30 u64 EightDup 34.3 -> 32.5 ms)
            cut_kbuf(false);
            cut_stripes();
            cut_kbuf(true);
        }
    }
    uint32_t slot = 0, treeb = 0, wk = 0;
    uint64_t bufoff = 0, cntoff = 0;
    for (size_t i = 0; i < segs.size(); ++i) {
        const Seg& s = segs[i];
        TaskD t{};
        t.off = s.off;
        t.m = s.m;
        const uint32_t k = kk[i];
        t.k = k;
        t.kbuf = kb[i];
        t.alpha = alpha_for<DT>(s.m, R, k);
        t.seed = mix64(R.seed ^ mix64(((uint64_t)level << 48) ^ s.off));
        const uint64_t nb = (s.m + b - 1) / b;
        const uint64_t ns = nss[i];
        t.stripe_begin = (uint32_t)L.stripes.size();
        t.nstripes = (uint32_t)ns;
        t.cnt_begin = (uint32_t)cntoff;
        cntoff += ns * t.kbuf;
        for (uint64_t q = 0; q < ns; ++q) {
            StripeD sd{};
            sd.task = (uint32_t)i;
            sd.blk_begin = (uint32_t)(nb * q / ns);
            sd.blk_end = (uint32_t)(nb * (q + 1) / ns);
            sd.buf_off = bufoff;
            bufoff += (uint64_t)2 * t.kbuf * b;   // partial buffers and side area, kbuf blocks each
            L.stripes.push_back(sd);
        }
        const uint64_t w = 4 * wgroups[i];
        t.worker_begin = wk;
        t.nworkers = (uint32_t)w;
        wk += (uint32_t)w;
        t.slot_begin = slot;
        slot += t.kbuf;
        t.tree_begin = treeb;
        treeb += k;
        L.tasks.push_back(t);
    }
    // classification launch order: longest stripes first, so that the
    // workgroups dispatched last are the short ones (longest processing
    // time first).  A stripe's cost is its length plus about 2k blocks:
    // the blocks filled in the side area, moved into the stripe at the end,
    // and the partly filled blocks moved to the partial buffers.
    // Up to kExactOrder stripes are sorted exactly (ties keep the stripe
    // order); above that (many small tasks) by classes of a quarter octave
    // of cost, which is as good for balance and linear in the stripe count.
    const size_t S = L.stripes.size();
    std::vector<uint64_t> cost(S);
    for (size_t q = 0; q < S; ++q) {
        const StripeD& sd = L.stripes[q];
        const TaskD& td = L.tasks[sd.task];
        const uint64_t e = std::min<uint64_t>((uint64_t)sd.blk_end * b, td.m) - (uint64_t)sd.blk_begin * b;
        cost[q] = e + 2 * std::min<uint64_t>(e, (uint64_t)td.k * b);
    }
    L.order.resize(S);
    for (size_t q = 0; q < S; ++q) L.order[q] = (uint32_t)q;
    if (S <= kExactOrder) {
        std::stable_sort(L.order.begin(), L.order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    } else {
        constexpr int NCLS = 4 * 64;
        auto cls = [&](uint64_t c) {          // 4 log2(c), rounded down, larger cost -> smaller class
            if (c == 0) return NCLS - 1;
            const int l = 63 - __builtin_clzll(c);
            const int frac = l >= 2 ? (int)((c >> (l - 2)) & 3) : (int)((c << (2 - l)) & 3);
            return NCLS - 1 - (4 * l + frac);
        };
        std::vector<uint32_t> start(NCLS + 1, 0);
        for (size_t q = 0; q < S; ++q) ++start[cls(cost[q]) + 1];
        for (int i = 0; i < NCLS; ++i) start[i + 1] += start[i];
        for (size_t q = 0; q < S; ++q) L.order[start[cls(cost[q])]++] = (uint32_t)q;
    }
    L.total_slots = slot;
    L.total_tree = treeb;
    L.total_workers = wk;
    L.total_buf = bufoff;
    L.total_cnt = cntoff;
}

template <int DT>
size_t level_bytes(const Level<DT>& L, uint32_t b) {
    using Key = typename Traits<DT>::Key;
    using Elem = typename Traits<DT>::Elem;
    const size_t T = L.tasks.size(), S = L.stripes.size();
    size_t off = 0;
    auto add = [&](size_t bytes) { off = Carve::size_of(off, bytes); };
    add(T * sizeof(TaskD));
    add(S * sizeof(StripeD));
    add(S * sizeof(uint32_t));
    add(T * sizeof(TaskS));
    add((L.total_slots + T) * sizeof(uint64_t));
    add(L.total_tree * sizeof(Key));
    add(L.total_tree * sizeof(Key));
    add((L.total_slots + T) * sizeof(uint32_t));
    add(L.total_slots * sizeof(BucketSlot));
    add(L.total_cnt * sizeof(uint32_t));
    add(S * sizeof(uint32_t));
    add(L.total_slots);
    return off + 256;
}

template <int DT>
void carve_level(Level<DT>& L, void* base, void* misc, void* data, void* bufs, const Resolved& R,
                 uint32_t level = 0) {
    using Key = typename Traits<DT>::Key;
    using Elem = typename Traits<DT>::Elem;
    const size_t T = L.tasks.size(), S = L.stripes.size();
    Carve cv(base);
    Ctx<DT>& c = L.c;
    c.data = (Elem*)data;
    // the host-written descriptors next to each other (one copy in), then
    // the task state and bounds the host reads back (one copy out)
    c.tasks = cv.take<TaskD>(T);
    c.stripes = cv.take<StripeD>(S);
    c.order = cv.take<uint32_t>(S);
    c.ts = cv.take<TaskS>(T);
    c.bounds = cv.take<uint64_t>(L.total_slots + T);
    c.tree = cv.take<Key>(L.total_tree);
    c.spl = cv.take<Key>(L.total_tree);
    c.delim = cv.take<uint32_t>(L.total_slots + T);
    c.slots = cv.take<BucketSlot>(L.total_slots);
    c.counts = cv.take<uint32_t>(L.total_cnt);
    c.stripe_full = cv.take<uint32_t>(S);
    L.fused_flags = cv.take<uint8_t>(L.total_slots);
    c.fused = nullptr;
    c.bufs = (Elem*)bufs;
    c.ntasks = (uint32_t)T;
    c.nstripes = (uint32_t)S;
    char* m = (char*)misc;
    c.err = (uint32_t*)m;
    c.stats = (unsigned long long*)(m + kStatsOffset + std::min(level, kStatLevels - 1) * kStatsBytes);
    c.b = R.b;
    c.spin_limit = R.spin;
    c.total_workers = L.total_workers;
    c.total_slots = L.total_slots;
    c.skip_inplace = (R.flags & IPS4O_FLAG_NO_SKIP) ? 0u : 1u;
    // classification in virtual tiles of two tiles below the first level,
    // where k = 512 or 1024 leaves runs of 8 to 16 keys per bucket and tile
    // (level 2 of 2^30 keys 7.7 -> 7.0 ms); on the first level (k = 256,
    // runs of 32) they gain nothing and slow presorted inputs down
    c.vtile = level >= 1 ? 1u : 0u;
    c.tree_cls = tree_cls_on() ? 1u : 0u;
}

// Kernel shapes per element type.
// CNT/EPT: classification workgroup size and elements per thread per tile;
// BNT/BVT: base-case workgroup size and items per thread (BNT*BVT is the
// base-case capacity of the element type).
template <int DT> struct Shape;
template <> struct Shape<DT_U64> { static constexpr int CNT = 1024, EPT = 8, BNT = 1024, BVT = 16; };
template <> struct Shape<DT_F64> { static constexpr int CNT = 1024, EPT = 8, BNT = 1024, BVT = 16; };
template <> struct Shape<DT_PAIR> { static constexpr int CNT = 1024, EPT = 4, BNT = 1024, BVT = 8; };
template <> struct Shape<DT_QUARTET> { static constexpr int CNT = 1024, EPT = 2, BNT = 512, BVT = 8; };
template <> struct Shape<DT_BYTES100> { static constexpr int CNT = 512, EPT = 1, BNT = 512, BVT = 8; };

template <int DT, int WPL>
hipError_t launch_permute_wpl(const Ctx<DT>& c, hipStream_t st) {
    uint32_t grid = (c.total_workers + 3) / 4;
    hipLaunchKernelGGL((k_permute<DT, WPL>), dim3(grid), dim3(256), 0, st, c);
    return hipGetLastError();
}

template <int DT>
hipError_t launch_permute(const Ctx<DT>& c, hipStream_t st) {
    using TR = Traits<DT>;
    const uint32_t words = c.b * (uint32_t)(sizeof(typename TR::Elem) / sizeof(typename TR::Word));
    const uint32_t wpl = (words + 63) / 64;
    if (wpl <= 4) return launch_permute_wpl<DT, 4>(c, st);
    if (wpl <= 8) return launch_permute_wpl<DT, 8>(c, st);
    if (wpl <= 16) return launch_permute_wpl<DT, 16>(c, st);
    return launch_permute_wpl<DT, 32>(c, st);
}

struct LevelMarks {    // timer records whose byte counts are known after the level
    int fix = -1, permute = -1, cleanup = -1;
};

// First half of a level: descriptors, sampling, classification, bounds.
// With `stage` the descriptors go through that pinned buffer, so the copies
// do not wait for earlier work on the stream (the buffer must not be
// reused before they ran).
template <int DT>
int launch_level_head(ips4o_handle* h, Level<DT>& L, hipStream_t st, const HostTree<DT>* given, Timer& tm,
                      bool check, HostArena* stage) {
    using Key = typename Traits<DT>::Key;
    using Elem = typename Traits<DT>::Elem;
    constexpr int CNT = Shape<DT>::CNT, EPT = Shape<DT>::EPT;
    Ctx<DT>& c = L.c;
    const size_t T = L.tasks.size(), S = L.stripes.size();
    const void* src_tasks = L.tasks.data();
    const void* src_stripes = L.stripes.data();
    const void* src_order = L.order.data();
    if (stage) {
        // the device layout (tasks, stripes, order, carved in that order)
        // mirrored in the staging buffer: one copy
        const size_t bt = T * sizeof(TaskD), bs = S * sizeof(StripeD), bo = S * sizeof(uint32_t);
        const size_t os = (size_t)((const char*)c.stripes - (const char*)c.tasks);
        const size_t oo = (size_t)((const char*)c.order - (const char*)c.tasks);
        int rc = stage->ensure(oo + bo);
        if (rc) return rc;
        char* p = (char*)stage->p;
        std::memcpy(p, L.tasks.data(), bt);
        std::memcpy(p + os, L.stripes.data(), bs);
        std::memcpy(p + oo, L.order.data(), bo);
        HIP_TRY(hipMemcpyAsync((void*)c.tasks, p, oo + bo, hipMemcpyHostToDevice, st));
    } else {
        HIP_TRY(hipMemcpyAsync((void*)c.tasks, src_tasks, T * sizeof(TaskD), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync((void*)c.stripes, src_stripes, S * sizeof(StripeD), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync((void*)c.order, src_order, S * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    }
    if (given) {
        HIP_TRY(hipMemcpyAsync(c.tree, given->tree.data(), given->tree.size() * sizeof(Key), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(c.spl, given->spl.data(), given->spl.size() * sizeof(Key), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(c.ts, &given->ts, sizeof(TaskS), hipMemcpyHostToDevice, st));
    } else {
        // levels whose samples are all small (many small tasks) take an
        // instance with a small LDS sample array, several per CU
        uint64_t pmax = 1;
        for (const TaskD& t : L.tasks) pmax = std::max<uint64_t>(pmax, next_pow2((uint64_t)t.alpha * t.k - 1));
        int r = tm.begin(KK_SAMPLE);
        if (pmax <= kSmallSample)
            hipLaunchKernelGGL((k_sample<DT, 256, kSmallSample>), dim3(T), dim3(256), 0, st, c);
        else
            hipLaunchKernelGGL((k_sample<DT, 1024>), dim3(T), dim3(1024), 0, st, c);
        HIP_TRY(hipGetLastError());
        tm.end(r, 0.0);
    }
    uint64_t level_m = 0;
    for (const TaskD& t : L.tasks) level_m += t.m;
    const size_t cls_lds = sizeof(ClassifyLds<DT, CNT, EPT>);
    HIP_TRY(hipFuncSetAttribute((const void*)k_classify<DT, CNT, EPT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)cls_lds));
    int r = tm.begin(KK_CLASSIFY);
    hipLaunchKernelGGL((k_classify<DT, CNT, EPT>), dim3(S), dim3(CNT), cls_lds, st, c);
    HIP_TRY(hipGetLastError());
    tm.end(r, 2.0 * sizeof(Elem) * (double)level_m);
    if (check) {
        hipLaunchKernelGGL((k_check_classify<DT, 256>), dim3(S), dim3(256), 0, st, c);
        HIP_TRY(hipGetLastError());
    }
    r = tm.begin(KK_SCAN);
    hipLaunchKernelGGL((k_scan<DT, 1024>), dim3(T), dim3(1024), 0, st, c);
    HIP_TRY(hipGetLastError());
    tm.end(r, 0.0);
    return IPS4O_OK;
}

// Cleanup of a level: overhangs to the side area, then the free positions
// of every bucket filled, except the buckets flagged in c.fused (cleaned by
// the fused base case).
template <int DT>
int launch_level_cleanup(Level<DT>& L, hipStream_t st, Timer& tm, LevelMarks& mk, hipError_t* herr) {
    Ctx<DT>& c = L.c;
    const uint32_t T = (uint32_t)L.tasks.size();
    // a bucket has a source (under a block) per stripe, plus the overhang
    // and the overflow block; with many stripes the sources are split over
    // several workgroups
    uint32_t kmax = 0, nsmax = 1;
    for (const TaskD& t : L.tasks) {
        kmax = std::max(kmax, t.kbuf);
        nsmax = std::max(nsmax, t.nstripes);
    }
    const uint32_t parts = std::min<uint32_t>(32, std::max<uint32_t>(1, (nsmax + 2) / 16));
    mk.cleanup = tm.begin(KK_CLEANUP);
    for (uint32_t t0 = 0; t0 < T; t0 += 65535) {
        const uint32_t nt = std::min<uint32_t>(65535, T - t0);
        hipLaunchKernelGGL((k_overhang<DT, 256>), dim3((kmax + 3) / 4, nt), dim3(256), 0, st, c, t0);
        if ((*herr = hipGetLastError()) != hipSuccess) return IPS4O_ERR_HIP;
    }
    for (uint32_t t0 = 0; t0 < T; t0 += 65535) {
        const uint32_t nt = std::min<uint32_t>(65535, T - t0);
        if (nsmax + 2 <= 64)
            hipLaunchKernelGGL((k_cleanup_narrow<DT>), dim3((kmax + 3) / 4, nt), dim3(256), 0, st, c, t0);
        else
            hipLaunchKernelGGL((k_cleanup<DT, 256>), dim3(kmax * parts, nt), dim3(256), 0, st, c, parts, t0);
        if ((*herr = hipGetLastError()) != hipSuccess) return IPS4O_ERR_HIP;
    }
    tm.end(mk.cleanup, 0.0);
    return IPS4O_OK;
}

// Second half of a level: empty-block fix, block permutation and (unless
// the caller enqueues it later, with launch_level_cleanup) the cleanup.
template <int DT>
int launch_level_tail(ips4o_handle* h, Level<DT>& L, hipStream_t st, Timer& tm, LevelMarks& mk, bool check,
                      bool cleanup = true) {
    Ctx<DT>& c = L.c;
    const uint32_t T = (uint32_t)L.tasks.size();
    mk.fix = tm.begin(KK_FIX);
    {
        // one workgroup per bucket: 16 waves when tasks have many stripes
        // (many holes per bucket), else one wave
        uint32_t nsmax = 1, kmax = 0;
        for (const TaskD& t : L.tasks) {
            nsmax = std::max(nsmax, t.nstripes);
            kmax = std::max(kmax, t.kbuf);
        }
        for (uint32_t t0 = 0; t0 < T; t0 += 65535) {
            const uint32_t nt = std::min<uint32_t>(65535, T - t0);
            if (nsmax > 64)
                hipLaunchKernelGGL((k_fix_empty<DT, 1024, STRIPES_PER_TASK_MAX>), dim3(kmax, nt), dim3(1024), 0, st, c, t0);
            else
                hipLaunchKernelGGL((k_fix_empty<DT, 64, 64>), dim3(kmax, nt), dim3(64), 0, st, c, t0);
            HIP_TRY(hipGetLastError());
        }
    }
    HIP_TRY(hipGetLastError());
    tm.end(mk.fix, 0.0);
    mk.permute = tm.begin(KK_PERMUTE);
    HIP_TRY(launch_permute<DT>(c, st));
    tm.end(mk.permute, 0.0);
    if (check) {
        uint32_t kmax = 0;
        for (const TaskD& t : L.tasks) kmax = std::max(kmax, t.kbuf);
        for (uint32_t t0 = 0; t0 < T; t0 += 65535) {
            const uint32_t nt = std::min<uint32_t>(65535, T - t0);
            hipLaunchKernelGGL((k_check_permute<DT, 256>), dim3(kmax, nt), dim3(256), 0, st, c, t0);
            HIP_TRY(hipGetLastError());
        }
    }
    if (!cleanup) return IPS4O_OK;
    return launch_level_cleanup<DT>(L, st, tm, mk, &h->last_hip);
}

// Strictly in-place hand-off (Section 4.6): every bucket's largest element
// moved to its first entry, then each task's bucket boundaries overwritten
// by the ones a walk over those marks finds (k_walk), so that the next
// level is planned from what the data holds.  `elems`: the level's elements
// (read once by the marking).
template <int DT>
int launch_mark_walk(Level<DT>& L, hipStream_t st, Timer& tm, uint64_t elems, uint64_t cap, hipError_t* herr) {
    Ctx<DT>& c = L.c;
    const uint32_t T = (uint32_t)L.tasks.size();
    uint32_t kmax = 0;
    uint64_t ksum = 0;
    for (const TaskD& t : L.tasks) {
        kmax = std::max(kmax, t.kbuf);
        ksum += t.k;
    }
    // a workgroup per bucket where buckets are small; buckets of a million
    // elements and more (the top level) are cut into parts of about 2^18
    // elements whose maxima go to the stripe buffers, free once the cleanup
    // has run (the next level's classification fills them after the walk)
    using Key = typename Traits<DT>::Key;
    const uint64_t avg = elems / std::max<uint64_t>(ksum, 1);
    const uint32_t P = (uint32_t)std::min<uint64_t>(64, (avg + (1u << 18) - 1) >> 18);
    const size_t part_key_bytes = ((size_t)L.total_slots * P * sizeof(Key) + 255) & ~(size_t)255;
    const size_t part_pos_bytes = ((size_t)L.total_slots * P * sizeof(uint64_t) + 255) & ~(size_t)255;
    const bool parts = avg >= (1u << 20) && 2 * (part_key_bytes + part_pos_bytes) <=
                                                (size_t)L.total_buf * sizeof(typename Traits<DT>::Elem);
    // maxima, their positions, minima, their positions
    Key* pk = (Key*)c.bufs;
    uint64_t* pp = (uint64_t*)((char*)c.bufs + part_key_bytes);
    Key* qk = (Key*)((char*)pp + part_pos_bytes);
    uint64_t* qp = (uint64_t*)((char*)qk + part_key_bytes);
    const int r = tm.begin(KK_MARK);
    for (uint32_t t0 = 0; t0 < T; t0 += 65535) {
        const uint32_t nt = std::min<uint32_t>(65535, T - t0);
        if (parts) {
            hipLaunchKernelGGL((k_mark_part<DT, 256, true>), dim3(kmax * P, nt), dim3(256), 0, st, c.data,
                               c.bounds, c.tasks, c.ts, t0, P, pk, pp, qk, qp, c.err);
            if ((*herr = hipGetLastError()) != hipSuccess) return IPS4O_ERR_HIP;
            hipLaunchKernelGGL((k_mark_pick<DT, true>), dim3((kmax + 255) / 256, nt), dim3(256), 0, st, c.data,
                               c.bounds, c.tasks, c.ts, t0, P, pk, pp, qk, qp);
        } else {
            hipLaunchKernelGGL((k_mark_max<DT, 256, true>), dim3(std::max(kmax, 1u), nt), dim3(256), 0, st,
                               c.data, (uint64_t)0, c.bounds, c.tasks, c.ts, t0, 0u, c.err);
        }
        if ((*herr = hipGetLastError()) != hipSuccess) return IPS4O_ERR_HIP;
    }
    hipLaunchKernelGGL((k_walk<DT, true>), dim3((T + 3) / 4), dim3(256), 0, st, c.data, c.bounds, c.tasks, c.ts,
                       T, cap, c.err);
    if ((*herr = hipGetLastError()) != hipSuccess) return IPS4O_ERR_HIP;
    tm.end(r, (double)sizeof(typename Traits<DT>::Elem) * (double)elems);
    return IPS4O_OK;
}

template <int DT>
int run_level(ips4o_handle* h, Level<DT>& L, hipStream_t st, const HostTree<DT>* given, Timer& tm,
              LevelMarks& mk, bool check) {
    int rc = launch_level_head<DT>(h, L, st, given, tm, check, nullptr);
    if (rc) return rc;
    return launch_level_tail<DT>(h, L, st, tm, mk, check);
}

// bytes of the launches whose amount of work is counted on the device
template <int DT>
void account_level(Timer& tm, const LevelMarks& mk, const unsigned long long* now,
                   const unsigned long long* before, uint32_t b) {
    const double s = (double)sizeof(typename Traits<DT>::Elem);
    tm.set_bytes(mk.permute, 2.0 * s * b * (double)(now[0] - before[0]));
    tm.set_bytes(mk.cleanup, 2.0 * s * (double)(now[2] - before[2]));
    tm.set_bytes(mk.fix, 2.0 * s * b * (double)(now[3] - before[3]));
}

int check_device_error(ips4o_handle* h, hipStream_t st) {
    uint32_t err[53] = {0};
    HIP_TRY(hipMemcpyAsync(err, h->misc.p, sizeof(err), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    h->last.fault_bits = err[0];
    if (err[0] && log_enabled())
        std::fprintf(stderr, "[ips4o] device fault bits %u, first: code %u (%u, %u, %u)\n", err[0], err[48],
                     err[49], err[50], err[51]);
    return err[0] ? IPS4O_ERR_DEVICE_FAULT : IPS4O_OK;
}

int reset_misc(ips4o_handle* h, hipStream_t st) {
    static_assert(kStatsBytes == STAT_SPREAD * 64, "counter block size");
    int rc = h->misc.ensure(kStatsOffset + kStatLevels * kStatsBytes);
    if (rc) return rc;
    HIP_TRY(hipMemsetAsync(h->misc.p, 0, kStatsOffset + kStatLevels * kStatsBytes, st));
    return IPS4O_OK;
}

// Read back the per-task state and bounds of a finished level.
template <int DT>
int read_level(ips4o_handle* h, Level<DT>& L, hipStream_t st, std::vector<TaskS>& ts,
               const uint64_t*& bounds, unsigned long long* stats) {
    const size_t T = L.tasks.size();
    ts.resize(T);
    const size_t nb = L.total_slots + T;
    int rc0 = h->hbounds.ensure(nb * sizeof(uint64_t));
    if (rc0) return rc0;
    HIP_TRY(hipMemcpyAsync(ts.data(), L.c.ts, T * sizeof(TaskS), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h->hbounds.p, L.c.bounds, nb * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    bounds = (const uint64_t*)h->hbounds.p;
    unsigned long long spread[STAT_SPREAD * 8];
    HIP_TRY(hipMemcpyAsync(spread, L.c.stats, sizeof(spread), hipMemcpyDeviceToHost, st));
    const int rc = check_device_error(h, st);
    for (int q = 0; q < 4; ++q) {
        stats[q] = 0;
        for (int r = 0; r < STAT_SPREAD; ++r) stats[q] += spread[r * 8 + q];
    }
    return rc;
}

// Base-case bins larger than half the capacity are sorted by one
// workgroup of BNT threads per CU; the others by workgroups of BNT/2
// threads holding half the LDS, two per CU, so that one workgroup's
// barriers and LDS latencies overlap the other's work.  Each size class
// runs the counting sort first; the bins it hands back (items crowded into
// a few digits) are merge-sorted by a second launch that reads their count
// from device memory.
template <int DT>
constexpr uint32_t small_bin_cap() {
    return (uint32_t)(Shape<DT>::BNT / 2) * Shape<DT>::BVT;
}

constexpr size_t kFailCounts = 256;     // misc: two base-case fallback counters
constexpr size_t kBaseChunk = size_t(1) << 20;   // base-case bins per round of launches

// With `bsrc` (FUSED) the bins come from the level whose context `c` is,
// and the counting sort cleans each bin's buckets before it reads the bin.
template <int DT, int NT, bool FUSED = false>
int launch_basecase(ips4o_handle* h, const Ctx<DT>& c, const SegD* segs, size_t nseg, uint32_t grid,
                    typename Traits<DT>::Elem* scr, SegD* fail, uint32_t* nfail, hipStream_t st,
                    const uint32_t* dev_nseg = nullptr, const BinSrc* bsrc = nullptr) {
    constexpr int BVT = Shape<DT>::BVT;
    using LB = BaseLds<DT, NT, BVT>;
    const size_t lds_count = LB::bytes(), lds_merge = LB::xchg_at + NT * sizeof(uint32_t);
    HIP_TRY(hipFuncSetAttribute((const void*)k_basecase_count<DT, NT, BVT, FUSED>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_count));
    HIP_TRY(hipFuncSetAttribute((const void*)k_basecase<DT, NT, BVT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_merge));
    hipLaunchKernelGGL((k_basecase_count<DT, NT, BVT, FUSED>), dim3(grid), dim3(NT), lds_count, st, c, segs,
                       (uint32_t)nseg, scr, fail, nfail, dev_nseg, bsrc);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_basecase<DT, NT, BVT>), dim3(grid), dim3(NT), lds_merge, st, c, (const SegD*)fail, 0u, scr,
                       (const uint32_t*)nfail);
    HIP_TRY(hipGetLastError());
    return IPS4O_OK;
}

// One chunk of at most kBaseChunk bins (bins[0..count)).  With `srcs`
// (srcs[i] the buckets of bins[i], none of them tiny) and `lc` (the context
// of the level that made the bins) the counting sort cleans the buckets
// first; `mark` receives the timer record of the chunk.
//
// With wait = false the call returns once the launches are enqueued: the
// staging buffers are then guarded by h->staged, and the next chunk waits
// for the copies out of them before it writes them again (or for the whole
// stream before it grows them).
template <int DT>
int run_basecase_chunk(ips4o_handle* h, void* d_data, const SegD* bins, size_t count, hipStream_t st,
                       Timer& tm, const BinSrc* srcs = nullptr, const Ctx<DT>* lc = nullptr,
                       int* mark = nullptr, bool wait = true) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    struct {
        const SegD* p;
        size_t n;
        const SegD* begin() const { return p; }
        const SegD* end() const { return p + n; }
        size_t size() const { return n; }
    } const list{bins, count};
    constexpr int BNT = Shape<DT>::BNT, BVT = Shape<DT>::BVT;
    static_assert(BNT * BVT == TR::kBaseCap, "base-case capacity");
    constexpr bool plain = (DT == DT_U64 || DT == DT_F64);
    const uint32_t half = small_bin_cap<DT>();
    // small bins first, then the large ones, then (u64/f64) the tiny ones
    // that one wave sorts in registers, staged in pinned memory
    const bool fused = srcs != nullptr;
    auto cls = [&](const SegD& sg) { return plain && !fused && sg.len <= kTinyBin ? 2 : sg.len <= half ? 0 : 1; };
    size_t ncls[3] = {0, 0, 0};
    for (const SegD& sg : list) ++ncls[cls(sg)];
    const size_t nsmall = ncls[0], nlarge = ncls[1], ntiny = ncls[2];
    const size_t srcb = fused ? list.size() * sizeof(BinSrc) : 0;
    if (h->staged_pending) {
        const bool grows = list.size() * sizeof(SegD) + srcb > h->hsegs.bytes ||
                           2 * list.size() * sizeof(SegD) + srcb > h->segs.bytes || !plain;
        if (grows) HIP_TRY(hipStreamSynchronize(st));      // buffers in use may be freed
        else HIP_TRY(hipEventSynchronize(h->staged));       // the copies out of hsegs have run
        h->staged_pending = false;
    }
    int rc = h->hsegs.ensure(list.size() * sizeof(SegD) + srcb);
    if (rc) return rc;
    {
        SegD* hs = (SegD*)h->hsegs.p;
        BinSrc* hb = (BinSrc*)(hs + list.size());
        size_t at[3] = {0, nsmall, nsmall + nlarge};
        for (size_t i = 0; i < list.size(); ++i) {
            const size_t to = at[cls(bins[i])]++;
            hs[to] = bins[i];
            if (fused) hb[to] = srcs[i];
        }
    }
    // the list, then room for the bins each size class hands back, then
    // (fused) the bins' buckets
    rc = h->segs.ensure(2 * list.size() * sizeof(SegD) + srcb);
    if (rc) return rc;
    const uint32_t g_small = (uint32_t)std::min<size_t>(nsmall, 2 * kBaseGrid);
    const uint32_t g_large = (uint32_t)std::min<size_t>(nlarge, kBaseGrid);
    Elem* scr = nullptr;
    if (!plain) {
        rc = h->rscratch.ensure(std::max((size_t)g_small * half, (size_t)g_large * TR::kBaseCap) * sizeof(Elem));
        if (rc) return rc;
        scr = (Elem*)h->rscratch.p;
    }
    HIP_TRY(hipMemcpyAsync(h->segs.p, h->hsegs.p, list.size() * sizeof(SegD), hipMemcpyHostToDevice, st));
    const BinSrc* d_src = nullptr;
    if (fused) {
        d_src = (const BinSrc*)((SegD*)h->segs.p + 2 * list.size());
        HIP_TRY(hipMemcpyAsync((void*)d_src, (SegD*)h->hsegs.p + list.size(), srcb, hipMemcpyHostToDevice, st));
    }
    const bool async = !wait && !log_enabled();
    if (async) {
        if (!h->staged) HIP_TRY(hipEventCreateWithFlags(&h->staged, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(h->staged, st));          // hsegs is free again once this fires
    }
    Ctx<DT> c{};
    if (lc) c = *lc;
    c.data = (Elem*)d_data;
    double elems = 0;
    for (const SegD& sg : list) elems += sg.len;
    SegD* d_segs = (SegD*)h->segs.p;
    SegD* fail = d_segs + list.size();
    uint32_t* nfail = (uint32_t*)((char*)h->misc.p + kFailCounts);
    HIP_TRY(hipMemsetAsync(nfail, 0, 2 * sizeof(uint32_t), st));     // bins handed back by this chunk
    int r = tm.begin(KK_BASE);
    if (mark) *mark = r;
    if (nsmall) {
        rc = fused ? launch_basecase<DT, BNT / 2, true>(h, c, d_segs, nsmall, g_small, scr, fail, nfail, st,
                                                         nullptr, d_src)
                   : launch_basecase<DT, BNT / 2>(h, c, d_segs, nsmall, g_small, scr, fail, nfail, st);
        if (rc) return rc;
    }
    if (nlarge) {
        rc = fused ? launch_basecase<DT, BNT, true>(h, c, d_segs + nsmall, nlarge, g_large, scr, fail + nsmall,
                                                     nfail + 1, st, nullptr, d_src + nsmall)
                   : launch_basecase<DT, BNT>(h, c, d_segs + nsmall, nlarge, g_large, scr, fail + nsmall,
                                              nfail + 1, st);
        if (rc) return rc;
    }
    if constexpr (plain) {
        if (ntiny) {
            const uint32_t g = (uint32_t)std::min<size_t>((ntiny + 3) / 4, 4 * kBaseGrid);
            hipLaunchKernelGGL((k_basecase_tiny<DT, kTinyBin / 64>), dim3(g), dim3(256), 0, st, c,
                               (const SegD*)(d_segs + nsmall + nlarge), (uint32_t)ntiny, (const uint32_t*)nullptr);
            HIP_TRY(hipGetLastError());
        }
    }
    tm.end(r, 2.0 * sizeof(Elem) * elems);
    if (async) h->staged_pending = true;
    else HIP_TRY(hipStreamSynchronize(st));   // the staged list must outlive the copy
    if (log_enabled()) {
        uint32_t nf[2] = {0, 0};
        HIP_TRY(hipMemcpy(nf, nfail, sizeof(nf), hipMemcpyDeviceToHost));
        std::fprintf(stderr, "[ips4o] base case%s: %zu small bins (%u merge-sorted), %zu large (%u merge-sorted), "
                     "%zu tiny\n", fused ? " (fused cleanup)" : "", nsmall, nf[0], nlarge, nf[1], ntiny);
    }
    return IPS4O_OK;
}

// The base case over every bin of a sort, kBaseChunk bins per round of
// launches, so that the device bin list stays within a fixed size.
template <int DT>
int run_basecase(ips4o_handle* h, void* d_data, std::vector<SegD>& list, const Resolved& R,
                 hipStream_t st, Timer& tm, uint32_t pass) {
    (void)R;
    if (list.empty()) return IPS4O_OK;
    uint64_t elems = 0;
    for (const SegD& sg : list) elems += sg.len;
    tm.set_pass(pass, elems);          // the pass after the last level
    for (size_t a = 0; a < list.size(); a += kBaseChunk) {
        const int rc = run_basecase_chunk<DT>(h, d_data, list.data() + a, std::min(kBaseChunk, list.size() - a),
                                              st, tm);
        if (rc) return rc;
    }
    return IPS4O_OK;
}

// The base case of the bins found so far, enqueued without waiting for it:
// their ranges are final and no later level touches them, so they are
// sorted behind the level just enqueued while the host waits for that
// level's bounds and plans from them.  The timer records go to `marks`;
// the caller moves them to the base-case pass once the number of levels is
// known.
template <int DT>
int run_basecase_early(ips4o_handle* h, void* d_data, std::vector<SegD>& list, hipStream_t st, Timer& tm,
                       std::vector<int>& marks, uint64_t* elems) {
    for (const SegD& sg : list) *elems += sg.len;
    for (size_t a = 0; a < list.size(); a += kBaseChunk) {
        int mk = -1;
        const int rc = run_basecase_chunk<DT>(h, d_data, list.data() + a, std::min(kBaseChunk, list.size() - a),
                                              st, tm, nullptr, nullptr, &mk, false);
        if (rc) return rc;
        marks.push_back(mk);
    }
    list.clear();
    return IPS4O_OK;
}

// The stripe buffers of a level in the arena all levels share.  A level
// runs only after the previous one on the same stream, so one region
// serves every level; when a level needs more than the arena holds, the
// work in flight is waited for before it is replaced (the first sort of a
// size only: the arena is kept).
template <int DT>
int ensure_bufs(ips4o_handle* h, const Level<DT>& L, hipStream_t st) {
    const size_t need = (size_t)L.total_buf * sizeof(typename Traits<DT>::Elem);
    if (need <= h->bufs.bytes) return IPS4O_OK;
    HIP_TRY(hipStreamSynchronize(st));
    return h->bufs.ensure_exact(need);
}

// Offset of a level's bounds from its task state in the workspace (they
// are carved one after the other, so one copy reads both back).
template <int DT>
size_t readback_bounds_off(const Level<DT>& L) {
    return (size_t)((const char*)L.c.bounds - (const char*)L.c.ts);
}

// Copies of a level's error word, task state and bounds into pinned memory,
// enqueued right after its scan; `ev` fires when they have arrived.  Layout
// in `dst`: the error words (256 bytes), then the task state and the bounds
// as they lie in the workspace (bounds at readback_bounds_off(L) from the
// task state).
template <int DT>
int enqueue_readback(ips4o_handle* h, Level<DT>& L, HostArena& dst, hipEvent_t ev, hipStream_t st) {
    const size_t nb = L.total_slots + L.tasks.size();
    const size_t ob = readback_bounds_off(L), bytes = ob + nb * sizeof(uint64_t);
    int rc = dst.ensure(256 + bytes);
    if (rc) return rc;
    char* p = (char*)dst.p;
    HIP_TRY(hipMemcpyAsync(p, h->misc.p, 256, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(p + 256, L.c.ts, bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(ev, st));
    return IPS4O_OK;
}

// The recursion over a list of independent subproblems in [0, n_end): the
// whole array, or the segments of a segmented sort.  A level's bounds are
// read back as soon as its scan is done; while its permutation and cleanup
// still run, the host turns them into the next level's plan (or the
// base-case bins) and enqueues that work behind them; the bins found by
// the earlier levels are sorted behind each new level's launches.  Levels
// alternate between two workspaces, so the one a new level takes was last
// used two levels before, which has finished.
template <int DT>
int run_sort_list_body(ips4o_handle* h, void* d_data, uint64_t n_end, std::vector<Seg> init, const Resolved& R,
                       bool segmented, hipStream_t st) {
    h->last = ips4o_stats{};
    int rc = reset_misc(h, st);
    if (rc) return rc;
    for (hipEvent_t& e : h->scanned)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // subproblems within the base-case capacity go there at once, each in
    // a bin of its own
    std::vector<SegD> base;
    std::vector<Seg> cur;
    for (const Seg& sg : init) {
        if (sg.m <= 1) continue;
        if (sg.m <= R.cap) {
            base.push_back(SegD{sg.off, (uint32_t)sg.m, 0});
            h->last.elements_base += sg.m;
        } else {
            cur.push_back(sg);
        }
    }
    // stripe buffers of a level: at most an eighth of the elements sorted
    // (or one stripe per task, when that needs more)
    uint64_t buf_budget = 0;
    for (const Seg& sg : init) buf_budget += sg.m;
    buf_budget = std::max<uint64_t>(buf_budget / kBufBudgetDiv + 1, budget_floor(h, R));
    uint32_t level = 0;
    Level<DT> levels[2];
    std::vector<LevelMarks> marks;
    // base case that cleans the buckets of its bins (Section 4,
    // Implementation Details), on request
    constexpr bool plain = (DT == DT_U64 || DT == DT_F64);
    // strictly in-place hand-off between levels (Section 4.6)
    const bool strict = (R.flags & IPS4O_FLAG_STRICT) != 0;
    const bool fuse = !strict && ((R.flags & IPS4O_FLAG_FUSE) || fuse_on());
    std::vector<BinSrc> srcs, fs;
    std::vector<SegD> fb;
    uint64_t fused_elems = 0;          // elements of base-case launches made during the levels
    std::vector<int> fused_marks;      // their timer records
    std::vector<uint32_t> level_tasks, level_stripes, level_workers, level_b;
    Timer tm(h, st, (R.flags & IPS4O_FLAG_TIMING) != 0);
    const bool check = (R.flags & IPS4O_FLAG_CHECK) != 0;
    // host time (IPS4O_LOG): planning and enqueueing, waiting for a level's
    // bounds, turning them into the next plan
    using clk = std::chrono::steady_clock;
    double t_plan = 0, t_wait = 0, t_next = 0, t_planlevel = 0, t_head = 0;
    auto since = [](clk::time_point a) { return std::chrono::duration<double, std::milli>(clk::now() - a).count(); };
    // the caller's segments within the base-case capacity are sorted while
    // the host plans the first level (many segments make that plan long)
    if (!cur.empty() && !base.empty()) {
        rc = run_basecase_early<DT>(h, d_data, base, st, tm, fused_marks, &fused_elems);
        if (rc) return rc;
    }
    while (!cur.empty()) {
        if (level >= kMaxLevels) return IPS4O_ERR_DEVICE_FAULT;
        const auto t0 = clk::now();
        const int par = (int)(level & 1);
        Level<DT>& L = levels[par];
        Arena& work = par ? h->work2 : h->work;
        HostArena& rb = par ? h->hbounds2 : h->hbounds;
        // the block size of this level: the caller's, doubled while its
        // largest subproblem has too many blocks for the permutation word
        Resolved RL = R;
        {
            uint64_t mmax = 0;
            for (const Seg& sg : cur) mmax = std::max<uint64_t>(mmax, sg.m);
            if (!scale_block<DT>(&RL, mmax)) return IPS4O_ERR_NOT_SUPPORTED;
        }
        level_b.push_back(RL.b);
        plan_level<DT>(L, cur, RL, level, level == 0, 0, segmented && level == 0, 0, buf_budget);
        t_planlevel += since(t0);
        rc = work.ensure(level_bytes<DT>(L, RL.b));
        if (rc) return rc;
        rc = ensure_bufs<DT>(h, L, st);
        if (rc) return rc;
        carve_level<DT>(L, work.p, h->misc.p, d_data, h->bufs.p, RL, level);
        {
            uint64_t lm = 0;
            for (const Seg& sg : cur) lm += sg.m;
            tm.set_pass(level, lm);
        }
        marks.emplace_back();
        const auto th = clk::now();
        rc = launch_level_head<DT>(h, L, st, nullptr, tm, check, par ? &h->hdesc2 : &h->hdesc);
        if (rc) return rc;
        t_head += since(th);
        if (!strict) {
            rc = enqueue_readback<DT>(h, L, rb, h->scanned[par], st);
            if (rc) return rc;
        }
        // the cleanup waits for the bounds when the base case cleans the
        // buckets of the level's bins
        rc = launch_level_tail<DT>(h, L, st, tm, marks.back(), check, !fuse);
        if (rc) return rc;
        if (strict) {
            // the plan comes from the buckets the walk finds once the
            // level is done, not from the partition's own bounds
            uint64_t lm = 0;
            for (const Seg& sg : cur) lm += sg.m;
            rc = launch_mark_walk<DT>(L, st, tm, lm, R.cap, &h->last_hip);
            if (rc) return rc;
            rc = enqueue_readback<DT>(h, L, rb, h->scanned[par], st);
            if (rc) return rc;
        }
        // the bins of the earlier levels follow on the stream: the device
        // sorts them while the host waits for this level's bounds and plans
        // from them
        if (!base.empty()) {
            rc = run_basecase_early<DT>(h, d_data, base, st, tm, fused_marks, &fused_elems);
            if (rc) return rc;
        }
        level_tasks.push_back((uint32_t)L.tasks.size());
        level_stripes.push_back((uint32_t)L.stripes.size());
        level_workers.push_back(L.total_workers);
        for (const Seg& sg : cur) h->last.elements_distributed += sg.m;
        // ---- the bounds are on the host once the scan has run
        t_plan += since(t0);
        const auto t1 = clk::now();
        HIP_TRY(hipEventSynchronize(h->scanned[par]));
        t_wait += since(t1);
        const auto t2 = clk::now();
        const char* rp = (const char*)rb.p;
        const size_t T = L.tasks.size();
        if (((const uint32_t*)rp)[0] != 0) {        // a fault so far: no plan from these bounds
            (void)check_device_error(h, st);
            return IPS4O_ERR_DEVICE_FAULT;
        }
        const TaskS* ts = (const TaskS*)(rp + 256);
        const uint64_t* bounds = (const uint64_t*)(rp + 256 + readback_bounds_off(L));
        std::vector<Seg> next;
        base.reserve(base.size() + L.total_slots);
        const size_t base_before = base.size();
        srcs.clear();
        const uint64_t bin_cap = std::min(R.cap, small_bin_cap<DT>());
        std::vector<uint64_t> sb;      // a task's walked bounds without their flags (strict)
        std::vector<uint8_t> sone;     // and which of its buckets hold one key value
        for (size_t t = 0; t < T; ++t) {
            const TaskD& td = L.tasks[t];
            const uint64_t* bd = bounds + td.slot_begin + t;
            const uint32_t K = ts[t].K;
            if (log_enabled() && t < 64)
                std::fprintf(stderr, "[ips4o]   level %u task %zu off %llu m %llu k %u alpha %u K %u eq %u stripes %u\n",
                             level, t, (unsigned long long)td.off, (unsigned long long)td.m, td.k, td.alpha, K,
                             ts[t].eq, td.nstripes);
            uint64_t eb = 0;
            // strictly in place: the walk's buckets carry no equality
            // flags; a task left in one bucket holds one key value (with
            // k >= 4 a partition of two or more distinct keys makes at
            // least two buckets), which is sorted already, and so does a
            // bucket the walk found with equal keys at its two ends
            const uint8_t* one = nullptr;
            if (strict) {
                if (K > (uint32_t)KMAX || K > td.kbuf) {
                    (void)check_device_error(h, st);
                    return IPS4O_ERR_DEVICE_FAULT;
                }
                sb.resize(K + 1);
                sone.assign(K, 0);
                for (uint32_t q = 0; q <= K; ++q) {
                    sb[q] = bd[q] & ~kOneKeyBit;
                    if (q < K) sone[q] = (bd[q] & kOneKeyBit) ? 1 : 0;
                }
                if (K >= 1 && sb[0] == 0 && sb[1] == td.m) continue;
                bd = sb.data();
                one = sone.data();
            }
            const size_t next_before = next.size();
            if (K > (uint32_t)KMAX || K > td.kbuf ||
                !split_task(td.off, td.m, cur[t].grp, K, !strict && ts[t].eq != 0, bd, R.cap, bin_cap, base, next,
                            &eb, &srcs, (uint32_t)t, one)) {
                (void)check_device_error(h, st);
                return IPS4O_ERR_DEVICE_FAULT;
            }
            // the subproblems of a task whose keys repeat size their buffers
            // for equality buckets (a hint of the task, not of its buckets)
            if (strict && ts[t].eq)
                for (size_t q = next_before; q < next.size(); ++q) next[q].dup = 1;
            h->last.elements_base += eb;
        }
        // the level's bins (but the ones one wave sorts) go to the fused
        // base case, which cleans their buckets; the cleanup kernels skip
        // those buckets
        fb.clear();
        fs.clear();
        if (fuse) {
            size_t keep = base_before;
            for (size_t i = base_before; i < base.size(); ++i) {
                const SegD sg = base[i];
                if (!plain || sg.len > kTinyBin) {
                    fb.push_back(sg);
                    fs.push_back(srcs[i - base_before]);
                } else {
                    base[keep++] = sg;
                }
            }
            base.resize(keep);
        }
        if (!fb.empty()) {
            rc = h->hfused.ensure(L.total_slots);
            if (rc) return rc;
            uint8_t* fl = (uint8_t*)h->hfused.p;
            std::memset(fl, 0, L.total_slots);
            for (const BinSrc& b : fs)
                for (uint32_t j = b.j0; j <= b.j1; ++j) fl[L.tasks[b.task].slot_begin + j] = 1;
            HIP_TRY(hipMemcpyAsync(L.fused_flags, fl, L.total_slots, hipMemcpyHostToDevice, st));
            L.c.fused = L.fused_flags;
        }
        if (fuse) {
            rc = launch_level_cleanup<DT>(L, st, tm, marks.back(), &h->last_hip);
            if (rc) return rc;
        }
        if (!fb.empty()) {
            for (const SegD& sg : fb) fused_elems += sg.len;
            for (size_t a = 0; a < fb.size(); a += kBaseChunk) {
                int mk = -1;
                rc = run_basecase_chunk<DT>(h, d_data, fb.data() + a, std::min(kBaseChunk, fb.size() - a), st, tm,
                                            fs.data() + a, &L.c, &mk);
                if (rc) return rc;
                fused_marks.push_back(mk);
            }
        }
        L.c.fused = nullptr;
        cur.swap(next);
        ++level;
        t_next += since(t2);
    }
    h->last.levels = level;
    const auto t3 = clk::now();
    // the base-case pass follows the last level; the fused and early
    // launches count there
    for (int mk : fused_marks) tm.move_to_pass(mk, level);
    if (fused_elems) tm.set_pass(level, fused_elems);
    rc = run_basecase<DT>(h, d_data, base, R, st, tm, level);       // ends with a stream synchronize
    if (rc) return rc;
    if (log_enabled())
        std::fprintf(stderr, "[ips4o] host ms: plan+enqueue %.3f, wait for bounds %.3f, next plan %.3f, "
                     "base case (to the end) %.3f; of the first: level plans %.3f, first halves %.3f\n", t_plan,
                     t_wait, t_next, since(t3), t_planlevel, t_head);
    rc = check_device_error(h, st);
    // per-level counters: block moves, skips, cleanup and fix element counts
    std::vector<unsigned long long> cnt(kStatLevels * kStatsBytes / 8);
    HIP_TRY(hipMemcpy(cnt.data(), (char*)h->misc.p + kStatsOffset, kStatLevels * kStatsBytes, hipMemcpyDeviceToHost));
    for (uint32_t l = 0; l < level; ++l) {
        unsigned long long now[4] = {0, 0, 0, 0}, zero[4] = {0, 0, 0, 0};
        if (l < kStatLevels) {
            const unsigned long long* blk = cnt.data() + (size_t)l * kStatsBytes / 8;
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < STAT_SPREAD; ++r) now[q] += blk[r * 8 + q];
        }
        account_level<DT>(tm, marks[l], now, zero, level_b[l]);
        h->last.block_moves += now[0];
        h->last.block_skips += now[1];
        if (log_enabled())
            std::fprintf(stderr, "[ips4o] level %u: %u tasks, %u stripes, %u workers, moves %llu skips %llu\n", l,
                         level_tasks[l], level_stripes[l], level_workers[l], now[0], now[1]);
    }
    if (!fused_marks.empty()) {
        // elements the fused base case placed while cleaning (word 4 of
        // every level's counters)
        unsigned long long fc = 0;
        for (uint32_t l = 0; l < kStatLevels; ++l)
            for (int r = 0; r < STAT_SPREAD; ++r) fc += cnt[(size_t)l * kStatsBytes / 8 + r * 8 + 4];
        tm.add_bytes(fused_marks[0], 2.0 * sizeof(typename Traits<DT>::Elem) * (double)fc);
    }
    tm.finish();
    return rc;
}

// The recursion, and on every way out a wait for base-case launches that
// were not waited for (an error can end the planning while they still read
// the handle's bin lists).
template <int DT>
int run_sort_list(ips4o_handle* h, void* d_data, uint64_t n_end, std::vector<Seg> init, const Resolved& R,
                  bool segmented, hipStream_t st) {
    const int rc = run_sort_list_body<DT>(h, d_data, n_end, std::move(init), R, segmented, st);
    if (h->staged_pending) {
        const hipError_t e = hipStreamSynchronize(st);
        h->staged_pending = false;
        if (e != hipSuccess && rc == IPS4O_OK) {
            h->last_hip = e;
            return IPS4O_ERR_HIP;
        }
    }
    return rc;
}

template <int DT>
int run_sort(ips4o_handle* h, void* d_data, uint64_t n, const ips4o_params* p, hipStream_t st) {
    Resolved R;
    ips4o_params pm;
    p = merged_params(h, DT, p, &pm);
    int rc = resolve<DT>(p, &R);
    if (rc) return rc;
    h->last = ips4o_stats{};
    if (n <= 1) return IPS4O_OK;
    return run_sort_list<DT>(h, d_data, n, std::vector<Seg>{Seg{0, n, 0, 0}}, R, false, st);
}

// Segment i is [offs[i], offs[i + 1]); the offsets were checked by the caller.
template <int DT>
int run_sort_segmented(ips4o_handle* h, void* d_data, const uint64_t* offs, uint32_t nseg, const ips4o_params* p,
                       hipStream_t st) {
    Resolved R;
    ips4o_params pm;
    p = merged_params(h, DT, p, &pm);
    int rc = resolve<DT>(p, &R);
    if (rc) return rc;
    h->last = ips4o_stats{};
    std::vector<Seg> segs;
    uint64_t mmax = 0;
    for (uint32_t i = 0; i < nseg; ++i)
        if (offs[i + 1] - offs[i] > 1) {
            segs.push_back(Seg{offs[i], offs[i + 1] - offs[i], i, 0});
            mmax = std::max<uint64_t>(mmax, offs[i + 1] - offs[i]);
        }
    if (segs.empty()) return IPS4O_OK;
    {
        Resolved RT = R;      // refuse before any device work if no block size fits
        if (!scale_block<DT>(&RT, mmax)) return IPS4O_ERR_NOT_SUPPORTED;
    }
    return run_sort_list<DT>(h, d_data, offs[nseg], std::move(segs), R, true, st);
}

template <int DT>
int run_distribute(ips4o_handle* h, void* d_data, uint64_t n, const void* h_split, uint32_t m, int eq,
                   uint64_t* h_bounds, uint32_t* nb_out, const ips4o_params* p, hipStream_t st) {
    Resolved R;
    ips4o_params pm;
    p = merged_params(h, DT, p, &pm);
    int rc = resolve<DT>(p, &R);
    if (rc) return rc;
    if (!scale_block<DT>(&R, n)) return IPS4O_ERR_NOT_SUPPORTED;
    HostTree<DT> ht;
    rc = build_host_tree<DT>(h_split, m, eq, n, R.b, &ht);
    if (rc) return rc;
    const uint32_t K = ht.ts.K;
    h->last = ips4o_stats{};
    if (n == 0) {
        for (uint32_t i = 0; i <= K; ++i) h_bounds[i] = 0;
        if (nb_out) *nb_out = K;
        return IPS4O_OK;
    }
    rc = reset_misc(h, st);
    if (rc) return rc;
    Level<DT> L;
    std::vector<Seg> cur{Seg{0, n}};
    plan_level<DT>(L, cur, R, 0, true, ht.ts.kt, false, ht.ts.K,
                   std::max<uint64_t>(n / kBufBudgetDiv + 1, budget_floor(h, R)));
    rc = h->work.ensure(level_bytes<DT>(L, R.b));
    if (rc) return rc;
    rc = ensure_bufs<DT>(h, L, st);
    if (rc) return rc;
    carve_level<DT>(L, h->work.p, h->misc.p, d_data, h->bufs.p, R);
    Timer tm(h, st, (R.flags & IPS4O_FLAG_TIMING) != 0);
    LevelMarks mk;
    tm.set_pass(0, n);
    rc = run_level<DT>(h, L, st, &ht, tm, mk, (R.flags & IPS4O_FLAG_CHECK) != 0);
    if (rc) return rc;
    std::vector<TaskS> ts;
    const uint64_t* bounds = nullptr;     // pinned, valid until the next level's readback
    unsigned long long stats[4] = {0, 0, 0, 0}, zero[4] = {0, 0, 0, 0};
    rc = read_level<DT>(h, L, st, ts, bounds, stats);
    account_level<DT>(tm, mk, stats, zero, R.b);
    tm.finish();
    h->last.levels = 1;
    h->last.block_moves = stats[0];
    h->last.block_skips = stats[1];
    h->last.elements_distributed = n;
    if (rc) return rc;
    for (uint32_t i = 0; i <= K; ++i) h_bounds[i] = bounds[i];
    if (nb_out) *nb_out = K;
    return IPS4O_OK;
}

template <int DT>
int run_classify(ips4o_handle* h, const void* d_data, uint64_t n, const void* h_split, uint32_t m, int eq,
                 uint32_t* d_out, hipStream_t st) {
    using Key = typename Traits<DT>::Key;
    using Elem = typename Traits<DT>::Elem;
    HostTree<DT> ht;
    int rc = build_host_tree<DT>(h_split, m, eq, n, 1, &ht);
    if (rc) return rc;
    if (n == 0) return IPS4O_OK;
    // workspace: one task descriptor, task state, tree, splitters
    const size_t need = 4096 + 2 * KT_MAX * sizeof(Key);
    rc = h->work.ensure(need);
    if (rc) return rc;
    Carve cv(h->work.p);
    Ctx<DT> c{};
    c.data = (Elem*)d_data;
    TaskD td{};
    c.tasks = cv.take<TaskD>(1);
    c.ts = cv.take<TaskS>(1);
    c.tree = cv.take<Key>(KT_MAX);
    c.spl = cv.take<Key>(KT_MAX);
    HIP_TRY(hipMemcpyAsync((void*)c.tasks, &td, sizeof(td), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.ts, &ht.ts, sizeof(TaskS), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.tree, ht.tree.data(), ht.tree.size() * sizeof(Key), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.spl, ht.spl.data(), ht.spl.size() * sizeof(Key), hipMemcpyHostToDevice, st));
    uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL((k_bucket_ids<DT, 256>), dim3(grid), dim3(256), 0, st, c, n, d_out);
    HIP_TRY(hipGetLastError());
    // the host copies above read stack memory: finish them before returning
    HIP_TRY(hipStreamSynchronize(st));
    return IPS4O_OK;
}

template <int DT>
int run_select(ips4o_handle* h, const void* d_data, uint64_t n, const ips4o_params* p, void* h_out,
               uint32_t* nu_out, int* eq_out, hipStream_t st) {
    using Key = typename Traits<DT>::Key;
    using Elem = typename Traits<DT>::Elem;
    Resolved R;
    ips4o_params pm;
    p = merged_params(h, DT, p, &pm);
    int rc = resolve<DT>(p, &R);
    if (rc) return rc;
    rc = reset_misc(h, st);
    if (rc) return rc;
    Level<DT> L;
    std::vector<Seg> cur{Seg{0, n}};
    plan_level<DT>(L, cur, R, 0, true, 0);
    L.tasks[0].seed = R.seed;   // the caller's stream, not a derived one
    rc = h->work.ensure(level_bytes<DT>(L, R.b));
    if (rc) return rc;
    carve_level<DT>(L, h->work.p, h->misc.p, (void*)d_data, nullptr, R);    // sampling only
    HIP_TRY(hipMemcpyAsync((void*)L.c.tasks, L.tasks.data(), sizeof(TaskD), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_sample<DT, 1024>), dim3(1), dim3(1024), 0, st, L.c);
    HIP_TRY(hipGetLastError());
    TaskS ts{};
    std::vector<Key> spl(L.tasks[0].k);
    HIP_TRY(hipMemcpyAsync(&ts, L.c.ts, sizeof(TaskS), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(spl.data(), L.c.spl, spl.size() * sizeof(Key), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    // keys back to whole elements: the key fields are the element's leading
    // words for every type except f64 (inverse totalOrder image) and the
    // 100-byte records (big-endian bytes)
    char* out = (char*)h_out;
    for (uint32_t i = 0; i < ts.nuniq; ++i) {
        Elem e;
        std::memset(&e, 0, sizeof(e));
        const Key& k = spl[i];
        if constexpr (DT == DT_F64) {
            e = Traits<DT_F64>::unkey(k.v);
        } else if constexpr (DT == DT_BYTES100) {
            e.w[0] = bswap32((uint32_t)(k.hi >> 32));
            e.w[1] = bswap32((uint32_t)k.hi);
            e.w[2] = bswap32(k.lo << 16);
        } else if constexpr (DT == DT_U64) {
            e = k.v;
        } else if constexpr (DT == DT_PAIR) {
            e.w[0] = k.v;
        } else {
            e.w[0] = k.a; e.w[1] = k.b; e.w[2] = k.c;
        }
        std::memcpy(out + (size_t)i * sizeof(Elem), &e, sizeof(Elem));
    }
    *nu_out = ts.nuniq;
    *eq_out = (int)ts.eq;
    return check_device_error(h, st);
}

// Upper bound of the device workspace a handle holds after sorting n
// elements (ips4o_sort of n elements, ips4o_sort_segmented of n elements in
// all, ips4o_distribute of n elements), derived from the planning rules
// above; it does not depend on the keys.
//   stripe buffers (exact arena): every level plans at most
//     max(n/kBufBudgetDiv + 1, one stripe of k buckets per CU, what one
//     stripe per task with kbuf = k needs);
//     the top level of one array needs 2 KMAX b per stripe, at least
//     ceil(nb / kStripeBlocksMax) stripes; a deeper task of m > cap elements
//     has k < 4m/cap (adaptive_k), so one stripe per task needs below
//     8 b n / cap, plus 2 KT_MAX b per extra stripe of huge tasks.
//   per-level descriptors (two arenas, 25 % slack): a deeper level has at
//     most n/(cap+1) tasks, sum k <= 4n/cap + 2 per task, sum kbuf <= 2 sum k,
//     at most kLevelStripes + tasks + nb/kStripeBlocksMax stripes, and counts
//     for every stripe's kbuf buckets (at most the stripe buffers / 2b).
//   base-case bin list: at most kBaseChunk bins at once, twice (with the bins
//     handed to the merge sort); record scratch: one bin capacity per
//     workgroup of the base-case grids; the error and counter words.
template <int DT>
size_t workspace_bound(uint64_t n, const Resolved& R, uint32_t num_cus) {
    using TR = Traits<DT>;
    const uint64_t s = sizeof(typename TR::Elem), ks = sizeof(typename TR::Key);
    const uint64_t b0 = R.b, cap = R.cap;
    if (n <= 1) return 0;
    // block sizes: the top level's (scaled for n), and the deeper levels'
    // (scaled only when a subproblem can be large enough to need it)
    Resolved RT = R;
    (void)scale_block<DT>(&RT, n);
    const uint64_t b = RT.b;
    const uint64_t bd = n >= WR_MAX_BLOCKS * b0 ? b : b0;
    auto slack = [](uint64_t x) { return x + x / 4; };
    auto al = [](uint64_t x) { return x + 256; };
    const uint64_t nb = (n + b - 1) / b;
    const uint64_t huge = nb / kStripeBlocksMax + 1;          // stripes forced by stripe length
    uint64_t bufs = 0, work = 0;
    if (n > cap) {
        const uint64_t budget = std::max<uint64_t>(n / kBufBudgetDiv + 1, 2ull * R.k * b0 * (uint64_t)num_cus);
        const uint64_t root = 2 * (uint64_t)KMAX * b * std::max<uint64_t>(huge, R.stripes);
        const uint64_t deep = 8 * bd * n / cap + 1 + 2 * (uint64_t)KT_MAX * bd * huge;
        bufs = std::max(budget, std::max(root, deep));
        const uint64_t T = n / (cap + 1) + 1;
        const uint64_t sumk = std::max<uint64_t>((uint64_t)KT_MAX, 4 * n / cap + 2 * T);
        const uint64_t sumkb = 2 * sumk;
        const uint64_t S = std::max<uint64_t>(STRIPES_PER_TASK_MAX, kLevelStripes + T + huge);
        const uint64_t counts = bufs / (2 * b0) + 1;
        const uint64_t lv = al(T * sizeof(TaskD)) + al(S * sizeof(StripeD)) + al(T * sizeof(TaskS)) +
                            2 * al(sumk * ks) + al((sumkb + T) * 8) + al((sumkb + T) * 4) +
                            al(sumkb * sizeof(BucketSlot)) + al(counts * 4) + 2 * al(S * 4) + al(sumkb) + 256;
        work = 2 * slack(lv);
    }
    const uint64_t misc = slack(kStatsOffset + (uint64_t)kStatLevels * kStatsBytes);
    const uint64_t bins = std::min<uint64_t>(n / 2 + 1, kBaseChunk);
    const uint64_t segs = slack(bins * (2 * sizeof(SegD) + sizeof(BinSrc)));
    uint64_t recs = 0;
    if (DT != DT_U64 && DT != DT_F64)
        recs = slack(std::max(std::min<uint64_t>(bins, 2 * kBaseGrid) * small_bin_cap<DT>(),
                                 std::min<uint64_t>(bins, kBaseGrid) * (uint64_t)TR::kBaseCap) * s);
    return (size_t)(bufs * s + work + misc + segs + recs);
}

// n elements fit the permutation's block indices with some block size.
template <int DT>
int check_blocks(uint64_t n, const ips4o_params* params) {
    Resolved R;
    int rc = resolve<DT>(params, &R);
    if (rc) return rc;
    return scale_block<DT>(&R, n) ? IPS4O_OK : IPS4O_ERR_NOT_SUPPORTED;
}

template <int DT>
int workspace_query(uint64_t n, const ips4o_params* params, uint32_t num_cus, size_t* bytes) {
    Resolved R;
    int rc = resolve<DT>(params, &R);
    if (rc) return rc;
    if (!scale_block<DT>(&R, n)) return IPS4O_ERR_NOT_SUPPORTED;
    *bytes = workspace_bound<DT>(n, R, num_cus);
    return IPS4O_OK;
}

int check_ptr(const void* p, uint64_t n, int dt) {
    if (n > 0 && !p) return IPS4O_ERR_INVALID_ARG;
    if (p && ((uintptr_t)p % elem_align(dt))) return IPS4O_ERR_INVALID_ARG;
    return IPS4O_OK;
}

int check_params(const ips4o_params* params, int dtype) {
    Resolved R;
    switch (dtype) {
    case DT_U64: return resolve<DT_U64>(params, &R);
    case DT_F64: return resolve<DT_F64>(params, &R);
    case DT_PAIR: return resolve<DT_PAIR>(params, &R);
    case DT_QUARTET: return resolve<DT_QUARTET>(params, &R);
    case DT_BYTES100: return resolve<DT_BYTES100>(params, &R);
    }
    return IPS4O_ERR_INVALID_ARG;
}

template <int DT>
int check_splitter_order(const void* h_split, uint32_t m) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    const char* src = (const char*)h_split;
    typename TR::Key prev{};
    for (uint32_t i = 0; i < m; ++i) {
        Elem e;
        std::memcpy(&e, src + (size_t)i * sizeof(Elem), sizeof(Elem));
        typename TR::Key k = TR::key(e);
        if (i > 0 && k < prev) return IPS4O_ERR_INVALID_ARG;
        prev = k;
    }
    return IPS4O_OK;
}

int set_device(ips4o_handle* h) {
    HIP_TRY(hipSetDevice(h->device));
    return IPS4O_OK;
}

}  // namespace

// ---------------------------------------------------- sort without allocation
// For callers that cannot allocate (code under graph capture, tight serving
// loops): ips4o_sort_small sorts one base-case bin with its bin list, its
// merge-sort hand-back counters and its record scratch in this file-scope
// array, which every GPU the library runs on holds until the process ends.
// Host code never uses the array's name as an address: ips4o_create asks
// for the current device's address once per device (hipGetSymbolAddress)
// and every launch gets that pointer.
constexpr size_t kSmallBytes = 512 * 1024;
constexpr size_t kSmallRecords = 256;       // offset of the record scratch
static __device__ __align__(256) unsigned char scratch[kSmallBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_small_mu;
void* g_small_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (current), fetched once.
int small_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_small_mu);
    if (device < 0 || device >= kMaxDevices) return IPS4O_ERR_NOT_SUPPORTED;
    if (!g_small_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IPS4O_ERR_HIP;
        g_small_ptr[device] = p;
    }
    *out = g_small_ptr[device];
    return IPS4O_OK;
}

// Bin list [0] = the whole array, hand-back counters cleared (a kernel
// rather than a memset, so that the call can be captured in a graph).
__global__ void k_small_setup(SegD* bins, uint32_t* nfail, uint64_t n) {
    if (threadIdx.x == 0) {
        SegD sd;
        sd.off = 0;
        sd.len = (uint32_t)n;
        sd.pad = 0;
        bins[0] = sd;
        nfail[0] = 0;
        nfail[1] = 0;
    }
}

template <int DT>
int run_sort_small(ips4o_handle* h, void* d_data, uint64_t n, hipStream_t st) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    constexpr int BNT = Shape<DT>::BNT;
    constexpr bool plain = (DT == DT_U64 || DT == DT_F64);
    static_assert(kSmallRecords + (size_t)TR::kBaseCap * sizeof(Elem) <= kSmallBytes, "record scratch fits");
    if (n > (uint64_t)TR::kBaseCap) return IPS4O_ERR_NOT_SUPPORTED;
    if (n <= 1) return IPS4O_OK;
    char* base = (char*)h->small;
    SegD* bins = (SegD*)base;                      // [0] the bin, [1] handed back to the merge sort
    uint32_t* nfail = (uint32_t*)(base + 64);
    Elem* scr = plain ? nullptr : (Elem*)(base + kSmallRecords);
    hipLaunchKernelGGL(k_small_setup, dim3(1), dim3(64), 0, st, bins, nfail, n);
    HIP_TRY(hipGetLastError());
    Ctx<DT> c{};
    c.data = (Elem*)d_data;
    if (plain && n <= kTinyBin) {
        if constexpr (plain) {
            hipLaunchKernelGGL((k_basecase_tiny<DT, kTinyBin / 64>), dim3(1), dim3(256), 0, st, c,
                               (const SegD*)bins, 1u, (const uint32_t*)nullptr);
            HIP_TRY(hipGetLastError());
        }
        return IPS4O_OK;
    }
    if (n <= small_bin_cap<DT>()) return launch_basecase<DT, BNT / 2>(h, c, bins, 1, 1, scr, bins + 1, nfail, st);
    return launch_basecase<DT, BNT>(h, c, bins, 1, 1, scr, bins + 1, nfail + 1, st);
}

}  // namespace

// Segmented sort of segments within the base-case capacity, planned on the
// device (bins from the caller's device offsets, launches that read their
// bin counts from device memory): no host round trip, so the call can be
// captured in a HIP graph.  The first call for a segment count allocates the
// bin lists; later calls for as many segments or fewer allocate nothing.
template <int DT>
int run_sort_small_segments(ips4o_handle* h, void* d_data, const uint64_t* d_offs, uint32_t nseg, hipStream_t st) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    constexpr int BNT = Shape<DT>::BNT;
    constexpr bool plain = (DT == DT_U64 || DT == DT_F64);
    const uint32_t half = small_bin_cap<DT>();
    int rc = h->misc.ensure(kStatsOffset + kStatLevels * kStatsBytes);
    if (rc) return rc;
    // lists of the three classes, then the hand-back lists of the two
    // counting-sort classes, then eight counters
    const size_t list_bytes = 5 * (size_t)nseg * sizeof(SegD) + 64;
    rc = h->segs.ensure(list_bytes);
    if (rc) return rc;
    Elem* scr = nullptr;
    if (!plain) {
        rc = h->rscratch.ensure(std::max((size_t)2 * kBaseGrid * half, (size_t)kBaseGrid * TR::kBaseCap) * sizeof(Elem));
        if (rc) return rc;
        scr = (Elem*)h->rscratch.p;
    }
    SegD* lists = (SegD*)h->segs.p;
    uint32_t* cnt = (uint32_t*)((char*)h->segs.p + 5 * (size_t)nseg * sizeof(SegD));
    uint32_t* err = (uint32_t*)h->misc.p;
    hipLaunchKernelGGL((k_small_segments_setup<DT>), dim3(1), dim3(256), 0, st, cnt, err);
    HIP_TRY(hipGetLastError());
    const uint32_t gb = std::max<uint32_t>(1, std::min<uint32_t>((nseg + 255) / 256, 4096));
    hipLaunchKernelGGL((k_small_segments_bins<DT>), dim3(gb), dim3(256), 0, st, d_offs, nseg, half,
                       (uint32_t)TR::kBaseCap, plain ? kTinyBin : 0u, lists, cnt, err);
    HIP_TRY(hipGetLastError());
    Ctx<DT> c{};
    c.data = (Elem*)d_data;
    SegD* fail = lists + 3 * (size_t)nseg;
    const uint32_t g_small = std::min<uint32_t>(nseg, 2 * kBaseGrid), g_large = std::min<uint32_t>(nseg, kBaseGrid);
    rc = launch_basecase<DT, BNT / 2>(h, c, lists, 0, g_small, scr, fail, cnt + 3, st, cnt + 0);
    if (rc) return rc;
    rc = launch_basecase<DT, BNT>(h, c, lists + nseg, 0, g_large, scr, fail + nseg, cnt + 4, st, cnt + 1);
    if (rc) return rc;
    if constexpr (plain) {
        const uint32_t g = std::min<uint32_t>((nseg + 3) / 4, 4 * kBaseGrid);
        hipLaunchKernelGGL((k_basecase_tiny<DT, kTinyBin / 64>), dim3(g), dim3(256), 0, st, c,
                           (const SegD*)(lists + 2 * (size_t)nseg), 0u, (const uint32_t*)(cnt + 2));
        HIP_TRY(hipGetLastError());
    }
    return IPS4O_OK;
}

// The marking and the search of the strictly in-place recursion (Section
// 4.6) on caller-given buckets and positions.
template <int DT>
int run_mark_bucket_max(ips4o_handle* h, void* d_data, uint64_t n, const uint64_t* d_bounds, uint32_t nb,
                        hipStream_t st) {
    int rc = reset_misc(h, st);
    if (rc) return rc;
    hipLaunchKernelGGL((k_mark_max<DT, 1024>), dim3(std::min<uint32_t>(nb, 1u << 20), 1), dim3(1024), 0, st,
                       (typename Traits<DT>::Elem*)d_data, n, d_bounds, (const TaskD*)nullptr,
                       (const TaskS*)nullptr, 0u, nb, (uint32_t*)h->misc.p);
    HIP_TRY(hipGetLastError());
    return check_device_error(h, st);
}

template <int DT>
int run_search_next_largest(ips4o_handle* h, const void* d_data, uint64_t n, const uint64_t* d_pos,
                            uint64_t count, uint64_t* d_out, hipStream_t st) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>((count + 3) / 4, 1u << 16);
    hipLaunchKernelGGL((k_search_next<DT>), dim3(grid), dim3(256), 0, st,
                       (const typename Traits<DT>::Elem*)d_data, n, d_pos, count, d_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return IPS4O_OK;
}

#define DISPATCH(dt, CALL)                                   \
    switch (dt) {                                            \
    case DT_U64: { constexpr int D = DT_U64; return CALL; }  \
    case DT_F64: { constexpr int D = DT_F64; return CALL; }  \
    case DT_PAIR: { constexpr int D = DT_PAIR; return CALL; } \
    case DT_QUARTET: { constexpr int D = DT_QUARTET; return CALL; } \
    case DT_BYTES100: { constexpr int D = DT_BYTES100; return CALL; } \
    default: return IPS4O_ERR_INVALID_ARG;                   \
    }

extern "C" {

int ips4o_create(int hip_device, ips4o_handle** out) {
    if (!out) return IPS4O_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return IPS4O_ERR_NOT_SUPPORTED;
    if (hip_device < 0 || hip_device >= count) return IPS4O_ERR_INVALID_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return IPS4O_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return IPS4O_ERR_NOT_SUPPORTED;
    // this device's address of the array ips4o_sort_small works in (set-up
    // once per device, with the device current)
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return IPS4O_ERR_HIP;
    if (hipSetDevice(hip_device) != hipSuccess) return IPS4O_ERR_HIP;
    void* small = nullptr;
    const int rs = small_scratch(hip_device, &small);
    (void)hipSetDevice(prev);
    if (rs) return rs;
    ips4o_handle* h = new (std::nothrow) ips4o_handle();
    if (!h) return IPS4O_ERR_OUT_OF_MEMORY;
    h->device = hip_device;
    h->num_cus = prop.multiProcessorCount;
    h->small = small;
    *out = h;
    return IPS4O_OK;
}

void ips4o_destroy(ips4o_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->work.release();
    h->work2.release();
    h->bufs.release();
    h->hbounds2.release();
    h->hdesc.release();
    h->hdesc2.release();
    for (hipEvent_t& e : h->scanned)
        if (e) (void)hipEventDestroy(e);
    if (h->staged) (void)hipEventDestroy(h->staged);
    h->misc.release();
    h->segs.release();
    h->rscratch.release();
    h->hbounds.release();
    h->hsegs.release();
    h->hstage.release();
    delete h;
}

int ips4o_workspace_size(const ips4o_handle* h, int dtype, uint64_t n, const ips4o_params* params, size_t* bytes) {
    (void)h;
    if (!bytes) return IPS4O_ERR_INVALID_ARG;
    if (elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    int rc = check_params(params, dtype);
    if (rc) return rc;
    if (n >= kMaxElements) return IPS4O_ERR_NOT_SUPPORTED;
    ips4o_params pm;
    params = merged_params(h, dtype, params, &pm);
    DISPATCH(dtype, workspace_query<D>(n, params, h ? (uint32_t)h->num_cus : 256u, bytes));
}

int ips4o_set_default_params(ips4o_handle* h, int dtype, const ips4o_params* params) {
    if (!h || elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    if (!params) {
        h->dflt[dtype] = ips4o_params{};
        return IPS4O_OK;
    }
    const int rc = check_params(params, dtype);
    if (rc) return rc;
    h->dflt[dtype] = *params;
    h->dflt[dtype].flags = 0;
    return IPS4O_OK;
}

int ips4o_workspace_bytes(const ips4o_handle* h, size_t* bytes) {
    if (!h || !bytes) return IPS4O_ERR_INVALID_ARG;
    *bytes = h->work.bytes + h->work2.bytes + h->bufs.bytes + h->misc.bytes + h->segs.bytes + h->rscratch.bytes;
    return IPS4O_OK;
}

int ips4o_sort(ips4o_handle* h, void* d_data, uint64_t n, int dtype, const ips4o_params* params,
               void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, params);
    if (rc) return rc;
    if (n <= 1) return IPS4O_OK;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_sort<D>(h, d_data, n, params, st));
}

int ips4o_sort_small(ips4o_handle* h, void* d_data, uint64_t n, int dtype, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    if (elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    int rc = check_ptr(d_data, n, dtype);
    if (rc) return rc;
    if (n > ips4o_small_max(dtype)) return IPS4O_ERR_NOT_SUPPORTED;
    if (n <= 1) return IPS4O_OK;
    if (!h->small) return IPS4O_ERR_HIP;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_sort_small<D>(h, d_data, n, st));
}

int ips4o_sort_segmented_small(ips4o_handle* h, void* d_data, int dtype, const uint64_t* d_offsets,
                               uint32_t num_segments, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    if (elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    if (num_segments == 0) return IPS4O_OK;
    if (!d_offsets || ((uintptr_t)d_offsets & 7)) return IPS4O_ERR_INVALID_ARG;
    if (!d_data || ((uintptr_t)d_data % elem_align(dtype))) return IPS4O_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_sort_small_segments<D>(h, d_data, d_offsets, num_segments, st));
}

uint64_t ips4o_small_max(int dtype) {
    switch (dtype) {
    case DT_U64: return (uint64_t)Traits<DT_U64>::kBaseCap;
    case DT_F64: return (uint64_t)Traits<DT_F64>::kBaseCap;
    case DT_PAIR: return (uint64_t)Traits<DT_PAIR>::kBaseCap;
    case DT_QUARTET: return (uint64_t)Traits<DT_QUARTET>::kBaseCap;
    case DT_BYTES100: return (uint64_t)Traits<DT_BYTES100>::kBaseCap;
    }
    return 0;
}

int ips4o_sort_segmented(ips4o_handle* h, void* d_data, int dtype, const uint64_t* h_offsets, uint32_t num_segments,
                         const ips4o_params* params, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_segments(d_data, dtype, h_offsets, num_segments, params);
    if (rc) return rc;
    if (num_segments == 0 || h_offsets[num_segments] <= 1) return IPS4O_OK;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_sort_segmented<D>(h, d_data, h_offsets, num_segments, params, st));
}

int ips4o_distribute(ips4o_handle* h, void* d_data, uint64_t n, int dtype, const void* h_splitters,
                     uint32_t num_splitters, int equality_buckets, uint64_t* h_bounds_out,
                     uint32_t* num_buckets_out, const ips4o_params* params, void* hip_stream) {
    if (!h || !h_bounds_out) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, params);
    if (rc) return rc;
    rc = ips4o_check_splitters(h_splitters, num_splitters, dtype, equality_buckets);
    if (rc) return rc;
    if (n > 0) {
        rc = set_device(h);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_distribute<D>(h, d_data, n, h_splitters, num_splitters, equality_buckets,
                                      h_bounds_out, num_buckets_out, params, st));
}

int ips4o_sort_segmented_dev(ips4o_handle* h, void* d_data, int dtype, const uint64_t* d_offsets,
                             uint32_t num_segments, const ips4o_params* params, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    if (num_segments == 0) return IPS4O_OK;
    if (!d_offsets || ((uintptr_t)d_offsets & 7)) return IPS4O_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t bytes = ((size_t)num_segments + 1) * sizeof(uint64_t);
    rc = h->hstage.ensure(bytes);
    if (rc) return rc;
    // the table may be written by earlier work on the stream: copy in order
    HIP_TRY(hipMemcpyAsync(h->hstage.p, d_offsets, bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ips4o_sort_segmented(h, d_data, dtype, (const uint64_t*)h->hstage.p, num_segments, params, hip_stream);
}

int ips4o_distribute_dev(ips4o_handle* h, void* d_data, uint64_t n, int dtype, const void* d_splitters,
                         uint32_t num_splitters, int equality_buckets, uint64_t* d_bounds_out,
                         uint32_t* d_num_buckets_out, const ips4o_params* params, void* hip_stream) {
    if (!h || !d_bounds_out || ((uintptr_t)d_bounds_out & 7)) return IPS4O_ERR_INVALID_ARG;
    if (d_num_buckets_out && ((uintptr_t)d_num_buckets_out & 3)) return IPS4O_ERR_INVALID_ARG;
    const size_t s = elem_size(dtype);
    if (s == 0 || !d_splitters || ((uintptr_t)d_splitters % elem_align(dtype))) return IPS4O_ERR_INVALID_ARG;
    if (num_splitters < 1 || num_splitters > (uint32_t)KGIVEN_MAX) return IPS4O_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    // splitters to the host (the search tree is built there), in stream order
    const size_t sbytes = (size_t)num_splitters * s, bbytes = (size_t)(2 * KGIVEN_MAX + 2) * sizeof(uint64_t);
    rc = h->hstage.ensure(sbytes + bbytes + 64);
    if (rc) return rc;
    char* stage = (char*)h->hstage.p;
    HIP_TRY(hipMemcpyAsync(stage, d_splitters, sbytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    uint64_t* hb = (uint64_t*)(stage + ((sbytes + 63) & ~(size_t)63));
    uint32_t K = 0;
    rc = ips4o_distribute(h, d_data, n, dtype, stage, num_splitters, equality_buckets, hb, &K, params, hip_stream);
    if (rc) return rc;
    uint32_t* hk = (uint32_t*)(hb + K + 1);
    *hk = K;
    HIP_TRY(hipMemcpyAsync(d_bounds_out, hb, (size_t)(K + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if (d_num_buckets_out)
        HIP_TRY(hipMemcpyAsync(d_num_buckets_out, hk, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));      // the staging buffer is reused by the next call
    return IPS4O_OK;
}

int ips4o_classify(ips4o_handle* h, const void* d_data, uint64_t n, int dtype, const void* h_splitters,
                   uint32_t num_splitters, int equality_buckets, uint32_t* d_bucket_out, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, nullptr);
    if (rc) return rc;
    rc = ips4o_check_splitters(h_splitters, num_splitters, dtype, equality_buckets);
    if (rc) return rc;
    if (n > 0 && (!d_bucket_out || ((uintptr_t)d_bucket_out & 3))) return IPS4O_ERR_INVALID_ARG;
    if (n > 0) {
        rc = set_device(h);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_classify<D>(h, d_data, n, h_splitters, num_splitters, equality_buckets,
                                    d_bucket_out, st));
}

int ips4o_mark_bucket_max(ips4o_handle* h, void* d_data, uint64_t n, int dtype, const uint64_t* d_bounds,
                          uint32_t num_buckets, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, nullptr);
    if (rc) return rc;
    if (num_buckets == 0) return IPS4O_OK;
    if (!d_bounds || ((uintptr_t)d_bounds & 7)) return IPS4O_ERR_INVALID_ARG;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_mark_bucket_max<D>(h, d_data, n, d_bounds, num_buckets, st));
}

int ips4o_search_next_largest(ips4o_handle* h, const void* d_data, uint64_t n, int dtype, const uint64_t* d_pos,
                              uint64_t count, uint64_t* d_out, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, nullptr);
    if (rc) return rc;
    if (count == 0) return IPS4O_OK;
    if (!d_pos || !d_out || ((uintptr_t)d_pos & 7) || ((uintptr_t)d_out & 7)) return IPS4O_ERR_INVALID_ARG;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_search_next_largest<D>(h, d_data, n, d_pos, count, d_out, st));
}

int ips4o_select_splitters(ips4o_handle* h, const void* d_data, uint64_t n, int dtype,
                           const ips4o_params* params, void* h_splitters_out, uint32_t* num_unique_out,
                           int* equality_out, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = ips4o_check_args(d_data, n, dtype, params);
    if (rc) return rc;
    if (n < 1 || !h_splitters_out || !num_unique_out || !equality_out) return IPS4O_ERR_INVALID_ARG;
    rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DISPATCH(dtype, run_select<D>(h, d_data, n, params, h_splitters_out, num_unique_out, equality_out, st));
}

int ips4o_check_args(const void* d_data, uint64_t n, int dtype, const ips4o_params* params) {
    if (elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    int rc = check_ptr(d_data, n, dtype);
    if (rc) return rc;
    rc = check_params(params, dtype);
    if (rc) return rc;
    if (n >= kMaxElements) return IPS4O_ERR_NOT_SUPPORTED;
    DISPATCH(dtype, check_blocks<D>(n, params));
}

int ips4o_check_segments(const void* d_data, int dtype, const uint64_t* h_offsets, uint32_t num_segments,
                         const ips4o_params* params) {
    if (num_segments > 0 && !h_offsets) return IPS4O_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < num_segments; ++i)
        if (h_offsets[i + 1] < h_offsets[i]) return IPS4O_ERR_INVALID_ARG;
    return ips4o_check_args(d_data, num_segments ? h_offsets[num_segments] : 0, dtype, params);
}

int ips4o_check_splitters(const void* h_splitters, uint32_t num_splitters, int dtype, int equality_buckets) {
    if (elem_size(dtype) == 0) return IPS4O_ERR_INVALID_ARG;
    if (!h_splitters || num_splitters < 1 || num_splitters > (uint32_t)KGIVEN_MAX) return IPS4O_ERR_INVALID_ARG;
    if (equality_buckets != 0 && equality_buckets != 1) return IPS4O_ERR_INVALID_ARG;
    DISPATCH(dtype, check_splitter_order<D>(h_splitters, num_splitters));
}

int ips4o_sync(ips4o_handle* h, void* hip_stream) {
    if (!h) return IPS4O_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if (!h->misc.p) {
        HIP_TRY(hipStreamSynchronize(st));
        return IPS4O_OK;
    }
    return check_device_error(h, st);
}

const char* ips4o_status_string(int status) {
    switch (status) {
    case IPS4O_OK: return "ok";
    case IPS4O_ERR_INVALID_ARG: return "invalid argument";
    case IPS4O_ERR_OUT_OF_MEMORY: return "out of device memory";
    case IPS4O_ERR_HIP: return "HIP runtime error";
    case IPS4O_ERR_NOT_SUPPORTED: return "not supported (device is not gfx950, or n too large)";
    case IPS4O_ERR_DEVICE_FAULT: return "device fault: a kernel found an inconsistent state; data undefined";
    }
    return "unknown status";
}

int ips4o_last_kernel_stats(const ips4o_handle* h, ips4o_kernel_stat* out) {
    if (!h || !out) return IPS4O_ERR_INVALID_ARG;
    for (int i = 0; i < KK_N; ++i) out[i] = h->kstats[i];
    return IPS4O_OK;
}

int ips4o_last_pass_stats(const ips4o_handle* h, ips4o_pass_stat* out, uint32_t max_passes, uint32_t* num_passes) {
    if (!h || !num_passes || (max_passes > 0 && !out)) return IPS4O_ERR_INVALID_ARG;
    *num_passes = (uint32_t)h->pstats.size();
    for (uint32_t i = 0; i < max_passes && i < h->pstats.size(); ++i) out[i] = h->pstats[i];
    return IPS4O_OK;
}

int ips4o_last_stats(const ips4o_handle* h, ips4o_stats* out) {
    if (!h || !out) return IPS4O_ERR_INVALID_ARG;
    *out = h->last;
    return IPS4O_OK;
}

}  // extern "C"
