// gfx950 kernels of one in-place super scalar samplesort level (Section 4 of
// Axtmann, Witt, Ferizovic, Sanders, arXiv 1705.02257) and of the base case.
//
// A level partitions a list of independent subproblems ("tasks", each a
// contiguous segment of the array) in six launches:
//   k_sample      one workgroup per task: oversampled splitters, duplicate
//                 removal, equality flag, level-order search tree (Section 3,
//                 Preliminaries; Section 4, Sampling, Implementation Details)
//   k_classify    one workgroup per stripe: local classification into
//                 per-workgroup buffer blocks of b elements, full blocks
//                 gathered at the stripe front (Section 4.1)
//   k_scan        one workgroup per task: bucket boundaries and block
//                 delimiters from the per-stripe counts (Section 4.2)
//   k_fix_empty   one workgroup per bucket: move full blocks of buckets that
//                 cross stripe ends so every bucket is [full | empty]
//                 (Appendix A, empty block movement); sets (w_i, r_i)
//   k_permute     wavefront workers: the block permutation with atomic
//                 read/write pointers and per-bucket reader counts (Section 4.2)
//   k_cleanup     one workgroup per bucket: heads, tails, partial buffers and
//                 the overflow block (Section 4.3)
// and k_basecase sorts small subproblems inside LDS.
//
// Block indices are relative to the task's segment start; block q covers
// elements [q*b, (q+1)*b) of the segment, the last block may be partial.
#pragma once
#include <type_traits>

#include "planner.hpp"
#include "traits.hpp"
#include "wrword.hpp"

namespace ips4o {

constexpr int KT_MAX = 1024;    // search tree leaves (power of two)
constexpr int KMAX = 1024;      // logical buckets (with equality buckets 2 nuniq + 1)
constexpr int KGIVEN_MAX = 511; // caller-given splitters: 2*511 + 1 buckets fit KMAX
// sample capacity in LDS: a power of two, at most 128 KiB of keys
template <class Key>
constexpr int sample_max() {
    return sizeof(Key) <= 8 ? 16384 : (sizeof(Key) <= 16 ? 8192 : 4096);
}
constexpr int STRIPES_PER_TASK_MAX = 1024;
constexpr uint32_t NO_BUCKET = 0xffffffffu;

struct TaskD {                  // host-planned, one per task
    uint64_t off;               // first element of the segment
    uint64_t m;                 // segment length
    uint64_t seed;              // sampling stream
    uint32_t k;                 // requested tree leaves
    uint32_t alpha;             // oversampling factor
    uint32_t stripe_begin, nstripes;
    uint32_t worker_begin, nworkers;
    uint32_t slot_begin;        // first bucket slot (sum of kbuf over earlier tasks)
    uint32_t tree_begin;        // first tree slot (sum of k over earlier tasks)
    uint32_t kbuf;              // buckets the task's buffers, slots and counts hold (K <= kbuf)
    uint32_t cnt_begin;         // counts of stripe stripe_begin + q at cnt_begin + q * kbuf
};

struct StripeD {                // host-planned, one per stripe
    uint32_t task;
    uint32_t blk_begin, blk_end;
    uint32_t pad;
    uint64_t buf_off;           // element offset of this stripe's partial buffers (kbuf blocks;
                                // during classification followed by its side area of kbuf blocks)
};

struct TaskS {                  // device-written per task
    uint32_t K;                 // logical buckets
    uint32_t kt;                // tree leaves (power of two)
    uint32_t eq;                // equality buckets on
    uint32_t nuniq;             // splitters in spl[] (unique when eq)
    uint32_t nblocks;           // ceil(m / b)
    uint32_t ovf_bucket;        // bucket that filled the overflow block
    uint32_t pad0, pad1;
};

// Per-bucket permutation state, one 64-byte slot per bucket: the atomics of
// two buckets share at most a cache line, and a worker's scan over 64
// buckets reads 4 KiB (wider slots made the scans of levels with many
// buckets a large part of the permutation's memory traffic).
//
struct alignas(64) BucketSlot {
    uint64_t wr;        // w, r and readers, packed as above
    uint32_t unused;
    uint32_t flag;      // unused
    uint32_t rinit;     // r at the start of the permutation (last full block)
    uint32_t pad[11];
};
static_assert(sizeof(BucketSlot) == 64, "bucket slot size");

template <int DT>
struct Ctx {
    using T = Traits<DT>;
    using Elem = typename T::Elem;
    using Key = typename T::Key;
    Elem* data;
    const TaskD* tasks;
    uint32_t ntasks;
    uint32_t nstripes;
    const StripeD* stripes;
    TaskS* ts;
    Key* tree;                  // [sum k]: tree_begin + i, i in 1..kt-1
    Key* spl;                   // [sum k]: tree_begin + j, sorted splitters (padded)
    uint64_t* bounds;           // [sum (kbuf+1)]: slot_begin + task + i
    uint32_t* delim;            // same indexing as bounds
    BucketSlot* slots;          // [sum kbuf]: slot_begin + i
    uint32_t* counts;           // [stripes][kbuf of the stripe's task]
    uint32_t* stripe_full;      // [stripes] full blocks after classification
    const uint32_t* order;      // [stripes] classification launch order (largest first)
    Elem* bufs;                 // stripe bucket buffers
    uint32_t* err;              // device error word (0 = ok)
    unsigned long long* stats;  // [0] block moves, [1] skips, [2] cleanup placements, [3] fix moves
    uint32_t b;                 // elements per block
    uint32_t spin_limit;
    uint32_t total_workers;
    uint32_t total_slots;
    uint32_t skip_inplace;
    uint32_t vtile;             // classification: virtual tiles of 2 tiles (8-byte keys)
    const uint8_t* fused;       // [sum kbuf] (or null): bucket cleaned by the fused base case, not by k_cleanup
    uint32_t tree_cls;          // classification by the search-tree descent instead of the table
                                // (8-byte keys; for timing the two against each other)
};

// The overflow block of task t (Section 4.2: the partial last block of a
// segment is never written in place): the last side slot of the task's first
// stripe, free from the end of classification on; the overhang slots of the
// cleanup are slots 0 .. K-2 of the same side area (the last bucket, K-1,
// ends at the segment end and has no overhang), and K <= kbuf.
template <int DT>
__device__ inline typename Traits<DT>::Elem* ovf_block(const Ctx<DT>& c, const TaskD& td) {
    return c.bufs + c.stripes[td.stripe_begin].buf_off + ((uint64_t)2 * td.kbuf - 1) * c.b;
}

enum ErrCode : uint32_t {
    ERR_SPIN = 1, ERR_CLEANUP_COUNT = 2, ERR_PERMUTE_RANGE = 4, ERR_FIX = 8,
    // phase invariant checks (debug flag)
    ERR_CHECK_BLOCK = 16,   // a full block after classification mixes buckets
    ERR_CHECK_COUNT = 32,   // recounted buckets differ from the stored counts
    ERR_CHECK_PLACED = 64,  // after the permutation a block in [d_i, w_i) is not of bucket i
    ERR_SEGMENT = 128,      // a small-segment sort got a segment above the capacity, or decreasing offsets
    ERR_MARKS = 256         // bucket bounds beyond the array or decreasing, or a walk over marked
                            // buckets found more buckets than the partition made
};

__device__ inline void raise_err(uint32_t* err, uint32_t code) {
    __hip_atomic_fetch_or(err, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-level counters (0 block moves, 1 skipped in-place blocks, 2 elements
// placed by the cleanup, 3 empty-block fix moves), each kept in STAT_SPREAD
// copies on separate cache lines: per-bucket updates from many workgroups
// would otherwise serialize on one address.  The host sums the copies.
constexpr int STAT_SPREAD = 32;
__device__ inline void stat_add(unsigned long long* stats, int which, unsigned long long v, uint32_t key) {
    atomicAdd(&stats[(key % STAT_SPREAD) * 8 + which], v);
}

// first failure details for diagnostics: err[48..52) = {code, a, b, c}
__device__ inline void raise_err_at(uint32_t* err, uint32_t code, uint32_t a, uint32_t b, uint32_t c) {
    raise_err(err, code);
    if (__hip_atomic_fetch_add(err + 52, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        err[48] = code; err[49] = a; err[50] = b; err[51] = c;
    }
}

// Relaxed agent-scope atomics.  None of the kernels reads, within one
// launch, data another workgroup wrote in that launch, so no acquire or
// release (which would write back and invalidate the L2 of the issuing
// XCD) is needed; where an atomic must follow earlier memory operations
// the code waits for those to complete first (wait_vmem) and keeps the
// compiler from reordering (compiler_fence).
__device__ inline void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }
__device__ inline uint64_t atom_add64(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t atom_add32(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t atom_load64(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t atom_load32(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void atom_store32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// largest index t in [0, n) with begin(t) <= x, for a non-decreasing begin()
template <class F>
__device__ inline uint32_t upper_find(uint32_t n, uint64_t x, F begin) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) / 2;
        if (begin(mid) <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ block scan
// Exclusive scan of one value per thread over the workgroup (NT threads).
// `sh` needs NT/64 + 1 entries.  Returns the exclusive prefix; *total gets
// the sum.  Contains LDS-only barriers: call from every thread.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    constexpr int NW = NT / 64;
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= (uint32_t)d) inc += t;
    }
    if (lane == 63) sh[wid] = inc;
    lds_barrier();
    if (wid == 0) {
        uint32_t t = lane < NW ? sh[lane] : 0u, ti = t;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            uint32_t u = __shfl_up(ti, d, 64);
            if (lane >= (uint32_t)d) ti += u;
        }
        if (lane < NW) sh[lane] = ti - t;
        if (lane == NW - 1) sh[NW] = ti;
    }
    lds_barrier();
    uint32_t r = inc - v + sh[wid];
    *total = sh[NW];
    lds_barrier();
    return r;
}

// In-place exclusive scan of arr[0..n) in LDS (n <= NT * 4).  Returns total.
template <int NT>
__device__ inline uint32_t lds_excl_scan(uint32_t* arr, uint32_t n, uint32_t* sh) {
    const uint32_t per = (n + NT - 1) / NT;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t loc = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < n) loc += arr[b0 + i];
    uint32_t total;
    uint32_t pre = block_excl_scan<NT>(loc, sh, &total);
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < n) {
            uint32_t v = arr[b0 + i];
            arr[b0 + i] = pre;
            pre += v;
        }
    lds_barrier();
    return total;
}

// ------------------------------------------------------- classification
// Branchless descent through the implicit tree (Section 3): j = 1, then
// log2(kt) times j = 2j + [a_j <= e]; leaf = j - kt counts the (padded)
// splitters <= e.  With equality buckets (Section 4, many identical keys)
// one more comparison against the splitter just below decides between the
// equality bucket 2j-1 and the open bucket 2j.
template <class Key>
__device__ inline uint32_t classify_key(const Key& e, const Key* stree, const Key* sspl,
                                        uint32_t log_kt, uint32_t nuniq, uint32_t eq) {
    uint32_t j = 1;
    for (uint32_t l = 0; l < log_kt; ++l) j = 2 * j + (stree[j] <= e ? 1u : 0u);
    j -= (1u << log_kt);
    j = j < nuniq ? j : nuniq;
    if (!eq) return j;
    uint32_t is_eq = (j >= 1 && sspl[j > 0 ? j - 1 : 0] == e) ? 1u : 0u;
    return 2 * j - is_eq;
}

template <int DT>
struct TreeLds {
    typename Traits<DT>::Key tree[KT_MAX];
    typename Traits<DT>::Key spl[KT_MAX];
};

template <int DT>
__device__ inline void load_tree(const Ctx<DT>& c, const TaskD& td, uint32_t kt, uint32_t nuniq,
                                 TreeLds<DT>& L) {
    for (uint32_t i = threadIdx.x; i < kt; i += blockDim.x) {
        L.tree[i] = c.tree[td.tree_begin + i];
        L.spl[i] = c.spl[td.tree_begin + i];
    }
    __syncthreads();
}

__device__ inline uint32_t ilog2(uint32_t x) { return 31u - __clz(x); }

// ------------------------------------------------------------- sampling
// One workgroup per task.  Draws S = alpha*k - 1 sample keys at positions
// floor(h_i * m / 2^64) (h_i: splitmix64 of the task's stream), sorts them in
// LDS (bitonic network), picks s_i = sample[i*alpha - 1], removes
// duplicates, switches equality buckets on when there were any, pads the
// splitter array to a power-of-two tree and stores the level-order tree
// a_i = s_{(2p+1) kt / 2^(l+1)} (l = floor(log2 i), p = i - 2^l).
// SMAX: sample capacity of this instance (every task's alpha*k - 1,
// rounded up to a power of two, must fit).
template <int DT, int NT, int SMAX = sample_max<typename Traits<DT>::Key>()>
__global__ __launch_bounds__(NT) void k_sample(Ctx<DT> c) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    __shared__ Key smp[SMAX];
    __shared__ uint32_t isnew[KT_MAX];
    __shared__ uint32_t scan_sh[NT / 64 + 1];
    const TaskD td = c.tasks[blockIdx.x];
    const uint32_t k = td.k, alpha = td.alpha;
    const uint32_t S = alpha * k - 1;
    uint32_t P = 1;
    while (P < S) P <<= 1;
    {
        // every load of this thread issued before the first store
        constexpr int LPT = SMAX / NT;
        Key v[LPT];
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const uint32_t i = threadIdx.x + (uint32_t)q * NT;
            v[q] = TR::max_key();
            if (i < S) v[q] = TR::key(c.data[td.off + __umul64hi(splitmix64_at(td.seed, i), td.m)]);
        }
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const uint32_t i = threadIdx.x + (uint32_t)q * NT;
            if (i < P) smp[i] = v[q];
        }
    }
    __syncthreads();
    // bitonic sort, ascending, P a power of two
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += NT) {
                uint32_t i = (t / stride) * 2 * stride + (t % stride);
                uint32_t j = i + stride;
                bool up = ((i & size) == 0);
                Key a = smp[i], bb = smp[j];
                bool sw = up ? (bb < a) : (a < bb);
                if (sw) { smp[i] = bb; smp[j] = a; }
            }
            __syncthreads();
        }
    }
    // picks s_i = sample[i*step - 1], i = 1..kp-1, and duplicate removal;
    // returns the number of unique picks (isnew[i]: index among them)
    auto pick_unique = [&](uint32_t kp, uint32_t step) {
        for (uint32_t i = threadIdx.x; i < KT_MAX; i += NT) {
            uint32_t f = 0;
            if (i >= 1 && i < kp) f = (i == 1) ? 1u : (smp[(i - 1) * step - 1] == smp[i * step - 1] ? 0u : 1u);
            isnew[i] = f;
        }
        __syncthreads();
        return lds_excl_scan<NT>(isnew, KT_MAX, scan_sh);
    };
    uint32_t kp = k, step = alpha;
    uint32_t nuniq = pick_unique(kp, step);
    // equality buckets double the bucket count: when 2 nuniq + 1 would
    // exceed the kbuf buckets the task's buffers hold, every second pick is
    // used instead (k/2 picks, twice the oversampling, the same sample),
    // with equality buckets kept on, so K <= k - 1
    bool thinned = false;
    if (nuniq < kp - 1 && 2 * nuniq + 1 > td.kbuf) {
        kp = k / 2;
        step = 2 * alpha;
        thinned = true;
        __syncthreads();
        nuniq = pick_unique(kp, step);
    }
    // the unique picks move to the front of smp (all picks are read before
    // any is overwritten), padded with the largest pick to kt entries; the
    // splitter array and the level-order tree are written from there
    constexpr int PPT = (KT_MAX + NT - 1) / NT;
    Key pk[PPT];
    bool nw[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t i = 1 + threadIdx.x + (uint32_t)q * NT;
        nw[q] = false;
        if (i < kp) {
            pk[q] = smp[i * step - 1];
            nw[q] = (i == 1) || !(smp[(i - 1) * step - 1] == pk[q]);
        }
    }
    const Key last = smp[(kp - 1) * step - 1];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q)
        if (nw[q]) smp[isnew[1 + threadIdx.x + (uint32_t)q * NT]] = pk[q];
    const uint32_t eq = (thinned || nuniq < kp - 1) ? 1u : 0u;
    uint32_t kt = kp;
    if (eq) {
        kt = 2;
        while (kt < nuniq + 1) kt <<= 1;
    }
    __syncthreads();
    for (uint32_t j = nuniq + threadIdx.x; j < kt; j += NT) smp[j] = last;
    __syncthreads();
    Key* spl = c.spl + td.tree_begin;
    Key* tree = c.tree + td.tree_begin;
    for (uint32_t j = threadIdx.x; j < kt; j += NT) spl[j] = smp[j];
    for (uint32_t i = 1 + threadIdx.x; i < kt; i += NT) {
        const uint32_t l = ilog2(i), p = i - (1u << l);
        const uint32_t idx = ((2 * p + 1) * kt) >> (l + 1);   // 1-based splitter index
        tree[i] = smp[idx - 1];
    }
    if (threadIdx.x == 0) {
        TaskS s;
        s.K = eq ? 2 * nuniq + 1 : nuniq + 1;
        s.kt = kt;
        s.eq = eq;
        s.nuniq = nuniq;
        s.nblocks = (uint32_t)((td.m + c.b - 1) / c.b);
        s.ovf_bucket = NO_BUCKET;
        s.pad0 = s.pad1 = 0;
        c.ts[blockIdx.x] = s;
    }
}

// ------------------------------------------- lookup-table classification
// The same bucket as the tree descent, #{i < nuniq : s_i <= e} (and the
// equality rule on top), found with fewer LDS reads.  A table of LUT_N
// cells splits the range of the splitters' leading 64-bit words into equal
// parts: cell c holds the first splitter index lo_c whose leading word
// lies at or beyond the cell's start and the number n_c of splitters whose
// leading word lies inside the cell.  A key's cell follows from its leading
// word; the splitters before lo_c are all below the key and those from
// lo_c + n_c on all above it, so a binary search over the n_c candidates
// finishes the count.  Its step count is the same for every key of the
// workgroup (log2 of the largest n_c + 1): about two for spread-out
// splitters, log2 k when they crowd into one cell.
constexpr int LUT_BITS = 12;
constexpr uint32_t LUT_N = 1u << LUT_BITS;

__device__ inline uint64_t lead_word(const Key1& k) { return k.v; }
__device__ inline uint64_t lead_word(const Key3& k) { return k.a; }
__device__ inline uint64_t lead_word(const Key10& k) { return k.hi; }

struct LutParams {
    uint64_t w_lo;      // leading word of the smallest splitter
    uint32_t sh;        // cell = (w - w_lo) >> sh, clamped to [0, LUT_N)
    uint32_t steps;     // binary-search steps
    uint32_t tree;      // the table area holds the level-order search tree instead
};

// Builds lut[] from the sorted splitters spl[0..nuniq) in LDS; every thread
// of the workgroup calls it.  `red` is NT/64 + 1 words of LDS scratch.
template <class Key, int NT>
__device__ inline LutParams build_lut(const Key* spl, uint32_t nuniq, uint32_t* lut, uint32_t* red) {
    LutParams P;
    P.w_lo = nuniq ? lead_word(spl[0]) : 0;
    const uint64_t span = nuniq ? lead_word(spl[nuniq - 1]) - P.w_lo : 0;
    const uint32_t bits = span ? 64u - (uint32_t)__clzll(span) : 0u;
    P.sh = bits > (uint32_t)LUT_BITS ? bits - LUT_BITS : 0u;
    // first splitter index whose leading word is at or beyond w_lo + off
    auto first_at = [&](uint64_t off) {
        uint32_t lo = 0, hi = nuniq;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (lead_word(spl[mid]) - P.w_lo < off) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    uint32_t nmax = 0;
    for (uint32_t cidx = threadIdx.x; cidx < LUT_N; cidx += NT) {
        const uint32_t lo = cidx == 0 ? 0u : first_at((uint64_t)cidx << P.sh);
        const uint32_t hi = cidx + 1 == LUT_N ? nuniq : first_at((uint64_t)(cidx + 1) << P.sh);
        lut[cidx] = lo | ((hi - lo) << 16);
        nmax = max(nmax, hi - lo);
    }
    // workgroup maximum of n_c
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, (uint32_t)__shfl_xor(nmax, d, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nmax;
    __syncthreads();
    uint32_t m = 0;
    for (int w = 0; w < NT / 64; ++w) m = max(m, red[w]);
    P.steps = m ? 32u - (uint32_t)__clz(m) : 0u;     // ceil(log2(m + 1))
    __syncthreads();
    return P;
}

template <class Key, int EPT>
__device__ inline void classify_lut_batch(const Key (&k)[EPT], uint32_t (&out)[EPT], const Key* spl,
                                          const uint32_t* lut, const LutParams& P, uint32_t nuniq, uint32_t eq) {
    uint32_t base[EPT], len[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint64_t w = lead_word(k[e]);
        const uint64_t off = w > P.w_lo ? w - P.w_lo : 0;
        const uint64_t cl = off >> P.sh;
        const uint32_t cell = cl < LUT_N ? (uint32_t)cl : LUT_N - 1;
        const uint32_t v = lut[cell];
        base[e] = v & 0xffffu;
        len[e] = v >> 16;
    }
    for (uint32_t s = 0; s < P.steps; ++s) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const uint32_t half = len[e] >> 1;
            const bool go = len[e] > 0 && spl[base[e] + half] <= k[e];
            base[e] = go ? base[e] + half + 1 : base[e];
            len[e] = go ? len[e] - half - 1 : half;
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t leaf = base[e];
        uint32_t r = leaf;
        if (eq) {
            const uint32_t is_eq = (leaf >= 1 && spl[leaf > 0 ? leaf - 1 : 0] == k[e]) ? 1u : 0u;
            r = 2 * leaf - is_eq;
        }
        out[e] = r;
    }
}

// ------------------------------------------------------ local classification
// One workgroup per stripe (Section 4.1).  The workgroup keeps one buffer
// block of b elements per bucket; a full buffer block is a finished block of
// the stripe.  To write every element only once, the buffer block a bucket is
// filling ("open" block) is a block of the stripe's own space, and a full
// open block simply stays where it is.  A block location is either a block
// of a side area of K blocks (locations 0 .. K-1) or stripe block q
// (location K + q).  A tile's new blocks take, in allocation order, the next
// stripe blocks as long as those have been read (H stripe blocks used, R
// read: at most R - H of them), and the rest the next side blocks (G used).
// Side blocks are taken only when the stripe is used up to R, and then every
// allocated block beyond R is partly filled (full blocks hold data already
// read), so G never exceeds K.  Presorted data has one or two partly filled
// blocks at a time and keeps its order: only the first block of a bucket that
// starts in a tile whose stripe blocks are used up goes to the side area.
//   phase 1  tiles of NT*EPT elements: classify in registers, counting-sort
//            by bucket in LDS, write every element into its bucket's open
//            block or into new blocks allocated as above;
//   phase 2  move the content of every partly filled open block to the
//            bucket's partial buffer (its block becomes a hole); then the
//            full blocks outside stripe blocks [0, F) (those in the side
//            area and those at or beyond F), in location order, move into
//            the free stripe blocks below F, in order, so the stripe ends as
//            [F full blocks | empty blocks] with the partial buffers outside
//            it, exactly as the paper's local classification leaves it.
template <int DT, int NT, int EPT>
struct ClassifyLds {
    using Elem = typename Traits<DT>::Elem;
    typename Traits<DT>::Key spl[KT_MAX];   // sorted unique splitters
    uint32_t lut[LUT_N];                    // lo_c | n_c << 16
    LutParams lp;
    Elem tile[NT * EPT];
    uint16_t ids[NT * EPT];
    uint32_t cnt[KMAX];         // elements of the tile per bucket (atomic ranks)
    uint32_t fill[KMAX];        // phase 1: fill of the open block (b: none or full);
                                // phase 2: fill of the partial buffer
    uint32_t open[KMAX];        // phase 1: location of the open block
    uint32_t nfull[KMAX];       // phase 1: blocks allocated; then full blocks
    uint32_t off[KMAX];         // start of the bucket's run in the tile
    int32_t lim[KMAX];          // phase 1: tile positions p < lim go to the open block,
    int32_t lim2[KMAX];         // p < lim2 to new stripe blocks, the rest to new side blocks
    int32_t base0[KMAX];        // phase 1: location element of position p: base0 + p,
    int32_t base1[KMAX];        // base1 + p,
    int32_t base2[KMAX];        // base2 + p (location element: location * b + offset)
    uint32_t holes[KMAX];       // locations of evacuated open blocks
    uint64_t scan_sh[NT / 64 + 1];
    uint32_t wf;                // phase 1: stripe blocks used (H); phase 2: list length
    uint32_t gside;             // phase 1: side blocks used (G)
    uint32_t nholes;
    uint32_t nalloc;            // phase 2: list length
};

// Exclusive scan of one 64-bit value per thread over the workgroup.
template <int NT>
__device__ inline uint64_t block_excl_scan64(uint64_t v, uint64_t* sh, uint64_t* total) {
    constexpr int NW = NT / 64;
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(inc, d, 64);
        if (lane >= (uint32_t)d) inc += t;
    }
    if (lane == 63) sh[wid] = inc;
    lds_barrier();
    if (wid == 0) {
        uint64_t t = lane < NW ? sh[lane] : 0ull, ti = t;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            uint64_t u = __shfl_up(ti, d, 64);
            if (lane >= (uint32_t)d) ti += u;
        }
        if (lane < NW) sh[lane] = ti - t;
        if (lane == NW - 1) sh[NW] = ti;
    }
    lds_barrier();
    uint64_t r = inc - v + sh[wid];
    *total = sh[NW];
    lds_barrier();
    return r;
}

// Tree descent for EPT keys at once, level by level, so that the LDS loads
// of the EPT descents are independent of each other.
template <class Key, int EPT>
__device__ inline void classify_batch(const Key (&k)[EPT], uint32_t (&out)[EPT], const Key* stree,
                                      const Key* sspl, uint32_t log_kt, uint32_t nuniq, uint32_t eq) {
    uint32_t j[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) j[e] = 1;
    for (uint32_t l = 0; l < log_kt; ++l) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) j[e] = 2 * j[e] + (stree[j[e]] <= k[e] ? 1u : 0u);
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        uint32_t leaf = j[e] - (1u << log_kt);
        leaf = leaf < nuniq ? leaf : nuniq;
        uint32_t r = leaf;
        if (eq) {
            const uint32_t is_eq = (leaf >= 1 && sspl[leaf > 0 ? leaf - 1 : 0] == k[e]) ? 1u : 0u;
            r = 2 * leaf - is_eq;
        }
        out[e] = r;
    }
}

// Classify the tile held in x[] (tn valid elements) and rank every element
// within its bucket: one LDS atomic per wavefront when all its lanes share a
// bucket (skewed inputs), else one per element.  PACK: the rank goes into
// bits 10.. of bk[] (bucket < 1024) instead of rk[].
template <int DT, int NT, int EPT, bool FULL, bool PACK = false>
__device__ inline void classify_rank(ClassifyLds<DT, NT, EPT>& L, const typename Traits<DT>::Elem (&x)[EPT],
                                     uint32_t tn, uint32_t lkt, const TaskS& st, uint32_t (&bk)[EPT],
                                     uint32_t (&rk)[EPT]) {
    using TR = Traits<DT>;
    typename TR::Key kk[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) kk[e] = TR::key(x[e]);
    if (sizeof(typename TR::Key) == 8 && L.lp.tree)
        classify_batch<typename TR::Key, EPT>(kk, bk, reinterpret_cast<const typename TR::Key*>(L.lut), L.spl, lkt,
                                              st.nuniq, st.eq);
    else
        classify_lut_batch<typename TR::Key, EPT>(kk, bk, L.spl, L.lut, L.lp, st.nuniq, st.eq);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t p = e * NT + threadIdx.x;
        const bool valid = FULL || p < tn;
        const uint64_t vmask = __ballot(valid);
        const uint32_t b0 = __builtin_amdgcn_readfirstlane(bk[e]);
        const uint64_t same = __ballot(valid && bk[e] == b0);
        if (same == vmask) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
            uint32_t base = 0;
            if (below == 0 && valid) base = atomicAdd(&L.cnt[b0], (uint32_t)__popcll(same));
            base = __builtin_amdgcn_readfirstlane(base);
            if constexpr (PACK) bk[e] |= (base + below) << 10;
            else rk[e] = base + below;
        } else if (valid) {
            const uint32_t r = atomicAdd(&L.cnt[bk[e]], 1u);
            if constexpr (PACK) bk[e] |= r << 10;
            else rk[e] = r;
        }
    }
}

template <int DT, int NT, int EPT, bool FULL>
__device__ inline void scatter_tile(ClassifyLds<DT, NT, EPT>& L, const typename Traits<DT>::Elem (&x)[EPT],
                                    uint32_t tn, const uint32_t (&bk)[EPT], const uint32_t (&rk)[EPT]) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t p = e * NT + threadIdx.x;
        if (FULL || p < tn) {
            const uint32_t q = L.off[bk[e]] + rk[e];
            L.tile[q] = x[e];
            L.ids[q] = (uint16_t)bk[e];
        }
    }
}

template <int DT, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_classify(Ctx<DT> c) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    using Word = typename TR::Word;
    constexpr uint32_t TILE = NT * EPT;
    constexpr uint32_t PER = (KMAX + NT - 1) / NT;      // buckets per thread in the scans
    constexpr uint32_t WPE = sizeof(Elem) / sizeof(Word);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    auto& L = *reinterpret_cast<ClassifyLds<DT, NT, EPT>*>(smem_raw);

    const uint32_t sid = c.order[blockIdx.x];
    const StripeD sd = c.stripes[sid];
    const TaskD td = c.tasks[sd.task];
    const TaskS st = c.ts[sd.task];
    const uint32_t b = c.b, lb = ilog2(c.b), K = st.K, lkt = ilog2(st.kt);
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < st.nuniq; i += NT) L.spl[i] = c.spl[td.tree_begin + i];
    __syncthreads();
    if (sizeof(typename TR::Key) == 8 && c.tree_cls) {
        // the search tree a_1 .. a_{kt-1} (level order) in the table's place
        typename TR::Key* t = reinterpret_cast<typename TR::Key*>(L.lut);
        static_assert(sizeof(L.lut) >= KT_MAX * 8, "tree fits the table area");
        for (uint32_t i = 1 + threadIdx.x; i < st.kt; i += NT) t[i] = c.tree[td.tree_begin + i];
        if (threadIdx.x == 0) L.lp = LutParams{0, 0, 0, 1u};
        __syncthreads();
    } else {
        LutParams P = build_lut<typename TR::Key, NT>(L.spl, st.nuniq, L.lut, L.holes);
        P.tree = 0;
        if (threadIdx.x == 0) L.lp = P;
    }

    const uint64_t s_begin = (uint64_t)sd.blk_begin * b;
    const uint64_t s_end = ((uint64_t)sd.blk_end * b < td.m) ? (uint64_t)sd.blk_end * b : td.m;
    const uint32_t E = (uint32_t)(s_end - s_begin);         // stripe elements
    Elem* sp = c.data + td.off + s_begin;                   // the stripe
    Elem* buf = c.bufs + sd.buf_off;                        // partial buffers, bucket j at j*b
    Elem* side = buf + ((uint64_t)td.kbuf << lb);           // slots 0 .. K-1
    const int64_t KB = (int64_t)K << lb;
    // element e of slot space (slot e >> lb) in memory
    auto slot_elem = [&](int64_t e) -> Elem* { return e < KB ? side + e : sp + (e - KB); };

    for (uint32_t q = threadIdx.x; q < K; q += NT) {
        L.cnt[q] = 0; L.fill[q] = b; L.open[q] = 0; L.nfull[q] = 0;
    }
    if (threadIdx.x == 0) { L.wf = 0; L.gside = 0; L.nholes = 0; L.nalloc = 0; }
    __syncthreads();

    // ---- phase 1: the stripe, straight into open blocks.
    // Full tiles take a path without per-element guards: straight-line
    // loads and stores let the compiler wait for exactly the loads it needs
    // instead of every outstanding memory operation.
    Elem x[EPT];
    auto load_tile = [&](const Elem* src, uint32_t t0, uint32_t end) {
        const uint32_t rem = end > t0 ? end - t0 : 0u;
        if (rem >= TILE) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) x[e] = src[t0 + e * NT + threadIdx.x];
        } else {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t p = e * NT + threadIdx.x;
                if (p < rem) x[e] = src[t0 + p];
            }
        }
    };
    // per-bucket bookkeeping of a tile of tn keys starting at stripe
    // position t0 whose ranks are in cnt: run offsets, where each run
    // position goes (open block, new stripe blocks, new side blocks), the
    // counters cleared for the next tile; false if the side area would
    // overflow (checked before any write)
    auto plan_tile = [&](uint32_t t0, uint32_t tn) -> bool {
        {
            // per bucket: run offset (bits 0..19), 1 if it gets new blocks
            // (bits 20..39) and its new blocks (bits 40..63).  Stream
            // position pos = fill + rank lies in the open block while
            // pos < b, else in new block (pos >> lb) - 1 counted from the
            // bucket's first new block.  C of the tile's Tn new blocks take
            // stripe blocks H.. (C: stripe blocks read but not used yet),
            // E = Tn - C take side blocks G..: the first new block of each of
            // the last E buckets that get new blocks (presorted data then
            // keeps its order once phase 2 moves them into the holes left by
            // the partly filled blocks before them), or, when fewer buckets
            // than E get new blocks, the last E new blocks in scan order.
            const uint32_t H = L.wf, G = L.gside, R = (t0 + tn) >> lb;
            uint64_t v[PER], loc = 0;
#pragma unroll
            for (uint32_t q = 0; q < PER; ++q) {
                const uint32_t jb = threadIdx.x * PER + q;
                v[q] = 0;
                if (jb < K) {
                    const uint32_t cn = L.cnt[jb];
                    L.cnt[jb] = 0;              // ready for the next tile's ranks
                    const uint32_t nn = cn ? ((L.fill[jb] + cn - 1) >> lb) : 0u;
                    v[q] = ((uint64_t)nn << 40) | ((uint64_t)(nn ? 1u : 0u) << 20) | cn;
                }
                loc += v[q];
            }
            uint64_t total;
            uint64_t pre = block_excl_scan64<NT>(loc, L.scan_sh, &total);
            const uint32_t Tn = (uint32_t)(total >> 40), M = (uint32_t)(total >> 20) & 0xfffffu;
            const uint32_t C = R > H ? min(R - H, Tn) : 0u, E = Tn - C;
            const bool firsts = E <= M;                 // side blocks: first new blocks of the last E buckets
#pragma unroll
            for (uint32_t q = 0; q < PER; ++q) {
                const uint32_t jb = threadIdx.x * PER + q;
                if (jb < K) {
                    const int32_t o = (int32_t)(pre & 0xfffffu), r = (int32_t)(pre >> 40);
                    const uint32_t ib = (uint32_t)(pre >> 20) & 0xfffffu;     // buckets with new blocks before
                    const uint32_t f = L.fill[jb], cn = (uint32_t)v[q] & 0xfffffu, nn = (uint32_t)(v[q] >> 40);
                    const int32_t bi = (int32_t)b, fi = (int32_t)f, Ci = (int32_t)C;
                    const int32_t S0 = (int32_t)(K + H), G0 = (int32_t)G;
                    L.off[jb] = (uint32_t)o;
                    L.lim[jb] = o + bi - fi;
                    L.base0[jb] = (int32_t)(L.open[jb] << lb) - o + fi;
                    if (firsts) {
                        const bool chosen = nn && ib + E >= M;
                        const int32_t cj = ib + E > M ? (int32_t)(ib + E - M) : 0;   // chosen buckets before
                        if (chosen) {
                            // new block 0 -> side block G + cj, blocks 1.. -> stripe
                            L.lim2[jb] = o + 2 * bi - fi;
                            L.base1[jb] = (G0 + cj - 1) * bi - o + fi;
                            L.base2[jb] = (S0 + r - cj - 2) * bi - o + fi;
                        } else {
                            L.lim2[jb] = 0x7fffffff;
                            L.base1[jb] = (S0 + r - cj - 1) * bi - o + fi;
                            L.base2[jb] = 0;
                        }
                        if (nn) {
                            L.open[jb] = chosen ? (nn == 1 ? (uint32_t)(G0 + cj) : (uint32_t)(S0 + r - cj) + nn - 2)
                                                : (uint32_t)(S0 + r - cj) + nn - 1;
                            L.nfull[jb] += nn;
                        }
                    } else {
                        // the first C new blocks in scan order -> stripe, the rest -> side
                        L.lim2[jb] = o + (Ci - r + 1) * bi - fi;
                        L.base1[jb] = (S0 + r - 1) * bi - o + fi;
                        L.base2[jb] = (G0 + r - Ci - 1) * bi - o + fi;
                        if (nn) {
                            const uint32_t last = (uint32_t)r + nn - 1;
                            L.open[jb] = last < C ? K + H + last : G + (last - C);
                            L.nfull[jb] += nn;
                        }
                    }
                    if (cn) L.fill[jb] = ((f + cn - 1) & (b - 1)) + 1;
                    pre += v[q];
                }
            }
            if (threadIdx.x == 0) {
                L.wf = H + C;
                L.gside = G + E;
            }
        }
        lds_barrier();
        // never more side blocks than the side area holds (cannot happen:
        // see above); checked before any write
        if (L.gside > K) {
            if (threadIdx.x == 0) raise_err(c.err, ERR_CHECK_BLOCK);
            return false;
        }
        return true;
    };
    // memory location element of tile position p of bucket jb
    auto loc_of = [&](uint32_t p, uint32_t jb) -> int64_t {
        const int32_t pi = (int32_t)p;
        const int32_t base = pi < L.lim[jb] ? L.base0[jb] : (pi < L.lim2[jb] ? L.base1[jb] : L.base2[jb]);
        return (int64_t)(base + pi);
    };
    auto phase1_tile = [&](uint32_t t0, uint32_t tn, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        uint32_t bk[EPT], rk[EPT];
        classify_rank<DT, NT, EPT, FULL>(L, x, tn, lkt, st, bk, rk);
        lds_barrier();
        if (!plan_tile(t0, tn)) return false;
        scatter_tile<DT, NT, EPT, FULL>(L, x, tn, bk, rk);
        lds_barrier();
        if constexpr (FULL) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t p = e * NT + threadIdx.x;
                *slot_elem(loc_of(p, L.ids[p])) = L.tile[p];
            }
        } else {
            for (uint32_t p = threadIdx.x; p < tn; p += NT) *slot_elem(loc_of(p, L.ids[p])) = L.tile[p];
        }
        // no barrier here: the next tile's ranking only touches cnt (cleared
        // by plan_tile), and the barrier after it comes before anything this
        // loop reads is overwritten
        return true;
    };
    // A virtual tile of 2 TILE keys (8-byte keys only): x holds the first
    // TILE, x2 the second.  Both halves are ranked together (cnt counts on
    // across them), so every bucket's run is twice as long as in a tile
    // and its writes cover whole cache lines more often; the runs are then
    // scattered and written in two passes by tile position, positions
    // [0, TILE) first, through the one TILE-key LDS buffer.  Bucket and rank
    // of a key travel packed in one word (bucket < 1024, rank < 2^14).
    auto phase1_vtile = [&](uint32_t t0, const Elem (&x2)[EPT]) -> bool {
        static_assert(KMAX <= 1024 && 2 * TILE <= (1u << 22), "bucket and rank packed in one word");
        uint32_t br[EPT], br2[EPT], unused[EPT];
        classify_rank<DT, NT, EPT, true, true>(L, x, TILE, lkt, st, br, unused);
        classify_rank<DT, NT, EPT, true, true>(L, x2, TILE, lkt, st, br2, unused);
        lds_barrier();
        if (!plan_tile(t0, 2 * TILE)) return false;
#pragma unroll
        for (uint32_t h = 0; h < 2; ++h) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t j = br[e] & 1023u, q = L.off[j] + (br[e] >> 10) - h * TILE;
                if (q < TILE) { L.tile[q] = x[e]; L.ids[q] = (uint16_t)j; }
                const uint32_t j2 = br2[e] & 1023u, q2 = L.off[j2] + (br2[e] >> 10) - h * TILE;
                if (q2 < TILE) { L.tile[q2] = x2[e]; L.ids[q2] = (uint16_t)j2; }
            }
            lds_barrier();
#pragma unroll 2
            for (int e = 0; e < EPT; ++e) {
                const uint32_t p = e * NT + threadIdx.x;
                *slot_elem(loc_of(h * TILE + p, L.ids[p])) = L.tile[p];
            }
            if (h == 0) lds_barrier();      // the second pass overwrites tile and ids
        }
        return true;
    };
    uint32_t t0 = 0;
    if constexpr (sizeof(Elem) == 8) {
        if (c.vtile) {
            Elem x2[EPT];
            for (; t0 + 2 * TILE <= E; t0 += 2 * TILE) {
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    x[e] = sp[t0 + e * NT + threadIdx.x];
                    x2[e] = sp[t0 + TILE + e * NT + threadIdx.x];
                }
                if (!phase1_vtile(t0, x2)) return;
            }
        }
    }
    load_tile(sp, t0, E);
    {
        // steady state: the next tile is full too.  Its loads go to a second
        // register set at the start of the iteration; the body has no other
        // loads and no data-dependent branches around memory operations, so
        // waiting for those loads later does not wait for this tile's stores.
        Elem xn[EPT];
        for (; t0 + 2 * TILE <= E; t0 += TILE) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) xn[e] = sp[t0 + TILE + e * NT + threadIdx.x];
            if (!phase1_tile(t0, TILE, std::true_type{})) return;
#pragma unroll
            for (int e = 0; e < EPT; ++e) x[e] = xn[e];
        }
    }
    for (; t0 < E; t0 += TILE) {
        const uint32_t tn = (E - t0) < TILE ? (E - t0) : TILE;
        const bool ok = tn == TILE ? phase1_tile(t0, TILE, std::true_type{}) : phase1_tile(t0, tn, std::false_type{});
        if (!ok) return;
        if (t0 + TILE < E) load_tile(sp, t0 + TILE, E);
    }
    __syncthreads();        // phase 1's stores are read back in phase 2

    // ---- phase 2: evacuate partly filled open blocks ...
    for (uint32_t jb = threadIdx.x; jb < K; jb += NT) {
        const uint32_t f = L.fill[jb];
        if (f < b) {
            L.holes[atomicAdd(&L.nholes, 1u)] = L.open[jb];
            L.nfull[jb] -= 1;               // that block is not full
        } else {
            L.fill[jb] = 0;                 // the partial buffer stays empty
        }
    }
    __syncthreads();
    for (uint32_t jb = wid; jb < K; jb += NT / 64) {
        const uint32_t f = L.fill[jb];
        if (f == 0) continue;
        const Elem* src = slot_elem((int64_t)L.open[jb] << lb);
        Elem* dst = buf + ((uint64_t)jb << lb);
        for (uint32_t r = lane; r < f; r += 64) dst[r] = src[r];
    }
    __syncthreads();
    // ... then every full block outside stripe blocks [0, F) moves into a
    // free stripe block below F; both lists in location order (scratch in
    // the tile area), so that data that arrived in order keeps it
    const uint32_t H1 = L.wf, G1 = L.gside, O = L.nholes, F = G1 + H1 - O;
    __syncthreads();                                 // every wave has read wf, gside and nholes
    // hole bits: side blocks [0, K) in words [0, KW), stripe block q at bit
    // q of words [KW, KW + SW)
    uint32_t* hole_bits = reinterpret_cast<uint32_t*>(L.tile);
    const uint32_t KW = (K + 31) / 32, SW = (H1 + 31) / 32, nbits = KW + SW;
    // at most G1 <= K side blocks plus O <= K stripe blocks at or beyond F
    // move, into at most O holes plus F - H1 <= G1 unused stripe blocks
    uint32_t* mis = hole_bits + nbits;               // full blocks to move (locations)
    uint32_t* fre = mis + 2 * K;                     // free stripe blocks below F
    uint32_t* sh32 = reinterpret_cast<uint32_t*>(L.scan_sh);
    static_assert(sizeof(L.tile) >= 4 * (4 * KMAX + 1024), "phase 2 scratch in the tile area");
    if (nbits + 4 * K > sizeof(L.tile) / 4) {        // stripes of more than 2^15 blocks
        if (threadIdx.x == 0) raise_err(c.err, ERR_CHECK_BLOCK);
        return;
    }
    for (uint32_t i = threadIdx.x; i < nbits; i += NT) hole_bits[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < O; i += NT) {
        const uint32_t h = L.holes[i];
        const uint32_t bit = h < K ? h : 32 * KW + (h - K);
        atomicOr(&hole_bits[bit >> 5], 1u << (bit & 31));
    }
    __syncthreads();
    auto is_hole = [&](uint32_t bit) { return (hole_bits[bit >> 5] >> (bit & 31)) & 1u; };
    // full blocks to move, in location order: side blocks [0, G1), then
    // stripe blocks [F, H1)
    uint32_t nmis = 0, nfre = 0;
    const uint32_t top = H1 > F ? H1 - F : 0u;
    for (uint32_t u0 = 0; u0 < G1 + top; u0 += NT) {
        const uint32_t u = u0 + threadIdx.x;
        uint32_t fm = 0, loc = 0;
        if (u < G1 + top) {
            loc = u < G1 ? u : K + F + (u - G1);
            fm = is_hole(u < G1 ? u : 32 * KW + F + (u - G1)) ? 0u : 1u;
        }
        uint32_t tm;
        const uint32_t pm = block_excl_scan<NT>(fm, sh32, &tm);
        if (fm && nmis + pm < 2 * K) mis[nmis + pm] = loc;
        nmis += tm;
    }
    // free stripe blocks below F, in order: the holes (a word of hole bits
    // per thread), then the stripe blocks [H1, F) never used
    const uint32_t fw = (min(F, H1) + 31) / 32;
    for (uint32_t w0 = 0; w0 < fw; w0 += NT) {
        const uint32_t w = w0 + threadIdx.x;
        uint32_t word = 0;
        if (w < fw) {
            word = hole_bits[KW + w];
            const uint32_t lim_q = min(F, H1);
            if (32 * w + 32 > lim_q) word &= (lim_q - 32 * w >= 32) ? ~0u : ((1u << (lim_q - 32 * w)) - 1u);
        }
        uint32_t tf;
        uint32_t pf = block_excl_scan<NT>((uint32_t)__popc(word), sh32, &tf);
        while (word) {
            const uint32_t bit = (uint32_t)__ffs(word) - 1u;
            if (nfre + pf < 2 * K) fre[nfre + pf] = 32 * w + bit;
            ++pf;
            word &= word - 1u;
        }
        nfre += tf;
    }
    for (uint32_t q = H1 + threadIdx.x; q < F; q += NT)      // stripe blocks never used
        if (nfre + (q - H1) < 2 * K) fre[nfre + (q - H1)] = q;
    nfre += F > H1 ? F - H1 : 0u;
    __syncthreads();
    const uint32_t nmove = nmis;
    if (nmis != nfre || nmis > 2 * K) {
        if (threadIdx.x == 0) raise_err(c.err, ERR_CHECK_BLOCK);
    } else {
        for (uint32_t i = wid; i < nmove; i += NT / 64) {
            const Word* sw = reinterpret_cast<const Word*>(slot_elem((int64_t)mis[i] << lb));
            Word* dw = reinterpret_cast<Word*>(sp + ((uint64_t)fre[i] << lb));
            // eight words per lane in flight: all loads of a chunk before its stores
            for (uint32_t i0 = 0; i0 < b * WPE; i0 += 8 * 64) {
                Word tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t w = i0 + u * 64 + lane;
                    if (w < b * WPE) tmp[u] = sw[w];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t w = i0 + u * 64 + lane;
                    if (w < b * WPE) dw[w] = tmp[u];
                }
            }
        }
    }
    const uint32_t full_blocks = F;
    __syncthreads();
    uint32_t* cnt_out = c.counts + td.cnt_begin + (uint64_t)(sid - td.stripe_begin) * td.kbuf;
    for (uint32_t q = threadIdx.x; q < K; q += NT) cnt_out[q] = (L.nfull[q] << lb) + L.fill[q];
    if (threadIdx.x == 0) c.stripe_full[sid] = full_blocks;
}

// --------------------------------------------------------------- scan
// One workgroup per task: C_i = sum over stripes, bounds B_i (exclusive
// prefix), delimiters d_i = ceil(B_i / b) (Section 4.2).  Also resets the
// overflow owner of the task.  With few buckets the
// stripes are summed by NT / K thread groups side by side.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_scan(Ctx<DT> c) {
    // bucket totals are 64-bit: a bucket of a subproblem of 2^32 or more
    // elements (all-equal keys, say) can hold that many
    __shared__ uint64_t tot[KMAX];
    __shared__ uint64_t part[NT];
    __shared__ uint64_t sh[NT / 64 + 1];
    const uint32_t t = blockIdx.x;
    const TaskD td = c.tasks[t];
    const uint32_t K = c.ts[t].K;
    const uint32_t P = K <= NT / 2 ? NT / K : 1u;
    if (P > 1) {
        const uint32_t j = threadIdx.x % K, p = threadIdx.x / K;
        uint64_t s = 0;
        if (p < P)
            for (uint32_t q = p; q < td.nstripes; q += P) s += c.counts[td.cnt_begin + (uint64_t)q * td.kbuf + j];
        part[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < K) {
            uint64_t v = 0;
            for (uint32_t q = 0; q < P; ++q) v += part[q * K + threadIdx.x];
            tot[threadIdx.x] = v;
        }
    } else {
        for (uint32_t j = threadIdx.x; j < K; j += NT) {
            uint64_t s = 0;
            for (uint32_t q = 0; q < td.nstripes; ++q) s += c.counts[td.cnt_begin + (uint64_t)q * td.kbuf + j];
            tot[j] = s;
        }
    }
    __syncthreads();
    // exclusive prefix over the K totals, PER consecutive buckets a thread
    constexpr uint32_t PER = (KMAX + NT - 1) / NT;
    uint64_t loc = 0;
#pragma unroll
    for (uint32_t i = 0; i < PER; ++i) {
        const uint32_t j = threadIdx.x * PER + i;
        if (j < K) loc += tot[j];
    }
    uint64_t total;
    uint64_t pre = block_excl_scan64<NT>(loc, sh, &total);
    (void)total;
    uint64_t* bd = c.bounds + td.slot_begin + t;
    uint32_t* dl = c.delim + td.slot_begin + t;
#pragma unroll
    for (uint32_t i = 0; i < PER; ++i) {
        const uint32_t j = threadIdx.x * PER + i;
        if (j < K) {
            bd[j] = pre;
            dl[j] = (uint32_t)((pre + c.b - 1) / c.b);
            pre += tot[j];
        }
    }
    if (threadIdx.x == 0) {
        bd[K] = td.m;
        dl[K] = (uint32_t)((td.m + c.b - 1) / c.b);
        c.ts[t].ovf_bucket = NO_BUCKET;
    }
}

// ------------------------------------------------------ empty-block fix
// One workgroup per bucket (grid: bucket, task from task0; NSMAX bounds the
// stripes of a task).  Within the bucket's block range
// [d_i, d_{i+1}) the stripes contribute runs "full, then empty".  Count the
// full blocks occ; the first occ positions must all be full: the empty ones
// among them ("holes") receive, in order, the full blocks found at or after
// d_i + occ ("stragglers"), as in Appendix A.  Then w_i = d_i and
// r_i = d_i + occ - 1.
template <int DT, int NT, int NSMAX>
__global__ __launch_bounds__(NT) void k_fix_empty(Ctx<DT> c, uint32_t task0) {
    using Elem = typename Traits<DT>::Elem;
    using Word = typename Traits<DT>::Word;
    __shared__ uint32_t hpre[NSMAX + 1];
    __shared__ uint32_t spre[NSMAX + 1];
    __shared__ uint32_t occpre[NSMAX + 1];
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint32_t t = task0 + blockIdx.y;
    const TaskD td = c.tasks[t];
    const uint32_t j = blockIdx.x;
    const uint32_t K = c.ts[t].K;
    if (j >= K) return;
    if (td.nstripes > NSMAX) {                  // the launch chose the wrong variant
        if (threadIdx.x == 0) raise_err(c.err, ERR_FIX);
        return;
    }
    const uint32_t b = c.b;
    const uint32_t* dl = c.delim + td.slot_begin + t;
    const uint32_t d0 = dl[j], d1 = dl[j + 1];
    const uint32_t ns = td.nstripes;
    // per-stripe occupied counts inside [d0, d1)
    for (uint32_t q = threadIdx.x; q < ns; q += NT) {
        const StripeD sd = c.stripes[td.stripe_begin + q];
        uint32_t lo = sd.blk_begin > d0 ? sd.blk_begin : d0;
        uint32_t hi = sd.blk_end < d1 ? sd.blk_end : d1;
        uint32_t fe = sd.blk_begin + c.stripe_full[td.stripe_begin + q];
        uint32_t o = 0;
        if (lo < hi && fe > lo) o = (fe < hi ? fe : hi) - lo;
        occpre[q] = o;
    }
    __syncthreads();
    const uint32_t occ = lds_excl_scan<NT>(occpre, ns, sh);
    const uint32_t target = d0 + occ;
    for (uint32_t q = threadIdx.x; q < ns; q += NT) {
        const StripeD sd = c.stripes[td.stripe_begin + q];
        uint32_t lo = sd.blk_begin > d0 ? sd.blk_begin : d0;
        uint32_t hi = sd.blk_end < d1 ? sd.blk_end : d1;
        uint32_t fe = sd.blk_begin + c.stripe_full[td.stripe_begin + q];
        uint32_t h = 0, s = 0;
        if (lo < hi) {
            uint32_t oe = fe < lo ? lo : (fe < hi ? fe : hi);     // end of the full run
            uint32_t he = hi < target ? hi : target;               // holes: [oe, he)
            if (he > oe) h = he - oe;
            uint32_t sb = lo > target ? lo : target;               // stragglers: [sb, oe)
            if (oe > sb) s = oe - sb;
        }
        hpre[q] = h;
        spre[q] = s;
    }
    __syncthreads();
    const uint32_t nh = lds_excl_scan<NT>(hpre, ns, sh);
    const uint32_t nsg = lds_excl_scan<NT>(spre, ns, sh);
    if (nh != nsg && threadIdx.x == 0) raise_err(c.err, ERR_FIX);
    hpre[ns] = nh;
    spre[ns] = nsg;
    if (threadIdx.x == 0 && nh) stat_add(c.stats, 3, nh, blockIdx.x);
    __syncthreads();
    // moves: the x-th hole receives the x-th straggler; one wavefront per move
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Elem* seg = c.data + td.off;
    const uint32_t words = b * (uint32_t)(sizeof(Elem) / sizeof(Word));
    for (uint32_t x = wid; x < nh; x += NT / 64) {
        uint32_t qh = upper_find(ns, x, [&](uint32_t i) { return (uint64_t)hpre[i]; });
        while (qh + 1 < ns && hpre[qh + 1] <= x) ++qh;
        uint32_t qs = upper_find(ns, x, [&](uint32_t i) { return (uint64_t)spre[i]; });
        while (qs + 1 < ns && spre[qs + 1] <= x) ++qs;
        const StripeD sh_ = c.stripes[td.stripe_begin + qh];
        const StripeD ss_ = c.stripes[td.stripe_begin + qs];
        uint32_t lo_h = sh_.blk_begin > d0 ? sh_.blk_begin : d0;
        uint32_t fe_h = sh_.blk_begin + c.stripe_full[td.stripe_begin + qh];
        uint32_t oe_h = fe_h < lo_h ? lo_h : fe_h;
        uint32_t dst_blk = oe_h + (x - hpre[qh]);
        uint32_t lo_s = ss_.blk_begin > d0 ? ss_.blk_begin : d0;
        uint32_t sb = lo_s > target ? lo_s : target;
        uint32_t src_blk = sb + (x - spre[qs]);
        const uint64_t full_blocks = td.m / b;
        if (dst_blk >= full_blocks || src_blk >= full_blocks || dst_blk < d0 || src_blk >= d1) {
            if (lane == 0) raise_err(c.err, ERR_FIX);
            continue;
        }
        Word* dw = reinterpret_cast<Word*>(seg + (uint64_t)dst_blk * b);
        const Word* sw = reinterpret_cast<const Word*>(seg + (uint64_t)src_blk * b);
        // eight words per lane in flight: all loads of a chunk before its stores
        for (uint32_t i0 = 0; i0 < words; i0 += 8 * 64) {
            Word tmp[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t i = i0 + u * 64 + lane;
                if (i < words) tmp[u] = sw[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t i = i0 + u * 64 + lane;
                if (i < words) dw[i] = tmp[u];
            }
        }
    }
    // In-place prefix: the first full blocks of the range may hold bucket j
    // already (presorted inputs; a bucket that holds the whole task).  They
    // count as processed: w starts after them, so that no worker reads or
    // moves them.  A full block holds one bucket, so its first element
    // decides.
    __shared__ uint32_t first_foreign;
    const uint64_t* bd = c.bounds + td.slot_begin + t;
    const bool whole = bd[j + 1] - bd[j] == td.m;       // every block holds bucket j
    if (threadIdx.x == 0) first_foreign = c.skip_inplace ? occ : 0u;
    if (c.skip_inplace && occ > 0 && !whole) {
        __syncthreads();                        // this workgroup's moves above are visible
        using Key = typename Traits<DT>::Key;
        const TaskS st = c.ts[t];
        const Key* spl = c.spl + td.tree_begin;
        // bucket j is [lower, upper) of the keys, or one splitter value
        const uint32_t leaf = st.eq ? (j + 1) / 2 : j;
        const bool eq_bucket = st.eq && (j & 1);
        const bool has_lo = leaf >= 1, has_hi = leaf < st.nuniq;
        const Key klo = has_lo ? spl[leaf - 1] : Key{}, khi = has_hi ? spl[leaf] : Key{};
        auto in_bucket = [&](const Key& e) {
            if (eq_bucket) return e == klo;
            if (has_lo && (st.eq ? !(klo < e) : e < klo)) return false;
            return !has_hi || e < khi;
        };
        // the first block alone first: on unsorted inputs it decides
        for (uint32_t i0 = 0, step = 1; i0 < occ; i0 += step, step = NT) {
            const uint32_t i = i0 + threadIdx.x;
            if (threadIdx.x < step && i < occ && !in_bucket(Traits<DT>::key(seg[(uint64_t)(d0 + i) * b])))
                atomicMin(&first_foreign, i);
            __syncthreads();
            if (first_foreign < occ) break;
        }
        // A presorted range whose prefix ends at a few foreign blocks (a
        // stripe leaves its first allocated blocks at its end): list the nf
        // foreign blocks after the prefix (at most FMAX, else the range stays
        // as it is) and swap every foreign block below the last nf positions
        // with an in-place block among those positions; then the first
        // occ - nf blocks all hold bucket j and count as processed.
        const uint32_t p0 = first_foreign;
        if (p0 > 0 && p0 < occ) {
            constexpr uint32_t FMAX = NT >= 1024 ? 2048 : 128;
            __shared__ uint32_t flist[FMAX], ilist[FMAX];
            uint32_t nf = 0;
            bool fits = true;
            for (uint32_t base = p0; base < occ; base += NT) {
                const uint32_t i = base + threadIdx.x;
                const uint32_t f =
                    (i < occ && !in_bucket(Traits<DT>::key(seg[(uint64_t)(d0 + i) * b]))) ? 1u : 0u;
                uint32_t tot;
                const uint32_t pre = block_excl_scan<NT>(f, sh, &tot);
                if (nf + tot > FMAX) { fits = false; break; }        // tot is the same in every thread
                if (f) flist[nf + pre] = i;
                nf += tot;
            }
            if (fits) {
                // the in-place blocks among the last nf positions: as many as
                // the foreign blocks below them, which are flist[0 .. ni)
                const uint32_t lo = occ - nf;
                uint32_t ni = 0;
                for (uint32_t base = lo; base < occ; base += NT) {
                    const uint32_t i = base + threadIdx.x;
                    const uint32_t f =
                        (i < occ && in_bucket(Traits<DT>::key(seg[(uint64_t)(d0 + i) * b]))) ? 1u : 0u;
                    uint32_t tot;
                    const uint32_t pre = block_excl_scan<NT>(f, sh, &tot);
                    if (f) ilist[ni + pre] = i;
                    ni += tot;
                }
                __syncthreads();
                const uint32_t lane = threadIdx.x & 63;
                const uint32_t words = b * (uint32_t)(sizeof(Elem) / sizeof(Word));
                for (uint32_t x = threadIdx.x >> 6; x < ni; x += NT / 64) {
                    Word* pa = reinterpret_cast<Word*>(seg + (uint64_t)(d0 + flist[x]) * b);
                    Word* pb = reinterpret_cast<Word*>(seg + (uint64_t)(d0 + ilist[x]) * b);
                    for (uint32_t i0 = 0; i0 < words; i0 += 4 * 64) {
                        Word ta[4], tb[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t i = i0 + u * 64 + lane;
                            if (i < words) { ta[u] = pa[i]; tb[u] = pb[i]; }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t i = i0 + u * 64 + lane;
                            if (i < words) { pa[i] = tb[u]; pb[i] = ta[u]; }
                        }
                    }
                }
                if (threadIdx.x == 0) {
                    first_foreign = lo;
                    if (ni) stat_add(c.stats, 3, ni, blockIdx.x);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prefix = first_foreign;
        c.slots[td.slot_begin + j].wr = wr_pack((int64_t)d0 + prefix, (int64_t)d0 + occ - 1);
        c.slots[td.slot_begin + j].rinit = d0 + occ;   // one past the last full block
    }
}

// ------------------------------------------------------ block permutation
// Wavefront workers (Section 4.2).  A worker takes an unprocessed block from
// its primary bucket by decrementing r_p and counting itself as a reader of
// the bucket in the same atomic, loads the block and then leaves the reader
// count; it classifies the block's first element to get its destination
// bucket and increments w_dest: if the block at the old w_dest is
// unprocessed it swaps (reads that block, writes its own) and continues with
// the block it read, unless that block already belongs to dest, in which
// case it is left in place; if the old w_dest is empty it writes its block
// there (when the position held a full block at the start, only once no
// worker is reading a block of dest any more: the reader of that position
// may still be loading it) and goes back to the primary bucket.  w, r and
// the reader count live in one 64-bit word so that every update sees a
// consistent state.  A worker stops after a full cycle over the
// buckets finds no unprocessed block.  The partial last block of a segment is
// never written in place: the overflow block stands in for it.
template <int DT, int WPL>
__global__ __launch_bounds__(256) void k_permute(Ctx<DT> c) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    using Word = typename TR::Word;
    using Key = typename TR::Key;
    __shared__ TreeLds<DT> trl;
    const uint32_t lane = threadIdx.x & 63;
    // workers are planned in groups of four, so a workgroup serves one task
    // and shares one copy of its search tree in LDS
    const uint32_t g0 = blockIdx.x * 4;
    const uint32_t gw = g0 + (threadIdx.x >> 6);
    const uint32_t t = upper_find(c.ntasks, g0, [&](uint32_t i) { return (uint64_t)c.tasks[i].worker_begin; });
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t b = c.b, K = st.K, lkt = ilog2(st.kt);
    load_tree<DT>(c, td, st.kt, st.nuniq, trl);
    const Key* gtree = trl.tree;
    const Key* gspl = trl.spl;
    if (gw >= c.total_workers || gw >= td.worker_begin + td.nworkers) return;
    const uint32_t lw = gw - td.worker_begin;
    BucketSlot* sl = c.slots + td.slot_begin;
    const uint32_t* dl = c.delim + td.slot_begin + t;
    Elem* seg = c.data + td.off;
    constexpr uint32_t WPE = sizeof(Elem) / sizeof(Word);
    const uint32_t words = b * WPE;
    const bool partial = (td.m % b) != 0;
    const uint32_t last_blk = st.nblocks - 1;
    Word* ovf = reinterpret_cast<Word*>(ovf_block<DT>(c, td));

    // words of block blk that lie inside the segment (all of them except for
    // a partial last block, which is never unprocessed and so never read)
    auto valid_words = [&](uint32_t blk) -> uint32_t {
        uint64_t rest = td.m - (uint64_t)blk * b;
        return rest >= b ? words : (uint32_t)rest * WPE;
    };
    auto load_block = [&](uint32_t blk, Word (&r)[WPL]) {
        const Word* src = reinterpret_cast<const Word*>(seg + (uint64_t)blk * b);
        const uint32_t vw = valid_words(blk);
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            uint32_t w = lane + 64u * i;
            if (w < vw) r[i] = src[w];
        }
    };
    auto store_block = [&](uint32_t blk, const Word (&r)[WPL]) {
        Word* dst = (partial && blk == last_blk) ? ovf : reinterpret_cast<Word*>(seg + (uint64_t)blk * b);
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            uint32_t w = lane + 64u * i;
            if (w < words) dst[w] = r[i];
        }
    };
    // bucket of the first element of a block held in registers: its words
    // sit in lanes 0..WPE-1 of register 0
    auto first_bucket = [&](const Word (&r)[WPL]) -> uint32_t {
        Elem e;
        Word* ew = reinterpret_cast<Word*>(&e);
#pragma unroll
        for (uint32_t i = 0; i < WPE; ++i) {
            if constexpr (sizeof(Word) == 8) {
                uint32_t lo = read_lane((uint32_t)r[0], i), hi = read_lane((uint32_t)(r[0] >> 32), i);
                ew[i] = ((uint64_t)hi << 32) | lo;
            } else {
                ew[i] = read_lane((uint32_t)r[0], i);
            }
        }
        return classify_key(TR::key(e), gtree, gspl, lkt, st.nuniq, st.eq);
    };

    Word A[WPL], B[WPL];
    uint32_t p = (uint32_t)(((uint64_t)lw * K) / td.nworkers);
    unsigned long long moves = 0, skips = 0;
    const uint32_t limit = c.spin_limit;
    // claim block r_q of bucket q; on success the block is in A and the
    // worker no longer counts as a reader of q
    auto try_claim = [&](uint32_t q, uint32_t& dest) -> bool {
        uint64_t old = 0;
        if (lane == 0) old = atom_add64(&sl[q].wr, WR_CLAIM);
        old = bcast_u64(old);
        const int64_t w0 = wr_w(old), r0 = wr_r(old);
        if (r0 < w0) {
            if (lane == 0) (void)atom_add64(&sl[q].wr, ~0ull);     // readers - 1
            return false;
        }
        load_block((uint32_t)r0, A);
        compiler_fence();
        wait_vmem();          // the block is in registers before the worker stops reading
        compiler_fence();
        if (lane == 0) (void)atom_add64(&sl[q].wr, ~0ull);         // readers - 1
        dest = first_bucket(A);
        return true;
    };
    while (true) {
        // ---- fetch an unprocessed block: scan the buckets from the primary
        // one for a candidate and claim there.  (Claiming again directly
        // where the last claim succeeded saves the scan, but on presorted
        // inputs it piles every worker onto the same few buckets.)
        bool got = false;
        uint32_t destA = 0;
        for (uint32_t scanned = 0, width = 1; !got && scanned < K; width = 64) {
            // look at the primary bucket first, then at 64 buckets at once
            // (each look reads a slot's cache line)
            uint32_t q = p + lane;
            if (q >= K) q -= K;
            bool cand = false;
            if (lane < width && scanned + lane < K) {
                const uint64_t v = atom_load64(&sl[q].wr);
                cand = wr_r(v) >= wr_w(v);
            }
            uint64_t mask = __ballot(cand);
            if (mask == 0) {
                uint32_t adv = (K - scanned) < width ? (K - scanned) : width;
                scanned += adv;
                p += adv;
                if (p >= K) p -= K;
                continue;
            }
            uint32_t first = __ffsll((long long)mask) - 1;
            scanned += first;
            p += first;
            if (p >= K) p -= K;
            got = try_claim(p, destA);
        }
        if (!got) break;
        // ---- place the block, swapping along the way
        while (true) {
            uint64_t old = 0;
            if (lane == 0) old = atom_add64(&sl[destA].wr, WR_WONE);
            old = bcast_u64(old);
            const int64_t x = wr_w(old), r = wr_r(old);
            if (x >= (int64_t)dl[destA + 1] || x < 0) {   // cannot happen for consistent counts
                if (lane == 0) raise_err(c.err, ERR_PERMUTE_RANGE);
                break;
            }
            if (x <= r && partial && (uint32_t)x == last_blk) {   // never unprocessed
                if (lane == 0) raise_err(c.err, ERR_PERMUTE_RANGE);
                break;
            }
            if (x <= r) {
                // unprocessed block at x: read it, then decide
                load_block((uint32_t)x, B);
                wait_vmem();
                uint32_t destB = first_bucket(B);
                if (destB == destA && c.skip_inplace) {
                    ++skips;
                    continue;                       // already in place; w moved past it
                }
                store_block((uint32_t)x, A);
                ++moves;
#pragma unroll
                for (int i = 0; i < WPL; ++i) A[i] = B[i];
                destA = destB;
                continue;
            }
            // empty block at x.  If x was a full block when the permutation
            // started, a reader took it (r passed x before this w did) and
            // may still be loading it: wait until the bucket has no reader.
            // Readers that claim after this point find r < w and read
            // nothing, so the count only falls; blocks that were empty from
            // the start were never read.
            uint32_t spins = 0;
            uint64_t cur = old;
            while ((uint32_t)x < sl[destA].rinit && wr_readers(cur) != 0) {
                if (++spins > limit) {
                    if (lane == 0) raise_err(c.err, ERR_SPIN);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                uint64_t v = 0;
                if (lane == 0) v = atom_load64(&sl[destA].wr);
                cur = bcast_u64(v);
            }
            compiler_fence();
            store_block((uint32_t)x, A);
            ++moves;
            if (partial && (uint32_t)x == last_blk && lane == 0) c.ts[t].ovf_bucket = destA;
            break;
        }
    }
    if (lane == 0) {
        stat_add(c.stats, 0, moves, blockIdx.x);
        stat_add(c.stats, 1, skips, blockIdx.x);
    }
}

// ---------------------------------------------------------------- cleanup
// Section 4.3.  Bucket j owns [B_j, B_{j+1}).  After the permutation its
// full blocks fill [d_j b, w_j b), except that a block written to the
// partial last block went to the overflow block.  Elements still to place:
// the overhang [B_{j+1}, w_j b) (bucket-j data inside the head of bucket
// j+1, and of further buckets when those are smaller than a block), the
// partial buffers of every stripe of the task, and the overflow block if
// bucket j wrote it.  Free positions: the head [B_j, min(d_j b, B_{j+1}))
// and the tail after the full blocks.
//
// The paper's threads clean their buckets one after another.  Here every
// bucket is cleaned at once in two launches: k_overhang copies each
// overhang to a side slot (the side area of the task's first stripe, free
// once classification is over), so that k_cleanup can then fill every
// bucket's free positions with no ordering between buckets.
struct BucketGeom {
    uint64_t B0, B1;    // bucket bounds (segment-relative)
    uint64_t cs, ce;    // start and end of the correct full blocks
    uint64_t ohn;       // overhang elements at [B1, B1 + ohn)
    bool ovf_case;      // this bucket wrote the overflow block
};

template <int DT>
__device__ inline BucketGeom bucket_geom(const Ctx<DT>& c, uint32_t t, const TaskD& td, const TaskS& st,
                                         uint32_t j, bool* bad) {
    const uint32_t b = c.b;
    const uint64_t* bd = c.bounds + td.slot_begin + t;
    const uint32_t* dl = c.delim + td.slot_begin + t;
    BucketGeom g;
    g.B0 = bd[j];
    g.B1 = bd[j + 1];
    g.cs = (uint64_t)dl[j] * b;
    const uint64_t w = (uint64_t)wr_w(c.slots[td.slot_begin + j].wr);
    g.ovf_case = st.ovf_bucket == j;
    // with blocks the bucket holds at least b elements, so cs < B1; without
    // them the block region is empty at cs
    const bool has_blocks = w > dl[j];
    g.ce = !has_blocks ? g.cs : (g.ovf_case ? (uint64_t)(st.nblocks - 1) * b : w * b);
    g.ohn = (has_blocks && !g.ovf_case && g.ce > g.B1) ? g.ce - g.B1 : 0;
    *bad = g.B1 + g.ohn > td.m || g.ohn >= b;      // cannot happen for consistent state
    if (*bad) g.ohn = 0;
    return g;
}

// Overhang to the side slot of the task's first stripe: one wave per
// bucket; grid (bucket groups, tasks from task0).
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_overhang(Ctx<DT> c, uint32_t task0) {
    using Elem = typename Traits<DT>::Elem;
    const uint32_t t = task0 + blockIdx.y;
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t j = blockIdx.x * (NT / 64) + threadIdx.x / 64, lane = threadIdx.x & 63;
    if (j >= st.K) return;
    bool bad;
    const BucketGeom g = bucket_geom<DT>(c, t, td, st, j, &bad);
    if (bad) {
        if (lane == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
        return;
    }
    const Elem* src = c.data + td.off + g.B1;
    Elem* side = c.bufs + c.stripes[td.stripe_begin].buf_off + ((uint64_t)td.kbuf + j) * c.b;
    for (uint32_t i = lane; i < g.ohn; i += 64) side[i] = src[i];
}

// Where source element x of a bucket goes: the head first, then the tail.
struct FreeMap {
    uint64_t B0, tb, nhead;
    __device__ uint64_t operator()(uint64_t x) const { return x < nhead ? B0 + x : tb + (x - nhead); }
};

// Fill the free positions of buckets whose task has many stripes: grid
// (bucket * parts + part, tasks from task0), one workgroup per part; the
// bucket's sources [overhang | buffer of stripe 0 | ... | buffer of stripe
// ns-1 | overflow] are split into `parts` ranges of whole sources.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_cleanup(Ctx<DT> c, uint32_t parts, uint32_t task0) {
    using Elem = typename Traits<DT>::Elem;
    __shared__ uint32_t pre[STRIPES_PER_TASK_MAX + 3];
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint32_t t = task0 + blockIdx.y;
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t j = blockIdx.x / parts, part = blockIdx.x % parts;
    if (j >= st.K) return;
    if (c.fused && c.fused[td.slot_begin + j]) return;     // the fused base case cleans it
    const uint32_t b = c.b;
    bool bad;
    const BucketGeom g = bucket_geom<DT>(c, t, td, st, j, &bad);
    if (bad) {
        if (threadIdx.x == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
        return;
    }
    const uint32_t ns = td.nstripes, nq = ns + 2;
    for (uint32_t q = threadIdx.x; q < nq; q += NT) {
        uint32_t v;
        if (q == 0) v = (uint32_t)g.ohn;
        else if (q <= ns) v = c.counts[td.cnt_begin + (uint64_t)(q - 1) * td.kbuf + j] % b;
        else v = g.ovf_case ? b : 0;
        pre[q] = v;
    }
    __syncthreads();
    const uint32_t nsrc = lds_excl_scan<NT>(pre, nq, sh);
    pre[nq] = nsrc;     // every thread writes the same value
    __syncthreads();
    // free positions: head [B0, he) and tail [tb, B1)
    const uint64_t he = g.cs < g.B1 ? g.cs : g.B1;
    const uint64_t tb0 = g.ce > g.cs ? g.ce : g.cs;
    const uint64_t tb = tb0 < g.B1 ? tb0 : g.B1;
    const uint64_t nhead = he - g.B0, nfree = nhead + (g.B1 - tb);
    if (nfree != nsrc) {
        if (threadIdx.x == 0 && part == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
        return;
    }
    if (threadIdx.x == 0 && part == 0) stat_add(c.stats, 2, nsrc, blockIdx.x + blockIdx.y);
    const FreeMap fm{g.B0, tb, nhead};
    Elem* seg = c.data + td.off;
    const uint32_t q0 = (uint32_t)((uint64_t)nq * part / parts), q1 = (uint32_t)((uint64_t)nq * (part + 1) / parts);
    for (uint32_t q = q0; q < q1; ++q) {
        const uint32_t x0 = pre[q], n = pre[q + 1] - x0;
        if (n == 0) continue;
        const Elem* src = q == 0 ? c.bufs + c.stripes[td.stripe_begin].buf_off + ((uint64_t)td.kbuf + j) * b
                        : q <= ns ? c.bufs + c.stripes[td.stripe_begin + q - 1].buf_off + (uint64_t)j * b
                                  : ovf_block<DT>(c, td);
        for (uint32_t o = threadIdx.x; o < n; o += NT) seg[fm(x0 + o)] = src[o];
    }
}

// Cleanup of bucket j of task t (at most 62 stripes) by one wave: lane q
// holds source q's size and start, and every round places 64 U elements,
// all loads of a round issued before its stores, so a round costs one
// memory latency, not U.  Counts the elements placed in statistics word
// `which`.
template <int DT, int U>
__device__ inline void cleanup_bucket_wave(const Ctx<DT>& c, uint32_t t, const TaskD& td, const TaskS& st,
                                           uint32_t j, int which, uint32_t key) {
    using Elem = typename Traits<DT>::Elem;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t b = c.b;
    bool bad;
    const BucketGeom g = bucket_geom<DT>(c, t, td, st, j, &bad);
    if (bad) {
        if (lane == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
        return;
    }
    const uint32_t ns = td.nstripes, nq = ns + 2;
    uint32_t v = 0;
    uint64_t src_off = 0;                       // element offset in bufs (q <= ns)
    if (lane == 0) {
        v = (uint32_t)g.ohn;
        src_off = c.stripes[td.stripe_begin].buf_off + ((uint64_t)td.kbuf + j) * b;
    } else if (lane <= ns) {
        v = c.counts[td.cnt_begin + (uint64_t)(lane - 1) * td.kbuf + j] % b;
        src_off = c.stripes[td.stripe_begin + lane - 1].buf_off + (uint64_t)j * b;
    } else if (lane == ns + 1) {
        v = g.ovf_case ? b : 0;
    }
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(inc, d, 64);
        if (lane >= (uint32_t)d) inc += u;
    }
    const uint32_t nsrc = read_lane(inc, 63);
    const uint32_t x_lane = inc - v;
    const uint64_t he = g.cs < g.B1 ? g.cs : g.B1;
    const uint64_t tb0 = g.ce > g.cs ? g.ce : g.cs;
    const uint64_t tb = tb0 < g.B1 ? tb0 : g.B1;
    const uint64_t nhead = he - g.B0, nfree = nhead + (g.B1 - tb);
    if (nfree != nsrc) {
        if (lane == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
        return;
    }
    if (lane == 0 && nsrc) stat_add(c.stats, which, nsrc, key);
    const FreeMap fm{g.B0, tb, nhead};
    Elem* seg = c.data + td.off;
    const Elem* ovfp = ovf_block<DT>(c, td);
    for (uint32_t base = 0; base < nsrc; base += 64 * U) {
        uint32_t qs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) qs[u] = 0;
        for (uint32_t q = 1; q < nq; ++q) {
            const uint32_t xq = read_lane(x_lane, q);
#pragma unroll
            for (int u = 0; u < U; ++u) qs[u] = (base + lane + 64u * u >= xq) ? q : qs[u];
        }
        Elem r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = base + lane + 64u * u;
            const uint32_t q = qs[u];
            const uint32_t o = x - (uint32_t)__shfl(x_lane, q, 64);
            const uint64_t so = ((uint64_t)(uint32_t)__shfl((uint32_t)(src_off >> 32), q, 64) << 32) |
                                (uint32_t)__shfl((uint32_t)src_off, q, 64);
            if (x < nsrc) r[u] = q == ns + 1 ? ovfp[o] : c.bufs[so + o];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = base + lane + 64u * u;
            if (x < nsrc) seg[fm(x)] = r[u];
        }
    }
}

// The same for tasks with at most 62 stripes: one wave per bucket, four
// buckets per workgroup; grid (bucket groups, tasks from task0).
template <int DT>
__global__ __launch_bounds__(256) void k_cleanup_narrow(Ctx<DT> c, uint32_t task0) {
    const uint32_t t = task0 + blockIdx.y;
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t j = blockIdx.x * 4 + threadIdx.x / 64;
    if (j >= st.K) return;
    if (c.fused && c.fused[td.slot_begin + j]) return;     // the fused base case cleans it
    cleanup_bucket_wave<DT, 8>(c, t, td, st, j, 2, threadIdx.x / 64 + blockIdx.x + blockIdx.y);
}

// Cleanup of the buckets j0 .. j1 of one task (a base-case bin, Section 4,
// Implementation Details: the base case sorts a bucket right after the
// cleanup has filled it) by a whole workgroup: the placement of k_cleanup.
// With at most 62 stripes in the task every wave cleans buckets of its own
// (cleanup_bucket_wave), else the workgroup takes one bucket after the
// other.  `lds` holds STRIPES_PER_TASK_MAX + 4 + NT/64 + 1 words of scratch.
// The caller synchronizes before it reads the bin back.  Counts the elements
// placed in statistics word 4.
template <int DT, int NT>
__device__ inline void cleanup_bin(const Ctx<DT>& c, const BinSrc& bs, uint32_t* lds) {
    using Elem = typename Traits<DT>::Elem;
    const uint32_t t = bs.task;
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t b = c.b, ns = td.nstripes, nq = ns + 2;
    if (nq <= 64) {
        constexpr int U = sizeof(Elem) >= 64 ? 1 : (int)(64 / sizeof(Elem));
        for (uint32_t j = bs.j0 + threadIdx.x / 64; j <= bs.j1; j += NT / 64)
            cleanup_bucket_wave<DT, U>(c, t, td, st, j, 4, blockIdx.x + j);
        return;
    }
    uint32_t* pre = lds;
    uint32_t* sh = lds + STRIPES_PER_TASK_MAX + 4;
    Elem* seg = c.data + td.off;
    for (uint32_t j = bs.j0; j <= bs.j1; ++j) {
        bool bad;
        const BucketGeom g = bucket_geom<DT>(c, t, td, st, j, &bad);
        if (bad) {
            if (threadIdx.x == 0) raise_err(c.err, ERR_CLEANUP_COUNT);
            continue;
        }
        for (uint32_t q = threadIdx.x; q < nq; q += NT) {
            uint32_t v;
            if (q == 0) v = (uint32_t)g.ohn;
            else if (q <= ns) v = c.counts[td.cnt_begin + (uint64_t)(q - 1) * td.kbuf + j] % b;
            else v = g.ovf_case ? b : 0;
            pre[q] = v;
        }
        __syncthreads();
        const uint32_t nsrc = lds_excl_scan<NT>(pre, nq, sh);
        pre[nq] = nsrc;
        __syncthreads();
        const uint64_t he = g.cs < g.B1 ? g.cs : g.B1;
        const uint64_t tb0 = g.ce > g.cs ? g.ce : g.cs;
        const uint64_t tb = tb0 < g.B1 ? tb0 : g.B1;
        const uint64_t nhead = he - g.B0, nfree = nhead + (g.B1 - tb);
        if (nfree == nsrc) {
            if (threadIdx.x == 0 && nsrc) stat_add(c.stats, 4, nsrc, blockIdx.x + j);
            const FreeMap fm{g.B0, tb, nhead};
            for (uint32_t q = 0; q < nq; ++q) {
                const uint32_t x0 = pre[q], n = pre[q + 1] - x0;
                if (n == 0) continue;
                const Elem* src = q == 0 ? c.bufs + c.stripes[td.stripe_begin].buf_off + ((uint64_t)td.kbuf + j) * b
                                : q <= ns ? c.bufs + c.stripes[td.stripe_begin + q - 1].buf_off + (uint64_t)j * b
                                          : ovf_block<DT>(c, td);
                for (uint32_t o = threadIdx.x; o < n; o += NT) seg[fm(x0 + o)] = src[o];
            }
        } else if (threadIdx.x == 0) {
            raise_err(c.err, ERR_CLEANUP_COUNT);
        }
        __syncthreads();        // pre is rewritten for the next bucket
    }
}

// -------------------------------------------------------------- base case
// Subproblems of at most the base-case capacity are sorted inside one
// workgroup's LDS (u64/f64 sort the keys themselves, f64 through the
// bijective totalOrder image; records sort (key, index) items and then
// gather whole records from a per-workgroup scratch copy of the segment).
template <class Key>
struct KeyIdx {
    Key k;
    uint32_t i;
};

template <int DT>
struct BaseItem {                       // records: key and position
    using Key = typename Traits<DT>::Key;
    using T = KeyIdx<Key>;
    __device__ static bool less(const T& a, const T& b) { return a.k < b.k || (a.k == b.k && a.i < b.i); }
    __device__ static T maxv() { return T{Traits<DT>::max_key(), 0xffffffffu}; }
};
template <>
struct BaseItem<DT_U64> {
    using T = uint64_t;
    __device__ static bool less(T a, T b) { return a < b; }
    __device__ static T maxv() { return ~0ull; }
};
template <>
struct BaseItem<DT_F64> : BaseItem<DT_U64> {};

// One stage of compare-exchanges between x[i] and x[i ^ j] (i < i ^ j),
// ascending where `up(i)`.  For 64-bit integer items one operand of the
// selects passes through an empty asm statement: the selects then no longer
// match the min/max idiom, which the compiler would expand into two 64-bit
// comparisons per exchange; one comparison feeds all four 32-bit selects.
template <class BI, int VT, int J, class Up>
__device__ inline void cx_stage(typename BI::T (&x)[VT], Up up) {
    using T = typename BI::T;
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        const int l = i ^ J;
        if (l > i) {
            const T a = x[i], b = x[l];
            const bool w = up(i) ? BI::less(b, a) : BI::less(a, b);
            T a2 = a;
            if constexpr (std::is_same<T, uint64_t>::value) asm volatile("" : "+v"(a2));
            x[i] = w ? b : a2;
            x[l] = w ? a2 : b;
        }
    }
}

template <class BI, int VT, int K, int J>
__device__ inline void sort_network_stages(typename BI::T (&x)[VT]) {
    if constexpr (K <= VT) {
        if constexpr (J > 0) {
            cx_stage<BI, VT, J>(x, [](int i) { return (i & K) == 0; });
            sort_network_stages<BI, VT, K, J / 2>(x);
        } else {
            sort_network_stages<BI, VT, K * 2, K>(x);
        }
    }
}

// bitonic sort of VT items in registers, ascending
template <class BI, int VT>
__device__ inline void sort_network(typename BI::T (&x)[VT]) {
    sort_network_stages<BI, VT, 2, 1>(x);
}

template <class BI, int VT, int J>
__device__ inline void bitonic_merge_stages(typename BI::T (&x)[VT]) {
    if constexpr (J > 0) {
        cx_stage<BI, VT, J>(x, [](int) { return true; });
        bitonic_merge_stages<BI, VT, J / 2>(x);
    }
}

// sorts a bitonic sequence ascending (log2 VT half-cleaner stages)
template <class BI, int VT>
__device__ inline void bitonic_merge(typename BI::T (&x)[VT]) {
    bitonic_merge_stages<BI, VT, VT / 2>(x);
}

// Leading 64-bit word of a base-case item (the key itself for u64/f64).
__device__ inline uint64_t item_lead(uint64_t k) { return k; }
template <class Key>
__device__ inline uint64_t item_lead(const KeyIdx<Key>& it) { return lead_word(it.k); }

// LDS layout of the base case: the items first (CAP of them for the
// counting sort; CAP + CAP/VT + VT padded slots for the merge sort), then
// either the digit counters (RADIX words holding 2*RADIX = CAP 16-bit
// counters) or the merge-path starts.
template <int DT, int NT, int VT>
struct BaseLds {
    using It = typename BaseItem<DT>::T;
    static constexpr uint32_t CAP = NT * VT;
    static constexpr uint32_t LOG_CAP = CAP >= 16384 ? 14 : CAP >= 8192 ? 13 : CAP >= 4096 ? 12 : CAP >= 2048 ? 11 : 10;
    static constexpr uint32_t RADIX = 1u << (LOG_CAP - 1);
    static constexpr size_t merge_items = CAP + CAP / VT + VT;
    static constexpr size_t counters_at = CAP * sizeof(It);
    static constexpr size_t xchg_at = (merge_items * sizeof(It) + 15) & ~size_t(15);
    static constexpr size_t bytes() {
        const size_t r = counters_at + RADIX * sizeof(uint32_t);
        const size_t m = xchg_at + NT * sizeof(uint32_t);
        return r > m ? r : m;
    }
};

// Counting sort of each listed segment (at most NT*VT elements) inside one
// workgroup's LDS, on the top bits of the leading word: every thread holds
// VT items in registers; the span [lo, hi] of their leading words, less the
// low bits in which all of them agree, is split into 2^(log2 CAP) equal
// digit ranges (16-bit counters, two per LDS word),
// an LDS atomic per item counts its digit (and returns its rank in it), and
// after an exclusive scan each item goes to its digit's group.  Groups hold
// about one item; each item's final place is the group start plus the
// number of group members that precede it (smaller, or equal and placed
// earlier), counted with the items taken in group order.  Where a digit
// covers a single u64/f64 or Pair key value every group is a run of equal
// keys and needs no ranking.  A segment whose keys are all equal is left as it is.
// Segments whose ranking would cost more than WMAX compares per item (keys
// crowded into a few digits), and records with one leading word, are left
// untouched and appended to `fail` for k_basecase (merge sort).
// FUSED: the bins are base-case bins of the level just partitioned; before a
// bin is read the workgroup runs the cleanup of its buckets (bsrc[si]): the
// next bin is cleaned and its keys fetched while this one is written out.
template <int DT, int NT, int VT, bool FUSED = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_basecase_count(Ctx<DT> c, const SegD* segs, uint32_t nseg,
                                                       typename Traits<DT>::Elem* scratch, SegD* fail,
                                                       uint32_t* nfail, const uint32_t* dev_nseg,
                                                       const BinSrc* bsrc) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    using BI = BaseItem<DT>;
    using It = typename BI::T;
    using LB = BaseLds<DT, NT, VT>;
    constexpr bool kPlain = (DT == DT_U64 || DT == DT_F64);
    // 2*RADIX digits with 16-bit counters, two to a word (counts and
    // offsets stay below 2^16)
    // ranking inside the groups costs about the sum of the squared group
    // sizes; beyond WMAX per item the merge sort is cheaper, and beyond
    // SPREAD per item the items are ranked in group order
    constexpr uint32_t RADIX = LB::RADIX, NDIG = 2 * RADIX, WMAX = 16, SPREAD = 4, NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    It* items = reinterpret_cast<It*>(smem_raw);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(smem_raw + LB::counters_at);
    // reduction, scan and maximum scratch: the start of the item array,
    // which is free until the items are scattered into it
    uint32_t* scan_sh = reinterpret_cast<uint32_t*>(smem_raw);
    uint32_t* work_sh = scan_sh + 32;
    uint64_t* red = reinterpret_cast<uint64_t*>(smem_raw + 256);
    auto digit_start = [&](uint32_t d) { return (cnt[d >> 1] >> ((d & 1u) * 16u)) & 0xffffu; };
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    Elem* scr = scratch + (uint64_t)blockIdx.x * (NT * VT);
    // u64/f64: the next bin's keys are loaded before this bin is written
    // out, with loads and stores free of guards (indexes clamped to the
    // bin), so the wait for the loads does not include those stores
    Elem raw[kPlain ? VT : 1];
    SegD sg{};
    auto fetch = [&](uint32_t s2) {
        if constexpr (kPlain) {
            sg = segs[s2];
            const Elem* src = c.data + sg.off;
#pragma unroll
            for (int v = 0; v < VT; ++v) raw[v] = src[min((uint32_t)(v * NT) + tid, sg.len - 1)];
        } else {
            sg = segs[s2];
        }
    };
    if (dev_nseg) nseg = *dev_nseg;             // the count written by an earlier kernel
    // cleanup scratch: u64/f64 clean the next bin while this one's sorted
    // keys sit in the item array, in the counters; records clean a bin at
    // the start of its iteration, in the item array
    constexpr size_t kCleanWords = STRIPES_PER_TASK_MAX + 4 + NT / 64 + 1;
    static_assert(!FUSED || (kPlain ? LB::RADIX >= kCleanWords : LB::counters_at >= 4 * kCleanWords),
                  "cleanup scratch");
    if (blockIdx.x < nseg) {
        if constexpr (FUSED && kPlain) {
            cleanup_bin<DT, NT>(c, bsrc[blockIdx.x], cnt);
            __syncthreads();
        }
        fetch(blockIdx.x);
    }
    for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
        if constexpr (FUSED && !kPlain) {
            cleanup_bin<DT, NT>(c, bsrc[si], reinterpret_cast<uint32_t*>(smem_raw));
            __syncthreads();
        }
        const uint32_t len = sg.len;
        Elem* seg = c.data + sg.off;
        It x[VT];
        uint64_t lo = ~0ull, hi = 0;
#pragma unroll
        for (int v = 0; v < VT; ++v) {
            const uint32_t i = v * NT + tid;
            x[v] = BI::maxv();
            if (i < len) {
                if constexpr (kPlain) {
                    x[v] = TR::key(raw[v]).v;
                } else {
                    const Elem e = seg[i];
                    scr[i] = e;
                    x[v] = It{TR::key(e), i};
                }
                const uint64_t w = item_lead(x[v]);
                lo = w < lo ? w : lo;
                hi = w > hi ? w : hi;
            }
        }
        // span of the leading words over the segment
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const uint64_t l2 = __shfl_xor(lo, d, 64), h2 = __shfl_xor(hi, d, 64);
            lo = l2 < lo ? l2 : lo;
            hi = h2 > hi ? h2 : hi;
        }
        if (lane == 0) { red[2 * wid] = lo; red[2 * wid + 1] = hi; }
        for (uint32_t q = tid; q < RADIX; q += NT) cnt[q] = 0;            // NDIG 16-bit counters
        __syncthreads();
        lo = red[0];
        hi = red[1];
        for (uint32_t w = 1; w < NW; ++w) {
            lo = red[2 * w] < lo ? red[2 * w] : lo;
            hi = red[2 * w + 1] > hi ? red[2 * w + 1] : hi;
        }
        // the low bits in which every leading word agrees with lo
        // (integer-valued f64 keys agree in many): a second reduction, only
        // when the span is wider than the digit count
        uint32_t tz = 0;
        if (lo != hi && 64u - (uint32_t)__clzll(hi - lo) > LB::LOG_CAP) {
            uint64_t orx = 0;
#pragma unroll
            for (int v = 0; v < VT; ++v)
                if (v * NT + tid < len) orx |= item_lead(x[v]) - lo;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) orx |= __shfl_xor(orx, d, 64);
            if (lane == 0) red[4 * NW + wid] = orx;
            __syncthreads();
            orx = 0;
            for (uint32_t w = 0; w < NW; ++w) orx |= red[4 * NW + w];
            tz = (uint32_t)__builtin_ctzll(orx);
        }
        // all keys equal: already sorted; records with one leading word: merge sort
        bool radix = lo != hi;
        bool sorted = false;
        uint32_t dr[VT];                            // digit | arrival << 16, then the final place
        uint32_t sh = 0;
        bool exact = false, spread = true;
        if (radix) {
            // digits: (lead - lo) >> sh, where sh first drops the tz low
            // bits shared by every leading word (lead - lo has them zero)
            const uint64_t span = (hi - lo) >> tz;
            const uint32_t bits = 64u - (uint32_t)__clzll(span);
            const uint32_t over = bits > LB::LOG_CAP ? bits - LB::LOG_CAP : 0u;
            sh = tz + over;
            // one key value per digit: every group is a run of equal keys,
            // already in place once scattered -- for u64/f64 keys, and for
            // Pair records, whose key is the leading word (records with
            // equal keys may come out in any order: the sort is not stable)
            exact = (kPlain || DT == DT_PAIR) && over == 0;
#pragma unroll
            for (int v = 0; v < VT; ++v) {
                if (v * NT + tid < len) {
                    const uint32_t d = (uint32_t)((item_lead(x[v]) - lo) >> sh);
                    const uint32_t hs = (d & 1u) * 16u;
                    const uint32_t old = atomicAdd(&cnt[d >> 1], 1u << hs);
                    dr[v] = d | (((old >> hs) & 0xffffu) << 16);
                }
            }
            __syncthreads();
            // exclusive scan of the counters; ranking work (sum of squared
            // group sizes, each size clamped to 1024, the sum saturating)
            constexpr uint32_t PERC = RADIX / NT, SAT = 1u << 30;
            static_assert(PERC % 4 == 0, "counter words per thread");
            uint32_t cv[PERC], loc = 0, wk = 0;
            uint4* cnt4 = reinterpret_cast<uint4*>(cnt) + tid * (PERC / 4);
#pragma unroll
            for (uint32_t q = 0; q < PERC / 4; ++q) {
                const uint4 w4 = cnt4[q];
                cv[4 * q] = w4.x; cv[4 * q + 1] = w4.y; cv[4 * q + 2] = w4.z; cv[4 * q + 3] = w4.w;
            }
#pragma unroll
            for (uint32_t q = 0; q < PERC; ++q) {
                const uint32_t c0 = cv[q] & 0xffffu, c1 = cv[q] >> 16;
                const uint32_t k0 = min(c0, 1024u), k1 = min(c1, 1024u);
                loc += c0 + c1;
                wk += k0 * k0 + k1 * k1;
            }
            uint32_t total;
            uint32_t pre = block_excl_scan<NT>(loc, scan_sh, &total);
#pragma unroll
            for (uint32_t q = 0; q < PERC; ++q) {
                const uint32_t c0 = cv[q] & 0xffffu, c1 = cv[q] >> 16;
                const uint32_t p0 = pre, p1 = pre + c0;
                cv[q] = p0 | (p1 << 16);
                pre = p1 + c1;
            }
#pragma unroll
            for (uint32_t q = 0; q < PERC / 4; ++q)
                cnt4[q] = make_uint4(cv[4 * q], cv[4 * q + 1], cv[4 * q + 2], cv[4 * q + 3]);
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) wk = min(wk + (uint32_t)__shfl_xor((int)wk, d, 64), SAT);
            if (lane == 0) work_sh[wid] = wk;
            __syncthreads();
            wk = 0;
            for (uint32_t w = 0; w < NW; ++w) wk = min(wk + work_sh[w], SAT);
            radix = exact || wk <= WMAX * len;
            spread = wk <= SPREAD * len;
            __syncthreads();                        // scan_sh and work_sh are read
        }
        if (radix) {
            // each item to its group ...
#pragma unroll
            for (int v = 0; v < VT; ++v)
                if (v * NT + tid < len) items[digit_start(dr[v] & 0xffffu) + (dr[v] >> 16)] = x[v];
            if (!exact && !spread) {
                // ... then to its place inside the group, from the registers
                __syncthreads();
#pragma unroll
                for (int v = 0; v < VT; ++v) {
                    if (v * NT + tid < len) {
                        const uint32_t d = dr[v] & 0xffffu;
                        const uint32_t g0 = digit_start(d), g1 = d + 1 < NDIG ? digit_start(d + 1) : len;
                        const uint32_t pos = g0 + (dr[v] >> 16);
                        uint32_t rank = 0;
                        for (uint32_t j = g0; j < g1; ++j) {
                            const It z = items[j];
                            rank += (BI::less(z, x[v]) || (j < pos && !BI::less(x[v], z))) ? 1u : 0u;
                        }
                        dr[v] = g0 + rank;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < VT; ++v)
                    if (v * NT + tid < len) items[dr[v]] = x[v];
            } else if (!exact) {
                // ... or, where groups are large, with the items walked in
                // group order: the 64 lanes of a wave then rank members of
                // neighbouring groups, so a wave's scan is about as long as
                // the largest of them, not the largest group any of its
                // items fell into
                __syncthreads();
#pragma unroll
                for (int v = 0; v < VT; ++v) {
                    const uint32_t p = v * NT + tid;
                    if (p < len) {
                        const It y = items[p];
                        const uint32_t d = (uint32_t)((item_lead(y) - lo) >> sh);
                        const uint32_t g0 = digit_start(d), g1 = d + 1 < NDIG ? digit_start(d + 1) : len;
                        uint32_t rank = 0;
                        for (uint32_t j = g0; j < g1; ++j) {
                            const It z = items[j];
                            rank += (BI::less(z, y) || (j < p && !BI::less(y, z))) ? 1u : 0u;
                        }
                        x[v] = y;
                        dr[v] = g0 + rank;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < VT; ++v)
                    if (v * NT + tid < len) items[dr[v]] = x[v];
            }
            sorted = true;
        } else if (!(kPlain && lo == hi)) {
            if (tid == 0) fail[atomicAdd(nfail, 1u)] = sg;
        }
        __syncthreads();
        const SegD cur = sg;
        if (si + gridDim.x < nseg) {
            if constexpr (FUSED && kPlain) {
                // the counters are free now; the items hold this bin's output
                cleanup_bin<DT, NT>(c, bsrc[si + gridDim.x], cnt);
                __syncthreads();
            }
            fetch(si + gridDim.x);
        }
        if (sorted) {
            Elem* out = c.data + cur.off;
            if constexpr (kPlain) {
                // four at a time: the next bin's keys already occupy registers
#pragma unroll
                for (int v0 = 0; v0 < VT; v0 += 4) {
#pragma unroll
                    for (int v = v0; v < v0 + 4; ++v) {
                        const uint32_t i = min((uint32_t)(v * NT) + tid, cur.len - 1);
                        if constexpr (DT == DT_F64) out[i] = Traits<DT_F64>::unkey(items[i]);
                        else out[i] = items[i];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                for (uint32_t i = tid; i < cur.len; i += NT) out[i] = scr[items[i].i];
            }
        }
        __syncthreads();
    }
}

// Sort of each listed segment of at most 64 R u64/f64 keys by one wave:
// the keys in registers (element e = 64 r + lane, padded with the maximal
// key to 64 R), a bitonic sorting network whose exchanges at a distance of
// 64 or more pair two registers of one lane and whose shorter ones pair two
// lanes through shuffles (each lane keeps the minimum or the maximum), then
// written back.  No LDS and no barrier, so many bins run per CU at once.
template <int DT, int R>
__global__ __launch_bounds__(256) void k_basecase_tiny(Ctx<DT> c, const SegD* segs, uint32_t nseg,
                                                       const uint32_t* dev_nseg) {
    static_assert(DT == DT_U64 || DT == DT_F64, "plain keys only");
    if (dev_nseg) nseg = *dev_nseg;
    using TR = Traits<DT>;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
    for (uint32_t si = wave; si < nseg; si += nwaves) {
        const SegD sg = segs[si];
        uint64_t* seg = c.data + sg.off;
        uint64_t x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = (uint32_t)r * 64u + lane;
            x[r] = e < sg.len ? TR::key(seg[e]).v : ~0ull;
        }
#pragma unroll
        for (uint32_t k = 2; k <= 64u * R; k <<= 1) {
#pragma unroll
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                if (j >= 64) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int l = r ^ (int)(j >> 6);
                        if (l > r) {
                            const bool up = (((uint32_t)r * 64u + lane) & k) == 0;
                            const uint64_t a = x[r], b = x[l];
                            const bool w = up ? b < a : a < b;
                            x[r] = w ? b : a;
                            x[l] = w ? a : b;
                        }
                    }
                } else {
                    const bool lower = (lane & j) == 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x[r], (int)j, 64);
                        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x[r] >> 32), (int)j, 64);
                        const uint64_t y = ((uint64_t)hi << 32) | lo;
                        const bool up = (((uint32_t)r * 64u + lane) & k) == 0;
                        const bool take = lower == up ? y < x[r] : x[r] < y;
                        x[r] = take ? y : x[r];
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = (uint32_t)r * 64u + lane;
            if (e < sg.len) {
                if constexpr (DT == DT_F64) seg[e] = Traits<DT_F64>::unkey(x[r]);
                else seg[e] = x[r];
            }
        }
    }
}

// Merge sort of each listed segment (at most NT*VT elements; the count is
// read from `dev_nseg` when given) inside one workgroup's LDS.  The segment
// is padded to lenP (a multiple of VT) with maximal sentinels, so every
// thread owns exactly VT items and no access needs a bounds check.  Every
// thread sorts its VT items in registers with a bitonic network; then
// log2(len / VT) merge passes double the sorted runs.  In a pass each thread
// finds where its VT outputs start in the merge of its two runs by a binary
// search along its cross diagonal (merge path); the next thread's start,
// exchanged through LDS, says how many of the VT outputs come from each run,
// na from the first and VT - na from the second.  The thread loads those na
// items ascending followed by the VT - na items descending (a bitonic
// sequence holding exactly its outputs) and sorts them with a bitonic merge.
// Records break ties by index, so the sentinels (index 2^32 - 1) stay last.
template <int DT, int NT, int VT>
__global__ __launch_bounds__(NT) void k_basecase(Ctx<DT> c, const SegD* segs, uint32_t nseg,
                                                 typename Traits<DT>::Elem* scratch, const uint32_t* dev_nseg) {
    using TR = Traits<DT>;
    using Elem = typename TR::Elem;
    using BI = BaseItem<DT>;
    using It = typename BI::T;
    using LB = BaseLds<DT, NT, VT>;
    constexpr bool kPlain = (DT == DT_U64 || DT == DT_F64);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    It* items = reinterpret_cast<It*>(smem_raw);
    uint32_t* xchg = reinterpret_cast<uint32_t*>(smem_raw + LB::xchg_at);
    auto pidx = [](uint32_t i) { return i + i / VT; };   // one pad item per VT: fewer bank conflicts
    const uint32_t tid = threadIdx.x;
    const uint32_t base = tid * VT;
    It* const mine = items + pidx(base);
    if (dev_nseg) nseg = *dev_nseg;
    for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
        const SegD sg = segs[si];
        const uint32_t len = sg.len;
        const uint32_t lenP = (len + VT - 1) / VT * VT;
        Elem* seg = c.data + sg.off;
        Elem* scr = scratch + (uint64_t)blockIdx.x * (NT * VT);
        for (uint32_t i = tid; i < lenP; i += NT) {
            It v = BI::maxv();
            if (i < len) {
                const Elem e = seg[i];
                if constexpr (kPlain) {
                    v = TR::key(e).v;
                } else {
                    scr[i] = e;
                    v = It{TR::key(e), i};
                }
            }
            items[pidx(i)] = v;
        }
        __syncthreads();
        const uint32_t nthr = lenP / VT;
        It x[VT];
        if (tid < nthr) {
#pragma unroll
            for (int v = 0; v < VT; ++v) x[v] = mine[v];
            sort_network<BI, VT>(x);
        }
        for (uint32_t L = VT; L < lenP; L *= 2) {
            __syncthreads();
            if (tid < nthr) {
#pragma unroll
                for (int v = 0; v < VT; ++v) mine[v] = x[v];
            }
            __syncthreads();
            uint32_t lo2 = 0, a0 = 0, aCount = 0, b0 = 0, diag = 0;
            if (tid < nthr) {
                a0 = base & ~(2 * L - 1);
                aCount = min(L, lenP - a0);
                b0 = a0 + L;
                const uint32_t bCount = b0 >= lenP ? 0u : min(L, lenP - b0);
                diag = base - a0;
                lo2 = diag > bCount ? diag - bCount : 0u;
                uint32_t hi2 = diag < aCount ? diag : aCount;
                while (lo2 < hi2) {
                    const uint32_t mid = (lo2 + hi2) >> 1;
                    const It av = items[pidx(a0 + mid)];
                    const It bv = items[pidx(b0 + diag - 1 - mid)];
                    if (!BI::less(bv, av)) lo2 = mid + 1; else hi2 = mid;
                }
                xchg[tid] = lo2;
            }
            lds_barrier();
            if (tid < nthr) {
                // the next thread continues this merge unless this thread
                // ends it (end of both runs or of the padded segment)
                const uint32_t end = min(a0 + 2 * L, lenP);
                const uint32_t lo_next = base + VT < end ? xchg[tid + 1] : aCount;
                const uint32_t na = lo_next - lo2;
                const uint32_t ai = a0 + lo2, bi_last = b0 + (diag - lo2) + VT - 1;
#pragma unroll
                for (int v = 0; v < VT; ++v)
                    x[v] = items[pidx((uint32_t)v < na ? ai + v : bi_last - v)];
                bitonic_merge<BI, VT>(x);
            }
        }
        __syncthreads();
        if (tid < nthr) {
#pragma unroll
            for (int v = 0; v < VT; ++v) mine[v] = x[v];
        }
        __syncthreads();
        for (uint32_t i = tid; i < len; i += NT) {
            if constexpr (DT == DT_F64) seg[i] = Traits<DT_F64>::unkey(items[pidx(i)]);
            else if constexpr (DT == DT_U64) seg[i] = items[pidx(i)];
            else seg[i] = scr[items[pidx(i)].i];
        }
        __syncthreads();
    }
}

// ------------------------------------------ segmented sort of small segments
// Bins straight from a device offset table (segment i = [offs[i], offs[i+1]),
// each within the base-case capacity): every segment of 2 or more elements
// goes to the list of its size class (0: at most `half`, the small counting
// sort; 1: larger, the large one; 2: at most `tiny`, one wave), in any order;
// cnt[0..3) receive the list lengths (cleared beforehand by
// k_small_segments_setup).  A decreasing pair of offsets or a segment above
// `cap` raises ERR_SEGMENT and that segment is left as it is.
template <int DT>
__global__ __launch_bounds__(256) void k_small_segments_setup(uint32_t* cnt, uint32_t* err) {
    if (threadIdx.x < 8) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) err[0] = 0;
}

template <int DT>
__global__ __launch_bounds__(256) void k_small_segments_bins(const uint64_t* offs, uint32_t nseg, uint32_t half,
                                                             uint32_t cap, uint32_t tiny, SegD* lists, uint32_t* cnt,
                                                             uint32_t* err) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nseg; i += gridDim.x * 256) {
        const uint64_t a = offs[i], e = offs[i + 1];
        if (e < a || e - a > cap) {
            raise_err_at(err, ERR_SEGMENT, i, (uint32_t)(e - a), cap);
            continue;
        }
        const uint32_t len = (uint32_t)(e - a);
        if (len <= 1) continue;
        const uint32_t cls = len <= tiny ? 2u : (len <= half ? 0u : 1u);
        const uint32_t at = atomicAdd(&cnt[cls], 1u);
        SegD sd;
        sd.off = a;
        sd.len = len;
        sd.pad = 0;
        lists[(uint64_t)cls * nseg + at] = sd;
    }
}

// ------------------------------------------------ phase invariant checks
// Debug only.  After local classification (Section 4.1): every stripe is
// [full blocks | empty blocks], each full block holds one bucket, and the
// full blocks plus the partial buffers reproduce the stored counts.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_check_classify(Ctx<DT> c) {
    using TR = Traits<DT>;
    __shared__ TreeLds<DT> tr;
    __shared__ uint32_t hist[KMAX];
    const StripeD sd = c.stripes[blockIdx.x];
    const TaskD td = c.tasks[sd.task];
    const TaskS st = c.ts[sd.task];
    const uint32_t b = c.b, K = st.K, lkt = ilog2(st.kt);
    load_tree<DT>(c, td, st.kt, st.nuniq, tr);
    for (uint32_t j = threadIdx.x; j < K; j += NT) hist[j] = 0;
    __syncthreads();
    const uint32_t F = c.stripe_full[blockIdx.x];
    const typename TR::Elem* sp = c.data + td.off + (uint64_t)sd.blk_begin * b;
    if ((uint64_t)(sd.blk_begin + F) * b > td.m || sd.blk_begin + F > sd.blk_end) {
        if (threadIdx.x == 0) raise_err(c.err, ERR_CHECK_BLOCK);
        return;
    }
    for (uint64_t i = threadIdx.x; i < (uint64_t)F * b; i += NT) {
        const uint32_t bj = classify_key(TR::key(sp[i]), tr.tree, tr.spl, lkt, st.nuniq, st.eq);
        const uint32_t b0 = classify_key(TR::key(sp[(i / b) * b]), tr.tree, tr.spl, lkt, st.nuniq, st.eq);
        if (bj != b0) raise_err_at(c.err, ERR_CHECK_BLOCK, (uint32_t)i, bj, b0);
        atomicAdd(&hist[bj], 1u);
    }
    const uint32_t* cnt = c.counts + td.cnt_begin + (uint64_t)(blockIdx.x - td.stripe_begin) * td.kbuf;
    for (uint32_t j = 0; j < K; ++j) {
        const uint32_t f = cnt[j] % b;
        for (uint32_t r = threadIdx.x; r < f; r += NT) {
            const uint32_t bj = classify_key(TR::key(c.bufs[sd.buf_off + (uint64_t)j * b + r]), tr.tree, tr.spl,
                                             lkt, st.nuniq, st.eq);
            if (bj != j) raise_err_at(c.err, ERR_CHECK_COUNT, r, bj, j);
            atomicAdd(&hist[bj], 1u);
        }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < K; j += NT)
        if (hist[j] != cnt[j]) raise_err_at(c.err, ERR_CHECK_COUNT, j, hist[j], cnt[j]);
}

// After the block permutation (Section 4.2 invariant at the end): every
// block in [d_i, w_i) holds only elements of bucket i.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_check_permute(Ctx<DT> c, uint32_t task0) {
    using TR = Traits<DT>;
    __shared__ TreeLds<DT> tr;
    const uint32_t t = task0 + blockIdx.y;
    const TaskD td = c.tasks[t];
    const TaskS st = c.ts[t];
    const uint32_t j = blockIdx.x;
    if (j >= st.K) return;
    const uint32_t b = c.b, lkt = ilog2(st.kt);
    load_tree<DT>(c, td, st.kt, st.nuniq, tr);
    const uint32_t d0 = c.delim[td.slot_begin + t + j];
    const uint32_t w = (uint32_t)wr_w(c.slots[td.slot_begin + j].wr);
    const bool partial = (td.m % b) != 0;
    const typename TR::Elem* seg = c.data + td.off;
    for (uint32_t q = d0; q < w; ++q) {
        const typename TR::Elem* blk = (partial && q == st.nblocks - 1) ? ovf_block<DT>(c, td) : seg + (uint64_t)q * b;
        for (uint32_t r = threadIdx.x; r < b; r += NT) {
            const uint32_t bj = classify_key(TR::key(blk[r]), tr.tree, tr.spl, lkt, st.nuniq, st.eq);
            if (bj != j) raise_err_at(c.err, ERR_CHECK_PLACED, q, bj, j);
        }
    }
}

// --------------------------------------------------- bucket ids (classify)
// The bucket of every element by the classification k_classify performs:
// the lookup table over the splitters' leading words, then the binary search
// and the equality rule (classify_lut_batch), one element per lane.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_bucket_ids(Ctx<DT> c, uint64_t n, uint32_t* out) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    __shared__ Key spl[KT_MAX];
    __shared__ uint32_t lut[LUT_N];
    __shared__ uint32_t red[NT / 64 + 1];
    const TaskS st = c.ts[0];
    const TaskD td = c.tasks[0];
    for (uint32_t i = threadIdx.x; i < st.nuniq; i += NT) spl[i] = c.spl[td.tree_begin + i];
    __syncthreads();
    const LutParams P = build_lut<Key, NT>(spl, st.nuniq, lut, red);
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * NT) {
        const Key k[1] = {TR::key(c.data[i])};
        uint32_t bk[1];
        classify_lut_batch<Key, 1>(k, bk, spl, lut, P, st.nuniq, st.eq);
        out[i] = bk[0];
    }
}

// ------------------------------ strictly in-place recursion (Section 4.6)
// The partition leaves the largest element of every bucket in the bucket's
// first entry.  The end of a bucket is then the first later position that
// holds a larger key: every later bucket of the partition, and every bucket
// of an earlier level after it, holds only larger keys, so the positions
// holding larger keys form a suffix and can be searched for.  The
// recursion then needs no bucket boundaries beyond the partition that made
// them.

// Wavefront read of a key (every word of it) from lane `src`.
__device__ inline Key1 shfl_key(const Key1& k, int src) { return Key1{(uint64_t)__shfl(k.v, src, 64)}; }
__device__ inline Key3 shfl_key(const Key3& k, int src) {
    return Key3{(uint64_t)__shfl(k.a, src, 64), (uint64_t)__shfl(k.b, src, 64), (uint64_t)__shfl(k.c, src, 64)};
}
__device__ inline Key10 shfl_key(const Key10& k, int src) {
    return Key10{(uint64_t)__shfl(k.hi, src, 64), (uint32_t)__shfl((int)k.lo, src, 64), 0u};
}

// The first position in [lo, hi) holding a key larger than piv, or hi
// (searchNextLargest).  One wavefront.  The first round is the exponential
// search's probes lo + 2^l - 1, all at once, one per lane; given a guess g
// of the answer's distance from lo (the previous bucket's length, in a walk
// over buckets of similar size), half of the lanes probe the exponential
// positions and the other half a window of 32 evenly spaced positions
// around lo + g, and the answer lies in both brackets.  The bracket is then
// narrowed by 64-way search, each round probing 64 evenly spaced positions:
// about log_64 of the bucket size dependent loads instead of 2 log_2, one
// round fewer when the guess is close.  The result is the first larger key
// whenever the larger keys form a suffix of [lo, hi); otherwise some
// position in [lo, hi] whose key is larger (or hi).  Only positions in
// [lo, hi) are read.  Every lane returns the same value, and *found receives
// the key at the returned position when it is below hi (the probe that
// found it loaded it).
template <int DT>
__device__ inline uint64_t wave_next_larger(const typename Traits<DT>::Elem* data,
                                            const typename Traits<DT>::Key& piv, uint64_t lo, uint64_t hi,
                                            typename Traits<DT>::Key* found = nullptr, uint64_t guess = 0) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    if (lo >= hi) return hi;
    const uint32_t lane = lane_id();
    const uint64_t len = hi - lo;
    // lanes [0, ne) probe lo + 2^lane - 1; with a guess, lanes 32.. probe
    // lo + w0 + (lane - 32) * ws
    const uint32_t ne = guess ? 32u : 63u;
    const uint64_t ws = guess / 16 ? guess / 16 : 1;
    const uint64_t w0 = guess > 16 * ws ? guess - 16 * ws : 0;
    bool in;
    uint64_t pos;
    if (lane < ne) {
        in = (1ull << lane) <= len;
        pos = lo + (1ull << lane) - 1;
    } else {
        const uint64_t o = w0 + (uint64_t)(lane - 32) * ws;
        in = guess != 0 && o < len;
        pos = lo + o;
    }
    Key k{};
    bool big = false;
    if (in) {
        k = TR::key(data[pos]);
        big = piv < k;
    }
    const uint64_t mb = __ballot(big), mi = __ballot(in);
    const uint64_t lowm = ne == 63u ? ~0ull : 0xffffffffull;
    uint64_t below, above;
    int src = -1;
    {
        const uint64_t b = mb & lowm, i = mi & lowm;
        if (b) {
            const uint32_t f = (uint32_t)__builtin_ctzll(b);
            above = lo + (1ull << f) - 1;
            below = f ? lo + (1ull << (f - 1)) : lo;      // probe f-1 held no larger key
            src = (int)f;
        } else {
            const uint32_t l = 63u - (uint32_t)__builtin_clzll(i);   // lane 0 is always in range
            below = lo + (1ull << l);
            above = hi;
        }
    }
    if (ne == 32u) {
        const uint64_t b = mb >> 32, i = mi >> 32;
        if (b) {
            const uint32_t f = (uint32_t)__builtin_ctzll(b);
            const uint64_t a2 = lo + w0 + (uint64_t)f * ws;
            const uint64_t b2 = f ? lo + w0 + (uint64_t)(f - 1) * ws + 1 : lo;
            if (a2 < above) {
                above = a2;
                src = (int)(32 + f);
            }
            below = below > b2 ? below : b2;
        } else if (i) {
            const uint32_t l = 63u - (uint32_t)__builtin_clzll(i);
            const uint64_t b2 = lo + w0 + (uint64_t)l * ws + 1;
            below = below > b2 ? below : b2;
        }
    }
    Key ak{};
    if (src >= 0) ak = shfl_key(k, src);
    // invariant: no larger key in [lo, below) at a probed position, and
    // `above` is hi or holds a larger key (ak); [below, above) shrinks
    // each round
    while (below < above) {
        const uint64_t step = ((above - below) + 63) >> 6;
        const uint64_t q = below + (uint64_t)lane * step;
        const bool qin = q < above;
        bool qb = false;
        Key kq{};
        if (qin) {
            kq = TR::key(data[q]);
            qb = piv < kq;
        }
        const uint64_t m2 = __ballot(qb);
        if (m2) {
            const uint32_t f = (uint32_t)__builtin_ctzll(m2);
            const uint64_t nb = f ? below + (uint64_t)(f - 1) * step + 1 : below;
            above = below + (uint64_t)f * step;
            below = nb;
            ak = shfl_key(kq, (int)f);
        } else {
            const uint32_t last = (uint32_t)__builtin_popcountll(__ballot(qin)) - 1;
            below = below + (uint64_t)last * step + 1;
        }
    }
    if (found) *found = ak;
    return above;
}

// Wavefront exchange of a key (every word of it) with lane ^ d.
__device__ inline Key1 shfl_xor_key(const Key1& k, int d) { return Key1{(uint64_t)__shfl_xor(k.v, d, 64)}; }
__device__ inline Key3 shfl_xor_key(const Key3& k, int d) {
    return Key3{(uint64_t)__shfl_xor(k.a, d, 64), (uint64_t)__shfl_xor(k.b, d, 64), (uint64_t)__shfl_xor(k.c, d, 64)};
}
__device__ inline Key10 shfl_xor_key(const Key10& k, int d) {
    return Key10{(uint64_t)__shfl_xor(k.hi, d, 64), (uint32_t)__shfl_xor((int)k.lo, d, 64), 0u};
}

// (key, position) of the largest key, the smaller position among equal keys
template <typename Key>
__device__ inline void keep_max(Key& bk, uint64_t& bp, const Key& k, uint64_t p) {
    if (bk < k || (k == bk && p < bp)) {
        bk = k;
        bp = p;
    }
}

// (key, position) of the smallest key, the smaller position among equal keys
template <typename Key>
__device__ inline void keep_min(Key& bk, uint64_t& bp, const Key& k, uint64_t p) {
    if (k < bk || (k == bk && p < bp)) {
        bk = k;
        bp = p;
    }
}

// Bucket [lo, hi) of at least two elements: the element at pmax (holding
// its largest key) trades places with the first; with MIN, then the
// element holding its smallest key (pmin before the first exchange) with
// the last, so that a bucket of one key value shows it at its two ends.
// The first element keeps the largest key either way.
template <int DT, bool MIN>
__device__ inline void mark_ends(typename Traits<DT>::Elem* data, uint64_t lo, uint64_t hi, uint64_t pmax,
                                 uint64_t pmin) {
    using Elem = typename Traits<DT>::Elem;
    if (pmax != lo) {
        const Elem a = data[lo];
        data[lo] = data[pmax];
        data[pmax] = a;
    }
    if constexpr (MIN) {
        if (pmin == lo) pmin = pmax;            // the first element went to pmax
        if (pmin != lo && pmin != hi - 1) {
            const Elem a = data[hi - 1];
            data[hi - 1] = data[pmin];
            data[pmin] = a;
        }
    }
}

// The marking the partition owes (Section 4.6): in bucket j the first
// element with the largest key trades places with the bucket's first
// element (with MIN, then the first with the smallest key with the last:
// mark_ends).  One workgroup per bucket (grid x, strided over the buckets);
// grid y: the tasks of a level from t0, bounds relative to the task's
// offset (equality buckets, which hold one key, are left alone); with
// tasks == nullptr one list of nb buckets whose bounds[0..nb] are
// positions in [0, n).  Each lane keeps eight loads in flight; the lanes'
// extremes meet by wavefront exchanges, then across the waves in LDS.
template <int DT, int NT, bool MIN = false>
__global__ __launch_bounds__(NT) void k_mark_max(typename Traits<DT>::Elem* data, uint64_t n,
                                                 const uint64_t* bounds, const TaskD* tasks, const TaskS* ts,
                                                 uint32_t t0, uint32_t nb, uint32_t* err) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    constexpr int W = NT / 64;
    constexpr int U = 8;
    __shared__ Key sk[W], sk2[W];
    __shared__ uint64_t sp[W], sp2[W];
    const uint32_t t = t0 + blockIdx.y;
    uint64_t off = 0, end = n;
    const uint64_t* bd = bounds;
    uint32_t K = nb;
    bool eq = false;
    if (tasks) {
        const TaskD td = tasks[t];
        off = td.off;
        end = td.off + td.m;
        bd = bounds + td.slot_begin + t;
        K = ts[t].K;
        eq = ts[t].eq != 0;
    }
    const uint32_t tid = threadIdx.x, wave = tid / 64;
    for (uint32_t j = blockIdx.x; j < K; j += gridDim.x) {
        if (eq && (j & 1)) continue;
        const uint64_t lo = off + bd[j], hi = off + bd[j + 1];
        if (hi < lo || hi > end) {
            if (tid == 0) raise_err(err, ERR_MARKS);
            continue;
        }
        if (hi - lo < 2) continue;
        Key bk = TR::key(data[lo]), mk = bk;
        uint64_t bp = lo, mp = lo;
        uint64_t p = lo + tid;
        for (; p + (U - 1) * NT < hi; p += U * NT) {
            Key kq[U];
#pragma unroll
            for (int u = 0; u < U; ++u) kq[u] = TR::key(data[p + (uint64_t)u * NT]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                keep_max(bk, bp, kq[u], p + (uint64_t)u * NT);
                if constexpr (MIN) keep_min(mk, mp, kq[u], p + (uint64_t)u * NT);
            }
        }
        for (; p < hi; p += NT) {
            const Key kk = TR::key(data[p]);
            keep_max(bk, bp, kk, p);
            if constexpr (MIN) keep_min(mk, mp, kk, p);
        }
        for (int d = 32; d >= 1; d >>= 1) {
            const Key ko = shfl_xor_key(bk, d);
            const uint64_t po = (uint64_t)__shfl_xor(bp, d, 64);
            keep_max(bk, bp, ko, po);
            if constexpr (MIN) {
                const Key k2 = shfl_xor_key(mk, d);
                const uint64_t p2 = (uint64_t)__shfl_xor(mp, d, 64);
                keep_min(mk, mp, k2, p2);
            }
        }
        if (lane_id() == 0) {
            sk[wave] = bk;
            sp[wave] = bp;
            sk2[wave] = mk;
            sp2[wave] = mp;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < W; ++w) {
                keep_max(bk, bp, sk[w], sp[w]);
                if constexpr (MIN) keep_min(mk, mp, sk2[w], sp2[w]);
            }
            mark_ends<DT, MIN>(data, lo, hi, bp, mp);
        }
        __syncthreads();
    }
}

// The same marking for buckets of millions of elements, in two steps: each
// bucket is cut into P equal parts, one workgroup per part writes the part's
// first largest key and its position to pk/pp[(slot_begin + j) * P + q]
// (with MIN its first smallest to qk/qp at the same index; position ~0: an
// empty part, or a bucket left alone), then k_mark_pick marks the bucket's
// ends from the parts' extremes.  One workgroup per bucket is bound by what
// one CU keeps in flight, and the largest bucket sets the time; parts
// spread every bucket over the device.
template <int DT, int NT, bool MIN = false>
__global__ __launch_bounds__(NT) void k_mark_part(const typename Traits<DT>::Elem* data, const uint64_t* bounds,
                                                  const TaskD* tasks, const TaskS* ts, uint32_t t0, uint32_t P,
                                                  typename Traits<DT>::Key* pk, uint64_t* pp,
                                                  typename Traits<DT>::Key* qk, uint64_t* qp, uint32_t* err) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    constexpr int W = NT / 64;
    constexpr int U = 8;
    __shared__ Key sk[W], sk2[W];
    __shared__ uint64_t sp[W], sp2[W];
    const uint32_t t = t0 + blockIdx.y;
    const uint32_t j = blockIdx.x / P, q = blockIdx.x % P;
    const TaskD td = tasks[t];
    const TaskS st = ts[t];
    if (j >= st.K) return;
    const uint32_t tid = threadIdx.x;
    const uint64_t at = ((uint64_t)td.slot_begin + j) * P + q;
    const uint64_t* bd = bounds + td.slot_begin + t;
    const uint64_t lo = td.off + bd[j], hi = td.off + bd[j + 1];
    if (hi < lo || hi > td.off + td.m) {
        if (tid == 0) {
            pp[at] = ~0ull;
            if (q == 0) raise_err(err, ERR_MARKS);
        }
        return;
    }
    const uint64_t len = hi - lo, a = lo + len * q / P, b = lo + len * (q + 1) / P;
    if ((st.eq && (j & 1)) || len < 2 || a == b) {
        if (tid == 0) pp[at] = ~0ull;
        return;
    }
    Key bk = TR::key(data[a]), mk = bk;
    uint64_t bp = a, mp = a;
    uint64_t p = a + tid;
    for (; p + (U - 1) * NT < b; p += U * NT) {
        Key kq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) kq[u] = TR::key(data[p + (uint64_t)u * NT]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            keep_max(bk, bp, kq[u], p + (uint64_t)u * NT);
            if constexpr (MIN) keep_min(mk, mp, kq[u], p + (uint64_t)u * NT);
        }
    }
    for (; p < b; p += NT) {
        const Key kk = TR::key(data[p]);
        keep_max(bk, bp, kk, p);
        if constexpr (MIN) keep_min(mk, mp, kk, p);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const Key ko = shfl_xor_key(bk, d);
        const uint64_t po = (uint64_t)__shfl_xor(bp, d, 64);
        keep_max(bk, bp, ko, po);
        if constexpr (MIN) {
            const Key k2 = shfl_xor_key(mk, d);
            const uint64_t p2 = (uint64_t)__shfl_xor(mp, d, 64);
            keep_min(mk, mp, k2, p2);
        }
    }
    if (lane_id() == 0) {
        sk[tid / 64] = bk;
        sp[tid / 64] = bp;
        sk2[tid / 64] = mk;
        sp2[tid / 64] = mp;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < W; ++w) {
            keep_max(bk, bp, sk[w], sp[w]);
            if constexpr (MIN) keep_min(mk, mp, sk2[w], sp2[w]);
        }
        pk[at] = bk;
        pp[at] = bp;
        if constexpr (MIN) {
            qk[at] = mk;
            qp[at] = mp;
        }
    }
}

// One lane per bucket: the largest of the parts' maxima (the first position
// among equal keys; parts lie in position order) goes to the bucket's first
// entry, and with MIN the smallest of their minima to its last (mark_ends).
template <int DT, bool MIN = false>
__global__ __launch_bounds__(256) void k_mark_pick(typename Traits<DT>::Elem* data, const uint64_t* bounds,
                                                   const TaskD* tasks, const TaskS* ts, uint32_t t0, uint32_t P,
                                                   const typename Traits<DT>::Key* pk, const uint64_t* pp,
                                                   const typename Traits<DT>::Key* qk, const uint64_t* qp) {
    using TR = Traits<DT>;
    using Key = typename TR::Key;
    const uint32_t t = t0 + blockIdx.y;
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    const TaskD td = tasks[t];
    if (j >= ts[t].K) return;
    const uint64_t base = ((uint64_t)td.slot_begin + j) * P;
    bool have = false;
    Key bk{}, mk{};
    uint64_t bp = 0, mp = 0;
    for (uint32_t q = 0; q < P; ++q) {
        const uint64_t p = pp[base + q];
        if (p == ~0ull) continue;
        const Key k = pk[base + q];
        if (!have) {
            bk = k;
            bp = p;
            if constexpr (MIN) {
                mk = qk[base + q];
                mp = qp[base + q];
            }
            have = true;
        } else {
            keep_max(bk, bp, k, p);
            if constexpr (MIN) keep_min(mk, mp, qk[base + q], qp[base + q]);
        }
    }
    if (!have) return;
    const uint64_t* bd = bounds + td.slot_begin + t;
    mark_ends<DT, MIN>(data, td.off + bd[j], td.off + bd[j + 1], bp, mp);
}

// searchNextLargest for caller-given positions: out[q] = the first position
// after pos[q] in [0, n) holding a larger key than data[pos[q]], or n (also
// for pos[q] >= n).  One wavefront per query.
template <int DT>
__global__ __launch_bounds__(256) void k_search_next(const typename Traits<DT>::Elem* data, uint64_t n,
                                                     const uint64_t* pos, uint64_t count, uint64_t* out) {
    using TR = Traits<DT>;
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    for (uint64_t q = (uint64_t)blockIdx.x * 4 + threadIdx.x / 64; q < count; q += waves) {
        const uint64_t i = pos[q];
        uint64_t j = n;
        if (i < n) j = wave_next_larger<DT>(data, TR::key(data[i]), i + 1, n);
        if (lane_id() == 0) out[q] = j;
    }
}

// The buckets of each task of a level found again from the data alone, after
// k_mark_max: from the task's first element on, each bucket ends where the
// next larger key begins (the recursion of Section 4.6, without its
// sequential order: one wavefront per task).  The bucket boundaries
// overwrite the task's bounds[0..K] (relative to its offset): the c
// non-empty buckets found, then the task's end repeated (empty buckets).
// More buckets than the partition made means the marks are missing.  With
// MIN (the marking also put each bucket's smallest key last) a bucket above
// `cap` elements whose two ends hold equal keys is one key value, and its
// start carries kOneKeyBit.
constexpr uint64_t kOneKeyBit = 1ull << 63;
template <int DT, bool MIN = false>
__global__ __launch_bounds__(256) void k_walk(const typename Traits<DT>::Elem* data, uint64_t* bounds,
                                              const TaskD* tasks, const TaskS* ts, uint32_t ntasks,
                                              uint64_t cap, uint32_t* err) {
    using TR = Traits<DT>;
    const uint32_t t = blockIdx.x * 4 + threadIdx.x / 64;
    if (t >= ntasks) return;
    const uint32_t lane = lane_id();
    const TaskD td = tasks[t];
    const uint32_t K = ts[t].K;
    uint64_t* bd = bounds + td.slot_begin + t;
    const uint64_t hi = td.off + td.m;
    uint64_t i = td.off;
    uint32_t c = 0;
    // each search returns the key at the bucket start it finds, which is
    // the next search's pivot, and the bucket's length guides the next
    // search (the first one guesses the average)
    typename TR::Key piv = TR::key(data[i]);
    uint64_t guess = td.m / (K ? K : 1);
    while (i < hi) {
        if (c >= K) {
            if (lane == 0) raise_err(err, ERR_MARKS);
            return;
        }
        const typename TR::Key top = piv;
        const uint64_t j = wave_next_larger<DT>(data, piv, i + 1, hi, &piv, guess ? guess - 1 : 0);
        // with MIN, a bucket above the capacity whose last entry (its
        // smallest key) equals its first (its largest) holds one key value
        bool one = false;
        if constexpr (MIN) {
            if (j - i > cap) one = TR::key(data[j - 1]) == top;
        }
        if (lane == 0) bd[c] = (i - td.off) | (one ? kOneKeyBit : 0ull);
        guess = j - i;
        i = j;
        ++c;
    }
    for (uint32_t q = c + lane; q <= K; q += 64) bd[q] = td.m;
}

}  // namespace ips4o
