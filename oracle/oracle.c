/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, sequential CPU statement of what the in-place super scalar
 * samplesort of Axtmann, Witt, Ferizovic and Sanders ("In-place Parallel Super
 * Scalar Samplesort (IPS4o)", arXiv 1705.02257) computes.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library.
 *
 * Each function cites the passage it follows.  Where the method reaches a
 * result with a plain definition (a sorted arrangement, a bucket index, a
 * histogram, a prefix sum) the function is that definition written out, with
 * the C library's qsort as the one library step.
 *
 * Element types (Section 5, data types): U64 and F64 keys; Pair = {u64 key,
 * u64 payload}; Quartet = {u64 w0, w1, w2 key, u64 payload}, lexicographic;
 * 100Bytes = {10-byte key, 90-byte payload}, lexicographic (unsigned bytes).
 * F64 keys are ordered by IEEE 754 totalOrder, written out from its definition
 * (sign first; then magnitude, reversed for negative numbers).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_U64 = 0, OR_F64 = 1, OR_PAIR = 2, OR_QUARTET = 3, OR_BYTES100 = 4 };

size_t or_elem_size(int dtype) {
    switch (dtype) {
    case OR_U64: case OR_F64: return 8;
    case OR_PAIR: return 16;
    case OR_QUARTET: return 32;
    case OR_BYTES100: return 100;
    }
    return 0;
}

static int cmp_u64_val(uint64_t x, uint64_t y) { return (x > y) - (x < y); }

/* IEEE 754 totalOrder on binary64 bit patterns: every negative-signed value
 * precedes every positive-signed one; among positive-signed values a larger
 * magnitude field (exponent, then fraction, i.e. the low 63 bits read as an
 * unsigned integer) is larger, NaNs above +inf; among negative-signed values
 * the order of magnitudes is reversed, so -NaN < -inf < ... < -0 < +0. */
static int cmp_f64_total(uint64_t x, uint64_t y) {
    int sx = (int)(x >> 63), sy = (int)(y >> 63);
    if (sx != sy) return sx ? -1 : 1;
    uint64_t mx = x & 0x7fffffffffffffffULL, my = y & 0x7fffffffffffffffULL;
    int c = cmp_u64_val(mx, my);
    return sx ? -c : c;
}

static uint64_t ld64(const void *p) { uint64_t v; memcpy(&v, p, 8); return v; }

/* Three-way comparison of the keys of two elements of `dtype`. */
int or_compare(const void *a, const void *b, int dtype) {
    const unsigned char *x = (const unsigned char *)a, *y = (const unsigned char *)b;
    switch (dtype) {
    case OR_U64: case OR_PAIR: return cmp_u64_val(ld64(x), ld64(y));
    case OR_F64: return cmp_f64_total(ld64(x), ld64(y));
    case OR_QUARTET:
        for (int w = 0; w < 3; ++w) {
            int c = cmp_u64_val(ld64(x + 8 * w), ld64(y + 8 * w));
            if (c) return c;
        }
        return 0;
    case OR_BYTES100: {
        int c = memcmp(x, y, 10);
        return (c > 0) - (c < 0);
    }
    }
    return 0;
}

static int q_u64(const void *a, const void *b) { return or_compare(a, b, OR_U64); }
static int q_f64(const void *a, const void *b) { return or_compare(a, b, OR_F64); }
static int q_pair(const void *a, const void *b) { return or_compare(a, b, OR_PAIR); }
static int q_quartet(const void *a, const void *b) { return or_compare(a, b, OR_QUARTET); }
static int q_bytes(const void *a, const void *b) { return or_compare(a, b, OR_BYTES100); }

typedef int (*qcmp_t)(const void *, const void *);
static qcmp_t qcmp_for(int dtype) {
    switch (dtype) {
    case OR_U64: return q_u64;
    case OR_F64: return q_f64;
    case OR_PAIR: return q_pair;
    case OR_QUARTET: return q_quartet;
    case OR_BYTES100: return q_bytes;
    }
    return 0;
}

/* Problem statement (Section 1): arrange A[0..n) so that the keys are
 * non-decreasing under the total order.  The key sequence of the result is
 * unique; the order of payloads among equal keys is not (samplesort is not
 * stable).  Library step: qsort.  Returns 0, or -1 for a bad dtype. */
int or_sort(void *data, uint64_t n, int dtype) {
    qcmp_t c = qcmp_for(dtype);
    if (!c) return -1;
    if (n > 1) qsort(data, (size_t)n, or_elem_size(dtype), c);
    return 0;
}

/* The non-decreasing arrangement (Section 1) of n keys that are all
 * integers in [0, vmax): u64 values, or f64 values whose bit pattern is that
 * of such an integer converted to binary64 (so no -0, NaN or fraction).  Such
 * keys compare as the integers they hold under either order, so the sorted
 * arrangement holds every value v exactly count(v) times, in increasing v:
 * count, then write out (no comparisons).  This is how the integer-valued
 * inputs of Section 5 (Ones, RootDup, TwoDup, EightDup: values below n) are
 * sorted at sizes where qsort takes minutes.  counts: caller buffer of vmax
 * uint32.  Returns 0; -1 for a dtype other than u64/f64 or n >= 2^32; -2 when
 * a key is not such an integer (the data is then unchanged). */
int or_sort_small_integers(void *data, uint64_t n, int dtype, uint64_t vmax, uint32_t *counts) {
    if ((dtype != OR_U64 && dtype != OR_F64) || n >= (1ULL << 32)) return -1;
    unsigned char *d = (unsigned char *)data;
    for (uint64_t v = 0; v < vmax; ++v) counts[v] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t bits = ld64(d + 8 * i), v;
        if (dtype == OR_U64) {
            v = bits;
            if (v >= vmax) return -2;
        } else {
            double x;
            memcpy(&x, &bits, 8);
            if (!(x >= 0.0 && x < (double)vmax)) return -2;
            v = (uint64_t)x;
            double back = (double)v;
            uint64_t bb;
            memcpy(&bb, &back, 8);
            if (bb != bits) return -2;
        }
        counts[v]++;
    }
    uint64_t at = 0;
    for (uint64_t v = 0; v < vmax; ++v) {
        uint64_t bits = v;
        if (dtype == OR_F64) {
            double x = (double)v;
            memcpy(&bits, &x, 8);
        }
        for (uint32_t c = 0; c < counts[v]; ++c, ++at) memcpy(d + 8 * at, &bits, 8);
    }
    return 0;
}

/* Many independent problems (the subproblems of Section 4, given by the
 * caller): segment i is A[offs[i] .. offs[i+1]), each sorted on its own by
 * the problem statement above; elements outside [offs[0], offs[nseg]) are
 * untouched.  Returns 0, -1 for a bad dtype, -2 for decreasing offsets. */
int or_sort_segmented(void *data, const uint64_t *offs, uint32_t nseg, int dtype) {
    if (!qcmp_for(dtype)) return -1;
    for (uint32_t i = 0; i < nseg; ++i)
        if (offs[i + 1] < offs[i]) return -2;
    unsigned char *a = (unsigned char *)data;
    for (uint32_t i = 0; i < nseg; ++i)
        or_sort(a + offs[i] * or_elem_size(dtype), offs[i + 1] - offs[i], dtype);
    return 0;
}

/* Bucket of one element for splitters s_1..s_m (sorted, non-decreasing).
 *  eq == 0 (Section 3, Preliminaries): element e goes to bucket i when
 *     s_{i-1} <= e < s_i with s_0 = -inf and s_{m+1} = +inf, i.e. the bucket
 *     index is the number of splitters <= e, in [0, m].
 *  eq != 0 (Section 4, "The Case of Many Identical Keys", and "Implementation
 *     Details"): duplicates are removed first, giving unique u_1 < ... < u_m'.
 *     Elements equal to a splitter get a bucket of their own between the two
 *     open ranges around it; the buckets in order are
 *     (-inf,u_1), {u_1}, (u_1,u_2), {u_2}, ..., {u_m'}, (u_m',+inf),
 *     numbered 0 .. 2m'.  With j = #{u <= e}: 2j-1 if j >= 1 and u_j == e,
 *     else 2j. */
uint32_t or_bucket(const void *elem, int dtype, const void *splitters, uint32_t m, int eq) {
    size_t s = or_elem_size(dtype);
    const unsigned char *sp = (const unsigned char *)splitters;
    if (!eq) {
        uint32_t cnt = 0;
        for (uint32_t i = 0; i < m; ++i)
            if (or_compare(sp + i * s, elem, dtype) <= 0) ++cnt;
        return cnt;
    }
    uint32_t j = 0;            /* number of distinct splitter keys <= e */
    int last_equal = 0;        /* the largest such key equals e */
    for (uint32_t i = 0; i < m; ++i) {
        if (i > 0 && or_compare(sp + (i - 1) * s, sp + i * s, dtype) == 0) continue;
        int c = or_compare(sp + i * s, elem, dtype);
        if (c <= 0) { ++j; last_equal = (c == 0); }
    }
    return (j >= 1 && last_equal) ? 2 * j - 1 : 2 * j;
}

/* Number of logical buckets for the given splitters. */
uint32_t or_num_buckets(int dtype, const void *splitters, uint32_t m, int eq) {
    if (!eq) return m + 1;
    size_t s = or_elem_size(dtype);
    const unsigned char *sp = (const unsigned char *)splitters;
    uint32_t u = 0;
    for (uint32_t i = 0; i < m; ++i)
        if (i == 0 || or_compare(sp + (i - 1) * s, sp + i * s, dtype) != 0) ++u;
    return 2 * u + 1;
}

/* Bucket index of every element (the classification step, Section 4.1). */
int or_classify(const void *data, uint64_t n, int dtype, const void *splitters,
                uint32_t m, int eq, uint32_t *out) {
    size_t s = or_elem_size(dtype);
    if (!s) return -1;
    const unsigned char *d = (const unsigned char *)data;
    for (uint64_t i = 0; i < n; ++i) out[i] = or_bucket(d + i * s, dtype, splitters, m, eq);
    return 0;
}

/* Bucket sizes (the counts kept during local classification, Section 4.1)
 * and their exclusive prefix sum, the bucket boundaries (Section 4.2):
 * bounds[i] = sum of counts[0..i), bounds[K] = n. */
int or_bucket_bounds(const void *data, uint64_t n, int dtype, const void *splitters,
                     uint32_t m, int eq, uint64_t *counts, uint64_t *bounds) {
    size_t s = or_elem_size(dtype);
    if (!s) return -1;
    uint32_t K = or_num_buckets(dtype, splitters, m, eq);
    const unsigned char *d = (const unsigned char *)data;
    for (uint32_t i = 0; i < K; ++i) counts[i] = 0;
    for (uint64_t i = 0; i < n; ++i) counts[or_bucket(d + i * s, dtype, splitters, m, eq)]++;
    bounds[0] = 0;
    for (uint32_t i = 0; i < K; ++i) bounds[i + 1] = bounds[i] + counts[i];
    return 0;
}

/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014): the i-th (0-based) output
 * of the generator whose state starts at `seed`. */
uint64_t or_splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Sampling (Section 3, Preliminaries, and Section 4, "Sampling"): draw
 * alpha*k - 1 input elements at random, sort them, and pick the k-1 splitters
 * equidistantly: s_i = sample[i*alpha - 1] (1-based i, 0-based sample), so
 * that exactly alpha-1 sample elements lie strictly between two picks.  Then
 * (Section 4, "Implementation Details") duplicates are removed and equality
 * buckets are switched on exactly when there were duplicates.
 *
 * Sample positions: with replacement, position i = floor(h_i * n / 2^64) with
 * h_i = splitmix64 output i of stream `seed`.  Writes the m' unique splitters
 * (whole elements) to `out` (room for k-1), their number to *m_unique and the
 * equality flag to *eq.  `scratch` must hold alpha*k - 1 elements. */
int or_select_splitters(const void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha,
                        uint64_t seed, void *scratch, void *out, uint32_t *m_unique, int *eq) {
    size_t s = or_elem_size(dtype);
    if (!s || n == 0 || k < 2 || alpha < 1) return -1;
    const unsigned char *d = (const unsigned char *)data;
    unsigned char *smp = (unsigned char *)scratch, *o = (unsigned char *)out;
    uint64_t S = (uint64_t)alpha * k - 1;
    for (uint64_t i = 0; i < S; ++i) {
        uint64_t h = or_splitmix64_at(seed, i);
        uint64_t pos = (uint64_t)(((unsigned __int128)h * n) >> 64);
        memcpy(smp + i * s, d + pos * s, s);
    }
    or_sort(smp, S, dtype);
    uint32_t u = 0;
    for (uint32_t i = 1; i < k; ++i) {
        const unsigned char *pick = smp + ((uint64_t)i * alpha - 1) * s;
        if (u > 0 && or_compare(o + (u - 1) * s, pick, dtype) == 0) continue;
        memcpy(o + u * s, pick, s);
        ++u;
    }
    *m_unique = u;
    *eq = (u < k - 1);
    return 0;
}

/* Splitter selection for a stripe whose buffers hold at most kcap buckets
 * (kcap = 0: no limit).  With equality buckets (Section 4, "The Case of Many
 * Identical Keys") u unique splitters make K = 2u + 1 buckets, which can
 * exceed the k buffers of a thread; the paper does not say what happens
 * then.  Reading taken: when 2u + 1 > kcap, every second pick of the same
 * sorted sample is used instead -- k/2 buckets at twice the oversampling,
 * which draws the very same alpha*k - 1 sample elements -- and equality
 * buckets stay on, so K <= k - 1.  Otherwise the result is
 * or_select_splitters'. */
int or_select_splitters_capped(const void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha,
                               uint64_t seed, uint32_t kcap, void *scratch, void *out, uint32_t *m_unique,
                               int *eq) {
    int rc = or_select_splitters(data, n, dtype, k, alpha, seed, scratch, out, m_unique, eq);
    if (rc != 0 || kcap == 0 || !*eq || 2 * *m_unique + 1 <= kcap || k < 4) return rc;
    rc = or_select_splitters(data, n, dtype, k / 2, 2 * alpha, seed, scratch, out, m_unique, eq);
    *eq = 1;
    return rc;
}

/* The implicit search tree of super scalar samplesort (Section 3,
 * Preliminaries): for k a power of two and splitters s_1..s_{k-1}, the array
 * a_1..a_{k-1} is the complete binary search tree in level order with
 * a_1 = s_{k/2}, a_2 = s_{k/4}, a_3 = s_{3k/4}, and the children of a_i are
 * a_{2i} and a_{2i+1}.  Built recursively: node i holds the middle splitter of
 * the index range [lo, hi) it covers, its children the middles of the halves.
 * s[0..k-2] holds s_1..s_{k-1}; a[0..k-2] receives a_1..a_{k-1}. */
static void tree_fill(const uint64_t *s, uint64_t *a, uint32_t node, uint32_t lo, uint32_t hi,
                      uint32_t k) {
    if (node >= k) return;
    uint32_t mid = (lo + hi) / 2;      /* splitter index s_mid */
    a[node - 1] = s[mid - 1];
    tree_fill(s, a, 2 * node, lo, mid, k);
    tree_fill(s, a, 2 * node + 1, mid, hi, k);
}

void or_tree(const uint64_t *s, uint32_t k, uint64_t *a) { tree_fill(s, a, 1, 0, k, k); }

/* Branchless descent through that tree: j = 1, then log2(k) times
 * j = 2j + [a_j <= e]; the bucket is j - k.  (u64 keys.) */
uint32_t or_tree_descend(const uint64_t *a, uint32_t k, uint64_t e) {
    uint32_t j = 1;
    while (j < k) j = 2 * j + (a[j - 1] <= e ? 1u : 0u);
    return j - k;
}

/* ---- Section 4.6, From Almost In-Place to Strictly In-Place ----
 *
 * The partitioning step leaves the largest element of every bucket in the
 * bucket's first entry; the end of a bucket is then found from the data
 * alone, as the first later position holding a larger key, so the recursion
 * keeps no bucket boundaries. */

static void swap_elems(unsigned char *a, unsigned char *b, size_t s) {
    unsigned char t[128];
    memcpy(t, a, s);
    memcpy(a, b, s);
    memcpy(b, t, s);
}

/* The marking the partitioning step must do (Section 4.6): for every bucket
 * [bounds[b], bounds[b+1]) of at least two elements, the first element whose
 * key is the largest of the bucket trades places with the bucket's first
 * element.  bounds[0..nb] are absolute positions, non-decreasing.  Returns
 * 0, or -1 for a bad dtype or decreasing bounds. */
int or_mark_bucket_max(void *data, int dtype, const uint64_t *bounds, uint32_t nb) {
    size_t s = or_elem_size(dtype);
    if (!s) return -1;
    unsigned char *d = (unsigned char *)data;
    for (uint32_t b = 0; b < nb; ++b) {
        if (bounds[b + 1] < bounds[b]) return -1;
        uint64_t lo = bounds[b], hi = bounds[b + 1], best = lo;
        if (hi - lo < 2) continue;
        for (uint64_t p = lo + 1; p < hi; ++p)
            if (or_compare(d + p * s, d + best * s, dtype) > 0) best = p;
        if (best != lo) swap_elems(d + lo * s, d + best * s, s);
    }
    return 0;
}

/* searchNextLargest (Section 4.6): the first position j in [lo, hi) whose
 * key is larger than the key of `pivot` (an element outside the searched
 * range, typically A[lo-1]), or hi if there is none.  Exponential search
 * probes lo, lo+1, lo+3, lo+7, ... (offsets 2^t - 1) until a larger key or
 * the end, then bisection between the last two probes finds the first
 * larger key.  The result is that first position whenever the positions
 * of [lo, hi) holding larger keys form a suffix of it, as they do after a
 * marked partition: the pivot is the largest key of its bucket and every
 * later bucket holds only larger keys.  Otherwise it is some position in
 * [lo, hi].  *probes (if given) receives the number of keys compared. */
uint64_t or_search_next_largest(const void *pivot, const void *data, uint64_t lo, uint64_t hi, int dtype,
                                uint64_t *probes) {
    size_t s = or_elem_size(dtype);
    const unsigned char *d = (const unsigned char *)data;
    uint64_t cnt = 0;
    /* exponential phase: the first probe lo + 2^t - 1 that is >= hi or larger */
    uint64_t below = lo, step = 1;          /* every position in [lo, below) is known not larger */
    uint64_t above = hi;                    /* the answer is at most `above` */
    for (;;) {
        uint64_t p = lo + step - 1;
        if (p >= hi) break;
        ++cnt;
        if (or_compare(d + p * s, pivot, dtype) > 0) { above = p; break; }
        below = p + 1;
        step *= 2;
    }
    /* bisection over [below, above): the first position holding a larger key */
    while (below < above) {
        uint64_t mid = below + (above - below) / 2;
        ++cnt;
        if (or_compare(d + mid * s, pivot, dtype) > 0) above = mid;
        else below = mid + 1;
    }
    if (probes) *probes = cnt;
    return above;
}

/* Insertion sort of A[lo, hi): the base case below n0 (Section 4,
 * Implementation Details). */
static void insertion_sort(unsigned char *d, uint64_t lo, uint64_t hi, int dtype, size_t s) {
    unsigned char t[128];
    for (uint64_t i = lo + 1; i < hi; ++i) {
        memcpy(t, d + i * s, s);
        uint64_t j = i;
        while (j > lo && or_compare(d + (j - 1) * s, t, dtype) > 0) {
            memcpy(d + j * s, d + (j - 1) * s, s);
            --j;
        }
        memcpy(d + j * s, t, s);
    }
}

/* One partitioning step of A[lo, hi) as Section 4.6 requires it: splitters
 * from a sample (or_select_splitters, sample stream splitmix64 output lo of
 * `seed`), every element moved to its bucket (or_bucket) with the order
 * inside a bucket kept (the arrangement inside a bucket is not fixed by the
 * method; this one needs a buffer of hi - lo elements, which is no concern
 * of a checker), then the bucket maxima marked (or_mark_bucket_max).
 * Returns the number of non-empty buckets, or -1. */
static int partition_marked(unsigned char *d, uint64_t lo, uint64_t hi, int dtype, uint32_t k, uint32_t alpha,
                            uint64_t seed) {
    size_t s = or_elem_size(dtype);
    uint64_t m = hi - lo;
    unsigned char *smp = malloc(((size_t)alpha * k) * s), *spl = malloc((size_t)k * s), *tmp = malloc(m * s);
    uint64_t *bounds = malloc((2 * (size_t)k + 2) * sizeof(uint64_t));
    uint32_t *bk = malloc(m * sizeof(uint32_t));
    int rc = -1;
    if (!smp || !spl || !tmp || !bounds || !bk) goto out;
    uint32_t mu = 0;
    int eq = 0;
    if (or_select_splitters(d + lo * s, m, dtype, k, alpha, or_splitmix64_at(seed, lo), smp, spl, &mu, &eq))
        goto out;
    uint32_t K = or_num_buckets(dtype, spl, mu, eq);
    for (uint32_t b = 0; b <= K; ++b) bounds[b] = 0;
    for (uint64_t i = 0; i < m; ++i) {
        bk[i] = or_bucket(d + (lo + i) * s, dtype, spl, mu, eq);
        bounds[bk[i] + 1]++;
    }
    for (uint32_t b = 0; b < K; ++b) bounds[b + 1] += bounds[b];
    {
        uint64_t *fill = malloc(((size_t)K + 1) * sizeof(uint64_t));
        if (!fill) goto out;
        memcpy(fill, bounds, ((size_t)K + 1) * sizeof(uint64_t));
        for (uint64_t i = 0; i < m; ++i) memcpy(tmp + (fill[bk[i]]++) * s, d + (lo + i) * s, s);
        free(fill);
    }
    memcpy(d + lo * s, tmp, m * s);
    rc = 0;
    for (uint32_t b = 0; b <= K; ++b) bounds[b] += lo;
    for (uint32_t b = 0; b < K; ++b) rc += bounds[b + 1] > bounds[b];
    or_mark_bucket_max(d, dtype, bounds, K);
out:
    free(smp); free(spl); free(tmp); free(bounds); free(bk);
    return rc;
}

/* Sequential samplesort with the recursion emulated in constant space
 * (Section 4.6): i is the first element of the current bucket, j the first
 * element of the next one.  While elements remain: a bucket of fewer than
 * n0 elements is sorted by insertion sort and i moves to j; a larger one is
 * partitioned (k buckets, oversampling alpha), which makes its first bucket
 * the current one.  Either way the next j is searchNextLargest(A[i]) over
 * A[i+1, n): A[i] holds the largest key of its bucket, put there by the
 * partition that made the bucket.
 *
 * Reading (the loop as printed never ends on a range of equal keys, which
 * every partition leaves in one bucket): a partition that leaves all of
 * [i, j) in one bucket means the range holds a single key value, since with
 * k >= 3 a range of two or more distinct keys always falls into at least
 * two buckets (its smallest and largest sampled splitters classify apart,
 * or, with equality buckets, a key differing from the one repeated splitter
 * leaves that splitter's bucket).  Such a range is already sorted, and i
 * moves to j.
 *
 * stats (if given, 4 entries): partitions, insertion sorts, ranges found
 * constant, and keys compared by searchNextLargest.  Requires k >= 3,
 * alpha >= 1, n0 >= 1.  Returns 0, or -1. */
int or_sort_strict(void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha, uint64_t n0, uint64_t seed,
                   uint64_t *stats) {
    size_t s = or_elem_size(dtype);
    if (!s || k < 3 || alpha < 1 || n0 < 1) return -1;
    unsigned char *d = (unsigned char *)data, pivot[128];
    uint64_t st[4] = {0, 0, 0, 0};
    uint64_t i = 0, j = n;
    while (i < n) {
        if (j - i < n0) {
            insertion_sort(d, i, j, dtype, s);
            st[1]++;
            i = j;
        } else {
            int nonempty = partition_marked(d, i, j, dtype, k, alpha, seed);
            if (nonempty < 0) return -1;
            st[0]++;
            if (nonempty == 1) {        /* one key value: already sorted */
                st[2]++;
                i = j;
            }
        }
        if (i >= n) break;
        uint64_t pr = 0;
        memcpy(pivot, d + i * s, s);
        j = or_search_next_largest(pivot, d, i + 1, n, dtype, &pr);
        st[3] += pr;
    }
    if (stats) memcpy(stats, st, sizeof st);
    return 0;
}
