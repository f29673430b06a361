/*
 * Seeded synthetic input generators shared by the tests, the oracle checks and
 * the benchmark.  This file holds none of the sorting method's arithmetic: it
 * only produces the nine input distributions of the paper's experiments
 * (Section 5, "Experimental Results": Uniform, Exponential, AlmostSorted,
 * RootDup, TwoDup, EightDup, Sorted, ReverseSorted, Ones) for 8-byte keys and
 * for the record types Pair, Quartet and 100Bytes.
 *
 * Randomness: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used counter-based: value i of stream
 * `seed` is the i-th output (0-based) of the splitmix64 sequence whose state
 * starts at `seed`, i.e. mix(seed + (i + 1) * golden_gamma).
 *
 * Readings of the paper's definitions (the formulas are 1-based and partly
 * garbled in the source; these are the 0-based readings):
 *   Uniform      u64: h_i ;  f64: (h_i >> 11) * 2^-53 in [0, 1)
 *   Exponential  f64: -ln(1 - u_i) (rate 1);  u64: the bit pattern of that
 *                double (order preserving because it is >= 0)
 *   Sorted       u64: i*q + (h_i mod q), q = floor(2^64 / n);  f64: (i + u_i)/n
 *   ReverseSorted  Sorted read backwards
 *   AlmostSorted Sorted, then floor(sqrt(n)) swaps of index pairs drawn from
 *                stream seed ^ SWAP_STREAM, applied in order
 *   Ones         1 / 1.0
 *   RootDup      i mod floor(sqrt(n))
 *   TwoDup       (i^2 + floor(n/2)) mod n   (exact integer arithmetic)
 *   EightDup     (i^8 + floor(n/2)) mod n   (exact integer arithmetic)
 * Integer-valued distributions convert exactly to double (all values < 2^53).
 *
 * Records (payload = original index i, so that the output can be checked
 * without a second sort):
 *   Pair     {u64 key, u64 payload=i}
 *   Quartet  {u64 w0, w1, w2, u64 payload=i}; word j is the u64 distribution
 *            value drawn from stream seed + j (deterministic distributions give
 *            w0 = w1 = w2)
 *   100Bytes {u8 key[10], u8 rest[90]}: key = 80-bit value big-endian (Uniform:
 *            64 random bits followed by 16 more; other distributions: the u64
 *            value right-aligned in the 10 bytes), rest[0..8) = i little-endian,
 *            rest[8..90) = filler bytes from stream splitmix64(i).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define WL_GAMMA 0x9e3779b97f4a7c15ULL
#define WL_SWAP_STREAM 0x5157a9c3d2e1f0b7ULL
#define WL_HI_STREAM 0x0123456789abcdefULL

enum { WL_UNIFORM = 0, WL_EXPONENTIAL, WL_SORTED, WL_REVERSE, WL_ALMOST,
       WL_ONES, WL_ROOTDUP, WL_TWODUP, WL_EIGHTDUP, WL_NDIST };
enum { WL_U64 = 0, WL_F64 = 1, WL_PAIR = 2, WL_QUARTET = 3, WL_BYTES100 = 4 };

static inline uint64_t wl_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* i-th (0-based) output of the splitmix64 stream with initial state `seed`. */
uint64_t wl_splitmix64_at(uint64_t seed, uint64_t i) {
    return wl_mix(seed + (i + 1) * WL_GAMMA);
}

static inline double wl_unit(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

static uint64_t isqrt_floor(uint64_t n) {
    uint64_t r = (uint64_t)sqrt((double)n);
    while (r * r > n) --r;
    while ((r + 1) * (r + 1) <= n) ++r;
    return r;
}

static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((unsigned __int128)a * b) % m);
}

/* u64 value of distribution `dist` at position i (Sorted-family positions are
 * the monotone ones; the reversal and the swaps are applied by the caller). */
static uint64_t value_u64(int dist, uint64_t n, uint64_t seed, uint64_t i) {
    switch (dist) {
    case WL_UNIFORM: return wl_splitmix64_at(seed, i);
    case WL_EXPONENTIAL: {
        double x = -log(1.0 - wl_unit(wl_splitmix64_at(seed, i)));
        uint64_t b; memcpy(&b, &x, 8); return b;
    }
    case WL_SORTED: case WL_REVERSE: case WL_ALMOST: {
        uint64_t q = (n <= 1) ? ~0ULL : (uint64_t)(((unsigned __int128)1 << 64) / n);
        return i * q + wl_splitmix64_at(seed, i) % q;
    }
    case WL_ONES: return 1;
    case WL_ROOTDUP: return i % isqrt_floor(n);
    case WL_TWODUP: { uint64_t x = i % n; return (mulmod(x, x, n) + n / 2) % n; }
    case WL_EIGHTDUP: {
        uint64_t x = i % n, x2 = mulmod(x, x, n), x4 = mulmod(x2, x2, n), x8 = mulmod(x4, x4, n);
        return (x8 + n / 2) % n;
    }
    }
    return 0;
}

static double value_f64(int dist, uint64_t n, uint64_t seed, uint64_t i) {
    switch (dist) {
    case WL_UNIFORM: return wl_unit(wl_splitmix64_at(seed, i));
    case WL_EXPONENTIAL: return -log(1.0 - wl_unit(wl_splitmix64_at(seed, i)));
    case WL_SORTED: case WL_REVERSE: case WL_ALMOST:
        return ((double)i + wl_unit(wl_splitmix64_at(seed, i))) / (double)n;
    default: return (double)value_u64(dist, n, seed, i);
    }
}

/* position in the monotone sequence that lands at output index i */
static inline uint64_t src_index(int dist, uint64_t n, uint64_t i) {
    return dist == WL_REVERSE ? n - 1 - i : i;
}

static void apply_swaps(unsigned char *base, uint64_t n, size_t s, uint64_t seed) {
    uint64_t m = isqrt_floor(n);
    unsigned char tmp[128];
    for (uint64_t j = 0; j < m; ++j) {
        uint64_t a = wl_splitmix64_at(seed ^ WL_SWAP_STREAM, 2 * j) % n;
        uint64_t b = wl_splitmix64_at(seed ^ WL_SWAP_STREAM, 2 * j + 1) % n;
        memcpy(tmp, base + a * s, s);
        memcpy(base + a * s, base + b * s, s);
        memcpy(base + b * s, tmp, s);
    }
}

static size_t elem_size(int dtype) {
    switch (dtype) {
    case WL_U64: case WL_F64: return 8;
    case WL_PAIR: return 16;
    case WL_QUARTET: return 32;
    case WL_BYTES100: return 100;
    }
    return 0;
}

/* Fill out[0..count) with elements first .. first+count-1 of the n-element
 * array (n elements of the dtype's size in all).  Every element depends only
 * on n, the seed and its own index, except for AlmostSorted, whose swaps
 * reach across the whole array: that one is produced only whole
 * (first = 0, count = n).  Returns 0, or -1 on a bad argument.  The loop is
 * embarrassingly parallel and split with OpenMP when the library is built
 * with it; values do not depend on the thread count. */
int wl_generate_range(int dist, int dtype, uint64_t n, uint64_t seed, uint64_t first, uint64_t count,
                      void *out) {
    if (dist < 0 || dist >= WL_NDIST || elem_size(dtype) == 0 || (count && !out)) return -1;
    if (first > n || count > n - first) return -1;
    if (dist == WL_ALMOST && count && (first != 0 || count != n)) return -1;
    if (count == 0) return 0;
    size_t s = elem_size(dtype);
    unsigned char *base = (unsigned char *)out;
    int64_t nn = (int64_t)count;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < nn; ++ii) {
        uint64_t i = first + (uint64_t)ii, p = src_index(dist, n, i);
        unsigned char *e = base + (uint64_t)ii * s;
        if (dtype == WL_U64) {
            uint64_t v = value_u64(dist, n, seed, p); memcpy(e, &v, 8);
        } else if (dtype == WL_F64) {
            double v = value_f64(dist, n, seed, p); memcpy(e, &v, 8);
        } else if (dtype == WL_PAIR) {
            uint64_t w[2] = { value_u64(dist, n, seed, p), i }; memcpy(e, w, 16);
        } else if (dtype == WL_QUARTET) {
            uint64_t w[4] = { value_u64(dist, n, seed, p), value_u64(dist, n, seed + 1, p),
                              value_u64(dist, n, seed + 2, p), i };
            memcpy(e, w, 32);
        } else { /* WL_BYTES100 */
            uint64_t v = value_u64(dist, n, seed, p);
            uint64_t lo16 = dist == WL_UNIFORM ? (wl_splitmix64_at(seed ^ WL_HI_STREAM, p) & 0xffff) : 0;
            unsigned char key[10];
            if (dist == WL_UNIFORM) {
                for (int b = 0; b < 8; ++b) key[b] = (unsigned char)(v >> (56 - 8 * b));
                key[8] = (unsigned char)(lo16 >> 8); key[9] = (unsigned char)lo16;
            } else {
                key[0] = key[1] = 0;
                for (int b = 0; b < 8; ++b) key[2 + b] = (unsigned char)(v >> (56 - 8 * b));
            }
            memcpy(e, key, 10);
            for (int b = 0; b < 8; ++b) e[10 + b] = (unsigned char)(i >> (8 * b));
            for (int b = 18; b < 100; b += 8) {
                uint64_t f = wl_splitmix64_at(i, (uint64_t)(b - 18) / 8);
                int len = 100 - b < 8 ? 100 - b : 8;
                memcpy(e + b, &f, (size_t)len);
            }
        }
    }
    if (dist == WL_ALMOST) apply_swaps(base, n, s, seed);
    return 0;
}

/* Fill out[0..n) (n elements of the dtype's size).  Returns 0, or -1 on a bad
 * argument. */
int wl_generate(int dist, int dtype, uint64_t n, uint64_t seed, void *out) {
    if (n && !out) return -1;
    return wl_generate_range(dist, dtype, n, seed, 0, n, out);
}
