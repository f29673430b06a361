// Element and key traits of the five element types, and small wavefront
// helpers, for the gfx950 samplesort kernels.
//
// Every comparison the method makes is between keys (Section 1: a total order
// on the keys).  Keys are extracted once per element into a register type
// whose `<=` is the order:
//   U64      the value;
//   F64      the IEEE 754 totalOrder image of the bits (sign bit set: all bits
//            flipped; sign bit clear: only the sign bit flipped), compared as
//            an unsigned integer;
//   PAIR     word 0;
//   QUARTET  (w0, w1, w2) lexicographic;
//   BYTES100 bytes 0..9 read big-endian as an 80-bit unsigned (hi: bytes 0..7,
//            lo: bytes 8..9).
// Elements are moved as opaque words (u64, or u32 for the 100-byte records,
// whose start addresses are only 4-byte aligned).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ips4o {

enum DType : int { DT_U64 = 0, DT_F64 = 1, DT_PAIR = 2, DT_QUARTET = 3, DT_BYTES100 = 4 };

struct Key1 {
    uint64_t v;
};
__device__ __host__ inline bool operator<=(const Key1& a, const Key1& b) { return a.v <= b.v; }
__device__ __host__ inline bool operator<(const Key1& a, const Key1& b) { return a.v < b.v; }
__device__ __host__ inline bool operator==(const Key1& a, const Key1& b) { return a.v == b.v; }

struct Key3 {
    uint64_t a, b, c;
};
__device__ __host__ inline bool operator<(const Key3& x, const Key3& y) {
    return x.a < y.a || (x.a == y.a && (x.b < y.b || (x.b == y.b && x.c < y.c)));
}
__device__ __host__ inline bool operator==(const Key3& x, const Key3& y) {
    return x.a == y.a && x.b == y.b && x.c == y.c;
}
__device__ __host__ inline bool operator<=(const Key3& x, const Key3& y) { return !(y < x); }

struct Key10 {
    uint64_t hi;
    uint32_t lo;
    uint32_t pad;
};
__device__ __host__ inline bool operator<(const Key10& x, const Key10& y) {
    return x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo);
}
__device__ __host__ inline bool operator==(const Key10& x, const Key10& y) {
    return x.hi == y.hi && x.lo == y.lo;
}
__device__ __host__ inline bool operator<=(const Key10& x, const Key10& y) { return !(y < x); }

struct E16 {
    uint64_t w[2];
};
struct E32 {
    uint64_t w[4];
};
struct E100 {
    uint32_t w[25];
};

__device__ __host__ inline uint32_t bswap32(uint32_t x) {
    return (x >> 24) | ((x >> 8) & 0xff00u) | ((x << 8) & 0xff0000u) | (x << 24);
}

template <int DT>
struct Traits;

template <>
struct Traits<DT_U64> {
    using Elem = uint64_t;
    using Key = Key1;
    using Word = uint64_t;
    static constexpr int kWords = 1;
    static constexpr int kBaseCap = 16384;
    __device__ __host__ static Key key(const Elem& e) { return Key{e}; }
    __device__ __host__ static Key max_key() { return Key{~0ull}; }
};

template <>
struct Traits<DT_F64> {
    using Elem = uint64_t;
    using Key = Key1;
    using Word = uint64_t;
    static constexpr int kWords = 1;
    static constexpr int kBaseCap = 16384;
    __device__ __host__ static Key key(const Elem& e) {
        uint64_t flip = (uint64_t)((int64_t)e >> 63) | 0x8000000000000000ull;
        return Key{e ^ flip};
    }
    // inverse of key(): the top bit of the image tells the original sign
    __device__ __host__ static Elem unkey(uint64_t k) {
        return (k >> 63) ? (k ^ 0x8000000000000000ull) : ~k;
    }
    __device__ __host__ static Key max_key() { return Key{~0ull}; }
};

template <>
struct Traits<DT_PAIR> {
    using Elem = E16;
    using Key = Key1;
    using Word = uint64_t;
    static constexpr int kWords = 2;
    static constexpr int kBaseCap = 8192;
    __device__ __host__ static Key key(const Elem& e) { return Key{e.w[0]}; }
    __device__ __host__ static Key max_key() { return Key{~0ull}; }
};

template <>
struct Traits<DT_QUARTET> {
    using Elem = E32;
    using Key = Key3;
    using Word = uint64_t;
    static constexpr int kWords = 4;
    static constexpr int kBaseCap = 4096;
    __device__ __host__ static Key key(const Elem& e) { return Key{e.w[0], e.w[1], e.w[2]}; }
    __device__ __host__ static Key max_key() { return Key{~0ull, ~0ull, ~0ull}; }
};

template <>
struct Traits<DT_BYTES100> {
    using Elem = E100;
    using Key = Key10;
    using Word = uint32_t;
    static constexpr int kWords = 25;
    static constexpr int kBaseCap = 4096;
    __device__ __host__ static Key key(const Elem& e) {
        uint64_t hi = ((uint64_t)bswap32(e.w[0]) << 32) | bswap32(e.w[1]);
        uint32_t lo = bswap32(e.w[2]) >> 16;
        return Key{hi, lo, 0};
    }
    __device__ __host__ static Key max_key() { return Key{~0ull, 0xffffu, 0}; }
};

// ---------------------------------------------------------------- wavefront
__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint64_t bcast_u64(uint64_t v) {  // value of the first active lane
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t bcast_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <class K>
__device__ inline K bcast_key(const K& k) {
    K r;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&k);
    uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(K) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return r;
}

// value of register `v` in lane `src` (uniform result)
__device__ inline uint32_t read_lane(uint32_t v, uint32_t src) {
    return __builtin_amdgcn_readlane(v, src);
}

// wait for every outstanding vector memory operation of this wave
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Workgroup barrier that orders LDS only: waits for this wave's LDS
// operations (lgkmcnt 0) but not for its global loads and stores, so loads
// issued ahead of time stay in flight across it.  Use __syncthreads() where
// other waves must see this wave's global stores.
__device__ inline void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);     // lgkmcnt(0); vmcnt, expcnt unconstrained
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace ips4o
