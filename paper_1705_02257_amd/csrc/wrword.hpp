// The per-bucket word of the block permutation (Section 4.2), plain C++ so
// that the kernels and a CPU-only test program share it.
//
// The word `wr` packs the write pointer w, the read pointer r and the
// number of workers reading a block of the bucket (Section 4.2: the paper
// keeps (w, r) in one 128-bit word and a reader count per bucket): bits
// 39..63 w, bits 14..38 r + WR_RBIAS, bits 0..13 readers.  A claim adds
// WR_CLAIM (one more reader, r one lower) in a single atomic, so the count
// a writer sees always includes every reader whose claim it could conflict
// with.  r may fall below w by one per worker that finds the bucket empty
// (each worker at most once per bucket); the bias keeps those decrements
// from borrowing into w.  Block indices stay below WR_MAX_BLOCKS and a task
// has at most WR_MAX_READERS workers.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define HD __host__ __device__
#else
#define HD
#endif

namespace ips4o {

constexpr int WR_RSHIFT = 14, WR_WSHIFT = 39;
constexpr uint64_t WR_READER = 1ull;
constexpr uint64_t WR_RONE = 1ull << WR_RSHIFT;
constexpr uint64_t WR_WONE = 1ull << WR_WSHIFT;
constexpr uint64_t WR_CLAIM = WR_READER - WR_RONE;          // readers + 1, r - 1 (mod 2^64)
constexpr int64_t WR_RBIAS = 1ll << 15;
constexpr uint32_t WR_MAX_READERS = (1u << WR_RSHIFT) - 1;
constexpr uint64_t WR_MAX_BLOCKS = (1ull << (WR_WSHIFT - WR_RSHIFT)) - 2 * (uint64_t)WR_RBIAS;
HD inline uint64_t wr_pack(int64_t w, int64_t r) {
    return ((uint64_t)w << WR_WSHIFT) | ((uint64_t)(r + WR_RBIAS) << WR_RSHIFT);
}
HD inline int64_t wr_w(uint64_t v) { return (int64_t)(v >> WR_WSHIFT); }
HD inline int64_t wr_r(uint64_t v) {
    return (int64_t)((v >> WR_RSHIFT) & ((1ull << (WR_WSHIFT - WR_RSHIFT)) - 1)) - WR_RBIAS;
}
HD inline uint32_t wr_readers(uint64_t v) { return (uint32_t)(v & WR_MAX_READERS); }

}  // namespace ips4o
