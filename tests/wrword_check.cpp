// CPU check of the permutation's per-bucket word (csrc/wrword.hpp): the
// fields w, r and the reader count change only as the single 64-bit adds of
// the kernels intend, at the extremes of every field, and a simulated
// interleaving of claims, failed claims, reader exits and writes keeps the
// protocol's invariants.  Built with g++ and the host sanitizers by
// tests/test_planner.py; no GPU involved.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1705_02257_amd/csrc/wrword.hpp"

using namespace ips4o;

#define CHECK(cond, ...)                                      \
    do {                                                      \
        if (!(cond)) {                                        \
            std::fprintf(stderr, "FAIL line %d: ", __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                \
            std::fprintf(stderr, "\n");                       \
            std::exit(1);                                     \
        }                                                     \
    } while (0)

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}

static void fields(uint64_t v, int64_t w, int64_t r, uint32_t d, int line) {
    if (wr_w(v) != w || wr_r(v) != r || wr_readers(v) != d) {
        std::fprintf(stderr, "FAIL line %d: got w %lld r %lld readers %u, want %lld %lld %u\n", line,
                     (long long)wr_w(v), (long long)wr_r(v), wr_readers(v), (long long)w, (long long)r, d);
        std::exit(1);
    }
}

int main() {
    // extremes of every field survive every add the kernels make
    const int64_t wmax = (int64_t)WR_MAX_BLOCKS;
    const int64_t ws[] = {0, 1, 12345, wmax - 1, wmax};
    const int64_t rs_[] = {-1 - (int64_t)WR_MAX_READERS, -1, 0, 7, wmax - 1};
    const uint32_t ds[] = {0, 1, 100, WR_MAX_READERS - 1};
    for (int64_t w : ws)
        for (int64_t r : rs_)
            for (uint32_t d : ds) {
                uint64_t v = wr_pack(w, r) + d;
                fields(v, w, r, d, __LINE__);
                if (r > -1 - (int64_t)WR_MAX_READERS) fields(v + WR_CLAIM, w, r - 1, d + 1, __LINE__);
                if (d > 0) fields(v + ~0ull, w, r, d - 1, __LINE__);
                if (w < wmax) fields(v + WR_WONE, w + 1, r, d, __LINE__);
            }
    CHECK(WR_MAX_BLOCKS + (uint64_t)WR_RBIAS < (1ull << (WR_WSHIFT - WR_RSHIFT)), "r field too narrow");
    CHECK((uint64_t)WR_MAX_BLOCKS < (1ull << (64 - WR_WSHIFT)), "w field too narrow");

    // a simulated bucket: workers claim blocks from the top (r) and write
    // from the bottom (w) in random interleavings; a claim that finds r < w
    // fails and leaves its reader count again; every worker fails at most
    // once (after a failure it sees r < w and never claims again).  The
    // count a writer sees whenever it writes a block that was full at the
    // start includes every reader still loading such a block.
    for (int trial = 0; trial < 2000; ++trial) {
        const int64_t d0 = (int64_t)(rnd() % 1000), full = (int64_t)(rnd() % 300);
        const int64_t rinit = d0 + full;
        const int workers = 1 + (int)(rnd() % 64);
        uint64_t v = wr_pack(d0, rinit - 1);
        std::vector<int64_t> reading(workers, -1);   // block a worker is loading, or -1
        std::vector<bool> failed(workers, false);
        int64_t writes = 0;
        for (int step = 0; step < 20000; ++step) {
            const int who = (int)(rnd() % workers);
            const int what = (int)(rnd() % 3);
            if (what == 0 && reading[who] < 0 && !failed[who] && wr_r(v) >= wr_w(v)) {
                const uint64_t old = v;
                v += WR_CLAIM;
                if (wr_r(old) < wr_w(old)) {
                    failed[who] = true;
                    v += ~0ull;
                } else {
                    reading[who] = wr_r(old);
                }
            } else if (what == 1 && reading[who] >= 0) {
                reading[who] = -1;                      // load done: leave the count
                v += ~0ull;
            } else if (what == 2 && writes < full) {
                const uint64_t old = v;
                v += WR_WONE;
                ++writes;
                const int64_t x = wr_w(old);
                if (x > wr_r(old) && x < rinit) {
                    int live = 0;
                    for (int q = 0; q < workers; ++q) live += reading[q] >= 0;
                    CHECK((int)wr_readers(old) == live, "readers %u, live %d", wr_readers(old), live);
                    for (int q = 0; q < workers; ++q)
                        if (reading[q] == x) CHECK(wr_readers(old) > 0, "reader of %lld not counted", (long long)x);
                }
            }
            int live = 0;
            for (int q = 0; q < workers; ++q) live += reading[q] >= 0;
            CHECK((int)wr_readers(v) == live, "count %u, live readers %d", wr_readers(v), live);
            CHECK(wr_r(v) >= d0 - 1 - workers, "r fell too far");
        }
    }
    std::printf("wrword ok\n");
    return 0;
}
