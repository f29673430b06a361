"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a small C driver built together with oracle/oracle.c runs every
entry point on all five element types at small and ragged sizes (empty
arrays, empty segments, one splitter, duplicate splitters, k = 2 .. 1024
trees, empty and one-element buckets for the marking) and checks the plain properties of each result; any out-of-bounds
access, overflow or misaligned load aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

size_t or_elem_size(int dtype);
int or_compare(const void *a, const void *b, int dtype);
int or_sort(void *data, uint64_t n, int dtype);
int or_sort_segmented(void *data, const uint64_t *offs, uint32_t nseg, int dtype);
uint32_t or_num_buckets(int dtype, const void *splitters, uint32_t m, int eq);
int or_classify(const void *data, uint64_t n, int dtype, const void *splitters, uint32_t m, int eq,
                uint32_t *out);
int or_bucket_bounds(const void *data, uint64_t n, int dtype, const void *splitters, uint32_t m, int eq,
                     uint64_t *counts, uint64_t *bounds);
int or_select_splitters(const void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha, uint64_t seed,
                        void *scratch, void *out, uint32_t *m_unique, int *eq);
int or_select_splitters_capped(const void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha, uint64_t seed,
                               uint32_t kcap, void *scratch, void *out, uint32_t *m_unique, int *eq);
void or_tree(const uint64_t *s, uint32_t k, uint64_t *a);
uint32_t or_tree_descend(const uint64_t *a, uint32_t k, uint64_t e);
int or_sort_small_integers(void *data, uint64_t n, int dtype, uint64_t vmax, uint32_t *counts);
int or_mark_bucket_max(void *data, int dtype, const uint64_t *bounds, uint32_t nb);
uint64_t or_search_next_largest(const void *pivot, const void *data, uint64_t lo, uint64_t hi, int dtype,
                                uint64_t *probes);
int or_sort_strict(void *data, uint64_t n, int dtype, uint32_t k, uint32_t alpha, uint64_t n0, uint64_t seed,
                   uint64_t *stats);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
#define FAIL(msg) do { fprintf(stderr, "FAIL %s (line %d)\n", msg, __LINE__); return 1; } while (0)

static void fill(unsigned char *d, uint64_t n, size_t s, int few) {
    for (uint64_t i = 0; i < n * s; ++i) d[i] = (unsigned char)(few ? rnd() % 3 : rnd());
}

static int sorted(const unsigned char *d, uint64_t n, size_t s, int dt) {
    for (uint64_t i = 1; i < n; ++i)
        if (or_compare(d + (i - 1) * s, d + i * s, dt) > 0) return 0;
    return 1;
}

int main(void) {
    const uint64_t sizes[] = {0, 1, 2, 3, 17, 256, 1001};
    for (int dt = 0; dt < 5; ++dt) {
        const size_t s = or_elem_size(dt);
        for (int few = 0; few < 2; ++few)
            for (size_t zi = 0; zi < sizeof sizes / sizeof sizes[0]; ++zi) {
                const uint64_t n = sizes[zi];
                unsigned char *d = malloc(n * s + 1);
                fill(d, n, s, few);
                if (or_sort(d, n, dt) != 0 || !sorted(d, n, s, dt)) FAIL("or_sort");
                /* segments of random lengths, some empty */
                uint64_t offs[12];
                offs[0] = 0;
                for (int i = 1; i < 11; ++i) offs[i] = n ? offs[i - 1] + rnd() % (n / 8 + 1) : 0;
                for (int i = 1; i < 11; ++i) if (offs[i] > n) offs[i] = n;
                offs[11] = n;
                fill(d, n, s, few);
                if (or_sort_segmented(d, offs, 11, dt) != 0) FAIL("or_sort_segmented");
                for (int i = 0; i < 11; ++i)
                    if (!sorted(d + offs[i] * s, offs[i + 1] - offs[i], s, dt)) FAIL("segment order");
                /* splitters from the data (duplicates when few), with and
                   without equality buckets */
                if (n > 0) {
                    for (uint32_t m = 1; m <= 9; m += 4) {
                        unsigned char *sp = malloc(m * s);
                        for (uint32_t i = 0; i < m; ++i) memcpy(sp + i * s, d + (rnd() % n) * s, s);
                        or_sort(sp, m, dt);
                        for (int eq = 0; eq < 2; ++eq) {
                            const uint32_t K = or_num_buckets(dt, sp, m, eq);
                            uint32_t *b = malloc(n * sizeof *b);
                            uint64_t *cnt = malloc(K * sizeof *cnt), *bd = malloc((K + 1) * sizeof *bd);
                            if (or_classify(d, n, dt, sp, m, eq, b) != 0) FAIL("or_classify");
                            for (uint64_t i = 0; i < n; ++i) if (b[i] >= K) FAIL("bucket range");
                            if (or_bucket_bounds(d, n, dt, sp, m, eq, cnt, bd) != 0) FAIL("or_bucket_bounds");
                            if (bd[0] != 0 || bd[K] != n) FAIL("bounds ends");
                            free(b); free(cnt); free(bd);
                        }
                        free(sp);
                    }
                    for (uint32_t k = 2; k <= 64; k *= 4) {
                        const uint32_t alpha = 3;
                        unsigned char *scr = malloc((alpha * k - 1) * s), *out = malloc((k - 1) * s);
                        uint32_t mu = 0; int eq = 0;
                        if (or_select_splitters(d, n, dt, k, alpha, 77 + k, scr, out, &mu, &eq) != 0)
                            FAIL("or_select_splitters");
                        if (mu < 1 || mu > k - 1 || !sorted(out, mu, s, dt)) FAIL("splitters");
                        if (or_select_splitters_capped(d, n, dt, k, alpha, 77 + k, k, scr, out, &mu, &eq) != 0)
                            FAIL("or_select_splitters_capped");
                        if (mu < 1 || (eq ? 2 * mu + 1 : mu + 1) > k || !sorted(out, mu, s, dt))
                            FAIL("capped splitters");
                        free(scr); free(out);
                    }
                }
                free(d);
            }
    }
    /* the implicit tree against a linear count, k = 2 .. 1024 */
    for (uint32_t k = 2; k <= 1024; k *= 2) {
        uint64_t *sp = malloc((k - 1) * sizeof *sp), *a = malloc((k - 1) * sizeof *a);
        for (uint32_t i = 0; i + 1 < k; ++i) sp[i] = rnd() % 4096;
        or_sort(sp, k - 1, 0);
        or_tree(sp, k, a);
        for (int t = 0; t < 200; ++t) {
            const uint64_t e = rnd() % 4100;
            uint32_t c = 0;
            for (uint32_t i = 0; i + 1 < k; ++i) c += sp[i] <= e;
            if (or_tree_descend(a, k, e) != c) FAIL("tree descent");
        }
        free(sp); free(a);
    }
    /* counting sort of small integers (u64 and integer-valued f64), sizes
       0 .. 1001 with vmax down to 1, and a refused key */
    for (int dt = 0; dt < 2; ++dt)
        for (size_t zi = 0; zi < sizeof sizes / sizeof sizes[0]; ++zi) {
            const uint64_t n = sizes[zi], vmax = 1 + rnd() % 40;
            uint64_t *d = malloc(n * 8 + 8);
            uint32_t *cnt = malloc(vmax * sizeof *cnt);
            for (uint64_t i = 0; i < n; ++i) {
                const uint64_t v = rnd() % vmax;
                if (dt == 0) d[i] = v; else { double x = (double)v; memcpy(&d[i], &x, 8); }
            }
            if (or_sort_small_integers(d, n, dt, vmax, cnt) != 0) FAIL("or_sort_small_integers");
            if (!sorted((unsigned char *)d, n, 8, dt)) FAIL("small integers order");
            if (n > 0) {
                if (dt == 0) d[n - 1] = vmax; else { double x = 0.5; memcpy(&d[n - 1], &x, 8); }
                if (or_sort_small_integers(d, n, dt, vmax, cnt) != -2) FAIL("a bad key accepted");
            }
            free(d); free(cnt);
        }
    /* the strictly in-place recursion: marking, searchNextLargest, the loop */
    for (int dt = 0; dt < 5; ++dt)
        for (uint64_t n = 0; n < 300; n += 37) {
            const size_t s = or_elem_size(dt);
            unsigned char *d = malloc(n * s + 1);
            for (uint64_t i = 0; i < n * s; ++i) d[i] = (unsigned char)(rnd() % 3);
            uint64_t bd[6] = {0, n / 5, n / 5, n / 2, n - n / 7, n};
            if (or_mark_bucket_max(d, dt, bd, 5) != 0) FAIL("or_mark_bucket_max");
            for (int b = 0; b < 5; ++b)
                for (uint64_t p = bd[b]; p < bd[b + 1]; ++p)
                    if (or_compare(d + p * s, d + bd[b] * s, dt) > 0) FAIL("marked entry not the largest");
            if (n > 1) {
                uint64_t pr = 0, j = or_search_next_largest(d, d, 1, n, dt, &pr);
                if (j < 1 || j > n) FAIL("or_search_next_largest range");
            }
            uint64_t stats[4];
            if (or_sort_strict(d, n, dt, 4, 1, 3, 5, stats) != 0 || !sorted(d, n, s, dt)) FAIL("or_sort_strict");
            free(d);
        }
    printf("ok\n");
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    probe = subprocess.run([gcc] + flags + ["-x", "c", "-", "-o", str(tmp_path / "probe")],
                           input="int main(void){return 0;}", capture_output=True, text=True)
    if probe.returncode != 0:
        pytest.skip("gcc cannot link the sanitizer runtimes here")
    subprocess.run([gcc] + flags + ["-o", str(exe), str(drv), ORACLE_C], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-2000:]
