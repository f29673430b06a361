"""Pins of the CPU oracle against what the paper and the mathematics fix:
brute force on tiny inputs, the IEEE totalOrder listing, hand-worked bucket
examples, the tree layout the paper prints, published splitmix64 outputs and
invariants that a dropped term, a wrong sign or index, or a transposed
operand would break."""
import itertools
import math

import numpy as np
import pytest

from conftest import golden_lines

DTYPES = ["u64", "f64", "pair", "quartet", "bytes100"]
F64_ORDER = [int(row[0], 16) for row in golden_lines("f64_total_order.txt")]


# ---------------------------------------------------------------- helpers
def _mk(dtype, keys, payloads=None):
    """Build a host array of `dtype` whose i-th key is keys[i] (int, or a bit
    pattern index into F64_ORDER for f64, or a tuple for quartet)."""
    n = len(keys)
    pay = list(range(n)) if payloads is None else payloads
    if dtype == "u64":
        return np.array(keys, dtype=np.uint64)
    if dtype == "f64":
        return np.array([F64_ORDER[k] for k in keys], dtype=np.uint64).view(np.float64)
    if dtype == "pair":
        return np.array([[k, p] for k, p in zip(keys, pay)], dtype=np.uint64).reshape(n, 2)
    if dtype == "quartet":
        return np.array([[k[0], k[1], k[2], p] for k, p in zip(keys, pay)],
                        dtype=np.uint64).reshape(n, 4)
    if dtype == "bytes100":
        a = np.zeros((n, 100), dtype=np.uint8)
        for i, (k, p) in enumerate(zip(keys, pay)):
            a[i, :10] = np.frombuffer(bytes(k), dtype=np.uint8)
            a[i, 10:18] = np.frombuffer(int(p).to_bytes(8, "little"), dtype=np.uint8)
        return a
    raise ValueError(dtype)


def _pykey(dtype, rec):
    """Python-level key of one record, independent of the oracle's C code."""
    if dtype == "u64":
        return int(rec)
    if dtype == "f64":
        return F64_ORDER.index(int(np.float64(rec).view(np.uint64)))
    if dtype == "pair":
        return int(rec[0])
    if dtype == "quartet":
        return (int(rec[0]), int(rec[1]), int(rec[2]))
    if dtype == "bytes100":
        return bytes(rec[:10].tobytes())
    raise ValueError(dtype)


def _records(dtype, arr):
    if arr.ndim == 1:
        return [arr[i].tobytes() for i in range(arr.shape[0])]
    return [arr[i].tobytes() for i in range(arr.shape[0])]


def _brute_force_sorted_set(dtype, arr):
    """All permutations of arr whose key sequence is non-decreasing."""
    n = arr.shape[0]
    keys = [_pykey(dtype, arr[i]) for i in range(n)]
    recs = _records(dtype, arr)
    good = set()
    for perm in itertools.permutations(range(n)):
        if all(keys[perm[i]] <= keys[perm[i + 1]] for i in range(n - 1)):
            good.add(tuple(recs[p] for p in perm))
    return good, keys


def _random_keys(dtype, n, rng, alphabet=None):
    if dtype == "f64":
        return list(rng.integers(0, len(F64_ORDER), n)) if alphabet is None else \
            [alphabet[i] for i in rng.integers(0, len(alphabet), n)]
    if alphabet is not None:
        vals = [alphabet[i] for i in rng.integers(0, len(alphabet), n)]
    else:
        vals = [int(v) for v in rng.integers(0, 2**63, n, dtype=np.uint64)]
    if dtype == "quartet":
        return [(v, (v * 7) % 3, v % 2) for v in vals]
    if dtype == "bytes100":
        return [bytes([0, v % 3, 0, 0, 0, 0, 0, 0, 0, (v * 5) % 7]) for v in vals]
    return vals


# ------------------------------------------------------ brute-force sorting
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7])
def test_sort_brute_force_distinct(oracle_mod, dtype, n):
    rng = np.random.default_rng(100 + n)
    if dtype == "f64":
        keys = list(rng.choice(len(F64_ORDER), n, replace=False))
    else:
        keys = _random_keys(dtype, n, rng)
    arr = _mk(dtype, keys)
    out = oracle_mod.sort(arr, dtype)
    good, _ = _brute_force_sorted_set(dtype, arr)
    assert len(good) == 1 or n == 0 or len(set(_pykey(dtype, arr[i]) for i in range(n))) < n
    assert tuple(_records(dtype, out)) in good


@pytest.mark.parametrize("dtype", DTYPES)
def test_sort_brute_force_alphabet_012(oracle_mod, dtype):
    """Every array over a 3-letter alphabet up to n = 5, and some at n = 6:
    the oracle's output is one of the non-decreasing permutations, and all of
    those share one key sequence."""
    alph = [0, 1, 2] if dtype != "f64" else [9, 10, 11]   # -0.0, +0.0, +min_subnormal
    cases = []
    for n in range(1, 6):
        cases += list(itertools.product(range(3), repeat=n))
    rng = np.random.default_rng(7)
    cases += [tuple(rng.integers(0, 3, 6)) for _ in range(20)]
    for c in cases:
        if dtype == "quartet":
            keys = [(0, alph[i] // 2, alph[i] % 2) for i in c]
        elif dtype == "bytes100":
            keys = [bytes([0] * 9 + [alph[i]]) for i in c]
        else:
            keys = [alph[i] for i in c]
        arr = _mk(dtype, keys)
        good, _ = _brute_force_sorted_set(dtype, arr)
        key_seqs = {tuple(_pykey(dtype, np.frombuffer(r, dtype=arr.dtype).reshape(arr.shape[1:]))
                          for r in g) for g in good}
        assert len(key_seqs) == 1
        assert tuple(_records(dtype, oracle_mod.sort(arr, dtype))) in good


@pytest.mark.parametrize("dtype", ["u64", "quartet", "bytes100"])
def test_sort_segmented_brute_force(oracle_mod, dtype):
    """Every way to cut a 6-element array into segments (and to leave a
    prefix and a suffix outside them): each segment comes out as one of its
    own non-decreasing permutations, and nothing outside the segments moves."""
    n = 6
    rng = np.random.default_rng(11)
    keys = [(int(v) % 3, int(v) % 2, 0) if dtype == "quartet" else
            (bytes([0] * 9 + [int(v) % 4]) if dtype == "bytes100" else int(v) % 5)
            for v in rng.integers(0, 60, n)]
    arr = _mk(dtype, keys, payloads=list(range(n)))
    for lo in range(0, 2):
        for hi in range(n - 1, n + 1):
            inner = hi - lo
            for cuts in itertools.product([0, 1], repeat=inner - 1):
                offs = [lo] + [lo + i + 1 for i, c in enumerate(cuts) if c] + [hi]
                out = oracle_mod.sort_segmented(arr, offs, dtype)
                assert _records(dtype, out[:lo]) == _records(dtype, arr[:lo])
                assert _records(dtype, out[hi:]) == _records(dtype, arr[hi:])
                for a, b in zip(offs[:-1], offs[1:]):
                    good, _ = _brute_force_sorted_set(dtype, arr[a:b])
                    assert tuple(_records(dtype, out[a:b])) in good


def test_sort_segmented_invariants(oracle_mod, workloads_mod):
    """Random layouts with empty and one-element segments: every segment
    holds its own elements (no element crosses a cut), in numpy's sorted
    order; one segment over everything is the full sort."""
    rng = np.random.default_rng(3)
    n = 20000
    arr = workloads_mod.generate("twodup", "u64", n, 5)
    for trial in range(5):
        cuts = np.sort(rng.integers(0, n, 40 + 30 * trial)).astype(np.uint64)
        offs = np.concatenate([[0], cuts, cuts[:3], [n]]).astype(np.uint64)
        offs.sort()
        out = oracle_mod.sort_segmented(arr, offs, "u64")
        for a, b in zip(offs[:-1].astype(int), offs[1:].astype(int)):
            assert np.array_equal(out[a:b], np.sort(arr[a:b]))
    assert np.array_equal(oracle_mod.sort_segmented(arr, [0, n], "u64"), oracle_mod.sort(arr, "u64"))
    with pytest.raises(ValueError):
        oracle_mod.sort_segmented(arr, [0, 10, 5, n], "u64")


def test_f64_total_order_listing(oracle_mod):
    """IEEE 754 totalOrder: a shuffled copy of the listing sorts back to it,
    and -0.0 precedes +0.0 as distinct bit patterns."""
    ref = np.array(F64_ORDER, dtype=np.uint64)
    rng = np.random.default_rng(3)
    for _ in range(5):
        shuf = ref[rng.permutation(ref.shape[0])]
        out = oracle_mod.sort(shuf.view(np.float64), "f64").view(np.uint64)
        assert np.array_equal(out, ref)
    a = np.array([0x0000000000000000], dtype=np.uint64).view(np.float64)
    b = np.array([0x8000000000000000], dtype=np.uint64).view(np.float64)
    assert oracle_mod.compare(b, a, "f64") == -1


def test_f64_agrees_with_numeric_order_on_ordinary_values(oracle_mod):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(5000) * 1e3
    out = oracle_mod.sort(x, "f64")
    assert np.array_equal(out, np.sort(x))


# ---------------------------------------------------- invariants at scale
@pytest.mark.parametrize("dtype", DTYPES)
def test_sort_invariants_random(oracle_mod, workloads_mod, dtype):
    """Sortedness by the Python-level key, record integrity through the
    payload index, and a permutation of the payloads."""
    n = 3000
    arr = workloads_mod.generate("rootdup" if dtype != "u64" else "uniform", dtype, n,
                                 seed=1234)
    out = oracle_mod.sort(arr, dtype)
    keys = [_pykey(dtype, out[i]) for i in range(n)] if dtype != "f64" else \
        list(out.view(np.uint64).astype(object))
    if dtype == "f64":   # rootdup values are non-negative: totalOrder = numeric
        assert np.all(np.diff(out) >= 0)
    else:
        assert all(keys[i] <= keys[i + 1] for i in range(n - 1))
    if dtype in ("pair", "quartet"):
        pay = out[:, -1].astype(np.int64)
        assert np.array_equal(np.sort(pay), np.arange(n))
        assert np.array_equal(out, arr[pay])
    elif dtype == "bytes100":
        pay = out[:, 10:18].copy().view(np.uint64).ravel().astype(np.int64)
        assert np.array_equal(np.sort(pay), np.arange(n))
        assert np.array_equal(out, arr[pay])
    else:
        assert np.array_equal(np.sort(out.view(np.uint64)), np.sort(arr.view(np.uint64))) \
            if dtype == "u64" else np.array_equal(np.sort(out), np.sort(arr))


def test_sort_u64_matches_numpy(oracle_mod, workloads_mod):
    for dist in workloads_mod.DISTRIBUTIONS:
        arr = workloads_mod.generate(dist, "u64", 20000, seed=5)
        assert np.array_equal(oracle_mod.sort(arr, "u64"), np.sort(arr))


# ---------------------------------------------------- bucket rule pins
def test_bucket_rule_hand_worked(oracle_mod):
    rows = golden_lines("bucket_rule.txt")
    sp = np.array([10, 20, 20, 30], dtype=np.uint64)
    el = np.array([int(r[0]) for r in rows], dtype=np.uint64)
    assert list(oracle_mod.classify(el, sp, "u64", False)) == [int(r[1]) for r in rows]
    assert list(oracle_mod.classify(el, sp, "u64", True)) == [int(r[2]) for r in rows]
    assert oracle_mod.num_buckets(sp, "u64", False) == 5
    assert oracle_mod.num_buckets(sp, "u64", True) == 7


@pytest.mark.parametrize("eq", [False, True])
def test_bucket_rule_properties(oracle_mod, eq):
    """Monotone in e; bucket boundaries sit exactly at the splitters; with
    equality buckets each splitter value has a bucket of its own (odd index)
    and no other value shares it."""
    rng = np.random.default_rng(21)
    for trial in range(30):
        m = int(rng.integers(1, 12))
        sp = np.sort(rng.integers(0, 40, m).astype(np.uint64))
        dom = np.arange(0, 45, dtype=np.uint64)
        b = oracle_mod.classify(dom, sp, "u64", eq)
        assert np.all(np.diff(b.astype(np.int64)) >= 0)
        K = oracle_mod.num_buckets(sp, "u64", eq)
        assert b.max() < K
        uniq = sorted(set(int(s) for s in sp))
        if not eq:
            for e, bi in zip(dom, b):
                lo = -1 if bi == 0 else int(sp[bi - 1])
                hi = 10**9 if bi == m else int(sp[bi])
                assert lo <= int(e) < hi
        else:
            assert K == 2 * len(uniq) + 1
            for e, bi in zip(dom, b):
                if int(e) in uniq:
                    assert bi % 2 == 1 and uniq[(bi - 1) // 2] == int(e)
                else:
                    assert bi % 2 == 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_bounds_agree_with_sorted_order(oracle_mod, workloads_mod, dtype):
    """Classifying the sorted array gives non-decreasing buckets that change
    exactly at the prefix-sum boundaries (two oracle routes must agree)."""
    n = 4000
    arr = workloads_mod.generate("twodup", dtype, n, seed=99)
    sp_idx = np.sort(np.random.default_rng(5).choice(n, 15, replace=False))
    srt = oracle_mod.sort(arr, dtype)
    sp = srt[sp_idx]
    for eq in (False, True):
        counts, bounds = oracle_mod.bucket_bounds(arr, sp, dtype, eq)
        assert int(counts.sum()) == n and int(bounds[-1]) == n
        assert np.array_equal(np.diff(bounds), counts)
        b = oracle_mod.classify(srt, sp, dtype, eq).astype(np.int64)
        assert np.all(np.diff(b) >= 0)
        for i in range(counts.shape[0]):
            assert np.all(b[int(bounds[i]):int(bounds[i + 1])] == i)


# ----------------------------------------------------------- tree pins
def test_tree_layout_printed_in_paper(oracle_mod):
    rows = golden_lines("tree_k8.txt")
    k = int(rows[0][0])
    s = np.array([int(x) for x in rows[1]], dtype=np.uint64)
    a = oracle_mod.tree(s, k)
    assert [int(x) for x in a] == [int(x) for x in rows[2]]


@pytest.mark.parametrize("k", [2, 4, 8, 16, 64, 256, 512])
def test_tree_first_entries_and_descent(oracle_mod, k):
    """a_1 = s_{k/2}, a_2 = s_{k/4}, a_3 = s_{3k/4}; the branchless descent
    returns #{s <= e} for every e of a small domain, also with duplicates."""
    rng = np.random.default_rng(k)
    for dup in (False, True):
        if dup:
            s = np.sort(rng.integers(0, 2 * k // 3 + 2, k - 1)).astype(np.uint64)
        else:
            s = np.sort(rng.choice(4 * k, k - 1, replace=False)).astype(np.uint64)
        a = oracle_mod.tree(s, k)
        assert int(a[0]) == int(s[k // 2 - 1])
        if k >= 4:
            assert int(a[1]) == int(s[k // 4 - 1]) and int(a[2]) == int(s[3 * k // 4 - 1])
        for e in range(0, 4 * k + 2):
            assert oracle_mod.tree_descend(a, k, e) == int(np.sum(s <= e))


# ------------------------------------------------------------ sampling
def test_splitmix64_published_values(oracle_mod, workloads_mod):
    for row in golden_lines("splitmix64.txt"):
        seed, outs = int(row[0]), [int(x) for x in row[1:]]
        assert [oracle_mod.splitmix64_at(seed, i) for i in range(len(outs))] == outs
        assert [workloads_mod.splitmix64_at(seed, i) for i in range(len(outs))] == outs


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair"])
def test_select_splitters_equidistant(oracle_mod, workloads_mod, dtype):
    """Splitters are sample[i*alpha - 1] of the sorted sample, the sample being
    drawn at floor(h_i * n / 2^64); re-derived here with the workloads module's
    own splitmix64 and numpy's sort."""
    n, k, alpha, seed = 5000, 16, 3, 77
    arr = workloads_mod.generate("uniform", dtype, n, seed=8)
    sp, eq = oracle_mod.select_splitters(arr, dtype, k, alpha, seed)
    pos = [(workloads_mod.splitmix64_at(seed, i) * n) >> 64 for i in range(alpha * k - 1)]
    sample = arr[pos]
    if dtype == "pair":
        keys = np.sort(sample[:, 0])
        got = sp[:, 0]
    else:
        keys = np.sort(sample)
        got = sp
    want = np.array([keys[i * alpha - 1] for i in range(1, k)])
    assert not eq and np.array_equal(got, want)


def test_select_splitters_duplicates_switch_on_equality(oracle_mod, workloads_mod):
    n = 4096
    ones = workloads_mod.generate("ones", "u64", n, seed=1)
    sp, eq = oracle_mod.select_splitters(ones, "u64", 256, 4, 3)
    assert eq and sp.shape[0] == 1 and int(sp[0]) == 1
    rd = workloads_mod.generate("rootdup", "u64", n, seed=1)   # 64 distinct keys
    sp, eq = oracle_mod.select_splitters(rd, "u64", 256, 4, 3)
    assert eq and np.all(np.diff(sp.astype(np.int64)) > 0) and sp.shape[0] <= 64
    assert oracle_mod.alpha_default(2**20) == 4 and oracle_mod.alpha_default(2**30) == 6


def test_select_splitters_capped_reading(oracle_mod, workloads_mod):
    """Equality buckets within the buffers (reading of Section 4, "The Case of
    Many Identical Keys", where 2u + 1 buckets can exceed the k buffers):
    re-derived from the sorted sample with numpy -- when 2u + 1 > kcap the
    splitters are every second pick, sample[2i*alpha - 1], deduplicated, with
    equality buckets on; otherwise the uncapped result -- and K <= kcap."""
    cases = 0
    for dist, n in [("rootdup", 20000), ("twodup", 4096), ("eightdup", 9000), ("uniform", 5000), ("ones", 777)]:
        arr = workloads_mod.generate(dist, "u64", n, seed=4)
        for k, alpha in [(4, 1), (16, 3), (64, 2), (256, 4)]:
            seed = 1000 + k
            pos = [(workloads_mod.splitmix64_at(seed, i) * n) >> 64 for i in range(alpha * k - 1)]
            sample = np.sort(arr[pos])
            picks = [int(sample[i * alpha - 1]) for i in range(1, k)]
            u = sorted(set(picks))
            eq_full = len(u) < k - 1
            sp, eq = oracle_mod.select_splitters(arr, "u64", k, alpha, seed, kcap=k)
            if eq_full and 2 * len(u) + 1 > k:
                half = sorted(set(int(sample[2 * i * alpha - 1]) for i in range(1, k // 2)))
                assert eq and [int(x) for x in sp] == half, (dist, k)
                cases += 1
            else:
                assert eq == eq_full and [int(x) for x in sp] == u, (dist, k)
            nb = 2 * sp.shape[0] + 1 if eq else sp.shape[0] + 1
            assert nb <= k
            sp2, eq2 = oracle_mod.select_splitters(arr, "u64", k, alpha, seed, kcap=2 * k - 1)
            assert eq2 == eq_full and [int(x) for x in sp2] == u
    assert cases >= 4       # the thinning was exercised


@pytest.mark.parametrize("dtype", ["u64", "f64"])
@pytest.mark.parametrize("dist", ["rootdup", "sorted", "reverse", "ones"])
def test_expected_sorted_range_is_a_slice(oracle_mod, workloads_mod, dtype, dist):
    """The chunked sorted arrangement (used for inputs too large for the
    host) equals slices of the counting / qsort routes, for square and
    non-square n, with chunks that split runs of equal keys."""
    for n in (1000, 4096, 65537, 100003):
        seed = 4242 + n
        whole = oracle_mod.sort(workloads_mod.generate(dist, dtype, n, seed), dtype)
        for first, count in [(0, n), (0, 1), (n - 1, 1), (17, 333), (n // 3, n // 2), (n, 0)]:
            got = oracle_mod.expected_sorted_range(dist, dtype, n, seed, first, count)
            assert np.array_equal(got.view(np.uint64), whole[first:first + count].view(np.uint64)), (n, first, count)
        parts = [oracle_mod.expected_sorted_range(dist, dtype, n, seed, f, min(999, n - f)) for f in range(0, n, 999)]
        assert np.array_equal(np.concatenate(parts).view(np.uint64), whole.view(np.uint64))
    with pytest.raises(ValueError):
        oracle_mod.expected_sorted_range(dist, dtype, 100, 1, 90, 11)


# ---------------------------------------------------------- generators
def test_generator_closed_forms(workloads_mod):
    n = 1 << 12
    g = workloads_mod.generate
    srt = g("sorted", "u64", n, 5)
    assert np.all(np.diff(srt.astype(object)) >= 0)
    assert np.array_equal(g("reverse", "u64", n, 5), srt[::-1])
    assert np.all(g("ones", "u64", n, 5) == 1) and np.all(g("ones", "f64", n, 5) == 1.0)
    m = math.isqrt(n)
    assert np.array_equal(g("rootdup", "u64", n, 5), np.arange(n, dtype=np.uint64) % m)
    i = np.arange(n, dtype=object)
    assert list(g("twodup", "u64", n, 5)) == list((i * i + n // 2) % n)
    assert list(g("eightdup", "u64", n, 5)) == list((i ** 8 + n // 2) % n)
    alm = g("almost", "u64", n, 5)
    assert np.count_nonzero(alm != srt) <= 2 * m
    assert np.array_equal(np.sort(alm), srt)
    fs = g("sorted", "f64", n, 5)
    assert np.all(np.diff(fs) >= 0) and fs[0] >= 0 and fs[-1] < 1
    ex = g("exponential", "f64", n, 5)
    assert np.all(ex >= 0) and abs(ex.mean() - 1.0) < 0.1
    assert np.array_equal(g("exponential", "u64", n, 5), ex.view(np.uint64))
    assert np.array_equal(g("twodup", "u64", 1000, 5), (np.arange(1000) ** 2 + 500) % 1000)


def test_generator_records_payload(workloads_mod):
    n = 1000
    p = workloads_mod.generate("uniform", "pair", n, 9)
    assert np.array_equal(p[:, 1], np.arange(n))
    assert np.array_equal(p[:, 0], workloads_mod.generate("uniform", "u64", n, 9))
    q = workloads_mod.generate("rootdup", "quartet", n, 9)
    assert np.array_equal(q[:, 3], np.arange(n)) and np.array_equal(q[:, 0], q[:, 1])
    b = workloads_mod.generate("rootdup", "bytes100", n, 9)
    assert np.array_equal(b[:, 10:18].copy().view(np.uint64).ravel(), np.arange(n))
    v = np.zeros(n, dtype=np.uint64)
    for j in range(2, 10):
        v = (v << np.uint64(8)) | b[:, j].astype(np.uint64)
    assert np.array_equal(v, np.arange(n, dtype=np.uint64) % math.isqrt(n))


def test_generator_range_is_a_slice(workloads_mod):
    """Chunked generation (used to upload inputs too large to hold whole on
    the host) gives exactly the slice of the whole array; AlmostSorted, whose
    swaps reach across the array, is refused in parts."""
    n = 50021
    for dist in workloads_mod.DISTRIBUTIONS:
        for dtype in workloads_mod.DTYPES:
            whole = workloads_mod.generate(dist, dtype, n, 31)
            if dist == "almost":
                with pytest.raises(ValueError):
                    workloads_mod.generate_range(dist, dtype, n, 31, 1, 10)
                assert np.array_equal(workloads_mod.generate_range(dist, dtype, n, 31, 0, n), whole)
                continue
            parts = [workloads_mod.generate_range(dist, dtype, n, 31, f, min(7001, n - f))
                     for f in range(0, n, 7001)]
            assert np.array_equal(np.concatenate(parts), whole), (dist, dtype)
    with pytest.raises(ValueError):
        workloads_mod.generate_range("uniform", "u64", n, 31, n - 5, 6)


# ------------------------------------- fast routes to the sorted output
# The full-size checks (2^30 keys) need the oracle's sorted arrangement in
# seconds; these routes are pinned here against brute force, the totalOrder
# listing, closed forms of the inputs and the qsort route.
@pytest.mark.parametrize("dtype", ["u64", "f64"])
def test_small_integers_brute_force(oracle_mod, dtype):
    """Counting sort of small integers: every array over {0, 1, 2} up to
    n = 5 and every permutation of 6 distinct values sorts to the one
    non-decreasing arrangement brute force finds."""
    def mk(vals):
        a = np.array(vals, dtype=np.uint64)
        return a if dtype == "u64" else a.astype(np.float64)
    cases = [list(c) for n in range(0, 6) for c in itertools.product(range(3), repeat=n)]
    cases += [list(p) for p in itertools.permutations([5, 0, 3, 9, 1, 7])][::37]
    for vals in cases:
        arr = mk(vals)
        got = oracle_mod.sort_small_integers(arr, dtype, 10)
        want = np.array(sorted(vals), dtype=np.uint64)
        want = want if dtype == "u64" else want.astype(np.float64)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), vals
        if len(vals) <= 5:
            good, _ = _brute_force_sorted_set(dtype, arr)
            assert tuple(_records(dtype, got)) in good and len(set(good)) == 1


@pytest.mark.parametrize("dtype", ["u64", "f64"])
@pytest.mark.parametrize("n", [2, 1000, 12345, 1 << 16])
def test_small_integers_rootdup_closed_form(oracle_mod, workloads_mod, dtype, n):
    """RootDup A[i] = i mod m, m = floor(sqrt(n)) (Section 5): the sorted
    output holds value v exactly floor((n - 1 - v) / m) + 1 times, in order."""
    m = math.isqrt(n)
    inp = workloads_mod.generate("rootdup", dtype, n, 1)
    got = oracle_mod.sort_small_integers(inp, dtype, n).view(np.uint64)
    reps = [(n - 1 - v) // m + 1 for v in range(m)]
    want = np.repeat(np.arange(m, dtype=np.uint64), reps)
    if dtype == "f64":
        want = want.astype(np.float64).view(np.uint64)
    assert sum(reps) == n
    assert np.array_equal(got, want)


def test_small_integers_refuses_other_keys(oracle_mod):
    """Keys that are not integers below vmax (a fraction, -0, NaN, a value
    at vmax) are refused and the input is left as it was."""
    for bad in ([1.0, 1.5], [0.0, -0.0], [2.0, float("nan")], [3.0, 10.0]):
        arr = np.array(bad, dtype=np.float64)
        with pytest.raises(ValueError):
            oracle_mod.sort_small_integers(arr, "f64", 10)
    with pytest.raises(ValueError):
        oracle_mod.sort_small_integers(np.array([3, 10], dtype=np.uint64), "u64", 10)


def test_total_order_np_listing(oracle_mod):
    """The numpy totalOrder route puts the special binary64 values in the
    order of the IEEE 754 totalOrder listing, from any starting order, and
    agrees with brute force on permutations of six of them."""
    listing = np.array(F64_ORDER, dtype=np.uint64)
    rng = np.random.default_rng(0)
    for _ in range(20):
        shuffled = listing[rng.permutation(listing.shape[0])].view(np.float64)
        got = oracle_mod.sort_total_order_np(shuffled, "f64").view(np.uint64)
        assert np.array_equal(got, listing)
    idx = [0, 3, len(F64_ORDER) // 2, len(F64_ORDER) - 4, len(F64_ORDER) - 1, 5]
    for perm in itertools.permutations(idx):
        arr = _mk("f64", list(perm))
        good, _ = _brute_force_sorted_set("f64", arr)
        got = oracle_mod.sort_total_order_np(arr, "f64")
        assert tuple(_records("f64", got)) in good


@pytest.mark.parametrize("dtype", ["u64", "f64"])
@pytest.mark.parametrize("dist", ["uniform", "exponential", "sorted", "reverse", "almost", "ones",
                                  "rootdup", "twodup", "eightdup"])
@pytest.mark.parametrize("n", [1, 2, 1000, (1 << 16) + 3])
def test_expected_sorted_matches_qsort(oracle_mod, workloads_mod, dtype, dist, n):
    """For every input distribution of Section 5 the fast route to the
    sorted output equals the qsort route (or_sort) bit for bit."""
    seed = workloads_mod.seed_for(1, dist, dtype)
    inp = workloads_mod.generate(dist, dtype, n, seed)
    want = oracle_mod.sort(inp, dtype)
    got = oracle_mod.expected_sorted(dist, dtype, n, seed)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
