"""Pins of the oracle's strictly in-place recursion (Section 4.6): the bucket
maxima a partition leaves in first entries, searchNextLargest by exponential
search and bisection, and the constant-space loop that sorts with them.

They are pinned to what the section and the mathematics fix: the largest
key of a bucket found by a Python maximum, the first larger key found by a
linear scan, searches that stay logarithmic in the bucket size, the sorted
arrangement (numpy's sort and brute force over permutations), and the
counts the loop must make on inputs whose course is known (a short array:
one insertion sort; one key value: one partition and nothing else)."""
import itertools
import math

import numpy as np
import pytest

from test_oracle import DTYPES, _mk, _pykey, _random_keys


def _keys(dtype, arr):
    return [_pykey(dtype, arr[i]) for i in range(arr.shape[0])]


def _marked_partition(dtype, rng, n, nbuckets, alphabet=None):
    """(array, bucket starts): keys sorted, cut into buckets between unequal
    keys, each bucket shuffled and its largest key moved to the front, built
    with Python's max (independent of the oracle's C code)."""
    keys = sorted(_random_keys(dtype, n, rng, alphabet), key=lambda k: k)
    arr = _mk(dtype, keys)
    kk = _keys(dtype, arr)
    order = sorted(range(n), key=lambda i: kk[i])
    arr = arr[order]
    kk = [kk[i] for i in order]
    changes = [i for i in range(1, n) if kk[i] != kk[i - 1]]
    cuts = sorted(rng.choice(changes, size=min(nbuckets - 1, len(changes)), replace=False)) if changes else []
    starts = [0] + [int(c) for c in cuts]
    bounds = starts + [n]
    out = arr.copy()
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        perm = lo + rng.permutation(hi - lo)
        out[lo:hi] = arr[perm]
        seg = _keys(dtype, out[lo:hi])
        top = max(range(hi - lo), key=lambda i: (seg[i], -i))    # first occurrence of the maximum
        tmp = out[lo].copy()
        out[lo] = out[lo + top]
        out[lo + top] = tmp
    return out, starts


def _same(a, b):
    return a.shape == b.shape and a.tobytes() == b.tobytes()


def _first_larger_linear(kk, i, hi):
    for j in range(i + 1, hi):
        if kk[j] > kk[i]:
            return j
    return hi


# ------------------------------------------------------------ marking
@pytest.mark.parametrize("dtype", DTYPES)
def test_mark_moves_first_maximum_to_front(oracle_mod, dtype):
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(0, 300))
        alphabet = None if trial % 2 else [3, 1, 4, 1, 5]
        arr = _mk(dtype, _random_keys(dtype, n, rng, alphabet))
        cuts = sorted(int(c) for c in rng.integers(0, n + 1, int(rng.integers(0, 9))))
        bounds = [0] + cuts + [n]
        out = oracle_mod.mark_bucket_max(arr, bounds, dtype)
        kin = _keys(dtype, arr)
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            expect = arr[lo:hi].copy()
            if hi - lo >= 2:
                top = max(range(hi - lo), key=lambda i: (kin[lo + i], -i))
                first = expect[0].copy()
                expect[0] = expect[top]
                expect[top] = first
            assert _same(out[lo:hi], expect), (trial, lo, hi)


def test_mark_rejects_decreasing_bounds(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.mark_bucket_max(np.arange(10, dtype=np.uint64), [0, 6, 4, 10], "u64")


# ------------------------------------------------------------ searchNextLargest
@pytest.mark.parametrize("dtype", DTYPES)
def test_search_finds_next_bucket_start(oracle_mod, dtype):
    rng = np.random.default_rng(5)
    for trial in range(8):
        n = int(rng.integers(1, 400))
        alphabet = None if trial % 2 else list(range(12))
        arr, starts = _marked_partition(dtype, rng, n, int(rng.integers(1, 20)), alphabet)
        kk = _keys(dtype, arr)
        ends = starts[1:] + [n]
        for s, e in zip(starts, ends):
            j, probes = oracle_mod.search_next_largest(arr, s, dtype)
            assert j == e == _first_larger_linear(kk, s, n), (trial, s)
            # exponential search then bisection: O(log) of the distance
            assert probes <= 2 * math.ceil(math.log2(e - s + 1)) + 2, (trial, s, e, probes)


def test_search_every_size_and_end(oracle_mod):
    """A bucket of m keys at most 5 (its maximum 5 first) followed by larger
    keys: the answer is m for every m, also when nothing larger follows."""
    rng = np.random.default_rng(2)
    for m in range(1, 200):
        body = list(rng.integers(0, 6, m - 1))
        for tail in (0, 1, 7):
            a = np.array([5] + body + list(range(6, 6 + tail)), dtype=np.uint64)
            j, _ = oracle_mod.search_next_largest(a, 0, "u64")
            assert j == m, (m, tail)
            if tail:
                j, _ = oracle_mod.search_next_largest(a, 0, "u64", hi=m + 1)
                assert j == m
            j, _ = oracle_mod.search_next_largest(a, 0, "u64", hi=m)
            assert j == m      # no larger key inside the bound: the bound


def test_search_equal_keys_are_not_larger(oracle_mod):
    a = np.array([4, 4, 4, 4, 9], dtype=np.uint64)
    assert oracle_mod.search_next_largest(a, 0, "u64")[0] == 4
    f = np.array([0.0, -0.0, 0.0, 1.0], dtype=np.float64)      # totalOrder: -0 < +0
    assert oracle_mod.search_next_largest(f, 1, "f64")[0] == 2
    assert oracle_mod.search_next_largest(f, 0, "f64")[0] == 3


# ------------------------------------------------------------ the loop
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [3, 4, 16])
def test_sort_strict_brute_force(oracle_mod, dtype, k):
    """Every arrangement of six elements with repeated keys, n0 = 2 so that
    the loop partitions, searches and skips constant ranges."""
    rng = np.random.default_rng(k)
    keys = _random_keys(dtype, 6, rng, [0, 0, 1, 2, 2, 2])
    base = _mk(dtype, keys)
    n = base.shape[0]
    want = sorted(_keys(dtype, base))
    seen = set()
    for perm in itertools.permutations(range(n)):
        if perm in seen:
            continue
        seen.add(perm)
        arr = base[list(perm)]
        out, _ = oracle_mod.sort_strict(arr, dtype, k=k, alpha=1, n0=2, seed=3)
        assert _keys(dtype, out) == want, perm
        assert sorted(x.tobytes() for x in out) == sorted(x.tobytes() for x in arr)


@pytest.mark.parametrize("dist", ["uniform", "exponential", "sorted", "reverse", "almost", "ones", "rootdup",
                                  "twodup", "eightdup"])
@pytest.mark.parametrize("dtype", ["u64", "f64"])
def test_sort_strict_matches_numpy(oracle_mod, workloads_mod, dist, dtype):
    for n, k, n0 in ((3000, 16, 16), (4097, 4, 64), (20000, 64, 32)):
        a = workloads_mod.generate(dist, dtype, n, 17)
        out, st = oracle_mod.sort_strict(a, dtype, k=k, alpha=2, n0=n0, seed=9)
        want = oracle_mod.sort_total_order_np(a, dtype)
        assert np.array_equal(out.view(np.uint64), want.view(np.uint64)), (n, k, n0)
        assert st["partitions"] >= 1


@pytest.mark.parametrize("dtype", ["pair", "quartet", "bytes100"])
def test_sort_strict_records(oracle_mod, workloads_mod, dtype):
    a = workloads_mod.generate("twodup", dtype, 3000, 4)
    out, _ = oracle_mod.sort_strict(a, dtype, k=16, alpha=2, n0=16, seed=1)
    ref = oracle_mod.sort(a, dtype)
    assert _keys(dtype, out) == _keys(dtype, ref)
    assert sorted(x.tobytes() for x in out) == sorted(x.tobytes() for x in a)


def test_sort_strict_counts(oracle_mod, workloads_mod):
    a = workloads_mod.generate("uniform", "u64", 100, 1)
    _, st = oracle_mod.sort_strict(a, "u64", k=16, alpha=2, n0=101, seed=1)
    assert st == {"partitions": 0, "small_sorts": 1, "constant": 0, "probes": 0}
    ones = np.ones(5000, dtype=np.uint64)
    _, st = oracle_mod.sort_strict(ones, "u64", k=16, alpha=2, n0=16, seed=1)
    assert st == {"partitions": 1, "small_sorts": 0, "constant": 1, "probes": 0}
    # distinct keys: no range is constant; every insertion sort follows a
    # search, and every search is logarithmic
    a = np.random.default_rng(3).permutation(20000).astype(np.uint64)
    _, st = oracle_mod.sort_strict(a, "u64", k=16, alpha=2, n0=16, seed=1)
    assert st["constant"] == 0
    searches = st["partitions"] + st["small_sorts"] - 1
    assert st["probes"] <= searches * (2 * math.ceil(math.log2(20000)) + 2)


def test_sort_strict_rejects_two_way(oracle_mod):
    """With k = 2 one splitter can leave a range of distinct keys in one
    bucket, so the constant-range reading needs k >= 3."""
    with pytest.raises(ValueError):
        oracle_mod.sort_strict(np.arange(10, dtype=np.uint64), "u64", k=2)


@pytest.mark.parametrize("k", [3, 4, 8])
def test_partition_of_distinct_keys_makes_two_buckets(oracle_mod, k):
    """The reading the loop's termination rests on: with k >= 3 buckets, a
    range holding two or more distinct keys never falls into a single
    bucket (splitters drawn from the range, duplicates switching equality
    buckets on).  Brute force over small ranges of few key values, every
    oversampling factor up to 3 and many sample streams."""
    rng = np.random.default_rng(40 + k)
    for trial in range(400):
        n = int(rng.integers(2, 24))
        a = rng.integers(0, int(rng.integers(2, 5)), n).astype(np.uint64)
        if np.unique(a).shape[0] < 2:
            continue
        alpha = int(rng.integers(1, 4))
        sp, eq = oracle_mod.select_splitters(a, "u64", k, alpha, int(rng.integers(0, 2**63)))
        counts, _ = oracle_mod.bucket_bounds(a, sp, "u64", eq)
        assert int((counts > 0).sum()) >= 2, (a.tolist(), sp.tolist(), eq)


def test_two_way_partition_can_leave_one_bucket(oracle_mod):
    """With k = 2 (one splitter) the same range can stay in one bucket,
    which is why the constant-range reading needs k >= 3."""
    a = np.array([1, 5, 5, 5], dtype=np.uint64)
    found = False
    for seed in range(200):
        sp, eq = oracle_mod.select_splitters(a, "u64", 2, 1, seed)
        counts, _ = oracle_mod.bucket_bounds(a, sp, "u64", eq)
        found |= int((counts > 0).sum()) == 1
    assert found
