"""Parity of the strictly in-place recursion (Section 4.6) on the GPU with
the CPU oracle, through the C ABI: the bucket-maximum marking (bytes
exact), searchNextLargest (positions exact), and sorts whose levels hand
over through those marks (IPS4O_FLAG_STRICT; keys bit-exact, records by
keys plus the payload-is-index check)."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import assert_sorted_like_oracle, env, from_dev, gpu_sort, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

DTYPES = ["u64", "f64", "pair", "quartet", "bytes100"]


def _bounds_dev(torch, bounds):
    return torch.from_numpy(np.ascontiguousarray(bounds, dtype=np.uint64).view(np.int64)).to("cuda:0")


def _marked_partition(dtype, n, k, seed):
    """A partition of a seeded input by the oracle's splitters, bucket order
    kept from the input, bucket maxima marked by the oracle: (array, bounds)."""
    inp = workloads.generate("twodup" if seed % 2 else "uniform", dtype, n, seed)
    sp, eq = oracle.select_splitters(inp, dtype, k, 2, seed)
    ids = oracle.classify(inp, sp, dtype, eq)
    _, bounds = oracle.bucket_bounds(inp, sp, dtype, eq)
    part = inp[np.argsort(ids, kind="stable")]
    return oracle.mark_bucket_max(part, bounds, dtype), bounds


@pytest.mark.parametrize("dtype", DTYPES)
def test_mark_bucket_max_parity(env, dtype):
    """Random buckets over a seeded input with repeated keys: empty ones, one
    element, and buckets long enough for every thread of a workgroup to see
    several tiles; bytes equal the oracle's."""
    torch, ips, h = env
    rng = np.random.default_rng(7)
    for n in (0, 1, 1000, 200003):
        inp = workloads.generate("eightdup", dtype, n, 31 + n)
        cuts = np.sort(rng.integers(0, n + 1, 40)) if n else np.zeros(0, dtype=np.int64)
        bounds = np.concatenate([[0], cuts, [n], [n]]).astype(np.uint64)
        print(f"[gpu] mark {dtype} n={n} buckets={bounds.shape[0] - 1}", flush=True)
        d = to_dev(torch, inp)
        ips.ips4o_mark_bucket_max(h, d, n, dtype, _bounds_dev(torch, bounds), bounds.shape[0] - 1)
        out = from_dev(d, inp)
        want = oracle.mark_bucket_max(inp, bounds, dtype)
        assert out.tobytes() == want.tobytes()


def test_mark_bucket_max_rejects_bounds_beyond_the_array(env):
    """Bounds past n are skipped by the kernel and reported (fault bit 256);
    the data is untouched."""
    torch, ips, h = env
    inp = workloads.generate("uniform", "u64", 5000, 3)
    d = to_dev(torch, inp)
    with pytest.raises(ips.Ips4oError):
        ips.ips4o_mark_bucket_max(h, d, 5000, "u64", _bounds_dev(torch, [0, 100, 6000]), 2)
    assert ips.ips4o_last_stats(h)["fault_bits"] & 256
    out = from_dev(d, inp)
    want = oracle.mark_bucket_max(inp, [0, 100], "u64")
    assert out.tobytes() == want.tobytes()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,k", [(3001, 4), (100003, 64), (1 << 20, 256)])
def test_search_next_largest_parity(env, dtype, n, k):
    """From every bucket's first entry of a marked partition the search
    finds the next bucket's first entry (the oracle's exponential search and
    bisection, and the partition's own bounds); positions at or past n give n."""
    torch, ips, h = env
    arr, bounds = _marked_partition(dtype, n, k, n + k)
    starts = np.unique(bounds[:-1][bounds[:-1] < bounds[1:]]).astype(np.uint64)
    nxt = np.array([b for b in bounds[1:] if b > 0], dtype=np.uint64)
    nxt = np.unique(nxt)
    queries = np.concatenate([starts, [n, n + 5]]).astype(np.uint64)
    print(f"[gpu] search {dtype} n={n} k={k} queries={queries.shape[0]}", flush=True)
    d = to_dev(torch, arr)
    dq = _bounds_dev(torch, queries)
    do = torch.zeros(queries.shape[0], dtype=torch.int64, device="cuda:0")
    ips.ips4o_search_next_largest(h, d, n, dtype, dq, queries.shape[0], do)
    got = do.cpu().numpy().view(np.uint64)
    # the partition's bounds: each non-empty bucket ends where the next starts
    assert np.array_equal(got[:starts.shape[0]], nxt)
    assert np.all(got[starts.shape[0]:] == n)
    # the oracle's search on a sample of the starts
    for q in starts[:: max(1, starts.shape[0] // 64)]:
        assert int(got[np.searchsorted(starts, q)]) == oracle.search_next_largest(arr, int(q), dtype)[0]


STRICT_CASES = [
    ("u64", "uniform", 1 << 22, None), ("u64", "twodup", 3000017, None), ("u64", "ones", 1000003, None),
    ("u64", "rootdup", 2000003, None), ("u64", "sorted", 1 << 21, None), ("u64", "uniform", 1000003, {"base_cap": 1000}),
    ("f64", "exponential", 1 << 21, {"k": 16}), ("f64", "eightdup", 1 << 21, None), ("f64", "almost", 1000003, None),
    ("pair", "uniform", 600011, None), ("quartet", "rootdup", 400009, None), ("bytes100", "twodup", 200003, None),
]


@pytest.mark.parametrize("dtype,dist,n,params", STRICT_CASES)
def test_sort_strict(env, dtype, dist, n, params):
    """Sorts whose levels are planned from the buckets found by the walk over
    the marks equal the oracle; the timed call's mark pass is accounted."""
    torch, ips, h = env
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(3, dist, dtype))
    base = dict(params or {})
    print(f"[gpu] strict sort {dtype} {dist} n={n} params={params}", flush=True)
    for flags in (ips.FLAG_STRICT, ips.FLAG_STRICT | 4, ips.FLAG_STRICT | ips.FLAG_TIMING):
        out = gpu_sort(env, inp, dtype, dict(base, flags=flags))
        assert_sorted_like_oracle(out, inp, dtype)
    st = ips.ips4o_last_stats(h)
    ks = ips.ips4o_last_kernel_stats(h)
    if st["levels"]:
        s = ips.ELEM_BYTES[ips.DTYPES[dtype]]
        assert ks["mark"]["launches"] == st["levels"]
        assert ks["mark"]["alg_bytes"] == s * st["elements_distributed"]


def test_sort_strict_matches_default_levels(env):
    """On distinct keys no bucket is an equality bucket, so the strict
    hand-off plans the same levels as the default one."""
    torch, ips, h = env
    n = 1 << 23
    inp = workloads.generate("uniform", "u64", n, 99)
    gpu_sort(env, inp, "u64", None)
    ref = ips.ips4o_last_stats(h)
    out = gpu_sort(env, inp, "u64", {"flags": ips.FLAG_STRICT})
    st = ips.ips4o_last_stats(h)
    assert np.array_equal(out, np.sort(inp))
    assert st["levels"] == ref["levels"]
    assert st["elements_distributed"] == ref["elements_distributed"]
    assert st["elements_base"] == ref["elements_base"]


def test_sort_strict_needs_four_buckets(env):
    torch, ips, h = env
    d = torch.zeros(1 << 16, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ips.Ips4oError):
        ips.ips4o_sort(h, d, 1 << 16, "u64", {"k": 2, "flags": ips.FLAG_STRICT})


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair"])
@pytest.mark.parametrize("dist", ["uniform", "eightdup"])
def test_sort_segmented_strict(env, dtype, dist):
    """A segmented sort with the strictly in-place hand-off: every segment
    above the base-case capacity is a subproblem of the top level, and its
    buckets are found by walking the marks inside the segment only."""
    from test_gpu_segmented import BASE_CAP, _layout, assert_segments_like_oracle, gpu_sort_segmented
    cap = BASE_CAP[dtype]
    sizes = [0, 1, 17, cap, cap + 1, 3 * cap + 7, 40 * cap + 3, 2, 9 * cap, 0]
    sizes = list(np.random.default_rng(len(dtype) + len(dist)).permutation(sizes))
    offs, n = _layout(sizes, lead=13, trail=29)
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(3, dist, dtype))
    torch, ips, h = env
    print(f"[gpu] strict segmented {dtype} {dist} n={n} segments={len(sizes)}", flush=True)
    out = gpu_sort_segmented(env, inp, offs, dtype, {"flags": ips.FLAG_STRICT})
    assert_segments_like_oracle(out, inp, offs, dtype)


@pytest.mark.parametrize("dtype,dist,n", [("u64", "eightdup", 1 << 22), ("u64", "rootdup", 1 << 22),
                                          ("f64", "eightdup", 3000017), ("pair", "rootdup", 1 << 21)])
def test_sort_strict_skips_one_key_buckets(env, dtype, dist, n):
    """The sort's marking also puts each bucket's smallest key last, so the
    walk recognises a bucket above the base-case capacity that holds one key
    by its two ends: equality buckets are not partitioned again, and the
    strict hand-off distributes exactly the elements the default one does."""
    torch, ips, h = env
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(3, dist, dtype))
    print(f"[gpu] strict one-key buckets {dtype} {dist} n={n}", flush=True)
    gpu_sort(env, inp, dtype, None)
    ref = ips.ips4o_last_stats(h)
    out = gpu_sort(env, inp, dtype, {"flags": ips.FLAG_STRICT})
    st = ips.ips4o_last_stats(h)
    assert_sorted_like_oracle(out, inp, dtype)
    assert st["levels"] == ref["levels"]
    assert st["elements_distributed"] == ref["elements_distributed"]
