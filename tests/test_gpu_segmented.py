"""Parity of the segmented sort (ips4o_sort_segmented, through the C ABI)
with the CPU oracle: every segment sorted on its own, keys bit-exact,
records checked by payload (payload = original index), elements outside the
segments untouched."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import env, from_dev, keys_of, payload_of, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

BASE_CAP = {"u64": 16384, "f64": 16384, "pair": 8192, "quartet": 4096, "bytes100": 4096}


def gpu_sort_segmented(env, arr, offsets, dtype, params=None):
    torch, ips, h = env
    d = to_dev(torch, arr)
    ips.ips4o_sort_segmented(h, d, offsets, dtype, params)
    torch.cuda.synchronize()
    return from_dev(d, arr)


def assert_segments_like_oracle(out, inp, offsets, dtype):
    ref = oracle.sort_segmented(inp, offsets, dtype)
    assert np.array_equal(keys_of(out, dtype), keys_of(ref, dtype)), "keys differ from the oracle"
    if dtype in ("u64", "f64"):
        assert np.array_equal(out.view(np.uint64), ref.view(np.uint64))
        return
    pay = payload_of(out, dtype)
    assert np.array_equal(out, inp[pay]), "a record was torn or mixed"
    n = inp.shape[0]
    lo, hi = int(offsets[0]), int(offsets[-1])
    assert np.array_equal(pay[:lo], np.arange(lo)) and np.array_equal(pay[hi:], np.arange(hi, n))
    for a, b in zip(np.asarray(offsets[:-1], dtype=np.int64), np.asarray(offsets[1:], dtype=np.int64)):
        assert np.array_equal(np.sort(pay[a:b]), np.arange(a, b)), "an element left its segment"


def _layout(sizes, lead=0, trail=0):
    offs = np.concatenate([[lead], lead + np.cumsum(sizes)]).astype(np.uint64)
    return offs, int(offs[-1]) + trail


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "quartet", "bytes100"])
@pytest.mark.parametrize("dist", ["uniform", "twodup"])
def test_segmented_mixed_sizes(env, dtype, dist):
    """Empty, one-element, tiny, base-case-sized (both bin classes, at and
    around the capacity) and multi-level segments side by side, in random
    order, between a prefix and a suffix that must stay as they are."""
    cap = BASE_CAP[dtype]
    sizes = [0, 1, 2, 17, 500, cap // 2, cap // 2 + 1, cap - 1, cap, cap + 1, 3 * cap + 7, 40 * cap + 3, 0, 5]
    rng = np.random.default_rng(len(dtype) + len(dist))
    sizes = list(rng.permutation(sizes))
    offs, n = _layout(sizes, lead=13, trail=29)
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(3, dist, dtype))
    print(f"[gpu] segmented {dtype} {dist} n={n} segments={len(sizes)}", flush=True)
    out = gpu_sort_segmented(env, inp, offs, dtype)
    assert_segments_like_oracle(out, inp, offs, dtype)


@pytest.mark.parametrize("dtype", ["u64", "pair"])
def test_segmented_many_small(env, dtype):
    """Thousands of small segments of uniform keys: base-case bins must not
    merge neighbouring segments (their key ranges overlap)."""
    rng = np.random.default_rng(21)
    sizes = rng.integers(0, 3000, 3000)
    offs, n = _layout(sizes)
    inp = workloads.generate("uniform", dtype, n, 77)
    print(f"[gpu] segmented {dtype} many small n={n}", flush=True)
    out = gpu_sort_segmented(env, inp, offs, dtype)
    assert_segments_like_oracle(out, inp, offs, dtype)


def test_segmented_equal_large_neighbours(env):
    """Equal-sized multi-level segments with identical key distributions:
    their buckets at every level interleave in key order but must stay in
    their own segment."""
    sizes = [200003] * 6
    offs, n = _layout(sizes)
    one = workloads.generate("uniform", "u64", sizes[0], 99)
    inp = np.concatenate([np.random.default_rng(i).permutation(one) for i in range(6)])
    print(f"[gpu] segmented u64 equal neighbours n={n}", flush=True)
    out = gpu_sort_segmented(env, inp, offs, "u64")
    assert_segments_like_oracle(out, inp, offs, "u64")


def test_segmented_log_uniform_sizes_and_params(env):
    """Segment sizes 2^U[4, 17.6] (the batched workload's shape) with three
    distributions mixed, under the default and a few other parameters."""
    rng = np.random.default_rng(5)
    sizes = np.floor(2.0 ** rng.uniform(4, 17.63, 400)).astype(np.int64)
    offs, n = _layout(sizes)
    parts = []
    for i, m in enumerate(sizes):
        dist = ["uniform", "twodup", "sorted"][i % 3]
        parts.append(workloads.generate(dist, "u64", int(m), 1000 + i))
    inp = np.concatenate(parts)
    for params in [None, {"k": 16}, {"block_bytes": 512}, {"base_cap": 1000}, {"workers": 64}]:
        print(f"[gpu] segmented u64 log-uniform n={n} params={params}", flush=True)
        out = gpu_sort_segmented(env, inp, offs, "u64", params)
        assert_segments_like_oracle(out, inp, offs, "u64")


def test_segmented_matches_plain_sort_for_one_segment(env):
    torch, ips, h = env
    n = 1 << 20
    inp = workloads.generate("exponential", "f64", n, 3)
    out = gpu_sort_segmented(env, inp, [0, n], "f64")
    assert np.array_equal(out.view(np.uint64), oracle.sort(inp, "f64").view(np.uint64))


def test_segmented_rejects_decreasing_offsets(env):
    torch, ips, h = env
    d = to_dev(torch, np.zeros(100, dtype=np.uint64))
    with pytest.raises(Exception):
        ips.ips4o_sort_segmented(h, d, [0, 50, 40, 100], "u64")


@pytest.mark.parametrize("dtype", ["u64", "pair"])
def test_segmented_device_offsets(env, dtype):
    """The offset table in device memory (ips4o_sort_segmented_dev), written
    by the caller's stream just before the call: the same result as the
    oracle's per-segment sort."""
    torch, ips, h = env
    cap = BASE_CAP[dtype]
    rng = np.random.default_rng(11)
    sizes = list(rng.permutation([0, 1, 3, 900, cap, cap + 1, 5 * cap + 3, 17, 0]))
    offs, n = _layout(sizes, lead=5, trail=7)
    inp = workloads.generate("uniform", dtype, n, workloads.seed_for(3, "uniform", dtype) + 1)
    d = to_dev(torch, inp)
    d_offs = torch.zeros(len(offs), dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream()
    d_offs.copy_(torch.from_numpy(offs.view(np.int64)), non_blocking=False)
    print(f"[gpu] segmented (device offsets) {dtype} n={n}", flush=True)
    ips.ips4o_sort_segmented_dev(h, d, d_offs, len(sizes), dtype, None, stream)
    torch.cuda.synchronize()
    assert_segments_like_oracle(from_dev(d, inp), inp, offs, dtype)


def _small_layout(dtype, nseg, seed):
    cap = BASE_CAP[dtype]
    rng = np.random.default_rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(0, np.log2(cap), nseg)).astype(np.int64)
    sizes[:6] = [0, 1, 2, cap // 2, cap // 2 + 1, cap]       # every size class and its edges
    rng.shuffle(sizes)
    return _layout(list(sizes), lead=3, trail=4)


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "bytes100"])
def test_segmented_small_device_planned(env, dtype):
    """ips4o_sort_segmented_small: bins made on the device from the device
    offsets, every segment sorted on its own like the oracle's."""
    torch, ips, h = env
    offs, n = _small_layout(dtype, 3000 if dtype in ("u64", "f64") else 600, 5)
    inp = workloads.generate("twodup", dtype, n, workloads.seed_for(3, "twodup", dtype) + 2)
    d = to_dev(torch, inp)
    d_offs = torch.from_numpy(offs.view(np.int64).copy()).to("cuda:0")
    stream = torch.cuda.current_stream()
    print(f"[gpu] segmented small {dtype} n={n} segments={len(offs) - 1}", flush=True)
    ips.ips4o_sort_segmented_small(h, d, d_offs, len(offs) - 1, dtype, stream)
    ips.ips4o_sync(h, stream)
    assert_segments_like_oracle(from_dev(d, inp), inp, offs, dtype)


def test_segmented_small_graph_replays(env):
    """The small-segment sort captured once in a HIP graph (torch.cuda.CUDAGraph)
    and replayed several times, the input restored and the result checked
    against the oracle between replays (eager work in between)."""
    torch, ips, h = env
    offs, n = _small_layout("u64", 5000, 9)
    inp = workloads.generate("uniform", "u64", n, 31)
    pristine = to_dev(torch, inp)
    d = pristine.clone()
    d_offs = torch.from_numpy(offs.view(np.int64).copy()).to("cuda:0")
    want = oracle.sort_segmented(inp, offs, "u64")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ips.ips4o_sort_segmented_small(h, d, d_offs, len(offs) - 1, "u64", s)   # sizes the bin lists
    s.synchronize()
    d.copy_(pristine)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print(f"[gpu] capture small-segment sort, {len(offs) - 1} segments", flush=True)
    with torch.cuda.graph(g, stream=s):
        ips.ips4o_sort_segmented_small(h, d, d_offs, len(offs) - 1, "u64", s)
    for rep in range(3):
        d.copy_(pristine)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = d.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want.view(np.uint64)), f"replay {rep}"
    ips.ips4o_sync(h, None)


def test_segmented_small_oversize_reported(env):
    torch, ips, h = env
    cap = BASE_CAP["u64"]
    offs = np.array([0, 100, 100 + cap + 1, 200 + cap + 1], dtype=np.uint64)
    inp = workloads.generate("uniform", "u64", int(offs[-1]), 3)
    d = to_dev(torch, inp)
    d_offs = torch.from_numpy(offs.view(np.int64).copy()).to("cuda:0")
    stream = torch.cuda.current_stream()
    ips.ips4o_sort_segmented_small(h, d, d_offs, 3, "u64", stream)
    with pytest.raises(ips.Ips4oError) as e:
        ips.ips4o_sync(h, stream)
    assert e.value.status == -5 and ips.ips4o_last_stats(h)["fault_bits"] & 128
    out = from_dev(d, inp).view(np.uint64)
    src = inp.view(np.uint64)
    assert np.array_equal(out[:100], np.sort(src[:100]))                     # the others are sorted
    assert np.array_equal(out[100 + cap + 1:], np.sort(src[100 + cap + 1:]))
    assert np.array_equal(out[100:100 + cap + 1], src[100:100 + cap + 1])    # the oversized one is untouched
