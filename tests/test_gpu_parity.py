"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Keys are compared bit-exactly; bucket boundaries and bucket ids exactly;
records by keys exactly plus payload checks (payload = original index, so the
output must be a permutation whose every record equals the input record its
payload names).  Sizes span several tiles and blocks with ragged tails."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

DISTS = workloads.DISTRIBUTIONS
SHAPE_TAIL = {"u64": (), "f64": (), "pair": (2,), "quartet": (4,), "bytes100": (100,)}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_02257_amd as ips
    oracle.build()
    workloads.build()
    h = ips.handle(0)
    return torch, ips, h


def to_dev(torch, arr):
    flat = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
    return torch.from_numpy(flat.copy()).to("cuda:0")


def from_dev(t, like):
    return t.cpu().numpy().view(like.dtype).reshape(like.shape)


def gpu_sort(env, arr, dtype, params=None):
    torch, ips, h = env
    d = to_dev(torch, arr)
    ips.ips4o_sort(h, d, arr.shape[0], dtype, params)
    torch.cuda.synchronize()
    return from_dev(d, arr)


def keys_of(arr, dtype):
    if dtype in ("u64", "f64"):
        return arr.view(np.uint64)
    if dtype == "pair":
        return arr[:, :1]
    if dtype == "quartet":
        return arr[:, :3]
    return arr[:, :10]


def payload_of(arr, dtype):
    if dtype in ("pair", "quartet"):
        return arr[:, -1].astype(np.int64)
    return arr[:, 10:18].copy().view(np.uint64).ravel().astype(np.int64)


def same_multiset(a, b):
    """Equal as multisets of whole elements (rows compared bytewise)."""
    rb = a.dtype.itemsize * (a.shape[1] if a.ndim == 2 else 1)
    va = np.ascontiguousarray(a).view(np.dtype((np.void, rb))).ravel()
    vb = np.ascontiguousarray(b).view(np.dtype((np.void, rb))).ravel()
    return np.array_equal(np.sort(va), np.sort(vb))


def assert_sorted_like_oracle(out, inp, dtype):
    ref = oracle.sort(inp, dtype)
    assert np.array_equal(keys_of(out, dtype), keys_of(ref, dtype)), "keys differ from the oracle"
    if dtype in ("u64", "f64"):
        assert np.array_equal(out.view(np.uint64), ref.view(np.uint64))
    else:
        pay = payload_of(out, dtype)
        assert np.array_equal(np.sort(pay), np.arange(inp.shape[0]))
        assert np.array_equal(out, inp[pay]), "a record was torn or mixed"


# ------------------------------------------------------------- full sort
@pytest.mark.parametrize("dtype", ["u64", "f64"])
@pytest.mark.parametrize("dist", DISTS)
def test_sort_2pow20_all_distributions(env, dtype, dist):
    """The small configuration: 2^20 keys, k = 256, b = 2 KiB, every
    distribution, keys bit-exact against the oracle."""
    n = 1 << 20
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(0, dist, dtype))
    print(f"[gpu] sort {dtype} {dist} n={n}", flush=True)
    out = gpu_sort(env, inp, dtype, {"k": 256, "block_bytes": 2048})
    assert_sorted_like_oracle(out, inp, dtype)


@pytest.mark.parametrize("dtype,dist,params", [
    ("u64", "uniform", None), ("u64", "sorted", None), ("f64", "exponential", None),
    ("u64", "uniform", {"k": 2}), ("u64", "twodup", {"k": 2}), ("f64", "almost", {"k": 2})])
def test_sort_2pow24_second_level(env, dtype, dist, params):
    """2^24 keys: a second level whose stripes hold several virtual tiles of
    16384 keys plus a remainder; with the default k its subproblems take
    k = 8, with k = 2 on the first level they take k = 1024.  Bit-exact
    against the oracle."""
    n = 1 << 24
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(2, dist, dtype))
    print(f"[gpu] sort {dtype} {dist} n=2^24 params={params}", flush=True)
    out = gpu_sort(env, inp, dtype, params)
    assert_sorted_like_oracle(out, inp, dtype)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 255, 256, 257, 4095, 16384, 16385, 65535, 65536,
                               65537, 100003, 262147, 1000003])
def test_sort_sizes_u64(env, n):
    inp = workloads.generate("uniform", "u64", n, 1000 + n)
    print(f"[gpu] sort u64 uniform n={n}", flush=True)
    out = gpu_sort(env, inp, "u64")
    assert_sorted_like_oracle(out, inp, "u64")


@pytest.mark.parametrize("dtype", ["pair", "quartet", "bytes100"])
@pytest.mark.parametrize("dist", ["uniform", "rootdup", "sorted", "ones"])
@pytest.mark.parametrize("n", [5000, 300007])
def test_sort_records(env, dtype, dist, n):
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(2, dist, dtype))
    print(f"[gpu] sort {dtype} {dist} n={n}", flush=True)
    out = gpu_sort(env, inp, dtype)
    assert_sorted_like_oracle(out, inp, dtype)


@pytest.mark.parametrize("n", [2, 63, 64, 65, 300, 511, 512, 513])
def test_sort_tiny_bins_with_extreme_keys(env, n):
    """Bins small enough for one wave: keys equal to the padding value (the
    largest u64; the f64 whose totalOrder image is the largest) sort with
    the rest."""
    rng = np.random.default_rng(n)
    u = rng.integers(0, 2**64, n, dtype=np.uint64)
    u[rng.integers(0, n, max(1, n // 5))] = np.uint64(2**64 - 1)
    out = gpu_sort(env, u, "u64")
    assert_sorted_like_oracle(out, u, "u64")
    f = u.copy()
    f[rng.integers(0, n, max(1, n // 5))] = np.uint64(0x7FFFFFFFFFFFFFFF)   # +NaN, largest image
    f[rng.integers(0, n, max(1, n // 7))] = np.uint64(0xFFFFFFFFFFFFFFFF)   # -NaN, smallest image
    fv = f.view(np.float64)
    out = gpu_sort(env, fv, "f64")
    assert_sorted_like_oracle(out, fv, "f64")


def test_sort_f64_special_values(env):
    """Signed zeros, infinities, NaNs with payloads and subnormals sort by
    IEEE totalOrder with their bit patterns intact."""
    rng = np.random.default_rng(5)
    specials = np.array([0x0000000000000000, 0x8000000000000000, 0x7ff0000000000000,
                         0xfff0000000000000, 0x7ff8000000000000, 0xfff8000000000000,
                         0x7ff0000000000001, 0xfff0000000000123, 0x0000000000000001,
                         0x8000000000000001, 0x000fffffffffffff, 0x7fefffffffffffff],
                        dtype=np.uint64)
    n = 200003
    base = workloads.generate("uniform", "u64", n, 77)
    idx = rng.integers(0, n, 30000)
    base[idx] = specials[rng.integers(0, specials.shape[0], idx.shape[0])]
    inp = base.view(np.float64)
    out = gpu_sort(env, inp, "f64")
    assert_sorted_like_oracle(out, inp, "f64")


def test_sort_robust_to_parameters(env):
    """The same input sorts to the same keys under different bucket counts,
    block sizes, stripe and worker counts (also fewer workers than a level
    has subproblems), and with skipping disabled."""
    n = 700001
    inp = workloads.generate("twodup", "u64", n, 31)
    ref = oracle.sort(inp, "u64")
    for params in [{"k": 2}, {"k": 16}, {"k": 512}, {"k": 1024}, {"block_bytes": 512}, {"block_bytes": 8192},
                   {"stripes": 1}, {"stripes": 7}, {"workers": 4}, {"workers": 64},
                   {"flags": 1}, {"alpha_x100": 100}, {"base_cap": 1000}, {"seed": 12345},
                   # a second level of 16 subproblems sharing 2 and 25 groups of four workers
                   {"k": 16, "base_cap": 1000, "workers": 8}, {"k": 16, "base_cap": 1000, "workers": 100}]:
        print(f"[gpu] sort u64 twodup n={n} params={params}", flush=True)
        out = gpu_sort(env, inp, "u64", params)
        assert np.array_equal(out, ref), params


def test_sort_equality_buckets_thinned(env):
    """k = 1024 on an input with about 700 distinct values: the 1023 picks
    hold duplicates but more than 511 unique values, so equality buckets
    would exceed the bucket limit and every second pick is used instead."""
    rng = np.random.default_rng(5)
    n = 1 << 20
    vals = np.sort(rng.integers(0, 2**64, 700, dtype=np.uint64))
    for dtype in ("u64", "f64"):
        inp = vals[rng.integers(0, 700, n)].copy()
        if dtype == "f64":
            inp = inp.view(np.float64)
            inp = np.where(np.isnan(inp), 1.5, inp)
        ref = oracle.sort(inp, dtype)
        print(f"[gpu] sort {dtype} 700 distinct values n={n} k=1024", flush=True)
        out = gpu_sort(env, inp, dtype, {"k": 1024})
        assert np.array_equal(out.view(np.uint64), ref.view(np.uint64)), dtype


def _clustered_keys(n, seed, clusters):
    """u64 keys spread over [0, 2^62) plus clusters: (size, width) puts
    `size` keys in [c, c + width) for a random c, so that they share one
    digit range of the base case's counting sort (width 1: all equal)."""
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << 62, n, dtype=np.uint64)
    pos = rng.permutation(n)
    at = 0
    for size, width in clusters:
        c = rng.integers(0, (1 << 62) - width, dtype=np.uint64)
        keys[pos[at:at + size]] = c + rng.integers(0, width, size, dtype=np.uint64)
        at += size
    return keys


def _with_keys(dtype, n, keys, seed):
    """An input of `dtype` whose leading key word is `keys` (payload =
    index; the other key words of a quartet and the last two key bytes of a
    100-byte record are few-valued, so that equal leading words still order
    by them)."""
    rng = np.random.default_rng(seed)
    if dtype == "u64":
        return keys.copy()
    if dtype == "f64":
        return (keys >> np.uint64(2)).view(np.float64)    # positive finite values
    inp = workloads.generate("uniform", dtype, n, seed)
    if dtype in ("pair", "quartet"):
        inp[:, 0] = keys
        if dtype == "quartet":
            inp[:, 1] = rng.integers(0, 3, n, dtype=np.uint64)
            inp[:, 2] = rng.integers(0, 3, n, dtype=np.uint64)
    else:
        inp[:, 0:8] = keys.astype(">u8").view(np.uint8).reshape(n, 8)
        inp[:, 8:10] = rng.integers(0, 3, (n, 2), dtype=np.uint8)
    return inp


# base-case capacity (and its half, the small bin class) per element type
BASE_CAP = {"u64": 16384, "f64": 16384, "pair": 8192, "quartet": 4096, "bytes100": 4096}


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "quartet", "bytes100"])
@pytest.mark.parametrize("shape", ["crowded", "equal_runs", "too_crowded", "narrow", "shared_low_bits"])
@pytest.mark.parametrize("which", ["small_bin", "large_bin", "levels"])
def test_sort_crowded_digit_groups(env, dtype, shape, which):
    """Inputs whose keys crowd into a few digit ranges of the base case:
    groups of 65 to 500 close keys (ranked in group order), long runs of
    equal keys, a group too large to rank (the bin goes to the merge sort),
    keys from a range narrower than the digit count (every digit one key
    value), and few-valued keys whose low 20 bits all agree (as integer
    valued doubles do); as one small or large bin, and through distribution
    levels."""
    cap = BASE_CAP[dtype]
    n = {"small_bin": cap // 2 - 37, "large_bin": cap - 5, "levels": 300007}[which]
    width = 1 << 30
    clusters = {"crowded": [(65, width), (130, width), (257, width), (min(500, n // 8), width), (80, 2)],
                "equal_runs": [(n // 4, 1), (n // 8, 1), (300, 1)],
                "too_crowded": [(n // 3, width), (90, width)], "narrow": [], "shared_low_bits": []}[shape]
    shapes = ["crowded", "equal_runs", "too_crowded", "narrow", "shared_low_bits"]
    seed = 8000 + 10 * list(BASE_CAP).index(dtype) + shapes.index(shape)
    keys = _clustered_keys(n, seed, clusters)
    if shape == "narrow":
        keys = np.uint64(1 << 50) + np.random.default_rng(seed).integers(0, 3000, n, dtype=np.uint64)
    if shape == "shared_low_bits":
        vals = np.random.default_rng(seed).integers(0, 2500, n, dtype=np.uint64) << np.uint64(20)
        keys = vals + np.uint64(0x5A5A5)
    inp = _with_keys(dtype, n, keys, seed)
    print(f"[gpu] sort {dtype} {shape} {which} n={n}", flush=True)
    out = gpu_sort(env, inp, dtype)
    assert_sorted_like_oracle(out, inp, dtype)


# ---------------------------------------------------- one distribution step
def _splitters(inp, dtype, m, seed, dup=False):
    srt = oracle.sort(inp, dtype)
    rng = np.random.default_rng(seed)
    pos = np.sort(rng.integers(0, inp.shape[0], m))
    if dup:
        pos[1::3] = pos[0::3][:pos[1::3].shape[0]]
        pos = np.sort(pos)
    return srt[pos]


@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "quartet", "bytes100"])
@pytest.mark.parametrize("eq", [False, True])
@pytest.mark.parametrize("m,n", [(1, 1000), (15, 65537), (255, 300001), (511, 1 << 18)])
def test_distribute_parity(env, dtype, eq, m, n):
    """Boundaries equal the oracle's exactly; each bucket's range holds exactly
    the elements the oracle's bucket rule assigns to it."""
    torch, ips, h = env
    dist = "rootdup" if eq else "uniform"
    inp = workloads.generate(dist, dtype, n, 4242 + m)
    sp = _splitters(inp, dtype, m, m, dup=eq)
    counts, bounds = oracle.bucket_bounds(inp, sp, dtype, eq)
    d = to_dev(torch, inp)
    print(f"[gpu] distribute {dtype} eq={eq} m={m} n={n}", flush=True)
    gb = ips.ips4o_distribute(h, d, n, dtype, sp, eq)
    out = from_dev(d, inp)
    assert np.array_equal(gb, bounds)
    ids = oracle.classify(out, sp, dtype, eq).astype(np.int64)
    want = np.repeat(np.arange(counts.shape[0]), counts.astype(np.int64))
    assert np.array_equal(ids, want)
    assert same_multiset(out, inp)


@pytest.mark.parametrize("dtype,eq", [("u64", False), ("f64", True), ("pair", True)])
def test_distribute_device_arrays(env, dtype, eq):
    """Splitters, bounds and bucket count in device memory
    (ips4o_distribute_dev): the oracle's bounds and bucket contents."""
    torch, ips, h = env
    n, m = 200003, 63
    dist = "rootdup" if eq else "uniform"
    inp = workloads.generate(dist, dtype, n, 77)
    sp = _splitters(inp, dtype, m, m, dup=eq)
    counts, bounds = oracle.bucket_bounds(inp, sp, dtype, eq)
    d = to_dev(torch, inp)
    d_sp = to_dev(torch, sp)
    d_bounds = torch.full((2 * m + 2,), -1, dtype=torch.int64, device="cuda:0")
    d_k = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    print(f"[gpu] distribute (device arrays) {dtype} eq={eq}", flush=True)
    ips.ips4o_distribute_dev(h, d, n, dtype, d_sp, m, eq, d_bounds, d_k)
    torch.cuda.synchronize()
    K = int(d_k.item())
    assert K == counts.shape[0]
    assert np.array_equal(d_bounds[:K + 1].cpu().numpy().view(np.uint64), bounds)
    out = from_dev(d, inp)
    ids = oracle.classify(out, sp, dtype, eq).astype(np.int64)
    assert np.array_equal(ids, np.repeat(np.arange(K), counts.astype(np.int64)))
    assert same_multiset(out, inp)


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 511, 513])
def test_distribute_tiny(env, n):
    torch, ips, h = env
    inp = workloads.generate("uniform", "u64", n, 9 + n)
    sp = np.sort(inp[: min(n, 5)]).astype(np.uint64)
    for eq in (False, True):
        counts, bounds = oracle.bucket_bounds(inp, sp, "u64", eq)
        d = to_dev(torch, inp)
        gb = ips.ips4o_distribute(h, d, n, "u64", sp, eq)
        out = from_dev(d, inp)
        assert np.array_equal(gb, bounds)
        ids = oracle.classify(out, sp, "u64", eq).astype(np.int64)
        assert np.array_equal(ids, np.repeat(np.arange(counts.shape[0]), counts.astype(np.int64)))


@pytest.mark.parametrize("trial", range(6))
def test_distribute_overhang_across_empty_buckets(env, trial):
    """Runs of equal splitters (no equality buckets) leave empty buckets right
    after a large one: the large bucket's last full block spills across all
    of them into the next bucket's head, which must not be overwritten before
    that spill has been saved."""
    torch, ips, h = env
    n = 200003 + 977 * trial
    inp = workloads.generate("uniform", "u64", n, 500 + trial)
    srt = np.sort(inp)
    rng = np.random.default_rng(trial)
    picks = np.sort(rng.integers(0, n, 40))
    sp = np.repeat(srt[picks], rng.integers(1, 6, picks.shape[0]))
    counts, bounds = oracle.bucket_bounds(inp, sp, "u64", False)
    d = to_dev(torch, inp)
    gb = ips.ips4o_distribute(h, d, n, "u64", sp, False, {"workers": 256})
    out = from_dev(d, inp)
    assert np.array_equal(gb, bounds)
    ids = oracle.classify(out, sp, "u64", False).astype(np.int64)
    assert np.array_equal(ids, np.repeat(np.arange(counts.shape[0]), counts.astype(np.int64)))


def test_sort_many_small_tasks_repeated(env):
    """Deep recursion with tiny tasks (base capacity 1000), several times."""
    n = 700001
    for rep, dist in enumerate(["uniform", "twodup", "uniform", "eightdup"]):
        inp = workloads.generate(dist, "u64", n, 31 + rep)
        out = gpu_sort(env, inp, "u64", {"base_cap": 1000})
        assert np.array_equal(out, np.sort(inp)), (rep, dist)


@pytest.mark.parametrize("dist", ["uniform", "twodup", "sorted", "ones", "eightdup"])
def test_phase_invariants_checked_on_device(env, dist):
    """With the debug flag the library verifies, after classification, that
    every stripe is [full blocks | empty blocks] with single-bucket full
    blocks and exact counts, and after the permutation that every block in
    [d_i, w_i) holds bucket i; any violation makes the call fail."""
    torch, ips, h = env
    for n, k in [(70001, 256), (300001, 16), (1 << 20, 256), (1 << 20, 512)]:
        inp = workloads.generate(dist, "u64", n, 77 + n)
        out = gpu_sort(env, inp, "u64", {"k": k, "flags": 4})
        assert np.array_equal(out, np.sort(inp)), (dist, n, k)
    for m in (3, 255, 511):
        inp = workloads.generate(dist, "u64", 200003, m)
        sp = _splitters(inp, "u64", m, m, dup=(dist != "uniform"))
        d = to_dev(torch, inp)
        gb = ips.ips4o_distribute(h, d, inp.shape[0], "u64", sp, dist != "uniform", {"flags": 4})
        _, bounds = oracle.bucket_bounds(inp, sp, "u64", dist != "uniform")
        assert np.array_equal(gb, bounds)


# ---------------------------------------- last level: fused cleanup
@pytest.mark.parametrize("dtype,dist,n,params", [
    ("u64", "uniform", 1 << 22, None), ("u64", "twodup", 3000017, None), ("f64", "eightdup", 1 << 21, None),
    ("u64", "rootdup", 2000003, None), ("u64", "uniform", 1000003, {"base_cap": 1000}),
    ("u64", "exponential", 1 << 22, {"k": 16}), ("f64", "almost", 1 << 21, {"block_bytes": 256}),
    ("pair", "uniform", 600011, None), ("quartet", "rootdup", 400009, None), ("bytes100", "twodup", 200003, None)])
def test_sort_fused_cleanup(env, dtype, dist, n, params):
    """With IPS4O_FLAG_FUSE the base case cleans the buckets of the bins it
    sorts (Section 4, Implementation Details).  The default call (a cleanup
    pass per level) and the fused one both equal the oracle; the fused one
    also passes the device's phase checks, and its timed base-case pass
    counts the elements it placed while cleaning."""
    torch, ips, h = env
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(3, dist, dtype))
    base = dict(params or {})
    print(f"[gpu] fused cleanup {dtype} {dist} n={n} params={params}", flush=True)
    for flags in (0, ips.FLAG_FUSE, ips.FLAG_FUSE | 4, ips.FLAG_FUSE | ips.FLAG_TIMING):
        out = gpu_sort(env, inp, dtype, dict(base, flags=flags))
        assert_sorted_like_oracle(out, inp, dtype)
    passes = ips.ips4o_last_pass_stats(h)
    assert passes and passes[-1]["base_case"]
    s = ips.ELEM_BYTES[ips.DTYPES[dtype]]
    st = ips.ips4o_last_stats(h)
    assert passes[-1]["elements"] == st["elements_base"]
    assert passes[-1]["alg_bytes"] >= 2.0 * s * st["elements_base"]


# ------------------------------------------------------- classification
@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "quartet", "bytes100"])
@pytest.mark.parametrize("eq", [False, True])
def test_classify_parity(env, dtype, eq):
    torch, ips, h = env
    n = 100003
    inp = workloads.generate("eightdup", dtype, n, 5)
    for m in (1, 2, 7, 64, 255, 511):
        sp = _splitters(inp, dtype, m, 100 + m, dup=True)
        d = to_dev(torch, inp)
        out = torch.zeros(n, dtype=torch.int32, device="cuda:0")
        ips.ips4o_classify(h, d, n, dtype, sp, eq, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.classify(inp, sp, dtype, eq)), (m, eq)


# -------------------------------------------------------------- sampling
@pytest.mark.parametrize("dtype", ["u64", "f64", "pair", "quartet", "bytes100"])
@pytest.mark.parametrize("dist", ["uniform", "rootdup", "ones"])
def test_select_splitters_parity(env, dtype, dist):
    torch, ips, h = env
    n = 200000
    inp = workloads.generate(dist, dtype, n, 3)
    for k in (2, 16, 256):
        alpha = oracle.alpha_default(n)
        seed = 0xABCDEF + k
        # a sort's first level holds buffers for min(2k, 1024) buckets
        want, weq = oracle.select_splitters(inp, dtype, k, alpha, seed, kcap=min(2 * k, 1024))
        d = to_dev(torch, inp)
        got, geq = ips.ips4o_select_splitters(h, d, n, dtype, {"k": k, "seed": seed, "alpha_x100": 100 * alpha},
                                              like=inp)
        assert geq == weq
        assert np.array_equal(keys_of(got, dtype), keys_of(want, dtype)), (k, dist)


def test_tensor_arguments_checked(env):
    """A view that is not contiguous or a tensor shorter than n elements is
    refused with ValueError before the library is called."""
    torch, ips, h = env
    d = torch.zeros(1000, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ValueError):
        ips.ips4o_sort(h, d[::2], 500, "u64")
    with pytest.raises(ValueError):
        ips.ips4o_sort(h, d, 1001, "u64")
    with pytest.raises(ValueError):
        ips.ips4o_sort(h, d.expand(4, 1000), 4000, "u64")
    with pytest.raises(ValueError):
        ips.ips4o_sort_segmented(h, d, [0, 600, 1200], "u64")
    ips.ips4o_sort(h, d, 1000, "u64")          # the exact size is accepted
