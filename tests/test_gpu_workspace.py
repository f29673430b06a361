"""Device workspace against its bound (Theorem 2: the extra space of the
method is O(k b) per thread, independent of n for a fixed thread count).

A fresh handle sorts one input; afterwards the workspace it holds
(ips4o_workspace_bytes) must not exceed what ips4o_workspace_size promised
before the call.  At the 2^30-key configuration the stripe buffers stay
within n/8 elements by construction, and the per-level descriptors and
bucket state add well under 1 % of the data, so the handle holds at most
0.135 n s there (the whole input is 8 GiB)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_02257_amd as ips
    workloads.build()
    return torch, ips


def _upload(torch, arr):
    flat = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
    return torch.from_numpy(flat.copy()).to("cuda:0")


@pytest.mark.parametrize("dtype,dist,log2n", [("u64", "uniform", 20), ("u64", "twodup", 24),
                                              ("f64", "eightdup", 24), ("u64", "ones", 22),
                                              ("pair", "rootdup", 22), ("quartet", "uniform", 21),
                                              ("bytes100", "uniform", 20)])
def test_sort_within_bound(env, dtype, dist, log2n):
    torch, ips = env
    n = 1 << log2n
    bound = ips.ips4o_workspace_size(dtype, n)
    inp = workloads.generate(dist, dtype, n, workloads.seed_for(2, dist, dtype))
    d = _upload(torch, inp)
    h = ips.ips4o_create(0)
    try:
        print(f"[gpu] workspace {dtype} {dist} n=2^{log2n}", flush=True)
        ips.ips4o_sort(h, d, n, dtype)
        torch.cuda.synchronize()
        held = ips.ips4o_workspace_bytes(h)
    finally:
        ips.ips4o_destroy(h)
    assert held <= bound, (held, bound)


def test_segmented_and_distribute_within_bound(env):
    torch, ips = env
    rng = np.random.default_rng(5)
    sizes = np.floor(2.0 ** rng.uniform(4, 20, 300)).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    inp = workloads.generate("uniform", "u64", n, 99)
    d = _upload(torch, inp)
    h = ips.ips4o_create(0)
    try:
        print(f"[gpu] workspace segmented n={n}", flush=True)
        ips.ips4o_sort_segmented(h, d, offs, "u64")
        torch.cuda.synchronize()
        assert ips.ips4o_workspace_bytes(h) <= ips.ips4o_workspace_size("u64", n)
    finally:
        ips.ips4o_destroy(h)
    m = 1 << 22
    inp = workloads.generate("uniform", "u64", m, 7)
    spl = np.sort(inp[rng.integers(0, m, 511)])
    d = _upload(torch, inp)
    h = ips.ips4o_create(0)
    try:
        print(f"[gpu] workspace distribute n={m}", flush=True)
        ips.ips4o_distribute(h, d, m, "u64", spl, True)
        torch.cuda.synchronize()
        assert ips.ips4o_workspace_bytes(h) <= ips.ips4o_workspace_size("u64", m)
    finally:
        ips.ips4o_destroy(h)


def test_sort_2pow30_workspace(env):
    """The 2^30 u64 Uniform sort on a fresh handle: within the query's bound
    and within n*s/8 (stripe buffers) + 1 % (descriptors, bucket state, bin
    list, counters) of the 8 GiB input; the output is checked against the
    oracle's sorted arrangement."""
    torch, ips = env
    n = 1 << 30
    bound = ips.ips4o_workspace_size("u64", n)
    seed = workloads.seed_for(1, "uniform", "u64")
    inp = workloads.generate("uniform", "u64", n, seed)
    d = torch.from_numpy(inp.view(np.int64)).to("cuda:0")
    h = ips.ips4o_create(0)
    try:
        print("[gpu] workspace u64 uniform n=2^30", flush=True)
        ips.ips4o_sort(h, d, n, "u64")
        torch.cuda.synchronize()
        held = ips.ips4o_workspace_bytes(h)
    finally:
        ips.ips4o_destroy(h)
    assert held <= bound, (held, bound)
    assert held <= 0.135 * n * 8, held / (n * 8)
    out = d.cpu().numpy().view(np.uint64)
    assert np.array_equal(out, oracle.sort_total_order_np(inp, "u64"))
    del d
    torch.cuda.empty_cache()
