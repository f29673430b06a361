"""The serving loop on the GPU: every request's result, sorted in a mix of
concurrent batches, equals the oracle's sort of that request alone (keys
bit-exact, pair payloads as a permutation of the request's own); the same
under a pool so small that batches run one at a time; and an oversized
request is rejected."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import env, from_dev, keys_of, payload_of, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _requests(torch, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dtype = ["u64", "f64", "pair"][int(rng.integers(0, 3))]
        n = int(2 ** rng.uniform(4, 20))
        dist = ["uniform", "twodup", "sorted", "rootdup"][i % 4]
        host = workloads.generate(dist, dtype, n, 5000 + i)
        if dtype == "u64":
            dev = torch.from_numpy(host.view(np.int64).copy()).to("cuda:0")
        elif dtype == "f64":
            dev = torch.from_numpy(host.copy()).to("cuda:0")
        else:
            dev = torch.from_numpy(host.view(np.int64).copy()).to("cuda:0")
        out.append((dtype, host, dev))
    torch.cuda.synchronize()
    return out


def _check(dtype, host, dev):
    got = dev.cpu().numpy().view(host.dtype).reshape(host.shape)
    ref = oracle.sort(host, dtype)
    assert np.array_equal(keys_of(got, dtype), keys_of(ref, dtype))
    if dtype == "pair":
        pay = payload_of(got, dtype)
        assert np.array_equal(np.sort(pay), np.arange(host.shape[0]))
        assert np.array_equal(got, host[pay])
    else:
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("pool", [64 << 30, 1 << 24])
def test_results_alone_and_in_the_mix(env, pool):
    torch, ips, h = env
    from paper_1705_02257_amd.serving import SortServer
    reqs = _requests(torch, 60, 11 if pool > 1 << 24 else 12)
    srv = SortServer(pool_bytes=pool, workers=3)
    handles = [srv.submit(dev, dtype) for dtype, _, dev in reqs]
    for r in handles:
        assert r.wait(120), "request did not finish"
    srv.close()
    print(f"[gpu] serving pool={pool}: {srv.batches} batches for {len(reqs)} requests", flush=True)
    assert all(r.error is None for r in handles), [r.error for r in handles if r.error]
    if pool > 1 << 24:
        assert srv.batches < len(reqs)          # requests were batched
    for (dtype, host, dev) in reqs:
        _check(dtype, host, dev)


def test_oversized_request_rejected(env):
    torch, ips, h = env
    from paper_1705_02257_amd.serving import SortServer
    srv = SortServer(pool_bytes=1 << 10, workers=1)
    big = torch.zeros(1 << 12, dtype=torch.int64, device="cuda:0")
    r = srv.submit(big, "u64")
    assert r.wait(10) and r.error == "rejected" and srv.rejected == 1
    small = torch.arange(100, 0, -1, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    r2 = srv.submit(small, "u64")
    assert r2.wait(60) and r2.error is None
    srv.close()
    assert torch.equal(small.cpu(), torch.arange(1, 101, dtype=torch.int64))


def test_submit_checks_the_tensor_and_orders_after_the_callers_stream(env):
    """A view that is not contiguous, or a tensor short of the request's
    bytes, is refused at submit; a tensor still being filled on the caller's
    stream when it is submitted is sorted only after that fill."""
    torch, ips, h = env
    from paper_1705_02257_amd.serving import SortServer
    srv = SortServer(workers=1)
    base = torch.zeros(1000, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ValueError):
        srv.submit(base[::2], "u64")
    with pytest.raises(ValueError):
        srv.submit(torch.zeros((10, 1), dtype=torch.int64, device="cuda:0"), "pair")
    n = 1 << 22
    host = workloads.generate("uniform", "u64", n, 0x5EB)
    src = torch.from_numpy(host.view(np.int64)).to("cuda:0")
    dst = torch.zeros_like(src)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(8):                 # keep the side stream busy, then fill dst last
            dst.copy_(src.flip(0))
        dst.copy_(src)
        r = srv.submit(dst, "u64")
    assert r.wait(60) and r.error is None
    srv.close()
    assert np.array_equal(dst.cpu().numpy().view(np.uint64), oracle.sort(host, "u64"))
