"""ips4o_sort_small, the sort that allocates nothing, through the C ABI.

On the same inputs its output must equal ips4o_sort's (keys bit-exact; for
records additionally the payloads a permutation of the indices and every
record intact), on two calls in a row of which the second is smaller, and a
fresh handle must hold no workspace afterwards."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CASES = [("u64", "uniform", 16384, 5000), ("u64", "twodup", 400, 37), ("f64", "exponential", 9000, 512),
         ("f64", "ones", 12000, 2), ("pair", "rootdup", 8192, 100), ("quartet", "uniform", 4096, 3000),
         ("bytes100", "uniform", 4096, 17)]


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_02257_amd as ips
    oracle.build()
    workloads.build()
    return torch, ips


def _upload(torch, arr):
    flat = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
    return torch.from_numpy(flat.copy()).to("cuda:0")


def _keys(arr, dtype):
    if dtype in ("u64", "f64"):
        return arr.view(np.uint64)
    return {"pair": arr[:, :1], "quartet": arr[:, :3], "bytes100": arr[:, :10]}[dtype]


def _payload(arr, dtype):
    if dtype in ("pair", "quartet"):
        return arr[:, -1].astype(np.int64)
    return arr[:, 10:18].copy().view(np.uint64).ravel().astype(np.int64)


@pytest.mark.parametrize("dtype,dist,n1,n2", CASES)
def test_small_sort_matches_sort(env, dtype, dist, n1, n2):
    torch, ips = env
    h = ips.ips4o_create(0)
    try:
        stream = torch.cuda.current_stream()
        for call, n in enumerate((n1, n2)):
            inp = workloads.generate(dist, dtype, n, workloads.seed_for(0, dist, dtype) + call)
            a, b = _upload(torch, inp), _upload(torch, inp)
            print(f"[gpu] sort_small {dtype} {dist} n={n} (call {call})", flush=True)
            ips.ips4o_sort_small(h, a, n, dtype, stream)
            ips.ips4o_sort(ips.handle(0), b, n, dtype, None, stream)   # another handle: h allocates nothing
            torch.cuda.synchronize()
            got = a.cpu().numpy().view(inp.dtype).reshape(inp.shape)
            ref = b.cpu().numpy().view(inp.dtype).reshape(inp.shape)
            assert np.array_equal(_keys(got, dtype), _keys(ref, dtype)), (dtype, n)
            assert np.array_equal(_keys(got, dtype), _keys(oracle.sort(inp, dtype), dtype))
            if dtype not in ("u64", "f64"):
                pay = _payload(got, dtype)
                assert np.array_equal(np.sort(pay), np.arange(n))
                assert np.array_equal(got, inp[pay]), "a record was torn or mixed"
        # nothing was allocated on this handle
        assert ips.ips4o_workspace_bytes(h) == 0
    finally:
        ips.ips4o_destroy(h)


def test_small_sort_refuses_large(env):
    torch, ips = env
    h = ips.handle(0)
    n = ips.ips4o_small_max("u64") + 1
    d = torch.zeros(n, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ips.Ips4oError) as e:
        ips.ips4o_sort_small(h, d, n, "u64")
    assert e.value.status == -4
