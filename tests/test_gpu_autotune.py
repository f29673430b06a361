"""The autotuner on the GPU: it times real sorts, records one of the
candidates, and a sort with the tuned parameters matches the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import env, from_dev, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def test_tune_and_use(env, tmp_path):
    torch, ips, h = env
    from paper_1705_02257_amd.autotune import Tuner
    cands = [{"k": 128, "block_bytes": 2048}, {"k": 256, "block_bytes": 1024}]
    t = Tuner(cache_path=str(tmp_path / "tune.json"))
    n = 1 << 22
    best = t.tune("u64", n, candidates=cands, reps=2)
    assert best in cands
    rec = t.table[Tuner.key("u64", n)]
    assert rec["ms"] > 0 and len(rec["candidates"]) == 2
    inp = workloads.generate("twodup", "u64", n, 99)
    d = to_dev(torch, inp)
    ips.ips4o_sort(h, d, n, "u64", Tuner(cache_path=str(tmp_path / "tune.json")).params("u64", n))
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(d, inp), oracle.sort(inp, "u64"))


def test_tuned_parameters_become_the_handle_default(env, tmp_path):
    """apply() installs the tuned set on a handle: a call with no parameters
    then runs with them (the sampling step returns at most k - 1 splitters
    for the tuned k), and sorts correctly."""
    torch, ips, h0 = env
    from paper_1705_02257_amd.autotune import Tuner
    cands = [{"k": 16, "block_bytes": 2048, "base_cap": 8192}, {"k": 32, "block_bytes": 1024, "base_cap": 16384}]
    t = Tuner(cache_path=str(tmp_path / "tune.json"))
    n = 1 << 21
    best = t.tune("u64", n, candidates=cands, reps=1)
    h = ips.ips4o_create(0)
    try:
        assert t.apply(h, "u64", n) == best
        inp = workloads.generate("uniform", "u64", n, 5)
        d = to_dev(torch, inp)
        sp, _ = ips.ips4o_select_splitters(h, d, n, "u64", None, like=inp)
        assert 1 <= sp.shape[0] <= best["k"] - 1
        ips.ips4o_sort(h, d, n, "u64")
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(d, inp), oracle.sort(inp, "u64"))
        ips.ips4o_set_default_params(h, "u64", None)
        sp, _ = ips.ips4o_select_splitters(h, d, n, "u64", None, like=inp)
        assert sp.shape[0] > best["k"]                  # the library default k = 256 again
    finally:
        ips.ips4o_destroy(h)
