"""The autotuner's bookkeeping on the CPU (a fake timer): the fastest
candidate wins, the table survives a round trip through its JSON cache, and
lookups fall back to the nearest tuned size class of the same type."""
from paper_1705_02257_amd.autotune import Tuner, size_class


def fake_timer(dtype, n, params):
    # pretend k = 512 with 2 KiB blocks is fastest for large inputs, k = 128 for small
    best_k = 512 if n >= 1 << 24 else 128
    return 1.0 + abs(params["k"] - best_k) / 1000 + abs(params["block_bytes"] - 2048) / 1e5


def test_fastest_candidate_recorded(tmp_path):
    path = str(tmp_path / "tune.json")
    t = Tuner(cache_path=path, timer=fake_timer)
    assert t.tune("u64", 1 << 26, reps=3) == {"k": 512, "block_bytes": 2048}
    assert t.tune("u64", 1 << 18, reps=1) == {"k": 128, "block_bytes": 2048}
    t2 = Tuner(cache_path=path)
    assert t2.params("u64", 1 << 26) == {"k": 512, "block_bytes": 2048}
    assert t2.params("u64", 3 << 24) == {"k": 512, "block_bytes": 2048}     # nearest class 2^26
    assert t2.params("u64", 1 << 19) == {"k": 128, "block_bytes": 2048}
    assert t2.params("pair", 1 << 26) is None
    rec = t2.table[Tuner.key("u64", 1 << 26)]
    assert len(rec["candidates"]) == 5 and rec["n"] == 1 << 26


def test_size_class():
    assert size_class(1) == 1 and size_class(1 << 20) == 20 and size_class(3 << 19) == 21


def test_search_space_spans_shapes_and_capacity():
    from paper_1705_02257_amd.autotune import search_space
    sp = search_space("u64")
    assert len(sp) == 36
    assert {p["base_cap"] for p in sp} == {8192, 16384}
    assert {p["k"] for p in sp} == {128, 256, 512} and {p["stripes"] for p in sp} == {0, 256}
    assert {p["base_cap"] for p in search_space("bytes100")} == {2048, 4096}


def test_default_params_need_a_handle():
    import paper_1705_02257_amd as ips
    assert ips.lib.ips4o_set_default_params(None, 0, None) == -1
