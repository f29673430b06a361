"""The serving loop's batching and admission policy, on the CPU (no
workers, fake requests): batches take the head's element type, skip other
types without losing their order, respect the batch and pool limits, and
release their bytes."""
import types

import pytest

torch = pytest.importorskip("torch")

from paper_1705_02257_amd.serving import SortServer


def fake(n, dtype="u64"):
    nb = n * (16 if dtype == "pair" else 8)
    return types.SimpleNamespace(n=n, nbytes=nb, dtype=dtype)


def server(**kw):
    kw.setdefault("count_workspace", False)
    kw.setdefault("params", None)
    return SortServer(workers=0, **kw)


def test_batches_take_the_head_type_in_order():
    s = server()
    reqs = [fake(10), fake(20, "pair"), fake(30), fake(40, "f64"), fake(50)]
    s.queue.extend(reqs)
    batch, held = s._take_batch()
    assert batch == [reqs[0], reqs[2], reqs[4]]
    assert held == 2 * 90 * 8 and s.inflight == held
    assert list(s.queue) == [reqs[1], reqs[3]]
    batch2, _ = s._take_batch()
    assert batch2 == [reqs[1]]


def test_batch_and_pool_limits():
    s = server(max_batch_bytes=100 * 8, pool_bytes=1000 * 8)
    reqs = [fake(60), fake(30), fake(20), fake(5)]
    s.queue.extend(reqs)
    batch, held = s._take_batch()
    assert batch == [reqs[0], reqs[1]]          # 60 + 30 fits, + 20 does not
    s.queue.clear()
    s.inflight = 998 * 8
    s.queue.extend([fake(5), fake(6)])
    assert s._take_batch() is None              # nothing fits beside the work in flight
    s.inflight = 0
    batch, held = s._take_batch()
    assert len(batch) == 2 and held == 2 * 11 * 8


def test_single_request_holds_its_bytes_only():
    s = server()
    s.queue.append(fake(7))
    batch, held = s._take_batch()
    assert len(batch) == 1 and held == 7 * 8 and s.inflight == held


def test_one_at_a_time_mode():
    s = server(batching=False)
    reqs = [fake(1), fake(2), fake(3)]
    s.queue.extend(reqs)
    assert s._take_batch()[0] == [reqs[0]]
    assert s._take_batch()[0] == [reqs[1]]


def test_submit_refuses_tensors_it_cannot_serve():
    """A tensor off the GPU or of an element type the server does not batch
    is refused at submit, before anything is queued."""
    s = server()
    with pytest.raises(ValueError):
        s.submit(torch.zeros(8, dtype=torch.int64), "u64")
    with pytest.raises(ValueError):
        s.submit(torch.zeros(8, dtype=torch.int64), "quartet")
    assert not s.queue and s.rejected == 0


def test_admission_counts_workspace():
    """With workspace counting a batch also holds what the library may add to
    its worker's handle (ips4o_workspace_size beyond what the handle holds),
    and the workspace handles keep between batches counts against the pool."""
    from paper_1705_02257_amd import ips4o_workspace_size
    n = 1 << 20
    bound = ips4o_workspace_size("u64", n)
    s = server(count_workspace=True, pool_bytes=1 << 40)
    s.queue.append(fake(n))
    batch, held = s._take_batch()
    assert held == n * 8 + bound
    s.inflight = 0
    s.queue.append(fake(n))
    batch, held = s._take_batch(ws_have=bound)      # the handle already holds enough
    assert held == n * 8
    # bytes fit the pool, bytes plus workspace do not: wait while others run
    s2 = server(count_workspace=True, pool_bytes=n * 8 + bound - 1)
    s2.inflight = 1
    s2.queue.append(fake(n))
    assert s2._take_batch() is None
    s2.inflight, s2.resident = 0, 0
    assert s2._take_batch() is not None             # alone it goes anyway
    s3 = server(count_workspace=True, pool_bytes=4 * n * 8 + 2 * bound)
    s3.resident = 4 * n * 8 + 2 * bound - 10        # workers hold nearly all of it
    s3.inflight = 1
    s3.queue.append(fake(1000))
    assert s3._take_batch() is None


def test_tuned_parameters_per_batch_size():
    """By default a request sorted on its own uses the shipped autotuner
    table's parameters for its element type and size class, and its
    workspace is bounded with those; a batch of several requests (one
    segmented sort) uses the library defaults; a worker whose last batch
    ran another configuration counts the whole bound (its buffers were
    sized for other parameters)."""
    from paper_1705_02257_amd import ips4o_workspace_size
    from paper_1705_02257_amd.autotune import TUNED, Tuner
    s = SortServer(workers=0, count_workspace=True, pool_bytes=1 << 40)
    t = Tuner(cache_path=TUNED)
    assert t.table, "the package ships a tuned table"
    for n in (1 << 20, 1 << 24, 1 << 30):
        assert s.params_for("u64", n) == t.params("u64", n)
    n = 1 << 20
    p = t.params("u64", n)
    bound = ips4o_workspace_size("u64", n, p)
    s.queue.append(fake(n))
    _, held = s._take_batch()
    assert held == n * 8 + bound
    s.inflight = 0
    s.queue.append(fake(n))
    _, held = s._take_batch(ws_have=bound, last=s.config_for("u64", n))
    assert held == n * 8                            # same configuration: the handle holds enough
    s.inflight = 0
    s.queue.append(fake(n))
    _, held = s._take_batch(ws_have=bound, last=s.config_for("u64", 1 << 30))
    if s.config_for("u64", 1 << 30) != s.config_for("u64", n):
        assert held == n * 8 + bound                # other parameters: the whole bound
    assert s.params_for("u64", n, single=False) is None    # batches: the library's per-segment choices
    s.inflight = 0
    s.queue.extend([fake(n), fake(n)])
    batch, held = s._take_batch()
    assert len(batch) == 2 and held == 2 * 2 * n * 8 + ips4o_workspace_size("u64", 2 * n)
    assert SortServer(workers=0, params=None).params_for("u64", n) is None
    assert SortServer(workers=0, params={"k": 64}).params_for("u64", n) == {"k": 64}
