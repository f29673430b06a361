"""Parity at the full sizes of the paper's experiments (Section 5).

* Key configuration: 2^30 keys, u64 and f64, each of the nine input
  distributions.  Every element of the GPU output is compared with the
  oracle's sorted arrangement of the same seeded input
  (oracle.expected_sorted: numpy's sort for Uniform and Exponential, the
  Sorted sequence for the three presorted inputs, counting for the integer
  inputs below n).  The oracle outputs are computed ahead in worker threads
  (its C and numpy calls release the interpreter lock), at most a few cells
  ahead so that the host holds a bounded number of 8 GiB arrays.
* 2^32 u64 keys (RootDup, ReverseSorted), checked in chunks against the
  oracle's chunkable closed forms.
* Record configuration: 2^28 Pair, Quartet and 100Bytes records with Uniform
  and RootDup keys, generated and uploaded in chunks.  The payload of every
  input record is its index, so three device-side checks together pin the
  output exactly: keys non-decreasing in the record order, payloads a
  permutation of [0, n), and every output record equal to the input record
  its payload names.
"""
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

N30 = 1 << 30
KEY_CELLS = [(dist, dtype) for dtype in ("u64", "f64") for dist in workloads.DISTRIBUTIONS]
RECORD_CELLS = [(dtype, dist) for dtype in ("pair", "quartet", "bytes100") for dist in ("uniform", "rootdup")]
CHUNK = 1 << 24


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_02257_amd as ips
    oracle.build()
    workloads.build()
    return torch, ips, ips.handle(0)


class Ahead:
    """Oracle outputs for the key cells, computed in worker threads at most
    `depth` cells ahead of the one being tested."""

    def __init__(self, cells, depth=3):
        self.cells, self.depth = list(cells), depth
        self.pool = ThreadPoolExecutor(max_workers=depth)
        self.fut = {}
        self.taken = set()
        self.lock = threading.Lock()

    def _want(self, i):
        for j in range(i, min(i + self.depth, len(self.cells))):
            c = self.cells[j]
            if c not in self.fut and c not in self.taken:
                dist, dtype = c
                self.fut[c] = self.pool.submit(oracle.expected_sorted, dist, dtype, N30,
                                               workloads.seed_for(1, dist, dtype))

    def get(self, cell):
        with self.lock:
            i = self.cells.index(cell)
            self._want(i)
            fut = self.fut.pop(cell)
            self.taken.add(cell)
        out = fut.result()
        with self.lock:
            self._want(i + 1)
        return out

    def close(self):
        self.pool.shutdown(wait=True, cancel_futures=True)
        self.fut.clear()


@pytest.fixture(scope="module")
def ahead():
    a = Ahead(KEY_CELLS)
    yield a
    a.close()


def first_difference(a, b):
    """Index of the first element where two equal-length u64 arrays differ,
    or None (compared in chunks to bound the temporaries)."""
    assert a.shape == b.shape
    for f in range(0, a.shape[0], CHUNK):
        x, y = a[f:f + CHUNK], b[f:f + CHUNK]
        ne = np.flatnonzero(x != y)
        if ne.size:
            return f + int(ne[0])
    return None


@pytest.mark.parametrize("dist,dtype", KEY_CELLS)
def test_sort_2pow30_matches_oracle(env, ahead, dist, dtype):
    """2^30 keys, default parameters (k = 256, b = 2 KiB): the output equals
    the oracle's sorted arrangement element by element (bit patterns; f64
    in IEEE totalOrder)."""
    torch, ips, h = env
    seed = workloads.seed_for(1, dist, dtype)
    print(f"[gpu] sort {dtype} {dist} n=2^30 seed={seed:#x}", flush=True)
    inp = workloads.generate(dist, dtype, N30, seed)
    d = torch.from_numpy(inp.view(np.int64)).to("cuda:0")
    del inp
    ips.ips4o_sort(h, d, N30, dtype)
    torch.cuda.synchronize()
    out = d.cpu().numpy().view(np.uint64)
    del d
    torch.cuda.empty_cache()
    want = ahead.get((dist, dtype)).view(np.uint64)
    at = first_difference(out, want)
    assert at is None, f"{dtype} {dist}: first difference at {at}: GPU {int(out[at]):#x}, oracle {int(want[at]):#x}"


@pytest.mark.parametrize("dist", ["reverse", "eightdup"])
def test_sort_2pow30_fused_cleanup(env, dist):
    """2^30 u64 keys with IPS4O_FLAG_FUSE (the base case cleans the buckets
    of its bins): equal element by element to the oracle's sorted
    arrangement (the Sorted sequence for ReverseSorted, counting for
    EightDup)."""
    torch, ips, h = env
    seed = workloads.seed_for(1, dist, "u64")
    print(f"[gpu] fused sort u64 {dist} n=2^30 seed={seed:#x}", flush=True)
    inp = workloads.generate(dist, "u64", N30, seed)
    d = torch.from_numpy(inp.view(np.int64)).to("cuda:0")
    del inp
    ips.ips4o_sort(h, d, N30, "u64", {"flags": ips.FLAG_FUSE})
    torch.cuda.synchronize()
    out = d.cpu().numpy().view(np.uint64)
    del d
    torch.cuda.empty_cache()
    want = oracle.expected_sorted(dist, "u64", N30, seed).view(np.uint64)
    at = first_difference(out, want)
    assert at is None, f"{dist}: first difference at {at}: GPU {int(out[at]):#x}, oracle {int(want[at]):#x}"


@pytest.mark.parametrize("dist,dtype", [("reverse", "u64"), ("eightdup", "u64"), ("rootdup", "f64")])
def test_sort_2pow30_strict(env, dist, dtype):
    """2^30 keys with IPS4O_FLAG_STRICT (each level planned from the buckets
    a walk over the bucket maxima finds, Section 4.6): equal element by
    element to the oracle's sorted arrangement.  EightDup leaves equality
    buckets above the base-case capacity, which the walk cannot tell apart:
    they are partitioned once more and found to hold one key."""
    torch, ips, h = env
    seed = workloads.seed_for(1, dist, dtype)
    print(f"[gpu] strict sort {dtype} {dist} n=2^30 seed={seed:#x}", flush=True)
    inp = workloads.generate(dist, dtype, N30, seed)
    d = torch.from_numpy(inp.view(np.int64)).to("cuda:0")
    del inp
    ips.ips4o_sort(h, d, N30, dtype, {"flags": ips.FLAG_STRICT})
    torch.cuda.synchronize()
    out = d.cpu().numpy().view(np.uint64)
    del d
    torch.cuda.empty_cache()
    want = oracle.expected_sorted(dist, dtype, N30, seed).view(np.uint64)
    at = first_difference(out, want)
    assert at is None, f"{dist}: first difference at {at}: GPU {int(out[at]):#x}, oracle {int(want[at]):#x}"


N32 = 1 << 32


@pytest.mark.parametrize("dist", ["rootdup", "reverse"])
def test_sort_2pow32_u64(env, dist):
    """2^32 u64 keys (32 GiB, the largest size of the paper's experiments;
    beyond 32-bit element counts): generated and uploaded in chunks, sorted,
    and compared chunk by chunk, element by element, with the oracle's
    sorted arrangement (closed form for RootDup, the Sorted sequence for
    ReverseSorted)."""
    torch, ips, h = env
    seed = workloads.seed_for(1, dist, "u64")
    chunk = 1 << 26
    print(f"[gpu] sort u64 {dist} n=2^32 seed={seed:#x}", flush=True)
    d = torch.empty(N32, dtype=torch.int64, device="cuda:0")
    for f in range(0, N32, chunk):
        part = workloads.generate_range(dist, "u64", N32, seed, f, chunk)
        d[f:f + chunk].copy_(torch.from_numpy(part.view(np.int64)))
    ips.ips4o_sort(h, d, N32, "u64")
    torch.cuda.synchronize()
    for f in range(0, N32, chunk):
        got = d[f:f + chunk].cpu().numpy().view(np.uint64)
        want = oracle.expected_sorted_range(dist, "u64", N32, seed, f, chunk)
        at = first_difference(got, want)
        assert at is None, f"{dist}: first difference at {f + at}: GPU {int(got[at]):#x}, oracle {int(want[at]):#x}"
    del d
    torch.cuda.empty_cache()


def upload_chunked(torch, dist, dtype, n, seed):
    """The n-record input on the device as raw bytes, generated and copied
    CHUNK records at a time."""
    s = workloads.ELEM_BYTES[dtype]
    d = torch.empty(n * s, dtype=torch.uint8, device="cuda:0")
    for f in range(0, n, CHUNK):
        c = min(CHUNK, n - f)
        part = workloads.generate_range(dist, dtype, n, seed, f, c)
        d[f * s:(f + c) * s].copy_(torch.from_numpy(part.reshape(-1).view(np.uint8)))
    return d


def key_columns(torch, rows, dtype):
    """Key of each record row as int64 columns, most significant first, each
    to be compared as unsigned."""
    if dtype == "pair":
        return [rows.view(torch.int64)[:, 0]]
    if dtype == "quartet":
        w = rows.view(torch.int64)
        return [w[:, 0], w[:, 1], w[:, 2]]
    b = rows[:, :10].to(torch.int64)
    hi = torch.zeros(rows.shape[0], dtype=torch.int64, device=rows.device)
    for j in range(8):
        hi = hi | (b[:, j] << (8 * (7 - j)))
    return [hi, (b[:, 8] << 8) | b[:, 9]]


def payload_column(torch, rows, dtype):
    if dtype in ("pair", "quartet"):
        return rows.view(torch.int64)[:, -1]
    b = rows[:, 10:18].to(torch.int64)
    p = torch.zeros(rows.shape[0], dtype=torch.int64, device=rows.device)
    for j in range(8):
        p = p | (b[:, j] << (8 * j))
    return p


def rows_nondecreasing(torch, cols):
    """Adjacent rows in order under the unsigned lexicographic order."""
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=cols[0].device)
    less = torch.zeros(cols[0].shape[0] - 1, dtype=torch.bool, device=cols[0].device)
    eq = torch.ones_like(less)
    for c in cols:
        a, b = c[:-1] ^ sign, c[1:] ^ sign
        less = less | (eq & (a < b))
        eq = eq & (a == b)
    return bool((less | eq).all())


@pytest.mark.parametrize("dtype,dist,flags", [(t, d, 0) for t, d in RECORD_CELLS] +
                         [("pair", "rootdup", 16), ("quartet", "uniform", 16)])
def test_sort_records_2pow28(env, dtype, dist, flags):
    """2^28 records at their full size (Pair 4.3 GB, Quartet 8.6 GB, 100Bytes
    26.8 GB): keys in order, payloads a permutation of the indices, every
    record intact; two cells also with the strictly in-place hand-off
    (flags 16, IPS4O_FLAG_STRICT)."""
    torch, ips, h = env
    n = 1 << 28
    s = workloads.ELEM_BYTES[dtype]
    seed = workloads.seed_for(2, dist, dtype)
    print(f"[gpu] sort {dtype} {dist} n=2^28 seed={seed:#x} flags={flags}", flush=True)
    d = upload_chunked(torch, dist, dtype, n, seed)
    d0 = d.clone()
    ips.ips4o_sort(h, d, n, dtype, {"flags": flags})
    torch.cuda.synchronize()
    rows, rows0 = d.view(n, s), d0.view(n, s)
    seen = torch.zeros(n, dtype=torch.bool, device="cuda:0")
    for f in range(0, n, CHUNK):
        c = min(CHUNK, n - f)
        blk = rows[f:min(n, f + c + 1)]          # one row of overlap with the next chunk
        assert rows_nondecreasing(torch, key_columns(torch, blk, dtype)), f"keys out of order near row {f}"
        pay = payload_column(torch, rows[f:f + c], dtype)
        assert bool(((pay >= 0) & (pay < n)).all()), f"payload out of range near row {f}"
        seen[pay] = True
        assert torch.equal(rows[f:f + c], rows0[pay]), f"a record was torn or mixed near row {f}"
    assert bool(seen.all()), "payloads are not a permutation of the indices"
    del d, d0, rows, rows0, seen
    torch.cuda.empty_cache()
