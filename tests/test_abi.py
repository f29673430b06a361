"""The C ABI library loads, exports every function include/ips4o.h declares,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ips4o.h")


@pytest.fixture(scope="module")
def ips():
    import paper_1705_02257_amd as ips
    return ips


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ips4o_\w+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for want in ["ips4o_create", "ips4o_destroy", "ips4o_sort", "ips4o_distribute",
                 "ips4o_classify", "ips4o_select_splitters", "ips4o_sync", "ips4o_status_string",
                 "ips4o_check_args", "ips4o_check_splitters"]:
        assert want in names


def test_library_exports_every_declared_symbol(ips):
    lib = ctypes.CDLL(ips.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_and_wraps_the_declared_api(ips):
    """The binding's export list is the header's, and each name has a
    Python function of the same name."""
    assert sorted(ips.EXPORTS) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(ips, name)), name


def test_library_is_gfx950_code():
    """The offload bundle of the built library targets gfx950 only."""
    blob = open(os.path.join(ROOT, "paper_1705_02257_amd", "libips4o.so"), "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx\w+)", blob))
    assert targets == {b"gfx950"}


def test_status_strings(ips):
    for code in [0, -1, -2, -3, -4, -5]:
        assert ips.ips4o_status_string(code) != "unknown status"
    assert ips.ips4o_status_string(-99) == "unknown status"


def _check(ips, ptr, n, dtype, **params):
    p = ips.Params()
    for k, v in params.items():
        setattr(p, k, v)
    return ips.lib.ips4o_check_args(ptr, n, dtype, ctypes.byref(p) if params else None)


def test_check_args(ips):
    ok, bad, unsup = 0, -1, -4
    assert _check(ips, 0x1000, 1 << 20, ips.U64) == ok
    assert _check(ips, None, 0, ips.U64) == ok                  # n = 0: NULL allowed
    assert _check(ips, None, 5, ips.U64) == bad                 # NULL with n > 0
    assert _check(ips, 0x1004, 5, ips.U64) == bad               # misaligned for 8-byte keys
    assert _check(ips, 0x1004, 5, ips.BYTES100) == ok           # 4-byte records
    assert _check(ips, 0x1002, 5, ips.BYTES100) == bad
    assert _check(ips, 0x1000, 5, 7) == bad                     # unknown dtype
    assert _check(ips, 0x1000, 1 << 32, ips.U64) == ok          # beyond 32-bit sizes
    assert _check(ips, 0x1000, 1 << 36, ips.U64) == unsup       # blocks beyond the pointer word
    assert _check(ips, 0x1000, 1 << 40, ips.U64) == unsup
    assert _check(ips, 0x1000, 1 << 31, ips.BYTES100) == unsup  # 64 records per block at most
    assert _check(ips, 0x1000, 1 << 30, ips.BYTES100) == ok
    assert _check(ips, 0x1000, 100, ips.U64, k=3) == bad        # not a power of two
    assert _check(ips, 0x1000, 100, ips.U64, k=2048) == bad     # above 1024
    assert _check(ips, 0x1000, 100, ips.U64, k=1024) == ok
    assert _check(ips, 0x1000, 100, ips.U64, block_bytes=4) == bad
    assert _check(ips, 0x1000, 100, ips.U64, block_bytes=1 << 14) == bad
    assert _check(ips, 0x1000, 100, ips.U64, base_cap=1) == bad
    assert _check(ips, 0x1000, 100, ips.U64, base_cap=1 << 20) == bad
    assert _check(ips, 0x1000, 100, ips.QUARTET, base_cap=4096) == ok
    assert _check(ips, 0x1000, 100, ips.U64, stripes=5000) == bad


def test_check_splitters(ips):
    lib = ips.lib
    s = np.array([1, 5, 5, 9], dtype=np.uint64)
    assert lib.ips4o_check_splitters(s.ctypes.data, 4, ips.U64, 0) == 0
    assert lib.ips4o_check_splitters(s.ctypes.data, 4, ips.U64, 1) == 0
    assert lib.ips4o_check_splitters(s.ctypes.data, 4, ips.U64, 2) == -1
    assert lib.ips4o_check_splitters(s.ctypes.data, 0, ips.U64, 0) == -1
    assert lib.ips4o_check_splitters(None, 4, ips.U64, 0) == -1
    u = np.array([1, 5, 4], dtype=np.uint64)
    assert lib.ips4o_check_splitters(u.ctypes.data, 3, ips.U64, 0) == -1
    # f64 order is totalOrder: -0.0 < +0.0 is sorted, +0.0 > -0.0 the other way is not
    f = np.array([-1.0, -0.0, 0.0, np.inf], dtype=np.float64)
    assert lib.ips4o_check_splitters(f.ctypes.data, 4, ips.F64, 0) == 0
    g = np.array([0.0, -0.0], dtype=np.float64)
    assert lib.ips4o_check_splitters(g.ctypes.data, 2, ips.F64, 0) == -1
    big = np.arange(512, dtype=np.uint64)
    assert lib.ips4o_check_splitters(big.ctypes.data, 512, ips.U64, 0) == -1
    assert lib.ips4o_check_splitters(big.ctypes.data, 511, ips.U64, 0) == 0
    # quartet keys are (w0, w1, w2) lexicographic; w3 is payload
    q = np.array([[1, 2, 3, 99], [1, 2, 4, 0], [1, 3, 0, 5]], dtype=np.uint64)
    assert lib.ips4o_check_splitters(q.ctypes.data, 3, ips.QUARTET, 0) == 0
    q2 = q[[1, 0, 2]].copy()
    assert lib.ips4o_check_splitters(q2.ctypes.data, 3, ips.QUARTET, 0) == -1
    # 100-byte keys: unsigned bytewise
    r = np.zeros((2, 100), dtype=np.uint8)
    r[0, 0] = 0x7f
    r[1, 0] = 0x80
    assert lib.ips4o_check_splitters(r.ctypes.data, 2, ips.BYTES100, 0) == 0
    assert lib.ips4o_check_splitters(r[::-1].copy().ctypes.data, 2, ips.BYTES100, 0) == -1


def test_check_segments(ips):
    lib = ips.lib
    ok = np.array([0, 5, 5, 17, 100], dtype=np.uint64)
    dev = ctypes.c_void_p(4096)        # only inspected for NULL and alignment
    assert lib.ips4o_check_segments(dev, ips.U64, ok.ctypes.data, 4, None) == 0
    assert lib.ips4o_check_segments(None, ips.U64, None, 0, None) == 0
    assert lib.ips4o_check_segments(dev, ips.U64, None, 3, None) == -1
    bad = np.array([0, 5, 4, 17], dtype=np.uint64)
    assert lib.ips4o_check_segments(dev, ips.U64, bad.ctypes.data, 3, None) == -1
    assert lib.ips4o_check_segments(None, ips.U64, ok.ctypes.data, 4, None) == -1
    assert lib.ips4o_check_segments(ctypes.c_void_p(4100), ips.U64, ok.ctypes.data, 4, None) == -1
    assert lib.ips4o_check_segments(dev, 9, ok.ctypes.data, 4, None) == -1
    huge = np.array([0, 1 << 40], dtype=np.uint64)
    assert lib.ips4o_check_segments(dev, ips.U64, huge.ctypes.data, 1, None) == -4
    big = np.array([0, 1 << 32], dtype=np.uint64)
    assert lib.ips4o_check_segments(dev, ips.U64, big.ctypes.data, 1, None) == 0
    # offsets may start past 0 (the elements before are left alone)
    late = np.array([7, 9, 30], dtype=np.uint64)
    assert lib.ips4o_check_segments(dev, ips.PAIR, late.ctypes.data, 2, None) == 0


def test_null_handle_rejected(ips):
    lib = ips.lib
    assert lib.ips4o_sort(None, None, 0, 0, None, None) == -1
    b = np.zeros(4, dtype=np.uint64)
    s = np.array([1], dtype=np.uint64)
    assert lib.ips4o_distribute(None, None, 0, 0, s.ctypes.data, 1, 0, b.ctypes.data, None, None,
                                None) == -1
    assert lib.ips4o_create(0, None) == -1
    assert lib.ips4o_sync(None, None) == -1
    o = np.array([0, 3], dtype=np.uint64)
    assert lib.ips4o_sort_segmented(None, None, 0, o.ctypes.data, 1, None, None) == -1


def test_create_without_gpu_is_an_error_not_a_crash(ips):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(1)
    rc = ips.lib.ips4o_create(0, ctypes.byref(h))
    assert rc in (-4, -1, -3) and h.value is None


def test_tensor_arguments_checked_before_the_library(ips):
    """Raw addresses pass through; a tensor that is not on a GPU is refused
    with ValueError before anything reaches the library."""
    import torch
    assert ips._addr(12345) == 12345 and ips._addr(None) is None
    with pytest.raises(ValueError):
        ips._addr(torch.zeros(4, dtype=torch.int64))
    with pytest.raises(ValueError):
        ips.ips4o_sort(None, torch.zeros(4, dtype=torch.int64), 4, "u64")


def test_check_wrappers(ips):
    """The Python check functions return the library's statuses."""
    assert ips.ips4o_check_args(0x1000, 1 << 20, "u64") == 0
    assert ips.ips4o_check_args(None, 5, "u64") == -1
    assert ips.ips4o_check_args(0x1000, 100, "u64", {"k": 3}) == -1
    assert ips.ips4o_check_segments(0x1000, "u64", [0, 50, 100]) == 0
    assert ips.ips4o_check_segments(0x1000, "u64", [0, 50, 40, 100]) == -1
    assert ips.ips4o_check_segments(None, "u64", []) == 0
    assert ips.ips4o_check_splitters(np.array([1, 2, 2, 3], np.uint64), "u64", True) == 0
    assert ips.ips4o_check_splitters(np.array([3, 1], np.uint64), "u64", False) == -1
    assert ips.ips4o_check_splitters(np.array([], np.uint64), "u64", False) == -1


def test_workspace_size_query(ips):
    """ips4o_workspace_size answers without a handle or a GPU: argument
    checks, nothing for n <= 1, and at the 2^30-key configuration a bound
    between the stripe buffers' share (n*s/8) and 0.18 n*s (the per-bucket
    state adds O(n / base_cap))."""
    import ctypes
    L = ips._L()
    v = ctypes.c_size_t()
    assert L.ips4o_workspace_size(None, 0, 100, None, None) == -1
    assert L.ips4o_workspace_size(None, 9, 100, None, ctypes.byref(v)) == -1
    assert L.ips4o_workspace_size(None, 0, 100, ips.Params(k=3), ctypes.byref(v)) == -1
    assert ips.ips4o_workspace_size("u64", 0) == 0 and ips.ips4o_workspace_size("u64", 1) == 0
    n = 1 << 30
    for dt, s in [("u64", 8), ("f64", 8), ("pair", 16)]:
        w = ips.ips4o_workspace_size(dt, n)
        assert n * s / 8 <= w <= 0.18 * n * s, (dt, w / (n * s))
    # larger arrays need no more than proportionally more
    a, b = ips.ips4o_workspace_size("u64", 1 << 28), ips.ips4o_workspace_size("u64", 1 << 29)
    assert a < b <= 2 * a + (1 << 26)


def test_small_sort_limits(ips):
    """The no-allocation sort's size limits are one base-case bin per type;
    a NULL handle is refused."""
    assert [ips.ips4o_small_max(d) for d in ("u64", "f64", "pair", "quartet", "bytes100")] == \
        [16384, 16384, 8192, 4096, 4096]
    assert ips.lib.ips4o_small_max(7) == 0
    assert ips.lib.ips4o_sort_small(None, ctypes.c_void_p(4096), 10, ips.U64, None) == -1
