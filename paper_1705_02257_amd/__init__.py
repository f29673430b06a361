"""Python binding of libips4o.so, the gfx950 in-place super scalar samplesort
(Axtmann, Witt, Ferizovic, Sanders, "In-place Parallel Super Scalar
Samplesort (IPS4o)", arXiv 1705.02257).

Argument marshalling only: every step of the sort runs in the HIP kernels of
the library.  The functions carry the C ABI's names (include/ips4o.h); array
arguments may be torch tensors on the handle's GPU (their data_ptr() is
passed) or raw device addresses as ints.  Host-side arrays (splitters,
bounds) are numpy arrays.  A nonzero status raises Ips4oError.  The library
must have been built (``python paper_1705_02257_amd/build.py``); the first
call without it raises ImportError -- there is no fallback path.
"""
import ctypes
import os

import numpy as np
# torch first: it brings its own HIP runtime, and libips4o.so must bind to
# that same runtime (it resolves libamdhip64.so.7 to the copy already loaded)
# so that device pointers and streams from torch are valid in the library
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libips4o.so")

U64, F64, PAIR, QUARTET, BYTES100 = 0, 1, 2, 3, 4
DTYPES = {"u64": U64, "f64": F64, "pair": PAIR, "quartet": QUARTET, "bytes100": BYTES100}
ELEM_BYTES = {U64: 8, F64: 8, PAIR: 16, QUARTET: 32, BYTES100: 100}
FLAG_NO_SKIP = 1
FLAG_FUSE = 8            # base-case kernels clean the buckets of their bins (off by default)
FLAG_STRICT = 16         # levels hand over through bucket maxima and searchNextLargest (Section 4.6)
DEFAULT_K = 256          # first-level buckets when params leave k at 0 ...
DEFAULT_K_SMALL = 128    # ... for arrays of fewer than 2^27 elements


def default_k(n: int) -> int:
    """The first level's bucket count the library uses for n elements when
    the parameters leave k at 0 (as documented for ips4o_params.k)."""
    return DEFAULT_K_SMALL if n < (1 << 27) else DEFAULT_K
DEFAULT_BLOCK_BYTES = 2048  # block size when params leave block_bytes at 0

#: C symbols the library exports (as declared in include/ips4o.h)
EXPORTS = ["ips4o_create", "ips4o_destroy", "ips4o_workspace_bytes", "ips4o_workspace_size", "ips4o_sort",
           "ips4o_sort_small", "ips4o_small_max", "ips4o_sort_segmented_dev", "ips4o_distribute_dev",
           "ips4o_sort_segmented_small", "ips4o_set_default_params",
           "ips4o_sort_segmented", "ips4o_distribute", "ips4o_classify", "ips4o_select_splitters",
           "ips4o_sync", "ips4o_status_string", "ips4o_last_stats", "ips4o_last_kernel_stats",
           "ips4o_last_pass_stats", "ips4o_mark_bucket_max", "ips4o_search_next_largest",
           "ips4o_check_args", "ips4o_check_splitters", "ips4o_check_segments"]


class Ips4oError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: status {status} ({ips4o_status_string(status)})")


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("block_bytes", ctypes.c_uint32),
                ("base_cap", ctypes.c_uint32), ("alpha_x100", ctypes.c_uint32),
                ("stripes", ctypes.c_uint32), ("workers", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("spin_limit", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("fault_bits", ctypes.c_uint32),
                ("block_moves", ctypes.c_uint64), ("block_skips", ctypes.c_uint64),
                ("elements_base", ctypes.c_uint64), ("elements_distributed", ctypes.c_uint64)]


KERNEL_KINDS = ["sample", "classify", "scan", "fix_empty", "permute", "cleanup", "basecase", "mark"]
FLAG_TIMING = 2


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class PassStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint32), ("base_case", ctypes.c_uint32),
                ("ms", ctypes.c_double), ("alg_bytes", ctypes.c_double), ("elements", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1705_02257_amd/build.py` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.ips4o_create.argtypes = [i32, ctypes.POINTER(vp)]
    L.ips4o_destroy.argtypes = [vp]
    L.ips4o_destroy.restype = None
    L.ips4o_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.ips4o_workspace_size.argtypes = [vp, i32, u64, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]
    L.ips4o_sort.argtypes = [vp, vp, u64, i32, ctypes.POINTER(Params), vp]
    L.ips4o_sort_small.argtypes = [vp, vp, u64, i32, vp]
    L.ips4o_sort_segmented_dev.argtypes = [vp, vp, i32, vp, u32, ctypes.POINTER(Params), vp]
    L.ips4o_sort_segmented_small.argtypes = [vp, vp, i32, vp, u32, vp]
    L.ips4o_set_default_params.argtypes = [vp, i32, ctypes.POINTER(Params)]
    L.ips4o_distribute_dev.argtypes = [vp, vp, u64, i32, vp, u32, i32, vp, vp, ctypes.POINTER(Params), vp]
    L.ips4o_small_max.argtypes = [i32]
    L.ips4o_small_max.restype = u64
    L.ips4o_sort_segmented.argtypes = [vp, vp, i32, vp, u32, ctypes.POINTER(Params), vp]
    L.ips4o_distribute.argtypes = [vp, vp, u64, i32, vp, u32, i32, vp, ctypes.POINTER(u32),
                                   ctypes.POINTER(Params), vp]
    L.ips4o_classify.argtypes = [vp, vp, u64, i32, vp, u32, i32, vp, vp]
    L.ips4o_select_splitters.argtypes = [vp, vp, u64, i32, ctypes.POINTER(Params), vp,
                                         ctypes.POINTER(u32), ctypes.POINTER(i32), vp]
    L.ips4o_mark_bucket_max.argtypes = [vp, vp, u64, i32, vp, u32, vp]
    L.ips4o_search_next_largest.argtypes = [vp, vp, u64, i32, vp, u64, vp, vp]
    L.ips4o_check_args.argtypes = [vp, u64, i32, ctypes.POINTER(Params)]
    L.ips4o_check_splitters.argtypes = [vp, u32, i32, i32]
    L.ips4o_check_segments.argtypes = [vp, i32, vp, u32, ctypes.POINTER(Params)]
    L.ips4o_sync.argtypes = [vp, vp]
    L.ips4o_status_string.argtypes = [i32]
    L.ips4o_status_string.restype = ctypes.c_char_p
    L.ips4o_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.ips4o_last_kernel_stats.argtypes = [vp, ctypes.POINTER(KernelStat)]
    L.ips4o_last_pass_stats.argtypes = [vp, ctypes.POINTER(PassStat), u32, ctypes.POINTER(u32)]
    for name in ["ips4o_create", "ips4o_workspace_bytes", "ips4o_workspace_size", "ips4o_sort_small",
                 "ips4o_sort_segmented_dev", "ips4o_distribute_dev", "ips4o_sort_segmented_small",
                 "ips4o_set_default_params", "ips4o_sort", "ips4o_sort_segmented", "ips4o_distribute",
                 "ips4o_classify", "ips4o_select_splitters", "ips4o_sync", "ips4o_last_stats",
                 "ips4o_check_args", "ips4o_check_splitters", "ips4o_check_segments",
                 "ips4o_last_kernel_stats", "ips4o_last_pass_stats", "ips4o_mark_bucket_max",
                 "ips4o_search_next_largest"]:
        getattr(L, name).restype = i32
    return L


_lib_cache = None


def _L():
    """The loaded library (loaded on first use; raises if it was never built)."""
    global _lib_cache
    if _lib_cache is None:
        _lib_cache = _load()
    return _lib_cache


def __getattr__(name):
    if name == "lib":
        return _L()
    raise AttributeError(name)


def _dtype(dt):
    return DTYPES[dt] if isinstance(dt, str) else int(dt)


def _addr(x, need_bytes=None, what="data"):
    """Device address of a torch tensor or of a raw address given as an int.
    A tensor must be on a GPU and contiguous (the library reads its bytes
    from data_ptr() on) and hold at least need_bytes bytes; anything else
    raises ValueError before the library is called."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError(f"{what}: a GPU tensor is needed, got one on {x.device}")
    if not x.is_contiguous():
        raise ValueError(f"{what}: the tensor must be contiguous")
    have = x.numel() * x.element_size()
    if need_bytes is not None and have < need_bytes:
        raise ValueError(f"{what}: {need_bytes} bytes needed, the tensor holds {have}")
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _params(p):
    if p is None:
        return None
    if isinstance(p, Params):
        return ctypes.byref(p)
    q = Params()
    for k, v in p.items():
        setattr(q, k, v)
    return ctypes.byref(q)


def _check(rc, where, h=None):
    if rc != 0:
        if rc == -5 and h is not None:
            where = f"{where} (fault bits {ips4o_last_stats(h)['fault_bits']})"
        raise Ips4oError(rc, where)


def n_elements(t, dtype):
    """Element count of a tensor laid out for `dtype` (rows for records)."""
    d = _dtype(dtype)
    if d in (U64, F64):
        return t.numel()
    return t.shape[0]


def ips4o_status_string(status: int) -> str:
    return _L().ips4o_status_string(status).decode()


def ips4o_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_L().ips4o_create(device, ctypes.byref(h)), "ips4o_create")
    return h.value


def ips4o_destroy(h: int) -> None:
    _L().ips4o_destroy(h)


def ips4o_workspace_bytes(h: int) -> int:
    v = ctypes.c_size_t()
    _check(_L().ips4o_workspace_bytes(h, ctypes.byref(v)), "ips4o_workspace_bytes")
    return v.value


def ips4o_workspace_size(dtype, n, params=None, h=None) -> int:
    """Upper bound of the device workspace a fresh handle holds after
    sorting n elements (no GPU needed)."""
    v = ctypes.c_size_t()
    _check(_L().ips4o_workspace_size(h, _dtype(dtype), int(n), _params(params), ctypes.byref(v)),
           "ips4o_workspace_size")
    return v.value


def ips4o_sort(h, data, n, dtype, params=None, stream=None) -> None:
    d = _dtype(dtype)
    _check(_L().ips4o_sort(h, _addr(data, n * ELEM_BYTES[d]), n, d, _params(params), _stream(stream)),
           "ips4o_sort", h)


def ips4o_small_max(dtype) -> int:
    """Largest element count ips4o_sort_small accepts for `dtype`."""
    return int(_L().ips4o_small_max(_dtype(dtype)))


def ips4o_sort_small(h, data, n, dtype, stream=None) -> None:
    """Sort data[0:n] in place like ips4o_sort, for n <= ips4o_small_max(dtype),
    with no allocation (the library's fixed per-GPU array; returns after
    enqueue on `stream`)."""
    d = _dtype(dtype)
    _check(_L().ips4o_sort_small(h, _addr(data, n * ELEM_BYTES[d]), int(n), d, _stream(stream)),
           "ips4o_sort_small", h)


def ips4o_sort_segmented(h, data, offsets, dtype, params=None, stream=None) -> None:
    """Sorts data[offsets[i]:offsets[i+1]] for every i, each on its own;
    `offsets` is a host sequence of non-decreasing element offsets."""
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = max(offs.shape[0] - 1, 0)
    d = _dtype(dtype)
    need = int(offs.max()) * ELEM_BYTES[d] if nseg else 0
    _check(_L().ips4o_sort_segmented(h, _addr(data, need), d, offs.ctypes.data if nseg else None, nseg,
                                     _params(params), _stream(stream)), "ips4o_sort_segmented", h)


def ips4o_distribute(h, data, n, dtype, splitters: np.ndarray, equality_buckets: bool,
                     params=None, stream=None) -> np.ndarray:
    sp = np.ascontiguousarray(splitters)
    m = sp.shape[0]
    bounds = np.zeros(2 * m + 2, dtype=np.uint64)
    K = ctypes.c_uint32(0)
    _check(_L().ips4o_distribute(h, _addr(data, n * ELEM_BYTES[_dtype(dtype)]), n, _dtype(dtype), sp.ctypes.data, m,
                                int(bool(equality_buckets)), bounds.ctypes.data, ctypes.byref(K),
                                _params(params), _stream(stream)), "ips4o_distribute", h)
    return bounds[:K.value + 1].copy()


def ips4o_sort_segmented_dev(h, data, d_offsets, num_segments, dtype, params=None, stream=None) -> None:
    """ips4o_sort_segmented with the offset table (num_segments + 1 uint64
    offsets) in a device tensor."""
    _check(_L().ips4o_sort_segmented_dev(h, _addr(data), _dtype(dtype),
                                         _addr(d_offsets, 8 * (num_segments + 1), "offsets"), num_segments,
                                         _params(params), _stream(stream)), "ips4o_sort_segmented_dev", h)


def ips4o_set_default_params(h, dtype, params=None) -> None:
    """Parameters every later call on h for `dtype` uses where it leaves a
    field 0 (None clears them)."""
    _check(_L().ips4o_set_default_params(h, _dtype(dtype), _params(params)), "ips4o_set_default_params")


def ips4o_sort_segmented_small(h, data, d_offsets, num_segments, dtype, stream=None) -> None:
    """Segments of at most ips4o_small_max(dtype) elements, planned on the
    device from a device offset table; returns after enqueue (capturable in a
    HIP graph once a first call has sized the handle's bin lists)."""
    _check(_L().ips4o_sort_segmented_small(h, _addr(data), _dtype(dtype),
                                           _addr(d_offsets, 8 * (num_segments + 1), "offsets"), num_segments,
                                           _stream(stream)), "ips4o_sort_segmented_small", h)


def ips4o_distribute_dev(h, data, n, dtype, d_splitters, num_splitters, equality_buckets: bool, d_bounds,
                         d_num_buckets=None, params=None, stream=None) -> None:
    """ips4o_distribute with splitters, bounds and bucket count in device tensors."""
    d = _dtype(dtype)
    _check(_L().ips4o_distribute_dev(h, _addr(data, n * ELEM_BYTES[d]), n, d,
                                     _addr(d_splitters, num_splitters * ELEM_BYTES[d], "splitters"), num_splitters,
                                     int(bool(equality_buckets)), _addr(d_bounds, 8 * (2 * num_splitters + 2), "bounds"),
                                     _addr(d_num_buckets, 4, "num_buckets"), _params(params), _stream(stream)),
           "ips4o_distribute_dev", h)


def ips4o_classify(h, data, n, dtype, splitters: np.ndarray, equality_buckets: bool, out,
                   stream=None) -> None:
    sp = np.ascontiguousarray(splitters)
    _check(_L().ips4o_classify(h, _addr(data, n * ELEM_BYTES[_dtype(dtype)]), n, _dtype(dtype), sp.ctypes.data,
                              sp.shape[0], int(bool(equality_buckets)), _addr(out, 4 * n, "out"),
                              _stream(stream)),
           "ips4o_classify")


def ips4o_mark_bucket_max(h, data, n, dtype, d_bounds, num_buckets, stream=None) -> None:
    """Move the first largest element of every bucket [d_bounds[b],
    d_bounds[b+1]) to the bucket's first entry (Section 4.6); d_bounds: a
    device tensor of num_buckets + 1 int64 positions."""
    d = _dtype(dtype)
    _check(_L().ips4o_mark_bucket_max(h, _addr(data, n * ELEM_BYTES[d]), n, d,
                                      _addr(d_bounds, 8 * (num_buckets + 1), "bounds") if num_buckets else None,
                                      num_buckets, _stream(stream)), "ips4o_mark_bucket_max", h)


def ips4o_search_next_largest(h, data, n, dtype, d_pos, count, d_out, stream=None) -> None:
    """d_out[q] = searchNextLargest from position d_pos[q] (Section 4.6): the
    first later position in [0, n) holding a larger key, or n; d_pos, d_out:
    device tensors of `count` int64."""
    d = _dtype(dtype)
    _check(_L().ips4o_search_next_largest(h, _addr(data, n * ELEM_BYTES[d]), n, d,
                                          _addr(d_pos, 8 * count, "positions") if count else None, count,
                                          _addr(d_out, 8 * count, "out") if count else None, _stream(stream)),
           "ips4o_search_next_largest", h)


def ips4o_select_splitters(h, data, n, dtype, params=None, stream=None, like: np.ndarray = None):
    """Returns (unique splitters as a host array shaped like one element row of
    `like` (or raw bytes rows), equality flag)."""
    d = _dtype(dtype)
    k = 1024                # room for any k (the call's, the handle default's or the library's)
    s = ELEM_BYTES[d]
    out = np.zeros((k - 1) * s, dtype=np.uint8)
    nu = ctypes.c_uint32(0)
    eq = ctypes.c_int(0)
    _check(_L().ips4o_select_splitters(h, _addr(data, n * ELEM_BYTES[d]), n, d, _params(params), out.ctypes.data,
                                      ctypes.byref(nu), ctypes.byref(eq), _stream(stream)),
           "ips4o_select_splitters")
    raw = out[:nu.value * s]
    if like is not None:
        raw = raw.view(like.dtype).reshape((nu.value,) + like.shape[1:])
    return raw, bool(eq.value)


def _raw_addr(x):
    """Address for the argument checks, which only inspect it (NULL and
    alignment): a tensor's data_ptr(), an int, or None."""
    if x is None or isinstance(x, int):
        return x
    return x.data_ptr()


def ips4o_check_args(data, n, dtype, params=None) -> int:
    """The status ips4o_sort would return for these arguments (0 when they
    are valid); no GPU needed."""
    return _L().ips4o_check_args(_raw_addr(data), n, _dtype(dtype), _params(params))


def ips4o_check_segments(data, dtype, offsets, params=None) -> int:
    """The status ips4o_sort_segmented would return for these arguments."""
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = max(offs.shape[0] - 1, 0)
    return _L().ips4o_check_segments(_raw_addr(data), _dtype(dtype), offs.ctypes.data if nseg else None,
                                     nseg, _params(params))


def ips4o_check_splitters(splitters: np.ndarray, dtype, equality_buckets) -> int:
    """The status ips4o_distribute / ips4o_classify would return for these
    caller-given splitters (host array of num_splitters elements)."""
    sp = np.ascontiguousarray(splitters)
    m = sp.shape[0]
    return _L().ips4o_check_splitters(sp.ctypes.data if m else None, m, _dtype(dtype), int(equality_buckets))


def ips4o_sync(h, stream=None) -> None:
    _check(_L().ips4o_sync(h, _stream(stream)), "ips4o_sync")


def ips4o_last_stats(h) -> dict:
    st = Stats()
    _check(_L().ips4o_last_stats(h, ctypes.byref(st)), "ips4o_last_stats")
    return {f: getattr(st, f) for f, _ in Stats._fields_}


def ips4o_last_kernel_stats(h) -> dict:
    """{kernel kind: {launches, ms, alg_bytes}} of the last timed call."""
    arr = (KernelStat * len(KERNEL_KINDS))()
    _check(_L().ips4o_last_kernel_stats(h, arr), "ips4o_last_kernel_stats")
    return {name: {"launches": arr[i].launches, "ms": arr[i].ms, "alg_bytes": arr[i].alg_bytes}
            for i, name in enumerate(KERNEL_KINDS)}


def ips4o_last_pass_stats(h) -> list:
    """[{launches, base_case, ms, alg_bytes, elements}] per pass of the last
    timed call: each distribution level, then the base case."""
    num = ctypes.c_uint32(0)
    _check(_L().ips4o_last_pass_stats(h, None, 0, ctypes.byref(num)), "ips4o_last_pass_stats")
    arr = (PassStat * max(1, num.value))()
    _check(_L().ips4o_last_pass_stats(h, arr, num.value, ctypes.byref(num)), "ips4o_last_pass_stats")
    return [{f: getattr(arr[i], f) for f, _ in PassStat._fields_} for i in range(num.value)]


_handles = {}


def handle(device: int = 0) -> int:
    """Process-wide handle for a device (created on first use)."""
    if device not in _handles:
        _handles[device] = ips4o_create(device)
    return _handles[device]


def sort_(tensor, dtype="u64", params=None, stream=None, device=None):
    """Sort a device tensor in place; returns the tensor."""
    dev = tensor.device.index if device is None else device
    ips4o_sort(handle(dev or 0), tensor, n_elements(tensor, dtype), dtype, params, stream)
    return tensor
