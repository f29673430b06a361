"""ORACLE -- test infrastructure only (loaded by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the product path).

Thin ctypes marshalling over ``oracle.c``: a plain sequential CPU statement of
what in-place super scalar samplesort computes.  The arithmetic lives in the C
file, each function citing its passage of the paper.  Shares no code with the
HIP library.

Arrays use the same host layouts as the workloads module: u64 -> uint64[n],
f64 -> float64[n], pair -> uint64[n,2], quartet -> uint64[n,4],
bytes100 -> uint8[n,100].  Splitters are whole elements of the same dtype.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DTYPES = {"u64": 0, "f64": 1, "pair": 2, "quartet": 3, "bytes100": 4}
ELEM_BYTES = {"u64": 8, "f64": 8, "pair": 16, "quartet": 32, "bytes100": 100}


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, vp, u32, i32 = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.or_sort.argtypes = [vp, u64, i32]; L.or_sort.restype = i32
        L.or_compare.argtypes = [vp, vp, i32]; L.or_compare.restype = i32
        L.or_sort_segmented.argtypes = [vp, vp, u32, i32]; L.or_sort_segmented.restype = i32
        L.or_sort_small_integers.argtypes = [vp, u64, i32, u64, vp]
        L.or_sort_small_integers.restype = i32
        L.or_bucket.argtypes = [vp, i32, vp, u32, i32]; L.or_bucket.restype = u32
        L.or_num_buckets.argtypes = [i32, vp, u32, i32]; L.or_num_buckets.restype = u32
        L.or_classify.argtypes = [vp, u64, i32, vp, u32, i32, vp]; L.or_classify.restype = i32
        L.or_bucket_bounds.argtypes = [vp, u64, i32, vp, u32, i32, vp, vp]
        L.or_bucket_bounds.restype = i32
        L.or_splitmix64_at.argtypes = [u64, u64]; L.or_splitmix64_at.restype = u64
        L.or_select_splitters.argtypes = [vp, u64, i32, u32, u32, u64, vp, vp,
                                          ctypes.POINTER(u32), ctypes.POINTER(i32)]
        L.or_select_splitters.restype = i32
        L.or_select_splitters_capped.argtypes = [vp, u64, i32, u32, u32, u64, u32, vp, vp,
                                                 ctypes.POINTER(u32), ctypes.POINTER(i32)]
        L.or_select_splitters_capped.restype = i32
        L.or_tree.argtypes = [vp, u32, vp]; L.or_tree.restype = None
        L.or_tree_descend.argtypes = [vp, u32, u64]; L.or_tree_descend.restype = u32
        L.or_mark_bucket_max.argtypes = [vp, i32, vp, u32]; L.or_mark_bucket_max.restype = i32
        L.or_search_next_largest.argtypes = [vp, vp, u64, u64, i32, ctypes.POINTER(u64)]
        L.or_search_next_largest.restype = u64
        L.or_sort_strict.argtypes = [vp, u64, i32, u32, u32, u64, u64, vp]
        L.or_sort_strict.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _n(a):
    return a.shape[0]


def sort(arr: np.ndarray, dtype: str) -> np.ndarray:
    """Sorted copy of arr (keys non-decreasing under the dtype's order)."""
    out = np.ascontiguousarray(arr).copy()
    if _load().or_sort(_ptr(out), _n(out), DTYPES[dtype]) != 0:
        raise ValueError(dtype)
    return out


def sort_segmented(arr: np.ndarray, offsets, dtype: str) -> np.ndarray:
    """Copy of arr with arr[offsets[i]:offsets[i+1]] sorted for every i."""
    out = np.ascontiguousarray(arr).copy()
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = max(offs.shape[0] - 1, 0)
    if nseg and int(offs[-1]) > out.shape[0]:
        raise ValueError("offsets beyond the array")
    rc = _load().or_sort_segmented(_ptr(out), _ptr(offs), nseg, DTYPES[dtype])
    if rc != 0:
        raise ValueError(f"or_sort_segmented: {rc}")
    return out


def sort_small_integers(arr: np.ndarray, dtype: str, vmax: int) -> np.ndarray:
    """Sorted copy of u64/f64 keys that are all integers in [0, vmax), by
    counting (or_sort_small_integers); raises ValueError otherwise."""
    out = np.ascontiguousarray(arr).copy()
    counts = np.empty(max(int(vmax), 1), dtype=np.uint32)
    rc = _load().or_sort_small_integers(_ptr(out), _n(out), DTYPES[dtype], int(vmax), counts.ctypes.data)
    if rc != 0:
        raise ValueError(f"or_sort_small_integers: {rc}")
    return out


_TOP = np.uint64(1 << 63)
_CHUNK = 1 << 24


def sort_total_order_np(arr: np.ndarray, dtype: str) -> np.ndarray:
    """Sorted copy of u64 or f64 keys with numpy's sort as the one library
    step (fast enough for 2^30 keys).  u64: numpy's unsigned order.  f64:
    IEEE 754 totalOrder through its order-preserving image as an unsigned
    integer -- a negative-signed pattern has all its bits flipped (larger
    magnitudes become smaller images), a positive-signed one only its sign
    bit (placing it above every negative one) -- sorted, then mapped back;
    a second statement of the order that or_compare writes out by cases."""
    if dtype == "u64":
        out = np.ascontiguousarray(arr, dtype=np.uint64).copy()
        out.sort()
        return out
    if dtype != "f64":
        raise ValueError(dtype)
    bits = np.ascontiguousarray(arr).view(np.uint64)
    img = np.empty_like(bits)
    for a in range(0, bits.shape[0], _CHUNK):
        x = bits[a:a + _CHUNK]
        flip = (x.view(np.int64) >> np.int64(63)).view(np.uint64) | _TOP     # all ones, or the sign bit
        np.bitwise_xor(x, flip, out=img[a:a + _CHUNK])
    img.sort()
    for a in range(0, img.shape[0], _CHUNK):
        y = img[a:a + _CHUNK]
        flip = (~(y.view(np.int64) >> np.int64(63))).view(np.uint64) | _TOP  # sign bit, or all ones
        np.bitwise_xor(y, flip, out=y)
    return img.view(np.float64)


def _nondecreasing(keys: np.ndarray, dtype: str) -> bool:
    if keys.shape[0] < 2:
        return True
    if dtype == "u64":
        k = keys.view(np.uint64)
    else:
        b = keys.view(np.uint64)
        k = b ^ ((b.view(np.int64) >> np.int64(63)).view(np.uint64) | _TOP)
    for a in range(0, k.shape[0] - 1, _CHUNK):
        seg = k[a:a + _CHUNK + 1]
        if not bool(np.all(seg[1:] >= seg[:-1])):
            return False
    return True


def expected_sorted(dist: str, dtype: str, n: int, seed: int) -> np.ndarray:
    """The sorted arrangement of workloads.generate(dist, dtype, n, seed)
    for u64/f64 keys by a route that stays fast at 2^30 keys (the inputs of
    Section 5, Experimental Results):
      uniform, exponential  numpy's sort (sort_total_order_np);
      sorted, reverse, almost  ReverseSorted is Sorted read backwards and
                  AlmostSorted is Sorted with pairs swapped, so the sorted
                  arrangement of all three is the Sorted sequence of the same
                  seed (checked to be non-decreasing here);
      ones, rootdup, twodup, eightdup  integers below n: counting
                  (sort_small_integers)."""
    import workloads
    if dtype not in ("u64", "f64"):
        raise ValueError(dtype)
    if dist in ("uniform", "exponential"):
        return sort_total_order_np(workloads.generate(dist, dtype, n, seed), dtype)
    if dist in ("sorted", "reverse", "almost"):
        out = workloads.generate("sorted", dtype, n, seed)
        if not _nondecreasing(out, dtype):
            raise ValueError("the Sorted input is not non-decreasing")
        return out
    if dist in ("ones", "rootdup", "twodup", "eightdup"):
        return sort_small_integers(workloads.generate(dist, dtype, n, seed), dtype, max(n, 2))
    raise ValueError(dist)


def expected_sorted_range(dist: str, dtype: str, n: int, seed: int, first: int, count: int) -> np.ndarray:
    """Elements first .. first+count-1 of the sorted arrangement of
    workloads.generate(dist, dtype, n, seed) for u64/f64 keys, computed
    without the rest of the array (for inputs too large to hold on the host):
      sorted, reverse  the Sorted sequence of the same seed, in chunks;
      rootdup          A[i] = i mod m with m = floor(sqrt(n)) (Section 5):
                       value v occurs floor((n - 1 - v) / m) + 1 times, so
                       position p holds the v whose cumulative count first
                       exceeds p;
      ones             all ones."""
    import math
    import workloads
    if dtype not in ("u64", "f64"):
        raise ValueError(dtype)
    if first < 0 or count < 0 or first + count > n:
        raise ValueError("range outside the array")
    if dist in ("sorted", "reverse"):
        return workloads.generate_range("sorted", dtype, n, seed, first, count)
    if dist == "ones":
        return np.ones(count, dtype=np.uint64 if dtype == "u64" else np.float64)
    if dist != "rootdup":
        raise ValueError(dist)
    m = math.isqrt(n)
    v = np.arange(m, dtype=np.uint64)
    occ = (np.uint64(n - 1) - v) // np.uint64(m) + np.uint64(1)
    ends = np.cumsum(occ)                     # ends[v] = positions holding values <= v
    if count == 0:
        return np.empty(0, dtype=np.uint64 if dtype == "u64" else np.float64)
    last = first + count                      # one past the range
    vf = int(np.searchsorted(ends, np.uint64(first), side="right"))
    vl = int(np.searchsorted(ends, np.uint64(last - 1), side="right"))
    lo = np.maximum(ends[vf:vl + 1] - occ[vf:vl + 1], np.uint64(first))
    hi = np.minimum(ends[vf:vl + 1], np.uint64(last))
    vals = np.repeat(np.arange(vf, vl + 1, dtype=np.uint64), (hi - lo).astype(np.int64))
    return vals if dtype == "u64" else vals.astype(np.float64)


def compare(a: np.ndarray, b: np.ndarray, dtype: str) -> int:
    a = np.ascontiguousarray(a); b = np.ascontiguousarray(b)
    return int(_load().or_compare(_ptr(a), _ptr(b), DTYPES[dtype]))


def num_buckets(splitters: np.ndarray, dtype: str, eq: bool) -> int:
    sp = np.ascontiguousarray(splitters)
    return int(_load().or_num_buckets(DTYPES[dtype], _ptr(sp), _n(sp), int(eq)))


def classify(arr: np.ndarray, splitters: np.ndarray, dtype: str, eq: bool) -> np.ndarray:
    a = np.ascontiguousarray(arr); sp = np.ascontiguousarray(splitters)
    out = np.empty(_n(a), dtype=np.uint32)
    rc = _load().or_classify(_ptr(a), _n(a), DTYPES[dtype], _ptr(sp), _n(sp), int(eq), _ptr(out))
    if rc != 0:
        raise ValueError(dtype)
    return out


def bucket_bounds(arr: np.ndarray, splitters: np.ndarray, dtype: str, eq: bool):
    """(counts[K], bounds[K+1]) of one distribution step with given splitters."""
    a = np.ascontiguousarray(arr); sp = np.ascontiguousarray(splitters)
    K = num_buckets(sp, dtype, eq)
    counts = np.zeros(K, dtype=np.uint64); bounds = np.zeros(K + 1, dtype=np.uint64)
    rc = _load().or_bucket_bounds(_ptr(a), _n(a), DTYPES[dtype], _ptr(sp), _n(sp), int(eq),
                                  counts.ctypes.data, bounds.ctypes.data)
    if rc != 0:
        raise ValueError(dtype)
    return counts, bounds


def splitmix64_at(seed: int, i: int) -> int:
    return int(_load().or_splitmix64_at(seed & (2**64 - 1), i))


def select_splitters(arr: np.ndarray, dtype: str, k: int, alpha: int, seed: int, kcap: int = 0):
    """(unique splitters as elements, equality flag) for k buckets, oversampling
    alpha; with kcap > 0 the bucket count is kept within kcap as
    or_select_splitters_capped states."""
    a = np.ascontiguousarray(arr)
    shape_tail = a.shape[1:]
    scratch = np.empty((alpha * k - 1,) + shape_tail, dtype=a.dtype)
    out = np.empty((k - 1,) + shape_tail, dtype=a.dtype)
    mu = ctypes.c_uint32(0); eq = ctypes.c_int(0)
    rc = _load().or_select_splitters_capped(_ptr(a), _n(a), DTYPES[dtype], k, alpha, seed & (2**64 - 1),
                                            int(kcap), _ptr(scratch), _ptr(out), ctypes.byref(mu),
                                            ctypes.byref(eq))
    if rc != 0:
        raise ValueError("select_splitters: bad arguments")
    return out[:mu.value].copy(), bool(eq.value)


def tree(splitters_u64: np.ndarray, k: int) -> np.ndarray:
    """Level-order search tree a_1..a_{k-1} of k-1 sorted u64 splitters."""
    s = np.ascontiguousarray(splitters_u64, dtype=np.uint64)
    assert s.shape[0] == k - 1
    a = np.empty(k - 1, dtype=np.uint64)
    _load().or_tree(_ptr(s), k, _ptr(a))
    return a


def tree_descend(a: np.ndarray, k: int, e: int) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return int(_load().or_tree_descend(_ptr(a), k, e))


def alpha_default(n: int) -> int:
    """Oversampling factor 0.2*log2(n), at least 1 (Section 4, Implementation Details)."""
    import math
    return max(1, int(0.2 * math.log2(n))) if n > 1 else 1


def mark_bucket_max(arr: np.ndarray, bounds, dtype: str) -> np.ndarray:
    """Copy of arr with the largest element of every bucket
    [bounds[b], bounds[b+1]) moved to the bucket's first entry
    (or_mark_bucket_max, Section 4.6)."""
    out = np.ascontiguousarray(arr).copy()
    bd = np.ascontiguousarray(bounds, dtype=np.uint64)
    nb = max(bd.shape[0] - 1, 0)
    if nb and int(bd[-1]) > out.shape[0]:
        raise ValueError("bounds beyond the array")
    if _load().or_mark_bucket_max(_ptr(out), DTYPES[dtype], _ptr(bd), nb) != 0:
        raise ValueError("or_mark_bucket_max: bad arguments")
    return out


def search_next_largest(arr: np.ndarray, i: int, dtype: str, hi: int = None):
    """(searchNextLargest(A[i], A, i+1, hi), keys compared) of Section 4.6,
    0-based: the first position after i holding a key larger than A[i]'s, or
    hi (default len(arr)) if none, by exponential search and bisection."""
    a = np.ascontiguousarray(arr)
    hi = _n(a) if hi is None else hi
    if not 0 <= i < hi <= _n(a):
        raise ValueError("position outside the array")
    pivot = a[i].copy()
    probes = ctypes.c_uint64(0)
    j = _load().or_search_next_largest(_ptr(np.ascontiguousarray(pivot)), _ptr(a), i + 1, hi, DTYPES[dtype],
                                       ctypes.byref(probes))
    return int(j), int(probes.value)


def sort_strict(arr: np.ndarray, dtype: str, k: int = 16, alpha: int = 2, n0: int = 16, seed: int = 1):
    """(sorted copy, stats) by sequential samplesort whose recursion is
    emulated in constant space through bucket maxima and searchNextLargest
    (or_sort_strict, Section 4.6).  stats: partitions, insertion sorts,
    ranges found constant, keys compared by the searches."""
    out = np.ascontiguousarray(arr).copy()
    st = np.zeros(4, dtype=np.uint64)
    rc = _load().or_sort_strict(_ptr(out), _n(out), DTYPES[dtype], k, alpha, n0, seed & (2**64 - 1),
                                st.ctypes.data)
    if rc != 0:
        raise ValueError("or_sort_strict: bad arguments")
    return out, {"partitions": int(st[0]), "small_sorts": int(st[1]), "constant": int(st[2]),
                 "probes": int(st[3])}
