"""Seeded synthetic inputs of the paper's nine distributions (Section 5) for the
key types u64/f64 and the record types Pair, Quartet and 100Bytes.

This module holds none of the sorting method's arithmetic; it is shared by the
tests, the oracle checks and the benchmark.  The generator is plain C
(``gen.c``) built with gcc into ``libworkloads.so`` next to this file.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libworkloads.so")

DISTRIBUTIONS = ["uniform", "exponential", "sorted", "reverse", "almost",
                 "ones", "rootdup", "twodup", "eightdup"]
DTYPES = {"u64": 0, "f64": 1, "pair": 2, "quartet": 3, "bytes100": 4}
ELEM_BYTES = {"u64": 8, "f64": 8, "pair": 16, "quartet": 32, "bytes100": 100}

#: Seed recipe: base + 1000*config + 10*distribution + dtype.
SEED_BASE = 0x1705022570


def seed_for(config: int, dist: str, dtype: str) -> int:
    return SEED_BASE + 1000 * config + 10 * DISTRIBUTIONS.index(dist) + DTYPES[dtype]


def build(force: bool = False) -> str:
    """Compile gen.c with gcc (OpenMP) into libworkloads.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.wl_generate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_void_p]
        lib.wl_generate.restype = ctypes.c_int
        lib.wl_generate_range.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        lib.wl_generate_range.restype = ctypes.c_int
        lib.wl_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.wl_splitmix64_at.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def empty(dtype: str, n: int) -> np.ndarray:
    """Host array laid out as the device expects for `dtype`."""
    if dtype == "u64":
        return np.empty(n, dtype=np.uint64)
    if dtype == "f64":
        return np.empty(n, dtype=np.float64)
    if dtype == "pair":
        return np.empty((n, 2), dtype=np.uint64)
    if dtype == "quartet":
        return np.empty((n, 4), dtype=np.uint64)
    if dtype == "bytes100":
        return np.empty((n, 100), dtype=np.uint8)
    raise ValueError(dtype)


def generate(dist: str, dtype: str, n: int, seed: int, out: np.ndarray = None) -> np.ndarray:
    """Return n elements of `dist` as `dtype` from `seed` (deterministic)."""
    arr = empty(dtype, n) if out is None else out
    assert arr.flags["C_CONTIGUOUS"] and arr.nbytes == n * ELEM_BYTES[dtype]
    rc = _load().wl_generate(DISTRIBUTIONS.index(dist), DTYPES[dtype], n, seed & (2**64 - 1),
                             arr.ctypes.data if n else None)
    if rc != 0:
        raise ValueError(f"wl_generate failed for {dist}/{dtype}/{n}")
    return arr


def generate_range(dist: str, dtype: str, n: int, seed: int, first: int, count: int,
                   out: np.ndarray = None) -> np.ndarray:
    """Elements first .. first+count-1 of generate(dist, dtype, n, seed),
    produced without the rest (AlmostSorted only whole: its swaps reach
    across the array)."""
    arr = empty(dtype, count) if out is None else out
    assert arr.flags["C_CONTIGUOUS"] and arr.nbytes == count * ELEM_BYTES[dtype]
    rc = _load().wl_generate_range(DISTRIBUTIONS.index(dist), DTYPES[dtype], n, seed & (2**64 - 1), first,
                                   count, arr.ctypes.data if count else None)
    if rc != 0:
        raise ValueError(f"wl_generate_range failed for {dist}/{dtype}/{n}/{first}+{count}")
    return arr


def splitmix64_at(seed: int, i: int) -> int:
    """i-th (0-based) output of the splitmix64 stream whose state starts at seed."""
    return int(_load().wl_splitmix64_at(seed & (2**64 - 1), i))
