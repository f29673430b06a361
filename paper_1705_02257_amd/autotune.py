"""Autotuner for the sort's tuning parameters.

Section 4 (Implementation Details) leaves the bucket count k, the block size
and the oversampling factor as parameters whose best values depend on the
machine and on the input.  Tuner times candidate parameter sets with
ips4o_sort on synthetic device-resident inputs of a size class (powers of
two) and element type, and keeps the fastest set per (element type, size
class) in a JSON cache.  params() looks a size up in the cache (the nearest
tuned class of the same element type), so callers can pass the result to
ips4o_sort or ips4o_sort_segmented.

The workgroup shapes of the kernels are fixed per element type when the
library is built; the tuner covers the parameters the C ABI exposes.
"""
import json
import math
import os
import time

DEFAULT_CANDIDATES = [
    {"k": 128, "block_bytes": 2048},
    {"k": 256, "block_bytes": 2048},
    {"k": 512, "block_bytes": 2048},
    {"k": 256, "block_bytes": 1024},
    {"k": 256, "block_bytes": 4096},
]


def size_class(n: int) -> int:
    """log2 of n rounded to the nearest integer (at least 1)."""
    return max(1, int(round(math.log2(max(n, 2)))))


class Tuner:
    """Per-(element type, size class) best parameters, tuned on demand."""

    def __init__(self, cache_path=None, device=0, timer=None):
        self.cache_path = cache_path
        self.device = device
        self.table = {}
        self._timer = timer            # (dtype, n, params) -> seconds; None: time on the GPU
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    @staticmethod
    def key(dtype: str, n: int) -> str:
        return f"{dtype}:{size_class(n)}"

    def params(self, dtype: str, n: int):
        """The tuned parameters of the nearest size class of `dtype`, or None."""
        want = size_class(n)
        best, dist = None, None
        for k, rec in self.table.items():
            dt, cls = k.split(":")
            if dt != dtype:
                continue
            d = abs(int(cls) - want)
            if dist is None or d < dist:
                best, dist = rec["params"], d
        return dict(best) if best is not None else None

    def tune(self, dtype: str, n: int, candidates=None, reps: int = 3, dist: str = "uniform"):
        """Times every candidate (median of `reps` sorts) and records the
        fastest for the size class of n; returns its parameters."""
        cands = candidates or DEFAULT_CANDIDATES
        timer, done = (self._timer, None) if self._timer else self._make_gpu_timer(dtype, n, dist)
        results = []
        try:
            for p in cands:
                ts = sorted(timer(dtype, n, p) for _ in range(reps))
                results.append((ts[len(ts) // 2], p))
        finally:
            if done:
                done()
        t_best, p_best = min(results, key=lambda r: r[0])
        self.table[self.key(dtype, n)] = {
            "params": dict(p_best), "ms": t_best * 1e3, "n": int(n),
            "candidates": [{"params": dict(p), "ms": t * 1e3} for t, p in results]}
        self.save()
        return dict(p_best)

    def save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
                f.write("\n")
            os.replace(tmp, self.cache_path)

    def _make_gpu_timer(self, dtype, n, dist):
        import numpy as np
        import torch

        import workloads
        from . import ips4o_create, ips4o_destroy, ips4o_sort

        workloads.build()
        host = workloads.generate(dist, dtype, n, 0x7E57 + n)
        raw = host.view(np.int64) if dtype in ("u64", "f64") else host.reshape(-1).view(np.uint8)
        pristine = torch.from_numpy(np.ascontiguousarray(raw)).to(f"cuda:{self.device}")
        work = torch.empty_like(pristine)
        h = ips4o_create(self.device)
        stream = torch.cuda.current_stream()

        def timer(dt, m, params):
            work.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ips4o_sort(h, work, m, dt, params, stream)
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        def done():
            torch.cuda.synchronize()
            ips4o_destroy(h)

        ips4o_sort(h, work, n, dtype, None, stream)      # first call allocates the workspace
        torch.cuda.synchronize()
        return timer, done
