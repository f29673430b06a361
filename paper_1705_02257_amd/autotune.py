"""Autotuner for the sort's tuning parameters.

Section 4 (Implementation Details) leaves the bucket count k, the block size
and the oversampling factor as parameters whose best values depend on the
machine and on the input.  Tuner times candidate parameter sets with
ips4o_sort on synthetic device-resident inputs of a size class (powers of
two) and element type, and keeps the fastest set per (element type, size
class) in a JSON cache.  params() looks a size up in the cache (the nearest
tuned class of the same element type); apply() installs it as the handle's
default (ips4o_set_default_params), so that every later call on that handle
that passes no parameters uses it.

search_space() spans the bucket count k, the block size, the number of
classification workgroups of the first level (stripes) and the base-case
capacity, which also picks the base-case workgroup shape: at half the
capacity every bin goes to the 512-lane instance that runs two workgroups
per CU, at the full capacity the larger bins go to the 1024-lane one.  Tile
sizes are fixed per element type when the library is built.
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


def search_space(dtype: str):
    """Every combination of k in {128, 256, 512}, 1, 2 or 4 KiB blocks,
    planner-chosen or 256 first-level stripes, and half or all of the
    base-case capacity."""
    from . import ips4o_small_max
    cap = ips4o_small_max(dtype)
    out = []
    for k in (128, 256, 512):
        for bb in (1024, 2048, 4096):
            for stripes in (0, 256):
                for bc in (cap // 2, cap):
                    out.append({"k": k, "block_bytes": bb, "stripes": stripes, "base_cap": bc})
    return out


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

    def apply(self, h, dtype: str, n: int):
        """Installs the tuned parameters of n's nearest size class as the
        defaults of handle h for `dtype`; returns them (None: nothing tuned)."""
        from . import ips4o_set_default_params
        p = self.params(dtype, n)
        if p is not None:
            ips4o_set_default_params(h, dtype, p)
        return p

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


#: parameters tuned on an MI355X (python -m paper_1705_02257_amd.autotune), shipped with the package
TUNED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def main(argv=None) -> int:
    """Tune the search space for the given element types and sizes on GPU 0
    and write the table (default: the shipped tuned.json)."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=TUNED)
    ap.add_argument("--dtype", nargs="+", default=["u64"])
    ap.add_argument("--log2n", type=int, nargs="+", default=[20, 24, 27, 30])
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    t = Tuner(cache_path=a.out)
    for dt in a.dtype:
        for lg in a.log2n:
            best = t.tune(dt, 1 << lg, candidates=search_space(dt), reps=a.reps)
            rec = t.table[Tuner.key(dt, 1 << lg)]
            print(f"[tune] {dt} 2^{lg}: {best} {rec['ms']:.3f} ms", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
