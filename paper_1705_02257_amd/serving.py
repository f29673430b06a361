"""Continuous-batching sort server over the segmented sort.

Requests are device tensors (u64, f64 or pair records) to be sorted in
place.  A request is admitted once the device memory it needs (its bytes,
twice over when it is staged with others, plus the library workspace the
batch may add to its worker's handle, from ips4o_workspace_size) fits the
pool budget beside the batches in flight and the workspace the workers'
handles already hold; admitted requests of one element type are gathered into
a batch, copied end to end into a staging buffer, sorted by one
ips4o_sort_segmented call and copied back (a batch of one request is sorted
where it lies).  Several workers, each with its own library handle and HIP
stream, run batches at the same time, so requests that arrive while others
are on the GPU start as soon as a worker and memory are free, and their work
overlaps on the device.  Latency runs from submit() to the completion of the
request's copy back.

A request tensor must be contiguous and on the server's GPU, and stay
untouched until wait() returns.  submit() records an event on the caller's
current stream, and the worker's stream waits for it, so work the caller
queued on that stream before submitting (filling the tensor) comes first.

The sorting itself is the library's (the recursion of Section 4 applied to
many independent arrays); this module only schedules.
"""
import collections
import os
import threading
import time

import numpy as np

from . import (ips4o_create, ips4o_destroy, ips4o_sort, ips4o_sort_segmented, ips4o_workspace_bytes,
               ips4o_workspace_size, n_elements)

ELEM_BYTES = {"u64": 8, "f64": 8, "pair": 16}


class Request:
    """One sort request; wait() blocks until it is done."""

    def __init__(self, tensor, dtype, ready=None):
        self.tensor = tensor
        self.dtype = dtype
        self.ready = ready              # event on the submitting stream
        self.n = n_elements(tensor, dtype)
        self.nbytes = self.n * ELEM_BYTES[dtype]
        self.t_submit = time.perf_counter()
        self.t_done = None
        self.error = None
        self.batch_size = 0
        self._done = threading.Event()

    def wait(self, timeout=None) -> bool:
        return self._done.wait(timeout)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_submit


class SortServer:
    """A request loop: submit() enqueues, worker threads batch and sort.

    pool_bytes: device bytes the server lets its work hold at once: the
    requests in flight, a batched request twice (its staging copy), and with
    count_workspace the library workspace of the workers' handles (what each
    holds, plus what a batch may add: its ips4o_workspace_size bound beyond
    what its worker holds); a request larger than the pool is rejected at
    submit; max_batch_bytes
    and max_batch: limits of one batch; workers: concurrent batches, one
    handle and stream each; batching=False sorts every request on its own,
    first come first served (the one-at-a-time reference); params: the
    sort parameters of a request sorted on its own -- "tuned" (the
    autotuner's table shipped with the package, tuned on single arrays and
    looked up by element type and size; library defaults where it has no
    entry), None (library defaults) or one ips4o_params dict; batches of
    several requests (one segmented sort) use the library defaults, which
    choose k per segment."""

    def __init__(self, device=0, pool_bytes=64 << 30, workers=2, max_batch_bytes=8 << 30, max_batch=4096,
                 batching=True, queue_limit=1 << 20, count_workspace=True, params="tuned"):
        import torch
        self.torch = torch
        self.device = device
        self.tuner = None
        self.fixed_params = None
        if params == "tuned":
            from .autotune import TUNED, Tuner
            if os.path.exists(TUNED):
                self.tuner = Tuner(cache_path=TUNED)
        elif params is not None:
            self.fixed_params = dict(params)
        self.pool_bytes = pool_bytes
        self.max_batch_bytes = max_batch_bytes
        self.max_batch = max_batch if batching else 1
        self.queue_limit = queue_limit
        self.queue = collections.deque()
        self.cond = threading.Condition()
        self.inflight = 0
        self.count_workspace = count_workspace
        self.resident = 0               # workspace the workers' handles hold between batches
        self.closed = False
        self.rejected = 0
        self.batches = 0
        self.completed = []
        self.threads = []
        self._errors = []
        for w in range(workers):
            t = threading.Thread(target=self._worker, name=f"sort-worker-{w}", daemon=True)
            t.start()
            self.threads.append(t)

    # ------------------------------------------------------------ clients
    def submit(self, tensor, dtype) -> Request:
        torch = self.torch
        if dtype not in ELEM_BYTES:
            raise ValueError(f"element type {dtype!r} is not served (one of {sorted(ELEM_BYTES)})")
        if not tensor.is_cuda or tensor.device.index != self.device:
            raise ValueError(f"the tensor must be on cuda:{self.device}, not {tensor.device}")
        if not tensor.is_contiguous():
            raise ValueError("the tensor must be contiguous")
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream(self.device))
        r = Request(tensor, dtype, ready)
        if tensor.numel() * tensor.element_size() < r.nbytes:
            raise ValueError(f"the tensor holds fewer than the {r.nbytes} bytes of {r.n} {dtype} elements")
        with self.cond:
            if self.closed:
                raise RuntimeError("server closed")
            if r.nbytes > self.pool_bytes or len(self.queue) >= self.queue_limit:
                self.rejected += 1
                r.error = "rejected"
                r._done.set()
                return r
            self.queue.append(r)
            self.cond.notify()
        return r

    def close(self):
        with self.cond:
            self.closed = True
            self.cond.notify_all()
        for t in self.threads:
            t.join()
        if self._errors:
            raise self._errors[0]

    # ------------------------------------------------------------ workers
    def params_for(self, dtype, n, single=True):
        """The parameters a request of n elements of dtype is sorted with
        (single: on its own; else a batch of n elements in all)."""
        if not single:
            return None
        if self.tuner is not None:
            return self.tuner.params(dtype, n)
        return self.fixed_params

    def config_for(self, dtype, n, single=True):
        """Element type and parameters of a batch of n elements."""
        p = self.params_for(dtype, n, single)
        return (dtype, tuple(sorted(p.items())) if p else None)

    def _growth(self, dtype, n, ws_have, last=None, single=True):
        """Workspace a batch of n elements may add to a handle holding
        ws_have after a batch of configuration `last` (config_for): the
        bound beyond what the handle holds when the configuration is the
        same, else the whole bound (the handle's buffers were sized for
        other parameters and may not cover this batch's)."""
        if not self.count_workspace:
            return 0
        bound = ips4o_workspace_size(dtype, n, self.params_for(dtype, n, single))
        if ws_have and last is not None and self.config_for(dtype, n, single) != last:
            return bound
        return max(0, bound - ws_have)

    def _take_batch(self, ws_have=0, last=None):
        """Called with the lock held: the head request plus the queue's later
        requests of its element type that fit the batch and pool limits, and
        the pool bytes the batch holds (its requests, twice over when they
        are staged together, plus the workspace it may add to a handle that
        holds ws_have after a batch of configuration `last`), or None when
        the head must wait for memory."""
        if not self.queue:
            return None
        head = self.queue[0]
        busy = self.inflight + self.resident
        if self.inflight > 0 and busy + head.nbytes + self._growth(head.dtype, head.n, ws_have, last) > self.pool_bytes:
            return None
        batch, total, elems = [self.queue.popleft()], head.nbytes, head.n
        keep = collections.deque()
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            if r.dtype != head.dtype:
                keep.append(self.queue.popleft())
                continue
            t2 = total + r.nbytes
            if t2 > self.max_batch_bytes or busy + 2 * t2 + self._growth(head.dtype, elems + r.n, ws_have, last, False) > \
                    self.pool_bytes:
                break
            batch.append(self.queue.popleft())
            total, elems = t2, elems + r.n
        self.queue.extendleft(reversed(keep))
        held = (2 * total if len(batch) > 1 else total) + self._growth(head.dtype, elems, ws_have, last, len(batch) == 1)
        self.inflight += held
        return batch, held

    def _worker(self):
        torch = self.torch
        torch.cuda.set_device(self.device)
        h = ips4o_create(self.device)       # a handle per worker: one call at a time each
        stream = torch.cuda.Stream(device=self.device)
        try:
            self._serve(h, stream)
        finally:
            stream.synchronize()
            ips4o_destroy(h)

    def _serve(self, h, stream):
        torch = self.torch
        ws_have = 0                     # workspace this worker's handle holds
        last = None                     # configuration of its last batch
        while True:
            with self.cond:
                got = None
                while got is None:
                    got = self._take_batch(ws_have, last)
                    if got is None:
                        if self.closed and not self.queue:
                            return
                        self.cond.wait(0.05)
            batch, held = got
            try:
                with torch.cuda.stream(stream):
                    self._run(h, stream, batch)
                stream.synchronize()
                now = time.perf_counter()
                for r in batch:
                    r.t_done = now
                    r.batch_size = len(batch)
            except Exception as e:          # surfaced by close()
                self._errors.append(e)
                for r in batch:
                    r.error = str(e)
            ws_now = ips4o_workspace_bytes(h)
            with self.cond:
                self.inflight -= held
                self.resident += ws_now - ws_have
                self.batches += 1
                self.completed.extend(batch)
                self.cond.notify_all()
            ws_have = ws_now
            last = self.config_for(batch[0].dtype, sum(r.n for r in batch), len(batch) == 1)
            for r in batch:
                r._done.set()

    def _run(self, h, stream, batch):
        torch = self.torch
        dtype = batch[0].dtype
        for r in batch:
            if r.ready is not None:
                stream.wait_event(r.ready)
        if len(batch) == 1:
            r = batch[0]
            ips4o_sort(h, r.tensor, r.n, dtype, self.params_for(dtype, r.n), stream)
            return
        sizes = [r.n for r in batch]
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        flat = [r.tensor.reshape(-1) for r in batch]
        staging = torch.cat(flat)
        ips4o_sort_segmented(h, staging, offs, dtype, self.params_for(dtype, int(offs[-1]), False), stream)
        words = [f.numel() for f in flat]
        at = 0
        for r, f, w in zip(batch, flat, words):
            f.copy_(staging[at:at + w])
            at += w
        del staging


def latency_summary(reqs):
    """p50 / p99 / max latency in ms over completed requests."""
    lat = np.array(sorted(r.latency for r in reqs if r.latency is not None))
    if lat.size == 0:
        return {"p50": None, "p99": None, "max": None}
    return {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
            "max": float(lat[-1] * 1e3)}
