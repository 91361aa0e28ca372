"""Several handles of one workload driven at once.

Independent solves (other loads, other parameter values) on a small
hierarchy leave most of the GPU idle: the coarse factorization is a chain of
panel steps, the coarse levels of a cycle are chains of small launches, and
every Krylov iteration waits for its Hessenberg column on the host.
``HandlePool`` keeps n hierarchies of the same configuration, each with its
own HIP stream, and runs the items of ``map`` on one host thread per handle,
so the handles' work interleaves on the device.  Every handle computes
exactly what a lone handle computes (its own launch shapes may differ, which
changes results only by rounding).

Each handle issues work on its own stream and, during a block
factorization, on one more stream per level; the HIP runtime maps a
process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default), and
streams sharing a queue run in order, so more queues can let the handles
overlap further (set it in the environment before the runtime starts).
Tensors that several items share must be complete before map is called.
"""
from __future__ import annotations

import threading

from . import fsgmg


class HandlePool:
    def __init__(self, cfg, w=None, n=4, device=0):
        import torch
        if n < 1:
            raise ValueError("a pool needs at least one handle")
        self.streams = [torch.cuda.Stream(device) for _ in range(n)]
        self.handles = []
        try:
            for s in self.streams:
                self.handles.append(fsgmg.Hierarchy(cfg, w, device=device, stream=s.cuda_stream))
        except Exception:
            self.close()
            raise
        self.device = device

    def __len__(self):
        return len(self.handles)

    def map(self, fn, items):
        """[fn(H, item) for item in items], item i on handle i % n; each
        handle takes its items in order on a host thread of its own, with its
        stream as torch's current stream.  The first exception raised by fn
        is re-raised after every thread has finished."""
        import torch
        items = list(items)
        out = [None] * len(items)
        errors = []

        def worker(k):
            H, s = self.handles[k], self.streams[k]
            try:
                with torch.cuda.device(self.device), torch.cuda.stream(s):
                    for i in range(k, len(items), len(self.handles)):
                        out[i] = fn(H, items[i])
                s.synchronize()
            except BaseException as e:   # noqa: BLE001 - handed to the caller
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(self.handles))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return out

    def close(self):
        for H in self.handles:
            H.close()
        self.handles = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
