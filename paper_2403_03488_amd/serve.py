"""Request loop with stage-level continuous batching on one GPU.

Requests (noisy uint8 images of any size, any sigma) arrive over time.  A
request is admitted when a slot is free and its device footprint (input,
output, workspace) fits the HBM budget; admission allocates its buffers and
starts the upload on the serving stream.  Every tick advances each in-flight
request by one of the seven stages (prep, match1, filter1, agg1, match2,
filter2, agg2) through bm3d_server_tick, which runs all requests that are at
the same stage in one batched launch -- so requests admitted while others
are mid-flight share launches with them.  A request completes when the event
recorded after the tick that ran its last stage has fired; latency is
arrival to that point.  Buffers are released at completion.

Everything on the device runs in the HIP library; this module only does the
scheduling and the torch allocations.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np

from . import bm3d

N_STAGES = 7


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    host_img: object        # pinned CPU uint8 tensor, HxW or HxWx3
    sigma: float
    # filled by the loop
    admitted: float = math.nan
    done: float = math.nan
    out: object = None      # device float32 result (kept if keep_outputs)
    buffers: object = None  # (device input, output, workspace) (kept if keep_buffers)

    @property
    def h(self):
        return self.host_img.shape[0]

    @property
    def w(self):
        return self.host_img.shape[1]

    @property
    def c(self):
        return 1 if self.host_img.dim() == 2 else self.host_img.shape[2]

    @property
    def mp(self):
        return self.h * self.w / 1e6


def footprint(h: int, w: int, c: int, p: bm3d.Params) -> int:
    """Device bytes one request holds while in flight."""
    return bm3d.workspace_size(h, w, c, p) + h * w * c + 4 * h * w * c


class ServingLoop:
    def __init__(self, p: bm3d.Params, max_slots: int = 32, hbm_budget: int = 16 << 30,
                 keep_outputs: bool = False, keep_buffers: bool = False):
        import torch
        self.torch = torch
        self.p = p
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.keep_outputs = keep_outputs
        self.keep_buffers = keep_buffers  # inspection: the request's workspace holds its groups
        self.server = bm3d.Server(max_slots, p)
        self.stream = torch.cuda.Stream()
        self.used = 0
        self.peak_used = 0
        self.ticks = 0
        self.tick_sizes = []

    def check_admissible(self, r: Request):
        need = footprint(r.h, r.w, r.c, self.p)
        if need > self.budget:
            raise ValueError("request %d needs %d bytes, more than the %d-byte budget"
                             % (r.rid, need, self.budget))

    def run(self, requests):
        """Serves the requests (sorted by arrival) in real time; returns them
        with admitted/done times filled in."""
        torch = self.torch
        for r in requests:
            self.check_admissible(r)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        active = []      # [req, stage, buffers]
        finishing = []   # [req, event, buffers]
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            while pending or waiting or active or finishing:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission: free slot and HBM footprint within budget
                while waiting and len(active) + len(finishing) < self.max_slots:
                    r = waiting[0]
                    need = footprint(r.h, r.w, r.c, self.p)
                    if self.used + need > self.budget:
                        break
                    waiting.popleft()
                    dev_img = torch.empty(r.host_img.shape, dtype=torch.uint8, device="cuda")
                    dev_img.copy_(r.host_img, non_blocking=True)
                    out = torch.empty(r.host_img.shape, dtype=torch.float32, device="cuda")
                    ws = torch.empty(bm3d.workspace_size(r.h, r.w, r.c, self.p), dtype=torch.uint8,
                                     device="cuda")
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                    r.admitted = time.perf_counter() - t0
                    active.append([r, 0, (dev_img, out, ws, need)])
                if active:
                    reqs = []
                    for r, stage, (dev_img, out, ws, _) in active:
                        reqs.append(bm3d.Request(dev_img.data_ptr(), out.data_ptr(), r.h, r.w, r.c,
                                                 float(r.sigma), ws.data_ptr(), ws.numel(), stage))
                    self.server.tick(reqs, self.stream)
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    self.ticks += 1
                    self.tick_sizes.append(len(reqs))
                    still = []
                    for item in active:
                        item[1] += 1
                        if item[1] == N_STAGES:
                            finishing.append([item[0], ev, item[2]])
                        else:
                            still.append(item)
                    active = still
                # completion
                if finishing:
                    keep = []
                    for r, ev, bufs in finishing:
                        if ev.query():
                            r.done = time.perf_counter() - t0
                            if self.keep_outputs or self.keep_buffers:
                                r.out = bufs[1]
                            if self.keep_buffers:
                                r.buffers = bufs[:3]
                            self.used -= bufs[3]
                        else:
                            keep.append([r, ev, bufs])
                    finishing = keep
                if not active and not waiting and pending and not finishing:
                    dt = pending[0].arrival - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
                elif not active and finishing:
                    time.sleep(0.0002)
        return requests


def summarize(requests, makespan=None):
    lat = np.array([r.done - r.arrival for r in requests]) * 1e3
    if makespan is None:
        makespan = max(r.done for r in requests) - min(r.arrival for r in requests)
    mp = sum(r.mp for r in requests)
    return {"requests": len(requests), "MP": mp, "makespan_s": makespan, "MPps": mp / makespan,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}


def serve_one_at_a_time(requests, p: bm3d.Params):
    """Baseline: the plain single-image path, one request at a time in
    arrival order (FCFS), in real time."""
    import torch
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for r in sorted(requests, key=lambda r: r.arrival):
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(0.0002)
            r.admitted = time.perf_counter() - t0
            dev_img = r.host_img.to("cuda", non_blocking=True)
            out = bm3d.denoise(dev_img, r.sigma, p, stream=stream)
            stream.synchronize()
            r.done = time.perf_counter() - t0
            del out, dev_img
    return requests
