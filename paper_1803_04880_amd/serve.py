"""Serving loop: continuous batching of protect / restore requests on one GPU.

Requests arrive over time (each names a device-resident buffer, or a pair of
fragments to restore).  The loop admits every arrived request that fits the
device-memory budget, plans the admitted protect requests and the admitted
restore requests as two batches (``batch.Batch``: one persistent launch per
direction over uneven buffers), launches them on a free stream (four by
default), and retires a launch when its completion event has fired,
releasing its memory and its stream.  While launches run on the GPU the host
plans and launches the next ones on the other streams, so planning overlaps
device work and a long request occupies one stream, not the device.  Every request's result
is exactly what a lone ``protect`` / ``restore`` call gives (the batch path
computes each item independently).

The per-request latency is arrival -> completion as seen by the host (the
event's completion is polled; the clock is ``time.perf_counter``).
``warmup()`` runs the batch kernels once on both streams before arrivals
start; ``launch_log`` keeps each launch's planning, launch and retire times
on the host clock and the device time of its kernels.
"""
from __future__ import annotations

import dataclasses
import gc
import time
from collections import deque

import torch

from . import default_width, geometry
from .batch import Batch


@dataclasses.dataclass
class Request:
    rid: int
    op: str                      # "protect" or "restore"
    arrival: float               # seconds from the start of the run
    n: int
    width: int
    levels: int
    key: bytes
    nonce: bytes
    x: torch.Tensor | None = None      # protect input (device)
    priv: torch.Tensor | None = None   # restore inputs (device)
    pub: torch.Tensor | None = None
    # results
    out_priv: torch.Tensor | None = None
    out_pub: torch.Tensor | None = None
    out: torch.Tensor | None = None
    done: float | None = None

    def device_bytes(self) -> int:
        g = geometry(self.n, self.width, self.levels)
        return g["priv_bytes"] + g["pub_bytes"] if self.op == "protect" else self.n


@dataclasses.dataclass
class _InFlight:
    reqs: list
    event: torch.cuda.Event
    bytes: int
    batches: list
    launched: float = 0.0        # host clock at launch (seconds from the run's start)
    planned: float = 0.0         # host clock when planning of the launch began
    gpu_start: torch.cuda.Event | None = None   # recorded before the batch kernels
    stream: torch.cuda.Stream | None = None      # returned to the free list at retirement


class Server:
    """Continuous-batching executor.  ``budget_bytes`` bounds the device
    memory of results in flight (outputs of admitted, unfinished requests);
    ``max_batch`` bounds the requests per launch; ``n_streams`` launches
    may run at once, each on its own stream, and a launch retires as soon as
    its own kernels have finished (whatever the state of the others)."""

    def __init__(self, budget_bytes: int = 64 << 30, max_batch: int = 512, device="cuda:0",
                 n_streams: int = 4):
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.free = deque(self.streams)
        self.in_use = 0
        self.inflight: list[_InFlight] = []
        self.batches_launched = 0
        self.on_complete = None   # called with each request when its batch has finished
        # per launch: (planning start, launch, retire) on the host clock,
        # device time of its kernels (ms), requests, bytes
        self.launch_log: list[tuple[float, float, float, float, int, int]] = []
        self._now = time.perf_counter

    def warmup(self, reserve_bytes: int = 4 << 30, large_bytes: int = 256 << 20):
        """Run one protect + restore batch on each stream and wait for it: a
        small buffer of every depth and one of ``large_bytes``, so that the
        first launches of the batch kernels, the streams' first timing events
        and the first plan uploads, small and large, happen before any request
        arrives; allocate and free ``reserve_bytes`` on each stream so that
        torch's caching allocator holds that much device memory for the
        results of the first launches."""
        for st in self.streams:
            with torch.cuda.stream(st):
                block = torch.empty(reserve_bytes, dtype=torch.uint8, device=self.device)
                del block
        key = bytes(16)
        for st in self.streams:
            with torch.cuda.stream(st):
                xs = [torch.full((4096 * lv + 17,), lv, dtype=torch.uint8, device=self.device)
                      for lv in (1, 2, 3, 4)]
                ws = [64] * 4
                lvs = [1, 2, 3, 4]
                if large_bytes:
                    xs.append(torch.zeros(large_bytes, dtype=torch.uint8, device=self.device))
                    ws.append(default_width(large_bytes))
                    lvs.append(3)
                b = Batch(xs, ws, lvs, [key] * len(xs), [key] * len(xs))
                start = torch.cuda.Event(enable_timing=True)
                start.record(st)
                b.protect(stream=st)
                b.restore(stream=st)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
            ev.synchronize()
            start.elapsed_time(ev)   # the first timing query, off the request path
            b.close()

    def _launch(self, reqs):
        prot = [r for r in reqs if r.op == "protect"]
        rest = [r for r in reqs if r.op == "restore"]
        stream = self.free.popleft()
        used = sum(r.device_bytes() for r in reqs)
        planned = self._now()
        batches = []
        with torch.cuda.stream(stream):
            # Both plans are built and uploaded (asynchronous copies on this
            # stream) before either batch is launched on the same stream; the
            # host does not wait for the device here.
            pb = rb = None
            if prot:
                pb = Batch([r.x for r in prot], [r.width for r in prot], [r.levels for r in prot],
                           [r.key for r in prot], [r.nonce for r in prot],
                           outs=[r.x for r in prot])   # protect never writes `out`
            if rest:
                outs = [torch.empty(r.n, dtype=torch.uint8, device=self.device) for r in rest]
                # restore reads only the fragments: the outputs stand in as inputs
                rb = Batch(outs, [r.width for r in rest], [r.levels for r in rest],
                           [r.key for r in rest], [r.nonce for r in rest],
                           privs=[r.priv for r in rest], pubs=[r.pub for r in rest], outs=outs)
            gpu_start = torch.cuda.Event(enable_timing=True)
            gpu_start.record(stream)
            if pb is not None:
                pb.protect(stream=stream)
                for r, p, q in zip(prot, pb.privs, pb.pubs):
                    r.out_priv, r.out_pub = p, q
                batches.append(pb)
            if rb is not None:
                rb.restore(stream=stream)
                for r, o in zip(rest, rb.outs):
                    r.out = o
                batches.append(rb)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        self.in_use += used
        self.inflight.append(_InFlight(reqs, ev, used, batches, self._now(), planned, gpu_start,
                                       stream))
        self.batches_launched += 1

    def _retire(self, now_fn, block=False):
        """Retire every launch whose kernels have finished; with ``block``,
        first wait for the oldest one."""
        if block and self.inflight:
            self.inflight[0].event.synchronize()
        keep = []
        for f in self.inflight:
            if not f.event.query():
                keep.append(f)
                continue
            t = now_fn()
            gpu_ms = f.gpu_start.elapsed_time(f.event) if f.gpu_start is not None else 0.0
            self.launch_log.append((f.planned, f.launched, t, gpu_ms, len(f.reqs), f.bytes))
            for r in f.reqs:
                r.done = t
                if self.on_complete is not None:
                    self.on_complete(r)
            for b in f.batches:
                b.close()
            self.in_use -= f.bytes
            self.free.append(f.stream)
        self.inflight = keep

    def run(self, requests, time_scale: float = 1.0):
        """Serve ``requests`` (sorted by arrival) in real time; returns the
        wall time of the run.  ``time_scale`` stretches arrival times."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        # the objects made so far (requests, tensors, plans) are long-lived:
        # collect once and move them out of the collector's generations, so
        # that no full collection over them interrupts the loop
        gc.collect()
        gc.freeze()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        self._now = now
        waiting: deque[Request] = deque()
        self.max_gap = (0.0, 0.0)   # longest host loop iteration (seconds) and its start
        t_prev = now()
        while pending or waiting or self.inflight:
            t = now()
            if t - t_prev > self.max_gap[0]:
                self.max_gap = (t - t_prev, t_prev)
            t_prev = t
            while pending and pending[0].arrival * time_scale <= t:
                waiting.append(pending.popleft())
            self._retire(now)
            take, room = [], self.budget - self.in_use
            while waiting and len(take) < self.max_batch:
                need = waiting[0].device_bytes()
                if need > room and (take or self.inflight):
                    break
                room -= need
                take.append(waiting.popleft())
            if take and self.free:
                self._launch(take)
            elif take:
                for r in reversed(take):   # every stream busy: keep them queued
                    waiting.appendleft(r)
                self._retire(now, block=True)
            elif not waiting and pending and not self.inflight:
                time.sleep(max(0.0, min(pending[0].arrival * time_scale - now(), 0.001)))
        self._retire(now, block=True)
        wall = now()
        gc.unfreeze()
        return wall
