"""Serving loop: forward-only renders of device-resident soups with
continuous batching.

Requests (soup, camera, resolution) arrive over time. The server keeps a
FIFO queue and a fixed number of stream slots (one library context and one
HIP stream each). Whenever a slot is free it takes the longest prefix of the
queue that fits the batch-size cap and the memory budget (admission by
memory: the bytes a request needs while in flight, against a configurable
fraction of the device memory that was free at start-up) and renders it
with ONE soup_render call, i.e. one binning pass and one raster launch over
every request of the batch, whatever soup each reads. A completion event
per batch is polled; requests that arrive while batches run join the next
launch (continuous batching), and the next launch can start on the other
stream while one batch still runs.

The policy (Scheduler) is separate from the device calls (a backend with
launch / done), so that it can be tested without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Ticket:
    rid: int
    soup: int
    view: object               # workloads.View
    arrival: float             # seconds on the run's clock
    need: int                  # bytes while in flight
    done: float = -1.0
    color: object = None


@dataclasses.dataclass
class Batch:
    tickets: List[Ticket]
    need: int
    handle: object             # backend's completion handle


def request_bytes(width: int, height: int, n_tris: int) -> int:
    """Device bytes a request needs while in flight, an upper bound: its
    colour output (12 B/px) and an allowance of 8 B/px for the per-tile
    counters and offsets and, in large batches, the binning chunks' per-tile
    slots; 128 B per triangle for its 64-byte setup record and its tile-list
    entries (the library's workspaces grow with 25% headroom). The GPU tests
    check it against what a render actually allocates: its colour buffer
    plus the workspaces of a fresh context."""
    P = int(width) * int(height)
    return P * (12 + 8) + int(n_tris) * 128


class Scheduler:
    """FIFO queue, stream slots, batch cap and memory budget."""

    def __init__(self, n_slots: int, max_batch: int, budget: int,
                 launch: Callable[[int, List[Ticket]], object], done: Callable[[object], bool],
                 finish: Callable[[object, List[Ticket]], None], clock: Callable[[], float]):
        assert n_slots >= 1 and max_batch >= 1 and budget > 0
        self.n_slots, self.max_batch, self.budget = n_slots, max_batch, budget
        self._launch, self._done, self._finish, self._clock = launch, done, finish, clock
        self.queue: collections.deque = collections.deque()
        self.slots: List[Optional[Batch]] = [None] * n_slots
        self.in_use = 0
        self.peak_in_use = 0          # the largest in_use seen after a launch
        self.peak_in_flight = 0       # ... and the most requests in flight at once
        self.batches = 0
        self.batch_sizes: List[int] = []

    def submit(self, t: Ticket) -> None:
        self.queue.append(t)

    @property
    def busy(self) -> bool:
        return any(b is not None for b in self.slots) or bool(self.queue)

    def _take(self) -> List[Ticket]:
        """Longest queue prefix within the batch cap and the free budget; a
        request larger than the whole budget is admitted alone when nothing
        else is in flight (it could never fit otherwise)."""
        out, need = [], 0
        free = self.budget - self.in_use
        while self.queue and len(out) < self.max_batch:
            t = self.queue[0]
            if need + t.need > free and not (not out and self.in_use == 0):
                break
            out.append(self.queue.popleft())
            need += t.need
        return out

    def poll(self) -> List[Ticket]:
        """Retire finished batches, then fill free slots. Returns the
        requests completed by this call (with their completion time)."""
        finished = []
        for i, b in enumerate(self.slots):
            if b is not None and self._done(b.handle):
                now = self._clock()
                self._finish(b.handle, b.tickets)
                for t in b.tickets:
                    t.done = now
                finished.extend(b.tickets)
                self.in_use -= b.need
                self.slots[i] = None
        for i in range(self.n_slots):
            if self.slots[i] is None and self.queue:
                batch = self._take()
                if not batch:
                    break
                need = sum(t.need for t in batch)
                self.in_use += need
                self.slots[i] = Batch(batch, need, self._launch(i, batch))
                self.batches += 1
                self.batch_sizes.append(len(batch))
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                self.peak_in_flight = max(self.peak_in_flight,
                                          sum(len(b.tickets) for b in self.slots if b is not None))
        return finished


class Server:
    """Device backend: one context and one stream per slot; soups resident.

    The screen-tile side is fixed (``tile``) or, with ``tile=None``, tuned per
    request resolution by ``tune_tiles`` (the forward's work unit is a tile
    region, so a small render wants small tiles to fill the GPU); a batch
    takes the tile of its largest request."""

    def __init__(self, soups, tile: Optional[int] = 16, n_streams: int = 2, max_batch: int = 16,
                 budget_fraction: float = 0.25, opts=None, keep_colors: bool = False,
                 budget_bytes: Optional[int] = None):
        import torch
        from . import _lib
        from . import raster as R
        self.torch, self.R = torch, R
        self.soups = list(soups)
        self.opts = opts if opts is not None else R.Opts(mode=1)
        self.keep_colors = keep_colors
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.tile = tile
        self.tile_by_res: Dict[tuple, int] = {}   # (width, height) -> tuned tile side
        self.ctxs = []
        for _ in range(n_streams):
            c = _lib.Ctx(torch.cuda.current_device())
            c.set_tile(tile if tile is not None else 16)
            self.ctxs.append(c)
        self.ctx_tile = [tile if tile is not None else 16] * n_streams
        free, _total = torch.cuda.mem_get_info()
        self.budget = int(budget_bytes) if budget_bytes is not None else int(budget_fraction * free)
        self.t0 = time.perf_counter()
        self.sched = Scheduler(n_streams, max_batch, self.budget, self._launch, self._done, self._finish,
                               self.clock)

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def reset_clock(self) -> None:
        self.t0 = time.perf_counter()

    def need(self, soup: int, view) -> int:
        return request_bytes(view.width, view.height, self.soups[soup].T)

    def tune_tiles(self, views: Sequence, reps: int = 5) -> Dict[tuple, dict]:
        """For each distinct resolution among ``views``, time one render of
        every soup at that view with every tile side (autotune.tune) and keep
        the fastest."""
        from . import autotune
        torch, R = self.torch, self.R
        out = {}
        for v in views:
            res = (int(v.width), int(v.height))
            if res in out:
                continue
            vs = R.Views.from_list([v])
            colors = [torch.empty(v.height, v.width, 3, dtype=torch.float32, device="cuda")]

            def step(vs=vs, colors=colors):   # on the current stream, which the tuner times
                for sc in self.soups:
                    R.render([sc], vs, self.opts, colors, ctx=self.ctxs[0])

            key = "serve-%dx%d-%s" % (res[0], res[1], ",".join(str(sc.T) for sc in self.soups))
            out[res] = autotune.tune(step, self.ctxs[0], key, reps=reps)
            self.tile_by_res[res] = int(out[res]["tile"])
        self.ctxs[0].set_tile(self.ctx_tile[0])
        return out

    def tile_for(self, tickets: List[Ticket]) -> int:
        if self.tile is not None or not self.tile_by_res:
            return self.tile if self.tile is not None else 16
        big = max(tickets, key=lambda t: t.view.width * t.view.height).view
        res = (int(big.width), int(big.height))
        if res in self.tile_by_res:
            return self.tile_by_res[res]
        px = big.width * big.height   # nearest tuned resolution by pixel count
        near = min(self.tile_by_res, key=lambda r: abs(r[0] * r[1] - px))
        return self.tile_by_res[near]

    def _launch(self, slot: int, batch: List[Ticket]):
        torch, R = self.torch, self.R
        s = self.streams[slot]
        views = R.Views.from_list([t.view for t in batch])
        scenes = [self.soups[t.soup] for t in batch]
        tile = self.tile_for(batch)
        if tile != self.ctx_tile[slot]:
            self.ctxs[slot].set_tile(tile)
            self.ctx_tile[slot] = tile
        with torch.cuda.stream(s):
            colors = [torch.empty(t.view.height, t.view.width, 3, dtype=torch.float32, device="cuda")
                      for t in batch]
            R.render(scenes, views, self.opts, colors, ctx=self.ctxs[slot], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, colors)

    @staticmethod
    def _done(handle) -> bool:
        return handle[0].query()

    def _finish(self, handle, tickets: List[Ticket]) -> None:
        if self.keep_colors:
            for t, c in zip(tickets, handle[1]):
                t.color = c

    def measure_request(self, soup: int, view) -> int:
        """Device bytes one render of this request allocates: its colour
        buffer plus what it grows a fresh context's workspaces to."""
        torch, R = self.torch, self.R
        from . import _lib
        ctx = _lib.Ctx(torch.cuda.current_device())
        ctx.set_tile(self.tile_for([Ticket(0, soup, view, 0.0, 0)]))
        c = torch.empty(view.height, view.width, 3, dtype=torch.float32, device="cuda")
        R.render([self.soups[soup]], R.Views.from_list([view]), self.opts, [c], ctx=ctx)
        torch.cuda.synchronize()
        n = ctx.workspace_bytes() + c.numel() * 4
        ctx.close()
        return n

    def render_alone(self, soup: int, view):
        """One request in its own call (reference for batching invariance)."""
        torch, R = self.torch, self.R
        c = torch.empty(view.height, view.width, 3, dtype=torch.float32, device="cuda")
        R.render([self.soups[soup]], R.Views.from_list([view]), self.opts, [c], ctx=self.ctxs[0],
                 stream=self.streams[0])
        self.streams[0].synchronize()
        return c


def run(server: Server, requests: Sequence, warmup_s: float = 0.0) -> Dict:
    """Open-loop replay of `requests` (workloads.Request, arrival times in
    seconds) in real time. Latency = completion observed by the host minus
    arrival. Requests arriving before warmup_s are served but not counted."""
    server.reset_clock()
    sched = server.sched
    tickets = [Ticket(i, r.soup, r.view, r.arrival_s, server.need(r.soup, r.view)) for i, r in enumerate(requests)]
    done: List[Ticket] = []
    i, n = 0, len(tickets)
    b0 = sched.batches
    while len(done) < n:
        now = server.clock()
        while i < n and tickets[i].arrival <= now:
            sched.submit(tickets[i])
            i += 1
        done.extend(sched.poll())
        if not sched.busy and i < n:
            # idle until the next arrival: sleep most of the gap, spin the rest
            gap = tickets[i].arrival - server.clock()
            if gap > 0.002:
                time.sleep(gap - 0.001)
    dur = max(t.done for t in done) if done else 0.0
    lat = np.array([t.done - t.arrival for t in done if t.arrival >= warmup_s]) * 1e3
    px = sum(t.view.width * t.view.height for t in done)
    sizes = sched.batch_sizes[b0:]
    return {
        "requests": len(lat),
        "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
        "mean_ms": round(float(lat.mean()), 3) if len(lat) else None,
        "max_ms": round(float(lat.max()), 3) if len(lat) else None,
        "throughput_rps": round(n / dur, 1) if dur > 0 else None,
        "mpixel_s": round(px / dur / 1e6, 1) if dur > 0 else None,
        "batches": len(sizes),
        "mean_batch": round(float(np.mean(sizes)), 2) if sizes else None,
        "peak_in_use_bytes": sched.peak_in_use,
        "peak_in_flight": sched.peak_in_flight,
    }
