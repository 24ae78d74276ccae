"""Continuous-batching server for energy + potential requests of mixed grid sizes.

Requests (density n, optional gradient, grid, cell) arrive over time.  The server keeps a pool of
S slots, each a HIP stream with its own library handles (one per grid/cell, created on first use
and kept resident with their FFT plans and kernel tables).  A request is admitted as soon as a slot
is free and the handle it needs fits in the HBM budget, counting every resident handle's work
buffers (`vdwxc_workspace_bytes`); otherwise it waits in arrival order.  Admitted requests run
concurrently on their slots' streams, so requests that arrive while others are on the GPU overlap
with them; completions are detected with stream events and free their slot immediately.

Every evaluation is deterministic (fixed-order reductions, no atomics), so a request's (E, v) is
bitwise the same alone or in the mix.

`submit` returns a `concurrent.futures.Future` that resolves to the finished Request (its `energy`
and `v` device tensors complete), or fails at once with ValueError when the request's handle alone
needs more than the whole HBM budget (it could never be admitted).
"""
from __future__ import annotations

import collections
import concurrent.futures
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import vdwxc


@dataclass
class Request:
    rid: int
    grid: tuple
    cell: np.ndarray
    n: torch.Tensor
    grad: torch.Tensor | None = None
    arrival: float = 0.0          # seconds from the start of the run
    # filled by the server
    admitted: float | None = None
    finished: float | None = None
    energy: torch.Tensor | None = None
    v: torch.Tensor | None = None
    slot: int | None = None
    future: concurrent.futures.Future | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Slot:
    index: int
    stream: torch.cuda.Stream
    handles: dict = field(default_factory=dict)
    busy: Request | None = None
    event: torch.cuda.Event | None = None


class Server:
    """S slots sharing an HBM budget (bytes) for the handles' work buffers."""

    def __init__(self, table, slots: int = 4, precision: str = "fp32", flavour: str = "DF1",
                 hbm_budget: float = 64e9):
        self.table = table
        self.precision = precision
        self.flavour = flavour
        self.budget = float(hbm_budget)
        self.slots = [_Slot(i, torch.cuda.Stream()) for i in range(slots)]
        self.resident = 0.0
        self.queue: collections.deque = collections.deque()
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.max_concurrent = 0
        self.peak_resident = 0.0

    # ---- memory accounting -----------------------------------------------------------------
    def _cost(self, grid) -> float:
        return float(vdwxc.workspace_bytes(grid, self.precision, self.table.nq))

    def _key(self, req):
        return (tuple(req.grid), tuple(np.asarray(req.cell, dtype=np.float64).ravel().round(12)))

    def _handle_for(self, slot: _Slot, req: Request, free_slots):
        """The slot's handle for this grid/cell, creating it if the budget allows; None if it cannot
        fit now.  To make room it evicts idle handles (this slot's first, then those of the other
        free slots), but only when evicting them does make room: otherwise nothing is evicted and
        the resident plans and tables stay."""
        key = self._key(req)
        h = slot.handles.get(key)
        if h is not None:
            return h
        need = self._cost(req.grid)
        if self.resident + need > self.budget:
            order = [slot] + [s for s in free_slots if s is not slot]
            victims = [(s, k) for s in order for k in s.handles]
            freeable = sum(self._cost(k[0]) for _, k in victims)
            if self.resident - freeable + need > self.budget:
                return None
            for s, k in victims:
                self.resident -= self._cost(k[0])
                s.handles.pop(k).close()
                if self.resident + need <= self.budget:
                    break
        with torch.cuda.stream(slot.stream):
            h = vdwxc.Functional(req.grid, req.cell, flavour=self.flavour, precision=self.precision,
                                 table=self.table, stream=slot.stream)
        slot.handles[key] = h
        self.resident += need
        self.peak_resident = max(self.peak_resident, self.resident)
        return h

    def warm(self, shapes):
        """Create every slot's handle for each (grid, cell) in `shapes` ahead of traffic, as far as
        the HBM budget allows (plans, tables and work buffers then stay resident), so that no
        request pays for a handle's set-up.  Returns the number of handles created."""
        made = 0
        for grid, cell in shapes:
            probe = Request(-1, tuple(grid), np.asarray(cell, dtype=np.float64), None)
            for slot in self.slots:
                key = self._key(probe)
                if key in slot.handles:
                    continue
                need = self._cost(probe.grid)
                if self.resident + need > self.budget:
                    return made
                with torch.cuda.stream(slot.stream):
                    slot.handles[key] = vdwxc.Functional(probe.grid, probe.cell, flavour=self.flavour,
                                                         precision=self.precision, table=self.table,
                                                         stream=slot.stream)
                self.resident += need
                self.peak_resident = max(self.peak_resident, self.resident)
                made += 1
        torch.cuda.synchronize()
        return made

    # ---- scheduling --------------------------------------------------------------------------
    def submit(self, req: Request) -> concurrent.futures.Future:
        """Queue a request; the returned Future resolves to the finished Request."""
        req.future = concurrent.futures.Future()
        need = self._cost(req.grid)
        if need > self.budget:
            req.future.set_exception(ValueError(
                f"request {req.rid}: grid {tuple(req.grid)} needs {need / 1e9:.3f} GB of work buffers, more than "
                f"the whole HBM budget of {self.budget / 1e9:.3f} GB"))
            self.rejected.append(req)
            return req.future
        self.queue.append(req)
        return req.future

    def _start(self, slot: _Slot, req: Request, h, now: float):
        req.admitted = now
        req.slot = slot.index
        req.v = torch.empty_like(req.n)
        req.energy = torch.empty(1, dtype=torch.float64, device=req.n.device)
        # inputs were produced on the default stream; order the slot's stream after them
        slot.stream.wait_stream(torch.cuda.default_stream())
        with torch.cuda.stream(slot.stream):
            h.potential_async(req.n, req.grad, req.v, req.energy)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.busy, slot.event = req, ev

    def poll(self, now: float) -> int:
        """Retire finished requests, then admit waiting ones in arrival order.  Returns the
        number of requests still queued or running."""
        for s in self.slots:
            if s.busy is not None and s.event.query():
                s.busy.finished = now
                self.done.append(s.busy)
                if s.busy.future is not None:
                    s.busy.future.set_result(s.busy)
                s.busy, s.event = None, None
        while self.queue:
            req = self.queue[0]
            free = [s for s in self.slots if s.busy is None]
            if not free:
                break
            # prefer a free slot that already holds a handle for this shape
            key = self._key(req)
            free.sort(key=lambda s: key not in s.handles)
            h = None
            for s in free:
                h = self._handle_for(s, req, free)
                if h is not None:
                    self._start(s, req, h, now)
                    break
            if h is None:
                break
            self.queue.popleft()
        running = sum(1 for s in self.slots if s.busy is not None)
        self.max_concurrent = max(self.max_concurrent, running)
        return len(self.queue) + running

    def run(self, requests, poll_interval: float = 2e-4):
        """Replay `requests` at their arrival times (seconds from now); returns a summary."""
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        i = 0
        while i < len(pending) or self.poll(time.perf_counter() - t0) > 0:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            self.poll(now)
            if i < len(pending) or self.queue or any(s.busy for s in self.slots):
                time.sleep(poll_interval)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if not self.done:
            return {"requests": 0, "rejected": len(self.rejected), "wall_s": wall}
        lat = np.array([r.latency for r in self.done])
        pts = sum(int(np.prod(r.grid)) for r in self.done)
        return {
            "requests": len(self.done),
            "rejected": len(self.rejected),
            "wall_s": wall,
            "req_per_s": len(self.done) / wall,
            "pts_per_s": pts / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_concurrent": self.max_concurrent,
            "peak_resident_bytes": self.peak_resident,
        }

    def close(self):
        for s in self.slots:
            for h in s.handles.values():
                h.close()
            s.handles.clear()
        self.resident = 0.0


def serving_shapes(grids=(48, 64, 96, 128, 160)):
    """The (grid, cell) pairs of the serving workload, for Server.warm."""
    from . import inputs
    out = []
    for g in grids:
        w = inputs.workload("serving", grid_n=int(g))
        out.append((w.grid, w.cell))
    return out


def poisson_requests(count: int, rate: float, seed: int, device="cuda", grids=(48, 64, 96, 128, 160)):
    """The serving workload: Poisson arrivals (mean `rate` per second), grid N uniform over
    `grids`, cell N * 0.15625 Angstrom, 50-400 Slater blobs each; densities and analytic gradients
    generated on the device before the clock starts."""
    from . import inputs
    rng = np.random.default_rng(inputs.SEED_BASE + 300 + seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for i in range(count):
        w = inputs.workload("serving", grid_n=int(rng.choice(grids)), seed_offset=1000 * seed + i)
        n, g = w.density(device=device)
        reqs.append(Request(i, w.grid, w.cell, n, g, arrival=float(t[i])))
    torch.cuda.synchronize()
    return reqs
