"""Continuous-batching server for energy + potential requests of mixed grid sizes.

Requests (density n, optional gradient, grid, cell) arrive over time.  The server keeps S slots,
each a HIP stream with one library handle per grid/cell.  Those handles own no work memory (they
hold only their plans and the tables shared between handles), so all of them stay resident.  The
work memory is a pool of buffers in size classes, planned once for the shapes the server is
warmed with and allocated before traffic: within the HBM budget, greedily the largest class that
still fits, at most one buffer per slot.  A request is admitted when a slot is free and a free
buffer of at least its size exists (the smallest such); the buffer is attached to the handle
(`vdwxc_set_workspace`: a pointer change and a flag-clearing kernel on the slot's stream), so
admission never allocates, frees, evicts or synchronises.  Waiting requests are admitted in arrival
order; a later request may start while an earlier one waits only in a buffer smaller than the
waiting request needs, so it never takes the buffer the earlier one waits for.  Admitted requests
run concurrently on their slots' streams; completions are detected with stream events and free
their slot and buffer at once.

Every evaluation is deterministic (fixed-order reductions, no atomics), so a request's (E, v) is
bitwise the same alone or in the mix, whichever buffer it ran in.

A server that is not warmed grows its pool on demand instead (up to one buffer per slot within the
budget, dropping idle buffers into torch's cache when a larger one is needed); that mode allocates
in the scheduler and is meant for tests and ad-hoc use.

`submit` returns a `concurrent.futures.Future` that resolves to the finished Request (its `energy`
and `v` device tensors complete), or fails at once with ValueError when no buffer the budget allows
could hold the request's work memory (it could never be admitted).
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
    buffer: int | None = None
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


@dataclass
class _Buffer:
    index: int
    size: int
    mem: torch.Tensor
    user: Request | None = None


def plan_pool(needs, budget: float, count: int) -> list[int]:
    """Buffer sizes for work memory needs `needs` (bytes) within `budget`: repeatedly the largest
    need that still fits, at most `count` buffers."""
    classes = sorted({int(x) for x in needs}, reverse=True)
    left, out = float(budget), []
    while len(out) < count:
        fit = [c for c in classes if c <= left]
        if not fit:
            break
        out.append(fit[0])
        left -= fit[0]
    return out


class Server:
    """S slots sharing a pool of work buffers of at most `hbm_budget` bytes."""

    def __init__(self, table, slots: int = 4, precision: str = "fp32", flavour: str = "DF1",
                 hbm_budget: float = 64e9):
        self.table = table
        self.precision = precision
        self.flavour = flavour
        self.budget = float(hbm_budget)
        self.slots = [_Slot(i, torch.cuda.Stream()) for i in range(slots)]
        self.buffers: list[_Buffer] = []
        self.frozen = False          # pool planned by warm(): no allocation after it
        self.resident = 0.0
        self.queue: collections.deque = collections.deque()
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.max_concurrent = 0
        self.peak_resident = 0.0

    # ---- memory ------------------------------------------------------------------------------
    def _cost(self, grid) -> int:
        return int(vdwxc.workspace_bytes(grid, self.precision, self.table.nq))

    def _key(self, grid, cell):
        return (tuple(grid), tuple(np.asarray(cell, dtype=np.float64).ravel().round(12)))

    def _add_buffer(self, size: int) -> _Buffer:
        mem = torch.empty(size, dtype=torch.uint8, device="cuda")
        buf = _Buffer(len(self.buffers), size, mem)
        self.buffers.append(buf)
        self.resident += size
        self.peak_resident = max(self.peak_resident, self.resident)
        return buf

    def _grow(self, need: int):
        """Unwarmed pool: a new buffer of `need` bytes if a slot's worth of buffers is not reached
        and the budget allows, dropping idle buffers (smallest first) to make room; else None."""
        if len(self.buffers) >= len(self.slots) and all(b.user is not None for b in self.buffers):
            return None
        idle = sorted((b for b in self.buffers if b.user is None), key=lambda b: b.size)
        free_bytes = self.budget - self.resident
        drop = []
        while (free_bytes < need or len(self.buffers) - len(drop) >= len(self.slots)) and idle:
            b = idle.pop(0)
            drop.append(b)
            free_bytes += b.size
        if free_bytes < need or len(self.buffers) - len(drop) >= len(self.slots):
            return None
        for b in drop:
            self.buffers.remove(b)
            self.resident -= b.size
        for i, b in enumerate(self.buffers):
            b.index = i
            if b.user is not None:
                b.user.buffer = i
        return self._add_buffer(need)

    def _handle(self, slot: _Slot, grid, cell):
        key = self._key(grid, cell)
        h = slot.handles.get(key)
        if h is None:
            with torch.cuda.stream(slot.stream):
                h = vdwxc.Functional(grid, cell, flavour=self.flavour, precision=self.precision, table=self.table,
                                     stream=slot.stream, own_workspace=False)
            slot.handles[key] = h
        return h

    def warm(self, shapes, evaluate: bool = True):
        """Plan and allocate the buffer pool for the (grid, cell) shapes of the expected traffic and
        create every slot's handle for each shape, before traffic.  With `evaluate`, every new
        handle also runs one evaluation of an empty cell (in the largest buffer) and every buffer one
        of the largest shape it holds, so that first-use costs are paid here.  Returns the number of
        handles created."""
        if not self.frozen:
            self.buffers.clear()
            self.resident = 0.0
            for size in plan_pool([self._cost(g) for g, _ in shapes], self.budget, len(self.slots)):
                self._add_buffer(size)
            self.frozen = True
        made = 0
        new = []
        for grid, cell in shapes:
            for slot in self.slots:
                if self._key(grid, cell) not in slot.handles:
                    new.append((slot, self._handle(slot, grid, cell), grid))
                    made += 1
        if evaluate and self.buffers:
            big = max(self.buffers, key=lambda b: b.size)
            runs = [(slot, h, grid, big) for slot, h, grid in new if self._cost(grid) <= big.size]
            for b in self.buffers:
                fits = [(self._cost(g), g, c) for g, c in shapes if self._cost(g) <= b.size]
                if fits and b is not big:
                    _, g, c = max(fits, key=lambda t: t[0])
                    runs.append((self.slots[0], self._handle(self.slots[0], g, c), g, b))
            for slot, h, grid, b in runs:
                n = torch.zeros(tuple(grid), dtype=torch.float64, device="cuda")
                v = torch.empty_like(n)
                e = torch.empty(1, dtype=torch.float64, device="cuda")
                slot.stream.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(slot.stream):
                    h.set_workspace(b.mem)
                    h.potential_async(n, None, v, e)
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        return made

    # ---- scheduling --------------------------------------------------------------------------
    def submit(self, req: Request) -> concurrent.futures.Future:
        """Queue a request; the returned Future resolves to the finished Request."""
        req.future = concurrent.futures.Future()
        need = self._cost(req.grid)
        largest = max([b.size for b in self.buffers], default=0)
        if (self.frozen and need > largest) or need > self.budget:
            req.future.set_exception(ValueError(
                f"request {req.rid}: grid {tuple(req.grid)} needs {need / 1e9:.3f} GB of work memory, more than "
                + (f"the pool's largest buffer ({largest / 1e9:.3f} GB)" if self.frozen else
                   f"the whole budget ({self.budget / 1e9:.3f} GB)")))
            self.rejected.append(req)
            return req.future
        self.queue.append(req)
        return req.future

    def _start(self, slot: _Slot, buf: _Buffer, req: Request, now: float):
        req.admitted = now
        req.slot = slot.index
        req.buffer = buf.index
        req.v = torch.empty_like(req.n)
        req.energy = torch.empty(1, dtype=torch.float64, device=req.n.device)
        h = self._handle(slot, req.grid, req.cell)
        # inputs were produced on the default stream; order the slot's stream after them
        slot.stream.wait_stream(torch.cuda.default_stream())
        with torch.cuda.stream(slot.stream):
            h.set_workspace(buf.mem)
            h.potential_async(req.n, req.grad, req.v, req.energy)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.busy, slot.event = req, ev
        buf.user = req

    def poll(self, now: float) -> int:
        """Retire finished requests, then admit waiting ones.  Returns the number of requests
        still queued or running."""
        for s in self.slots:
            if s.busy is not None and s.event.query():
                req = s.busy
                req.finished = now
                self.done.append(req)
                self.buffers[req.buffer].user = None
                s.busy, s.event = None, None
                if req.future is not None:
                    req.future.set_result(req)
        blocked_need = None   # work memory of the earliest request that is waiting
        kept = collections.deque()
        while self.queue:
            req = self.queue.popleft()
            free_slots = [s for s in self.slots if s.busy is None]
            if not free_slots:
                kept.append(req)
                kept.extend(self.queue)
                self.queue.clear()
                break
            need = self._cost(req.grid)
            cands = [b for b in self.buffers if b.user is None and b.size >= need
                     and (blocked_need is None or b.size < blocked_need)]
            if not cands and not self.frozen and blocked_need is None:
                grown = self._grow(need)
                if grown is not None:
                    cands = [grown]
            if not cands:
                if blocked_need is None:
                    blocked_need = need
                kept.append(req)
                continue
            buf = min(cands, key=lambda b: (b.size, b.index))
            # prefer a free slot that already holds a handle for this shape
            key = self._key(req.grid, req.cell)
            slot = min(free_slots, key=lambda s: (key not in s.handles, s.index))
            self._start(slot, buf, req, now)
        self.queue = kept
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
            "pool_buffer_bytes": [b.size for b in self.buffers],
        }

    def close(self):
        torch.cuda.synchronize()
        for s in self.slots:
            for h in s.handles.values():
                h.close()
            s.handles.clear()
        self.buffers.clear()
        self.frozen = False
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
