"""Continuous-batching solve server for KS lattice Boltzmann requests.

Each request asks for one periodic solve: scheme (D1Q5 or D1Q7), size N,
number of steps, precision ("fp64", or "fp32": by default served in the FP32
storage mode, populations in single precision with the density sum and the
rho^2 term in double; optionally in the split mode, rho in double and the
non-equilibrium part in single) and a seed for its initial density.

Admission is by device memory.  The server owns one device arena of
``budget_bytes``; an admitted request gets a block of exactly the bytes its own
state needs (two copies of N sites in its scheme and storage,
``kslb_instance_bytes``), and requests are admitted in arrival order while the
arena has room (the first request that does not fit waits, so large requests
are not starved by smaller ones behind them).  Any N the arena can hold is
accepted.  A block returns to the arena once the request's readout has
completed on the device.

Requests of one (scheme, storage) class run in one libkslb ensemble, on its own
stream, whose instances are descriptors bound to arena blocks
(``kslb_ensemble_bind``).  The server loop admits arrived requests (bind, then
initialise on the device, without synchronising), advances every class by one
round of up to ``round_steps`` steps (the ensemble launches one kernel per chunk
for all of the class's active requests, so requests admitted while others run
share their launches), and retires finished requests: their density is read out
on the class's stream and their completion is observed through an event.  Each
round takes the widest tiling (sites per lane) whose windows over the class's
active requests still fill the device, narrower ones while few requests run.
Classes run on separate streams, so their kernels overlap on the device.  The
per-site arithmetic is the library's, identical for a request alone and in any
mix.
"""
from __future__ import annotations

import bisect
import collections
import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from .ensemble import Ensemble
from .lattice import _prec

ALIGN = 256


def instance_bytes(n: int, q: int, precision) -> int:
    """Device bytes of one request's state (two copies), from the library."""
    b = _lib.fn("kslb_instance_bytes")(int(n), int(q), _prec(precision))
    if b == 0:
        raise ValueError("bad request shape n=%r q=%r precision=%r" % (n, q, precision))
    return int(b)


class Arena:
    """First-fit allocator of 256-byte aligned blocks over ``size`` bytes.

    Host bookkeeping only: offsets into one device buffer.  Free blocks are
    kept sorted by offset and merged with their neighbours on release."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self.free_off: List[int] = [0] if self.size else []
        self.free_len: List[int] = [self.size] if self.size else []
        self.used = 0
        self.peak = 0

    @staticmethod
    def rounded(nbytes: int) -> int:
        return (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN

    def alloc(self, nbytes: int) -> Optional[int]:
        need = self.rounded(nbytes)
        for k, ln in enumerate(self.free_len):
            if ln >= need:
                off = self.free_off[k]
                if ln == need:
                    del self.free_off[k], self.free_len[k]
                else:
                    self.free_off[k] += need
                    self.free_len[k] -= need
                self.used += need
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        ln = self.rounded(nbytes)
        k = bisect.bisect_left(self.free_off, off)
        if k < len(self.free_off) and self.free_off[k] < off + ln:
            raise ValueError("block [%d, %d) overlaps a free block" % (off, off + ln))
        if k > 0 and self.free_off[k - 1] + self.free_len[k - 1] > off:
            raise ValueError("block [%d, %d) overlaps a free block" % (off, off + ln))
        self.free_off.insert(k, off)
        self.free_len.insert(k, ln)
        self.used -= ln
        # merge with the following and the preceding free block
        if k + 1 < len(self.free_off) and self.free_off[k] + self.free_len[k] == self.free_off[k + 1]:
            self.free_len[k] += self.free_len[k + 1]
            del self.free_off[k + 1], self.free_len[k + 1]
        if k > 0 and self.free_off[k - 1] + self.free_len[k - 1] == self.free_off[k]:
            self.free_len[k - 1] += self.free_len[k]
            del self.free_off[k], self.free_len[k]

    def largest_free(self) -> int:
        return max(self.free_len, default=0)


@dataclass
class Result:
    index: int
    arrival: float
    admitted: float = math.nan
    completed: float = math.nan
    rho: Optional[object] = None        # device tensor (float64)
    event: Optional[object] = None
    finite: Optional[bool] = None       # False: the solve produced NaN/inf (retired alone)
    block: Optional[Tuple[int, int]] = None   # (offset, bytes) in the arena while it holds state

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


# Workgroup windows one class's launch should reach before it takes wider
# tiles: wide windows recompute less halo per site (the better throughput
# once the device is full), narrow ones split a few large requests over more
# workgroups (the shorter solve while it is not).
WINDOWS_TARGET = 128
LANES = 256


def tile_width(n, q: int, widths: Sequence[int], chunk: int, target: int = WINDOWS_TARGET) -> int:
    """Sites per lane for a round over requests of n sites: the first (widest)
    of ``widths`` at which the requests' tiles fill at least ``target``
    windows of LANES lanes, else the last.  A request of n sites takes
    ceil(n / valid) tiles of at most valid = LANES * width - 2 max|c| chunk
    sites, each with 2 max|c| chunk halo sites, at width sites per lane;
    small tiles share windows."""
    n = np.asarray(n, dtype=np.int64)
    h = 3 if q == 7 else 2
    for b in widths:
        valid = LANES * b - 2 * h * chunk
        if valid < b:
            continue
        tiles = -(-n // valid)
        lanes = -(-(n + tiles * 2 * h * chunk) // b)
        if int(lanes.sum()) >= target * LANES:
            return b
    return widths[-1]


class _Pool:
    """One (scheme, storage) class: an ensemble of request descriptors on its own stream."""

    def __init__(self, q: int, precision: str, dX: float, dT: float, slots: int, chunk: int, device,
                 tau: float = 0.0):
        import torch
        self.q, self.precision = q, precision
        self.chunk = chunk
        self.widths = {"fp64": (12, 8, 4), "fp32": (10, 8, 4)}.get(precision, (8, 4))
        self.width = None
        self.stream = torch.cuda.Stream(device=device)          # default priority
        # descriptors start bound to one-site placeholders in the ensemble's own buffer
        self.ens = Ensemble([1] * slots, q, precision, device=device, stream=self.stream)
        self.ens.set_physical(dX, dT, tau)
        self.ens.set_tiling(0, 0, chunk)
        self.free = list(range(slots))[::-1]
        self.remaining = np.zeros(slots, dtype=np.int64)
        self.owner: Dict[int, Result] = {}
        self.inflight: collections.deque = collections.deque()
        self.retired: collections.deque = collections.deque()   # readouts in stream order
        self.device = device

    def admit(self, res: Result, n: int, steps: int, rho0, ptr: int, nbytes: int) -> None:
        slot = self.free.pop()
        self.ens.bind(slot, n, ptr, nbytes)
        self.ens.init_rho(slot, rho0)        # device tensor: enqueued, no sync
        self.remaining[slot] = steps
        self.owner[slot] = res

    def pick_width(self) -> None:
        """Sites per lane for the next round: the widest tiling whose windows
        over the active requests reach WINDOWS_TARGET, else the narrowest.
        Every width computes the same bits."""
        width = tile_width(self.ens.n[list(self.owner)], self.q, self.widths, self.chunk)
        if width != self.width:
            self.ens.set_tiling(width, 0, 0)
            self.width = width

    def launch(self, round_steps: int) -> bool:
        import torch
        if not self.owner:
            return False
        self.pick_width()
        adv = np.minimum(self.remaining, round_steps)
        self.ens.advance(adv)
        self.remaining -= adv
        for slot in [s for s in self.owner if self.remaining[s] == 0]:
            res = self.owner.pop(slot)
            out = torch.empty(int(self.ens.n[slot]), dtype=torch.float64, device=self.device)
            self.ens.read_rho(slot, out)
            ev = torch.cuda.Event()
            ev.record(self.stream)
            res.rho, res.event = out, ev
            self.retired.append(res)
            self.free.append(slot)            # the descriptor is rebound at its next admission
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.inflight.append(ev)
        return True


@dataclass
class ServeStats:
    results: List[Result]
    wall: float
    site_updates: float
    queue_max: int = 0          # most requests waiting for admission at once
    queue_mean: float = 0.0     # time-averaged number waiting
    active_max: int = 0         # most requests holding state on the device at once
    arena_peak: int = 0         # most arena bytes held at once
    arena_bytes: int = 0

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results])
        done = np.isfinite(lat)
        lat_ms = lat[done] * 1e3
        wait = np.array([r.admitted - r.arrival for r in self.results])
        wait_ms = wait[np.isfinite(wait)] * 1e3
        pct = lambda a, q: float(np.percentile(a, q)) if a.size else None
        return {"requests": len(self.results), "completed": int(done.sum()),
                "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
                "mean_ms": float(lat_ms.mean()) if done.any() else None,
                "queue_wait_p50_ms": pct(wait_ms, 50), "queue_wait_p99_ms": pct(wait_ms, 99),
                "queue_depth_max": self.queue_max, "queue_depth_mean": self.queue_mean,
                "active_max": self.active_max, "arena_bytes": self.arena_bytes, "arena_peak_bytes": self.arena_peak,
                "wall_s": self.wall, "site_updates": self.site_updates,
                "achieved_glups": self.site_updates / self.wall / 1e9}


class SolveServer:
    """Request classes per (scheme, storage precision), admission by a device-memory budget,
    and the serving loop."""

    def __init__(self, dX: float, dT: float, budget_bytes: int = 4 << 30, slots: int = 2048, chunk: int = 64,
                 round_steps: int = 256, depth: int = 2, device="cuda:0",
                 classes: Optional[Sequence[Tuple[int, str]]] = None,
                 tau: Dict[int, float] = None, fp32_storage: str = "fp32"):
        import torch
        if fp32_storage not in ("fp32", "split"):
            raise ValueError("fp32 requests are served in the fp32 or split storage")
        self.dX, self.dT = dX, dT
        self.round_steps, self.depth = round_steps, depth
        self.device = device
        self.storage = {"fp64": "fp64", "fp32": fp32_storage}     # request precision -> storage mode
        if classes is None:
            classes = [(q, p) for q in (5, 7) for p in ("fp64", fp32_storage)]
        tau = tau or {}
        self.pools = {(q, p): _Pool(q, p, dX, dT, slots, chunk, device, tau.get(q, 0.0))
                      for q, p in classes}
        self.arena = Arena(budget_bytes)
        self.arena_buf = torch.empty(self.arena.size, dtype=torch.uint8, device=device)
        self.base = self.arena_buf.data_ptr()

    def request_bytes(self, r) -> int:
        return instance_bytes(r.n, r.q, self.storage[r.precision])

    def serve(self, requests, initial: Sequence, realtime: bool = True) -> ServeStats:
        """Serve ``requests`` (objects with arrival, q, n, steps, precision) whose initial
        densities ``initial[i]`` are already on the device."""
        import torch
        for r in requests:
            if self.arena.rounded(self.request_bytes(r)) > self.arena.size:
                raise ValueError("a request of %d sites needs more than the arena's %d bytes" % (r.n, self.arena.size))
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        pending = collections.deque(order)
        waiting: collections.deque = collections.deque()          # arrived, not admitted (arrival order)
        results = [Result(i, requests[i].arrival) for i in range(len(requests))]
        unfinished = set(range(len(requests)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: math.inf)
        q_max, q_area, q_last = 0, 0.0, 0.0      # admission queue depth statistics
        active, active_max = 0, 0
        while unfinished:
            now = clock()
            t_now = time.perf_counter() - t0
            q_area += len(waiting) * (t_now - q_last)
            q_last = t_now
            while pending and requests[pending[0]].arrival <= now:
                waiting.append(pending.popleft())
            q_max = max(q_max, len(waiting))
            progressed = False
            # admit in arrival order while memory (and a descriptor of the class) allows
            while waiting:
                i = waiting[0]
                r = requests[i]
                pool = self.pools[(r.q, self.storage[r.precision])]
                if not pool.free:
                    break
                nbytes = self.request_bytes(r)
                off = self.arena.alloc(nbytes)
                if off is None:
                    break
                waiting.popleft()
                results[i].admitted = clock() if realtime else 0.0
                results[i].block = (off, nbytes)
                pool.admit(results[i], r.n, r.steps, initial[i], self.base + off, nbytes)
                active += 1
                active_max = max(active_max, active)
                progressed = True
            for pool in self.pools.values():
                while pool.inflight and pool.inflight[0].query():
                    pool.inflight.popleft()
                if pool.owner and len(pool.inflight) < self.depth:
                    pool.launch(self.round_steps)
                    progressed = True
            for pool in self.pools.values():
                while pool.retired and pool.retired[0].event.query():
                    res = pool.retired.popleft()
                    res.completed = time.perf_counter() - t0
                    self.arena.release(*res.block)     # its readout has run: the memory is free
                    res.block = None
                    active -= 1
                    unfinished.discard(res.index)
                    progressed = True
            if not progressed:
                nxt = [p.inflight[0] for p in self.pools.values() if p.inflight]
                if nxt:
                    time.sleep(20e-6)
                elif pending:
                    dt = requests[pending[0]].arrival - clock()
                    if dt > 0:
                        time.sleep(min(dt, 1e-3))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for res in results:
            if res.rho is not None:
                res.finite = bool(torch.isfinite(res.rho).all().item())
        su = float(sum(r.n * r.steps for r in requests))
        return ServeStats(results, wall, su, q_max, q_area / wall if wall > 0 else 0.0, active_max,
                          self.arena.peak, self.arena.size)
