"""Continuous-batching solve server for KS lattice Boltzmann requests.

Each request asks for one periodic solve: scheme (D1Q5 or D1Q7), size N,
number of steps, precision ("fp64", or "fp32": by default served in the FP32
storage mode, populations in single precision with the density sum and the
rho^2 term in double; optionally in the split mode, rho in double and the
non-equilibrium part in single) and a seed for its initial density.
Requests of one (scheme, precision) class share a slot pool: one libkslb
ensemble whose instances are slots of a fixed capacity, on its own stream.

The server loop admits arrived requests into free slots (an admission resizes
the slot and initialises it on the device, without synchronising), advances
every pool by one round of up to `round_steps` steps (the ensemble launches one
kernel per chunk for all of the pool's active slots, so requests admitted
while others run share their launches), and retires finished requests: their
density is read out on the pool's stream and their completion is observed
through an event.  A slot is reused as soon as its readout is enqueued (stream
order protects it).  Pools run on separate streams, so their kernels overlap
on the device.  The per-site arithmetic is the library's, identical for a
request alone and in any mix.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .ensemble import Ensemble



@dataclass
class Result:
    index: int
    arrival: float
    admitted: float = math.nan
    completed: float = math.nan
    rho: Optional[object] = None        # device tensor (float64)
    event: Optional[object] = None
    finite: Optional[bool] = None       # False: the solve produced NaN/inf (retired alone)

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class _Pool:
    def __init__(self, q: int, precision: str, dX: float, dT: float, slots: int, capacity: int, chunk: int,
                 device, tau: float = 0.0):
        import torch
        self.q, self.precision = q, precision
        self.stream = torch.cuda.Stream(device=device)          # default priority
        self.ens = Ensemble([capacity] * slots, q, precision, device=device, stream=self.stream)
        self.ens.set_physical(dX, dT, tau)
        self.ens.set_tiling(0, 0, chunk)
        self.capacity = capacity
        self.free = list(range(slots))[::-1]
        self.remaining = np.zeros(slots, dtype=np.int64)
        self.owner: Dict[int, Result] = {}
        self.inflight: collections.deque = collections.deque()
        self.retired: collections.deque = collections.deque()   # readouts in stream order
        self.device = device

    def admit(self, res: Result, n: int, steps: int, rho0) -> None:
        slot = self.free.pop()
        self.ens.resize(slot, n)
        self.ens.init_rho(slot, rho0)        # device tensor: enqueued, no sync
        self.remaining[slot] = steps
        self.owner[slot] = res

    def launch(self, round_steps: int) -> bool:
        import torch
        if not self.owner:
            return False
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
            self.free.append(slot)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.inflight.append(ev)
        return True


@dataclass
class ServeStats:
    results: List[Result]
    wall: float
    site_updates: float
    queue_max: int = 0          # most requests waiting for a slot at once
    queue_mean: float = 0.0     # time-averaged number waiting

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
                "wall_s": self.wall, "site_updates": self.site_updates,
                "achieved_glups": self.site_updates / self.wall / 1e9}


class SolveServer:
    """Slot pools per (scheme, storage precision) class and the serving loop."""

    def __init__(self, dX: float, dT: float, slots: int = 256, capacity: int = 65536, chunk: int = 64,
                 round_steps: int = 256, depth: int = 2, device="cuda:0",
                 classes: Optional[Sequence[Tuple[int, str]]] = None,
                 tau: Dict[int, float] = None, fp32_storage: str = "fp32"):
        if fp32_storage not in ("fp32", "split"):
            raise ValueError("fp32 requests are served in the fp32 or split storage")
        self.dX, self.dT = dX, dT
        self.round_steps, self.depth = round_steps, depth
        self.device = device
        self.storage = {"fp64": "fp64", "fp32": fp32_storage}     # request precision -> storage mode
        if classes is None:
            classes = [(q, p) for q in (5, 7) for p in ("fp64", fp32_storage)]
        tau = tau or {}
        self.pools = {(q, p): _Pool(q, p, dX, dT, slots, capacity, chunk, device, tau.get(q, 0.0))
                      for q, p in classes}

    def serve(self, requests, initial: Sequence, realtime: bool = True) -> ServeStats:
        """Serve ``requests`` (objects with arrival, q, n, steps, precision) whose initial
        densities ``initial[i]`` are already on the device."""
        import torch
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        pending = collections.deque(order)
        waiting: Dict[Tuple[int, str], collections.deque] = {k: collections.deque() for k in self.pools}
        results = [Result(i, requests[i].arrival) for i in range(len(requests))]
        unfinished = set(range(len(requests)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: math.inf)
        q_max, q_area, q_last = 0, 0.0, 0.0      # admission queue depth statistics
        while unfinished:
            now = clock()
            t_now = time.perf_counter() - t0
            depth = sum(len(w) for w in waiting.values())
            q_area += depth * (t_now - q_last)
            q_last = t_now
            while pending and requests[pending[0]].arrival <= now:
                i = pending.popleft()
                r = requests[i]
                waiting[(r.q, self.storage[r.precision])].append(i)
            q_max = max(q_max, sum(len(w) for w in waiting.values()))
            progressed = False
            for key, pool in self.pools.items():
                w = waiting[key]
                while w and pool.free:
                    i = w.popleft()
                    r = requests[i]
                    results[i].admitted = clock() if realtime else 0.0
                    pool.admit(results[i], r.n, r.steps, initial[i])
                    progressed = True
                while pool.inflight and pool.inflight[0].query():
                    pool.inflight.popleft()
                if pool.owner and len(pool.inflight) < self.depth:
                    pool.launch(self.round_steps)
                    progressed = True
            for pool in self.pools.values():
                while pool.retired and pool.retired[0].event.query():
                    res = pool.retired.popleft()
                    res.completed = time.perf_counter() - t0
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
        return ServeStats(results, wall, su, q_max, q_area / wall if wall > 0 else 0.0)
