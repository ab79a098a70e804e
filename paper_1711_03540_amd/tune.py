"""Autotuner: picks kernel class, steps per launch, sites per lane and windows'
instance packing by timing candidates on the device.

All candidates give bitwise identical results (one shared site update), so the
tuner only compares speed.  Results are cached in a JSON file keyed by the
shape (scheme, precision, size or size histogram).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import inputs
from .ensemble import Ensemble
from .lattice import Lattice

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kslb_tune.json")


def _load(path: str) -> Dict:
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    json.dump(data, open(tmp, "w"), indent=1)
    os.replace(tmp, path)


def _time(fn, reps: int = 3) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_lattice(n: int, q: int = 7, precision: str = "fp64", steps: int = 2000, dX: float = math.pi / 16,
                 dT: float = 1e-4, cache: Optional[str] = DEFAULT_CACHE,
                 tile_steps: Iterable[int] = (0, 16, 32, 48, 64, 80, 96, 112),
                 span_steps: Iterable[int] = (0, 12, 18, 24)) -> Dict:
    """Best (kernel, steps_per_launch) for one periodic lattice of n sites
    (steps_per_launch is the exchange interval for SPAN; 0 = the library's
    default for the class)."""
    key = "lattice/q%d/%s/n%d" % (q, precision, n)
    data = _load(cache) if cache else {}
    if key in data:
        return data[key]
    rho0 = inputs.random_modes_ic(n, n * dX, seed=1)
    cands: List[Dict] = []
    lat = Lattice(n, q, precision).set_physical(dX, dT, 0.0)
    lat.init_rho(rho0)
    options = [("span", s) for s in span_steps] + [("resident", 0)] + [("tiled", s) for s in tile_steps]
    for kind, s in options:
        try:
            lat.set_kernel(kind, s)
        except Exception:
            continue
        aborted = lat.aborted_launches()
        t = _time(lambda: lat.advance(steps))
        if lat.aborted_launches() != aborted:
            # a multi-workgroup launch stopped early: its time is not a solve's
            lat.init_rho(rho0)
            continue
        cands.append({"kernel": kind, "steps_per_launch": s, "glups": n * steps / t / 1e9})
    best = max(cands, key=lambda c: c["glups"])
    out = {"best": best, "candidates": cands}
    if cache:
        data = _load(cache)
        data[key] = out
        _save(cache, data)
    return out


def tune_ensemble(sizes: Sequence[int], q: int = 7, precision: str = "fp64", steps: int = 512,
                  dX: float = math.pi / 16, dT: float = 1e-4, cache: Optional[str] = DEFAULT_CACHE,
                  sites_per_lane: Optional[Iterable[int]] = None,
                  chunks: Iterable[int] = (16, 24, 32, 40, 48, 64),
                  segments: Iterable[int] = (1, 4, 16, 64)) -> Dict:
    """Best (sites per lane, steps per chunk, tiles per window) for a ragged ensemble.
    sites_per_lane defaults to 12, 8 and 4 for FP64 storage, 10, 8 and 4 for FP32, 8
    and 4 otherwise."""
    if sites_per_lane is None:
        sites_per_lane = {"fp64": (12, 8, 4), "fp32": (10, 8, 4)}.get(precision, (8, 4))
    sizes = np.asarray(sizes, dtype=np.int64)
    hist = np.histogram(np.log2(sizes), bins=8, range=(0, 24))[0]
    key = "ensemble/q%d/%s/count%d/%s" % (q, precision, sizes.size, ",".join(map(str, hist)))
    data = _load(cache) if cache else {}
    if key in data:
        return data[key]
    ens = Ensemble(sizes, q, precision).set_physical(dX, dT, 0.0)
    for i, n in enumerate(sizes):
        ens.init_rho(i, inputs.random_modes_ic(int(n), int(n) * dX, seed=1000 + i))
    su = float(sizes.sum()) * steps
    cands: List[Dict] = []
    for B in sites_per_lane:
        for c in chunks:
            for m in segments:
                try:
                    ens.set_tiling(B, m, c)
                except Exception:
                    continue
                t = _time(lambda: ens.advance(np.full(sizes.size, steps)), reps=2)
                cands.append({"sites_per_lane": B, "steps_per_chunk": c, "max_segments": m,
                              "glups": su / t / 1e9})
    best = max(cands, key=lambda c: c["glups"])
    out = {"best": best, "candidates": cands}
    if cache:
        data = _load(cache)
        data[key] = out
        _save(cache, data)
    return out


def apply_ensemble(ens: Ensemble, tuned: Dict) -> Ensemble:
    b = tuned["best"]
    return ens.set_tiling(b["sites_per_lane"], b["max_segments"], b["steps_per_chunk"])


def apply_lattice(lat: Lattice, tuned: Dict) -> Lattice:
    b = tuned["best"]
    return lat.set_kernel(b["kernel"], b["steps_per_launch"])
