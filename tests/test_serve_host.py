"""Host-side logic of the solve server: statistics and the device-memory arena (no GPU)."""
import math

import numpy as np
import pytest

from paper_1711_03540_amd.serve import Arena, Result, ServeStats, instance_bytes


def test_summary_latency_and_queue_fields():
    res = []
    for i in range(100):
        r = Result(i, arrival=0.01 * i)
        r.admitted = r.arrival + 0.001 * (i % 10)
        r.completed = r.admitted + 0.1
        res.append(r)
    unfinished = Result(100, arrival=2.0)       # never completed: left out of latencies
    st = ServeStats(res + [unfinished], wall=2.5, site_updates=5e9, queue_max=7, queue_mean=1.25,
                    active_max=12, arena_peak=1 << 20, arena_bytes=1 << 22)
    s = st.summary()
    lat = np.array([r.completed - r.arrival for r in res]) * 1e3
    assert s["requests"] == 101 and s["completed"] == 100
    assert math.isclose(s["p50_ms"], np.percentile(lat, 50))
    assert math.isclose(s["p99_ms"], np.percentile(lat, 99))
    assert math.isclose(s["queue_wait_p99_ms"], np.percentile([0.001 * (i % 10) * 1e3 for i in range(100)], 99))
    assert s["queue_depth_max"] == 7 and s["queue_depth_mean"] == 1.25
    assert s["active_max"] == 12 and s["arena_peak_bytes"] == 1 << 20 and s["arena_bytes"] == 1 << 22
    assert math.isclose(s["achieved_glups"], 2.0)


def test_request_bytes_follow_the_state_layout():
    # two copies, each Q rows (FP64 / FP32) or a rho row plus Q float rows
    # (split), rows padded to 64 sites, each copy to 256 bytes
    assert instance_bytes(4096, 7, "fp64") == 2 * 7 * 4096 * 8
    assert instance_bytes(256, 5, "fp32") == 2 * 5 * 256 * 4
    assert instance_bytes(1000, 7, "split") == 2 * (1024 * 8 + 7 * 1024 * 4)
    assert instance_bytes(65536, 7, "fp64") == 2 * 7 * 65536 * 8
    with pytest.raises(ValueError):
        instance_bytes(0, 7, "fp64")


def test_arena_first_fit_alignment_and_merging():
    a = Arena(10_000)
    assert a.size == 9984                      # whole 256-byte blocks
    x = a.alloc(1000)                          # 1024 bytes
    y = a.alloc(256)
    z = a.alloc(3000)                          # 3072
    assert (x, y, z) == (0, 1024, 1280)
    assert a.used == 1024 + 256 + 3072 and a.peak == a.used
    assert a.alloc(9984) is None               # no room: the caller waits
    a.release(y, 256)
    assert a.alloc(512) == 4352                # the 256-byte hole is too small: first fit past it
    assert a.alloc(100) == 1024                # ... and a small block takes the hole
    a = Arena(4096)
    blocks = [a.alloc(1024) for _ in range(4)]
    assert blocks == [0, 1024, 2048, 3072] and a.alloc(1) is None
    for off in (1024, 3072, 0, 2048):          # out of order: neighbours merge back into one block
        a.release(off, 1000)
    assert a.used == 0 and a.free_off == [0] and a.free_len == [4096]
    with pytest.raises(ValueError):
        a.release(0, 256)                      # already free


def test_arena_holds_requests_up_to_its_budget():
    # admission by memory: a 4 GiB arena holds every N of the served stream,
    # including sizes beyond 65536 sites
    a = Arena(4 << 30)
    big = instance_bytes(1 << 20, 7, "fp64")
    assert a.alloc(big) == 0 and a.alloc(big) == big
    n_fit = 0
    while a.alloc(instance_bytes(65536, 7, "fp64")) is not None:
        n_fit += 1
    assert n_fit == ((4 << 30) - 2 * big) // instance_bytes(65536, 7, "fp64")


def test_tile_width_follows_load():
    from paper_1711_03540_amd.serve import tile_width
    # D1Q7, 64-step chunks: windows keep 3072 - 384 = 2688 (12 sites per
    # lane), 1664 (8) or 640 (4) sites
    assert tile_width([2688] * 128, 7, (12, 8, 4), 64) == 12
    assert tile_width([2688] * 127, 7, (12, 8, 4), 64) == 8      # 127 x 2 windows at 8 sites
    assert tile_width([1664] * 127, 7, (12, 8, 4), 64) == 4      # 127 x 3 windows at 4 sites
    assert tile_width([65536], 7, (12, 8, 4), 64) == 4           # one large request: the most windows
    assert tile_width([65536] * 6, 7, (12, 8, 4), 64) == 12      # 6 x 25 windows
    # D1Q5 keeps 2 x 2 x 64 = 256 halo sites: 2816 per 12-site window
    assert tile_width([2816] * 128, 5, (12, 8, 4), 64) == 12
    assert tile_width([2817] * 128, 5, (12, 8, 4), 64) == 12     # two tiles each, 278 lanes
    assert tile_width([2817] * 64, 5, (12, 8, 4), 64) == 4       # 69 windows at 12, 104 at 8
    # small requests share windows: 256 sites fill 54 lanes at 12 sites per
    # lane (106 windows for 500 requests) and 80 at 8 (156 windows)
    assert tile_width([256] * 500, 7, (12, 8, 4), 64) == 8
    assert tile_width([256] * 700, 7, (12, 8, 4), 64) == 12
    # FP32 and split classes choose between 8 and 4
    assert tile_width([1664] * 200, 7, (8, 4), 64) == 8
    assert tile_width([100] * 10, 7, (8, 4), 64) == 4
