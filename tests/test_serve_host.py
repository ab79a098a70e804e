"""Host-side logic of the solve server's statistics (no GPU)."""
import math

import numpy as np

from paper_1711_03540_amd.serve import Result, ServeStats


def test_summary_latency_and_queue_fields():
    res = []
    for i in range(100):
        r = Result(i, arrival=0.01 * i)
        r.admitted = r.arrival + 0.001 * (i % 10)
        r.completed = r.admitted + 0.1
        res.append(r)
    unfinished = Result(100, arrival=2.0)       # never completed: left out of latencies
    st = ServeStats(res + [unfinished], wall=2.5, site_updates=5e9, queue_max=7, queue_mean=1.25)
    s = st.summary()
    lat = np.array([r.completed - r.arrival for r in res]) * 1e3
    assert s["requests"] == 101 and s["completed"] == 100
    assert math.isclose(s["p50_ms"], np.percentile(lat, 50))
    assert math.isclose(s["p99_ms"], np.percentile(lat, 99))
    assert math.isclose(s["queue_wait_p99_ms"], np.percentile([0.001 * (i % 10) * 1e3 for i in range(100)], 99))
    assert s["queue_depth_max"] == 7 and s["queue_depth_mean"] == 1.25
    assert math.isclose(s["achieved_glups"], 2.0)
