"""Benchmark of the KS lattice Boltzmann hot path on one MI355X.

Default run: the largest single-GPU configuration, one D1Q7 lattice (the
paper's improved scheme) of N = 2^24 periodic sites on L = 32 pi 2^12
(dX = pi/128), 16 random Fourier modes of amplitude 0.1, dT = 2e-8, tau = 1,
FP64, 10^3 LB steps per solve on the halo-tiled kernel.  One benchmark step is
one whole solve: equilibrium init from a density already resident in HBM, the
LB steps, and the density readout into HBM.

The one JSON line also carries, for that lattice, the one-step (s = 1) kernel
and its fraction of the HBM roofline, the measured device peaks (a STREAM copy
and an LDS read microbenchmark) and the FP64 CPU oracle timed on a bounded
sample; and, as sub-objects under "configs", the other configurations, each
with its throughput, latency, roofline and CPU-oracle baseline: D1Q5 N = 256
and D1Q7 N = 4096 single lattices (the multi-workgroup kernel), the ragged
4096-instance ensemble in FP64 and FP32, and the served request stream at
2000 requests/s with a sweep of offered loads.

Other --workload values print their own JSON: a single configuration, or one
of the studies (table3, taumin, profiles, stats, lyapunov, lyapunov_spectrum,
serve_sweep).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GLUPS vs plain kernel at matched error; % HBM/LDS peak; p50/p99 solve latency"

# Published MI355X peaks.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6
N_CU = 256
N_SIMD = 4 * N_CU
CLOCK_GHZ = 2.4
TARGET_HBM_FRAC = 0.70      # the one-step kernel on the large lattice


# Algorithmic flops and FP64 instructions of one site update (an FMA counts 2
# flops and one instruction).  Population storage: density Q-1 adds; rho^2
# 1 mul; A_i rho 1 mul for c = 0 and one per +-c pair (A is even in c); one
# FMA per population with G != 0 (c = +-1, +-2) for G_i rho^2 + A_i rho; one
# FMA per population for (1 - omega) g_i + feq_i.  D1Q7: 6 adds + 5 muls +
# 11 FMAs = 22 instructions, 33 flops; D1Q5: 4 + 4 + 9 = 17, 26.  Rho-only
# storage (tau = 1, post-collision populations feq(rho)): each site's outgoing
# populations A_i rho + B_i rho^2 from its density (rho^2, A_0 rho and one
# A rho per pair, 4 FMAs), then the density sum over the Q incoming ones:
# D1Q7 1 + 4 + 4 + 6 = 15 instructions, 19 flops; D1Q5 1 + 3 + 4 + 4 = 12, 16.
# The conversions the FP32 and split storages add are not counted: they are
# overhead of the storage, not of the method.
def flops_per_site_update(q: int, precision: str = "fp64") -> int:
    if precision == "rho":
        return {7: 19, 5: 16}[q]
    return {7: 33, 5: 26}[q]


def valu_per_site_update(q: int, precision: str = "fp64") -> int:
    if precision == "rho":
        return {7: 15, 5: 12}[q]
    return {7: 22, 5: 17}[q]


# The ALU roofline of the path.  A wave64 FP64 instruction issues in 4 clocks
# on a 16-lane SIMD (64 FP64 lanes per CU per clock; the published 78.6 TFLOP/s
# counts every instruction as an FMA), so 1024 SIMDs x 16 lanes x 2.4 GHz /
# 22 = 1.79e12 D1Q7 updates/s is the issue ceiling, or 1024 x 16 x 2.4e9 x 33 /
# 22 = 59.0 TFLOP/s of the update's own flops.
def valu_ceiling_glups(q: int, simds: int = N_SIMD, precision: str = "fp64") -> float:
    return simds * CLOCK_GHZ * 16.0 / valu_per_site_update(q, precision)


def alu_peak_tflops(q: int, precision: str = "fp64", simds: int = N_SIMD) -> float:
    return valu_ceiling_glups(q, simds, precision) * flops_per_site_update(q, precision) / 1e3


ALU_PEAK_BASIS = ("FP64 VALU issue ceiling from unit counts and clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, "
                  "at the update's own flops per FP64 instruction (D1Q7 33 / 22, D1Q5 26 / 17, rho-only 19 / 15 "
                  "and 16 / 12); frac_of_published_fp64_peak is against 78.6 TFLOP/s, which counts every "
                  "instruction as an FMA")


# Algorithmic HBM bytes of one s = 1 step per site: read Q populations and
# write Q populations of the storage format.
def bytes_per_site_update(q: int, precision: str) -> int:
    return {"fp64": 2 * q * 8, "fp32": 2 * q * 4, "split": 2 * (8 + q * 4), "rho": 2 * 8}[precision]


# Algorithmic HBM bytes per site of one launch of a tiled solve, averaged over
# its `launches` launches: each reads and writes the state once, except that
# the first reads the initial density (8 B) instead of the state and the last
# also writes the density (8 B).
def solve_bytes_per_site_launch(q: int, precision: str, launches: int) -> float:
    full = bytes_per_site_update(q, precision)
    return (launches * full - (full // 2 - 8) + 8) / launches


WORKLOADS = {
    "all": (None, None),
    "d1q7_n16m": ("CFG_LARGE_Q7", "tiled"),
    "d1q7_n4096": ("CFG_RESIDENT_Q7", "span"),
    "d1q5_n256": ("CFG_SMALL_Q5", "span"),
    "ensemble": (None, None),
    "serve": (None, None),
    "serve_sweep": (None, None),
    "table3": (None, None),
    "stats": (None, None),
    "taumin": (None, None),
    "lyapunov": (None, None),
    "profiles": (None, None),
    "lyapunov_spectrum": (None, None),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed solves of the headline lattice (p50/p99 over them)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed solves")
    ap.add_argument("--workload", default="all", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "split", "rho"])
    ap.add_argument("--kernel", default=None, choices=["span", "resident", "tiled", "plain"])
    ap.add_argument("--tile-steps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the kernel class and steps per launch (lattice workloads) or the ensemble "
                         "tiling with the autotuner before timing (no cache)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the device-peak microbenchmarks")
    ap.add_argument("--instances", type=int, default=4096, help="ensemble workload: instances")
    ap.add_argument("--lb-steps", type=int, default=20000, help="ensemble workload: LB steps per instance")
    ap.add_argument("--chunk", type=int, default=0, help="ensemble/serve: steps per launch (0 = default)")
    ap.add_argument("--segments", type=int, default=0, help="ensemble: instance tiles per window (0 = default)")
    ap.add_argument("--requests", type=int, default=2000, help="serve workload: requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve workload: offered requests per second")
    ap.add_argument("--rates", default="250,500,1000,2000", help="serve_sweep: offered requests per second")
    ap.add_argument("--sweep-requests", type=int, default=1000, help="serve_sweep: requests per offered load")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serve: device-memory budget of admitted state")
    ap.add_argument("--round-steps", type=int, default=0, help="serve workload: steps per scheduling round (0 = default)")
    ap.add_argument("--serve-fp32", default="fp32", choices=["fp32", "split"],
                    help="serve workload: storage of the FP32 requests")
    ap.add_argument("--stats-t", type=int, default=1000, help="stats workload: final time T")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (reference kernel for HBM counters)")
    return ap.parse_args()


def log(msg: str) -> None:
    print("bench: " + msg, file=sys.stderr, flush=True)


def calibrate_copy():
    """A plain device-to-device copy of known size, to scale HBM byte counters."""
    import torch
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": 3}), flush=True)


KERNEL_SOURCE = os.path.join(ROOT, "paper_1711_03540_amd", "csrc", "kslb_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(kname: str, workload: str, precision: str, launch: dict = None):
    """HBM bytes per dispatch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs
    (scaled by the copy calibration); None when absent, when the kernel source
    changed since the counters were taken, or when this run's launch shape
    (steps per launch, workgroups; an ensemble's tiling) differs from the
    counted one."""
    import hashlib
    try:
        data = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    e = data.get("entries", {}).get("%s/%s/%s" % (kname, workload, precision))
    if not e or e.get("kernel_source_sha256") != sha:
        return None
    if launch is not None and any(launch.get(k) != v for k, v in e.get("launch", {}).items()):
        return None
    return e["fetch_bytes"] + e["write_bytes"]


# ---------------------------------------------------------------- CPU oracle baselines

def host_info() -> dict:
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_threads() -> int:
    """Worker threads for the multi-instance oracle legs: the host's cores, at
    most 16 (one GPU's share of a GPU host)."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_lattice(w, tau, budget_s: float = 10.0):
    """The FP64 CPU oracle on one lattice of the workload (single thread): the full
    solve, or its first steps when that would take longer than about budget_s."""
    import numpy as np

    import oracle
    rho0 = w.rho0()
    steps = w.steps
    sample = "one full solve: %d sites x %d steps" % (w.n, steps)
    est_rate = 6e7                             # site updates per second of one core (planning figure)
    if w.n * steps > budget_s * est_rate:
        steps = max(1, int(budget_s * est_rate // w.n))
        sample = "%d sites x the first %d of %d steps" % (w.n, steps, w.steps)
    times = []
    while len(times) < 5 and sum(times) < budget_s:
        t0 = time.perf_counter()
        oracle.solve_periodic(w.q, rho0, w.dX, w.dT, tau, steps)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    return {"value": w.n * steps / dt / 1e9, "unit": "GLUPS", "cores": 1, "kind": "oracle",
            "sample": sample + ", plain C FP64 oracle, median of %d trials: %.2f s (initialisation included)"
            % (len(times), dt), "trials_s": times, "host": host_info()}


def cpu_many(jobs, budget_s: float = 10.0):
    """The FP64 CPU oracle on independent solves (q, rho0, dX, dT, tau, steps),
    spread over cpu_threads() threads (the oracle releases the interpreter while
    it runs); the steps of every job are scaled down together when the whole
    sample would take longer than about budget_s.  Returns the rate and the
    scale applied."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    threads = cpu_threads()
    su = sum(len(j[1]) * j[5] for j in jobs)
    est = su / (6e7 * threads)
    scale = min(1.0, budget_s / est) if est > 0 else 1.0
    jobs = [(q, r, dX, dT, tau, max(1, int(steps * scale))) for q, r, dX, dT, tau, steps in jobs]
    su = sum(len(j[1]) * j[5] for j in jobs)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        list(pool.map(lambda j: oracle.solve_periodic(j[0], j[1], j[2], j[3], j[4], j[5]), jobs))
    dt = time.perf_counter() - t0
    return {"value": su / dt / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle", "seconds": dt,
            "site_updates": su, "step_scale": scale, "host": host_info()}


# ---------------------------------------------------------------- device peaks

def device_peaks() -> dict:
    """Measured HBM copy bandwidth and LDS read bytes per clock per CU
    (libkslb_probe), beside the published figures."""
    from paper_1711_03540_amd import probe
    hbm = probe.hbm_copy(4 << 30, reps=10)
    lds = probe.lds_bandwidth()
    log("peaks: copy %.0f GB/s, LDS %.1f B/clk/CU at %.2f GHz" %
        (hbm["best_gb_s"], lds["bytes_per_clk_per_cu"], lds["shader_ghz"]))
    return {"hbm_copy": hbm, "hbm_published_gb_s": PEAK_HBM_GBS, "lds": lds,
            "fp64_vector_published_tflops": PEAK_FP64_VECTOR_TFLOPS}


# ---------------------------------------------------------------- one lattice

def run_lattice(w, precision, kernel, solves, warmup, tile_steps=0, autotune=False, plain=True, cpu=True,
                peaks=None):
    """Time `solves` whole solves of one lattice (init from rho0 in HBM, w.steps LB
    steps, readout into HBM) and describe the dominant kernel against its roofline."""
    import numpy as np
    import torch

    from paper_1711_03540_amd.lattice import Lattice

    dev = torch.device("cuda:0")
    log("workload %s q=%d n=%d steps/solve=%d precision=%s kernel=%s" %
        (w.name, w.q, w.n, w.steps, precision, kernel))
    rho0 = torch.tensor(w.rho0(), dtype=torch.float64, device=dev)
    rho_out = torch.empty(w.n, dtype=torch.float64, device=dev)
    lat = Lattice(w.n, w.q, precision, device=dev)
    lat.set_physical(w.dX, w.dT, 0.0)
    lat.set_kernel(kernel, tile_steps)
    tuned = None
    if autotune:
        from paper_1711_03540_amd import tune
        tuned = tune.tune_lattice(w.n, w.q, precision, steps=min(w.steps, 2000), dX=w.dX, dT=w.dT, cache=None)
        tune.apply_lattice(lat, tuned)
        kernel = tuned["best"]["kernel"]
        log("autotuned %s" % tuned["best"])
    tau = lat.coefficients()["tau"]
    stream = lat.stream

    # one solve: kslb_solve (init from rho0, the steps, readout into rho_out;
    # on the tiled kernel the first and last launches carry the init and the
    # readout); the events bracket its launches
    def solve(ev=None):
        if ev is not None:
            ev[0].record(stream)
        lat.solve(rho0, w.steps, rho_out)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    aborted0 = lat.aborted_launches()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(solves)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(solves)]
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(solves)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(solves):
        starts[k].record(stream)
        solve(kev[k])
        ends[k].record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # every timed solve must have run to completion: no multi-workgroup launch
    # may have stopped early, and the last readout must be finite
    if lat.aborted_launches() != aborted0:
        raise SystemExit("bench: a multi-workgroup launch stopped early during the timed solves")
    if not bool(torch.isfinite(rho_out).all()):
        raise SystemExit("bench: non-finite density")
    lat_ms = np.array([starts[k].elapsed_time(ends[k]) for k in range(solves)])
    adv_ms = np.array([kev[k][0].elapsed_time(kev[k][1]) for k in range(solves)])
    site_updates = w.n * w.steps
    value = site_updates * solves / total / 1e9
    mass, bad = lat.diagnostics()
    if bad:
        raise SystemExit("bench: non-finite state")

    # launches per advance and the dominant kernel's average duration, from
    # the launch shape the library resolved for this lattice
    shape = lat.kernel()
    assert shape["kernel"] == kernel, shape
    launches = math.ceil(w.steps / shape["steps_per_launch"])
    units = w.n * w.steps / launches
    kname = {"resident": "k_ring", "span": "k_span", "tiled": "k_tile", "plain": "k_plain"}[kernel]
    kernel_ms = float(np.mean(adv_ms)) / launches
    if kernel == "plain":
        ach = bytes_per_site_update(w.q, precision) * units / (kernel_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": None}
    else:
        ach = flops_per_site_update(w.q, precision) * units / (kernel_ms * 1e-3) / 1e12
        peak = alu_peak_tflops(w.q, precision)
        roof = {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": None, "peak_basis": ALU_PEAK_BASIS,
                "frac_of_published_fp64_peak": ach / PEAK_FP64_VECTOR_TFLOPS}
        glups_kernel = units / (kernel_ms * 1e-3) / 1e9
        roof["valu_ceiling_glups"] = valu_ceiling_glups(w.q, precision=precision)
        if kernel in ("resident", "span"):
            # execution resources the launch can use: one workgroup of 8 waves
            # on one CU (4 SIMDs) for resident; one single-wave owner per SIMD
            # for span
            simds = 4 if kernel == "resident" else shape["workgroups"]
            if kernel == "span":
                roof["steps_between_exchanges"] = shape["exchange_steps"]
                roof["workgroups"] = simds
            roof["simds_used"] = simds
            roof["frac_of_used_simds"] = ach / alu_peak_tflops(w.q, precision, simds)
            roof["ns_per_step"] = kernel_ms * 1e6 / (w.steps / launches)
    if kernel == "tiled" and peaks:
        # the tile engine trades 12 (D1Q7) or 6 (D1Q5) populations per lane and
        # step through LDS (the rho-only state 2 H densities), each written once
        # and read once: 2 x 8 x 12 / 12 = 16 B per computed site update of 12
        # sites per lane (FP64), against the measured LDS read peak.  Sites per
        # lane from the launch: workgroups = ceil(N / (256 B - 2 H s)).
        hh = 3 if w.q == 7 else 2
        vals = 2 * hh if precision == "rho" else {7: 12, 5: 6}[w.q]
        per_lane = vals * (4 if precision == "fp32" else 8) * 2
        s_l = shape["steps_per_launch"]
        b_est = (w.n / shape["workgroups"] + 2 * hh * s_l) / 256.0
        sites = int(round(b_est))
        assert abs(b_est - sites) < 0.05 and -(-w.n // (256 * sites - 2 * hh * s_l)) == shape["workgroups"], shape
        win = 256 * sites
        valid = win - 2 * hh * s_l
        roof["sites_per_lane"] = sites
        lds_b = per_lane / sites * units * win / valid
        lp = peaks["lds"]["bytes_per_clk_per_cu"] * N_CU * peaks["lds"]["shader_ghz"] * 1e9
        roof["lds_bytes_per_launch"] = lds_b
        roof["lds_achieved_gb_s"] = lds_b / (kernel_ms * 1e-3) / 1e9
        roof["lds_frac_of_measured_peak"] = lds_b / (kernel_ms * 1e-3) / lp
    roof["traffic"] = measured_traffic(kname, w.name, precision,
                                       {k: shape[k] for k in ("steps_per_launch", "exchange_steps", "workgroups")})
    roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["traffic_algorithmic"] = (solve_bytes_per_site_launch(w.q, precision, launches) if kernel == "tiled"
                                   else bytes_per_site_update(w.q, precision)) * w.n
    roof["kernel"] = kname
    roof["launch_shape"] = shape
    roof["kernel_ms_avg"] = kernel_ms
    roof["algorithmic_per_site_update"] = (flops_per_site_update(w.q, precision) if kernel != "plain"
                                           else bytes_per_site_update(w.q, precision))
    roof["units_per_launch"] = units

    out = {
        "value": value, "unit": "GLUPS", "solves": solves, "warmup": warmup,
        "ms_per_solve": total / solves * 1e3,
        "config": {"workload": w.name, "scheme": "D1Q%d" % w.q, "n_sites": w.n, "lb_steps_per_solve": w.steps,
                   "dX": w.dX, "dT": w.dT, "tau": tau, "precision": precision, "kernel": kernel, "instances": 1},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "min": float(lat_ms.min())},
        "roofline": roof,
        "autotuned": tuned["best"] if tuned else None,
    }
    if plain and kernel != "plain":
        # plain one-step-per-launch kernel on the same lattice; bitwise identical results
        chk = min(w.steps, 2000 if w.n < (1 << 20) else 130)
        ref = Lattice(w.n, w.q, precision, device=dev).set_physical(w.dX, w.dT, 0.0).set_kernel("plain")
        ref.init_rho(rho0).advance(chk)
        lat.init_rho(rho0).advance(chk)
        same = bool(torch.equal(ref.save_state(), lat.save_state()))
        psteps = min(w.steps, 5000 if w.n < (1 << 20) else 200)
        ref.advance(psteps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ref.stream)
        ref.advance(psteps)
        e1.record(ref.stream)
        torch.cuda.synchronize()
        pg = w.n * psteps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        hbm = pg * bytes_per_site_update(w.q, precision)     # GB/s, algorithmic bytes
        pk = {"kernel": "k_plain", "glups": pg, "timed_lb_steps": psteps, "speedup": value / pg,
              "bitwise_identical_state_after_%d_steps" % chk: same,
              "hbm_gb_s": hbm, "hbm_frac": hbm / PEAK_HBM_GBS}
        rs = ref.kernel()
        pk["traffic"] = measured_traffic("k_plain", w.name, precision,
                                         {k: rs[k] for k in ("steps_per_launch", "exchange_steps", "workgroups")})
        pk["traffic_algorithmic"] = bytes_per_site_update(w.q, precision) * w.n
        if w.n >= (1 << 20):
            pk["hbm_frac_target"] = TARGET_HBM_FRAC
            pk["meets_target"] = hbm / PEAK_HBM_GBS >= TARGET_HBM_FRAC
            if peaks:
                pk["hbm_frac_of_measured_copy"] = hbm / peaks["hbm_copy"]["best_gb_s"]
        out["plain_kernel"] = pk
        ref.close()
        del ref
    # the one-step HBM roofline (2 Q b bytes per site update at 8 TB/s) that
    # temporal blocking lifts the solve above
    s1 = PEAK_HBM_GBS / bytes_per_site_update(w.q, precision)
    out["s1_hbm_roofline_glups"] = s1
    out["vs_s1_hbm_roofline"] = value / s1
    lat.close()
    del lat
    torch.cuda.synchronize()
    if cpu:
        out["cpu_baseline"] = cpu_lattice(w, tau)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    return out


# ---------------------------------------------------------------- ragged ensemble

def run_ensemble(precision, instances, lb_steps, solves=3, warmup=1, chunk=0, segments=0, autotune=False,
                 cpu=True):
    """Ragged ensemble: D1Q7 instances, N log-uniform in [512, 8192], dX = pi/16,
    dT = 1e-4, fitted tau, lb_steps steps each; one solve = batched init from
    densities in HBM, the steps, batched density readout into HBM; throughput
    against the plain one-step kernel on one instance of the mean size."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.ensemble import Ensemble
    from paper_1711_03540_amd.lattice import Lattice

    dev = torch.device("cuda:0")
    sizes = inputs.ensemble_shapes(instances, seed=2)
    dX, dT = math.pi / 16, 1e-4
    log("ensemble %d instances %s, %d steps" % (instances, precision, lb_steps))
    ens = Ensemble(sizes, 7, precision, device=dev).set_physical(dX, dT, 0.0)
    ens.set_tiling(0, segments, chunk)
    tuned = None
    if autotune:
        from paper_1711_03540_amd import tune
        tuned = tune.tune_ensemble(sizes, 7, precision, cache=None)
        tune.apply_ensemble(ens, tuned)
        log("autotuned ensemble tiling %s" % tuned["best"])
    tiling = ens.tiling()
    ics = [inputs.random_modes_ic(int(n), n * dX, seed=1000 + i) for i, n in enumerate(sizes)]
    rho_all = torch.tensor(np.concatenate(ics), device=dev)       # every instance's density, in HBM
    rho_out = torch.empty_like(rho_all)
    steps = np.full(len(sizes), lb_steps, dtype=np.int64)
    su = float(np.sum(sizes)) * lb_steps
    stream = ens.stream

    def solve():
        ens.init_rho_all(rho_all)       # one init launch for the whole ensemble
        ens.advance(steps)
        ens.rho_all(rho_out)            # one readout launch, into HBM

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(solves)]
    t0 = time.perf_counter()
    for k in range(solves):
        ev[k][0].record(stream)
        solve()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    if not bool(torch.isfinite(rho_out).all()):
        raise SystemExit("bench: non-finite ensemble density")
    sol_ms = np.array([a.elapsed_time(b) for a, b in ev])
    value = su * solves / total / 1e9
    tau = ens.tau
    # reduced storage: error of the smallest, median and largest instance
    # after the last solve against the same instances in GPU FP64 (norm-wise,
    # max |rho - rho_64| / max |rho_64|; FP64 itself is pinned to the oracle
    # by the parity tests)
    errors = None
    if precision != "fp64":
        order = np.argsort(sizes, kind="stable")
        pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
        ref = Ensemble([int(sizes[i]) for i in pick], 7, "fp64", device=dev).set_physical(dX, dT, 0.0)
        for k, i in enumerate(pick):
            ref.init_rho(k, torch.tensor(ics[i], device=dev))
        ref.advance(lb_steps)
        errors = {}
        out_host = rho_out.cpu().numpy()
        offs = np.concatenate([[0], np.cumsum(sizes)])
        for tag, k, i in zip(("smallest", "median", "largest"), range(3), pick):
            r64, got = ref.rho(k), out_host[offs[i]:offs[i + 1]]
            errors[tag] = {"instance": i, "n": int(sizes[i]),
                           "rel_err_vs_gpu_fp64": float(np.max(np.abs(got - r64)) / np.max(np.abs(r64)))}
        ref.close()
    # plain one-step kernel, one instance of the mean size (bitwise-identical arithmetic)
    nm = int(np.mean(sizes))
    lat = Lattice(nm, 7, precision, device=dev).set_physical(dX, dT, 0.0).set_kernel("plain")
    lat.init_rho(inputs.random_modes_ic(nm, nm * dX, seed=7)).advance(200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.advance(2000)
    torch.cuda.synchronize()
    plain = nm * 2000 / (time.perf_counter() - t0) / 1e9
    lat.close()
    fl = flops_per_site_update(7, precision)
    ach = fl * su / (float(np.mean(sol_ms)) * 1e-3) / 1e12
    peak = alu_peak_tflops(7, precision)
    out = {"workload": "ensemble_d1q7_%d" % len(sizes), "precision": precision, "value": value,
           "unit": "GLUPS", "ms_per_solve": 1e3 * total / solves, "solves": solves, "warmup": warmup,
           "site_updates_per_solve": su, "instances": len(sizes), "mean_n": float(np.mean(sizes)),
           "lb_steps": lb_steps, "tau": tau,
           "latency_ms": {"p50": float(np.percentile(sol_ms, 50)), "p99": float(np.percentile(sol_ms, 99))},
           "plain_one_instance_glups": plain, "speedup_vs_plain": value / plain,
           "errors": errors, "autotuned": tuned["best"] if tuned else None,
           # algorithmic flops of the site updates (halo re-computation not
           # counted) over the solve time from HIP events on the ensemble's
           # stream (init and readout included), against the FP64 issue ceiling
           "roofline": {"bound": "alu", "kernel": "k_ens", "achieved": ach, "peak": peak,
                        "unit": "TFLOP/s", "frac": ach / peak, "peak_basis": ALU_PEAK_BASIS,
                        "frac_of_published_fp64_peak": ach / PEAK_FP64_VECTOR_TFLOPS,
                        "traffic": measured_traffic("k_ens", "ensemble_d1q7_%d" % len(sizes), precision, tiling),
                        "tiling": tiling,
                        "traffic_unit": "bytes per chunk launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                        "traffic_algorithmic": bytes_per_site_update(7, precision) * float(np.sum(sizes))}}
    ens.close()
    if cpu:
        # a seeded 64-instance subset of the same ensemble, extrapolated
        from paper_1711_03540_amd.inputs import SplitMix64
        sm = SplitMix64(64)
        pick = []
        while len(pick) < min(64, len(sizes)):
            i = int(sm.uniform() * len(sizes))
            if i not in pick:
                pick.append(i)
        jobs = [(7, ics[i], dX, dT, tau, lb_steps) for i in pick]
        cb = cpu_many(jobs)
        cb["sample"] = ("a seeded subset of %d of the %d instances (N %d..%d), %d of the %d steps each, on %d "
                        "threads; the whole ensemble extrapolated at that rate" %
                        (len(pick), len(sizes), int(min(sizes[pick])), int(max(sizes[pick])),
                         max(1, int(lb_steps * cb["step_scale"])), lb_steps, cb["cores"]))
        cb["extrapolated_solve_s"] = su / (cb["value"] * 1e9)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = value / cb["value"]
    return out


# ---------------------------------------------------------------- serving

def run_serve(rate, requests, budget_gib=4.0, chunk=0, round_steps=0, serve_fp32="fp32", cpu=True):
    """Served request stream: Poisson arrivals at `rate`/s (the seeded stream of
    2000/s with its arrival times scaled), D1Q5/D1Q7, N log-uniform in [256,
    65536], 10^3..10^5 steps, FP32 (FP32 storage by default, split with
    serve_fp32="split") or FP64, dX = pi/16, dT = 1e-4; admission by a device
    memory budget of budget_gib."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.serve import SolveServer

    dev = torch.device("cuda:0")
    dX, dT = math.pi / 16, 1e-4
    reqs = inputs.request_stream(requests, seed=3)
    for r in reqs:                               # the same requests at another offered rate
        r.arrival *= 2000.0 / rate
    log("serve %d requests at %.0f/s" % (requests, rate))
    init = [torch.tensor(inputs.random_modes_ic(r.n, r.n * dX, seed=r.seed % (1 << 63)), device=dev)
            for r in reqs]
    srv = SolveServer(dX, dT, budget_bytes=int(budget_gib * (1 << 30)), chunk=chunk or 64,
                      round_steps=round_steps or 256, device=dev, fp32_storage=serve_fp32)
    warm = inputs.request_stream(8, seed=99, steps_lo=1000, steps_hi=1000)
    srv.serve(warm, [torch.tensor(inputs.random_modes_ic(r.n, r.n * dX, seed=5), device=dev) for r in warm],
              realtime=False)
    st = srv.serve(reqs, init, realtime=True)
    su = {5: 0.0, 7: 0.0}
    for r in reqs:
        su[r.q] += r.n * r.steps
    flops = sum(flops_per_site_update(q) * v for q, v in su.items())
    # the issue ceiling for this mix of schemes: the wall time the mix's FP64
    # instructions would take at full issue on every SIMD
    t_issue = sum(valu_per_site_update(q) * v for q, v in su.items()) / (N_SIMD * 16 * CLOCK_GHZ * 1e9)
    out = {"workload": "serve_%d_requests" % len(reqs), "rate_per_s": rate,
           "fp32_requests_storage": serve_fp32, "budget_bytes": srv.arena.size,
           "offered_glups": float(sum(r.n * r.steps for r in reqs) / reqs[-1].arrival / 1e9),
           "chunk_and_round_steps": {"q%d_%s" % k: [p.chunk, srv.round_steps] for k, p in srv.pools.items()}}
    out.update(st.summary())
    out["value"] = out["achieved_glups"]
    out["unit"] = "GLUPS"
    out["latency_ms"] = {"p50": out["p50_ms"], "p99": out["p99_ms"]}
    # the ensemble kernel's work (algorithmic flops of the site updates) over
    # the wall time of the whole served stream
    ach = flops / st.wall / 1e12
    peak = flops / t_issue / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "k_ens", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                       "frac": ach / peak, "peak_basis": ALU_PEAK_BASIS,
                       "frac_of_published_fp64_peak": ach / PEAK_FP64_VECTOR_TFLOPS, "traffic": None}
    if cpu:
        # the oracle on a seeded sample of 16 of the requests (FP64 arithmetic for all)
        from paper_1711_03540_amd.inputs import SplitMix64
        sm = SplitMix64(16)
        pick = []
        while len(pick) < min(16, len(reqs)):
            i = int(sm.uniform() * len(reqs))
            if i not in pick:
                pick.append(i)
        jobs = []
        for i in pick:
            r = reqs[i]
            tau = 1.0 if r.q == 5 else 0.0
            if tau <= 0.0:
                from paper_1711_03540_amd.lattice import tau_fit
                tau = tau_fit(7, dX, dT)
            jobs.append((r.q, init[i].cpu().numpy(), dX, dT, tau, r.steps))
        cb = cpu_many(jobs)
        part = "all" if cb["step_scale"] >= 1.0 else "a fraction %.3g" % cb["step_scale"]
        cb["sample"] = ("a seeded sample of %d requests, %s of each request's steps, on %d threads, one request "
                        "per thread at a time (FP64 oracle for every request; latency has no CPU analogue)"
                        % (len(pick), part, cb["cores"]))
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = out["value"] / cb["value"]
    del srv
    torch.cuda.synchronize()
    return out


def serve_sweep(rates, requests, budget_gib=4.0, serve_fp32="fp32"):
    """Offered load against achieved throughput, latency and queue depth."""
    rows = []
    for rate in rates:
        o = run_serve(rate, requests, budget_gib, serve_fp32=serve_fp32, cpu=False)
        rows.append({k: o[k] for k in ("rate_per_s", "offered_glups", "achieved_glups", "p50_ms", "p99_ms",
                                       "queue_wait_p50_ms", "queue_wait_p99_ms", "queue_depth_max",
                                       "queue_depth_mean", "active_max", "arena_peak_bytes", "completed",
                                       "requests", "wall_s")})
        log("sweep %s" % json.dumps(rows[-1]))
    return {"workload": "serve_sweep_%d_requests" % requests, "budget_gib": budget_gib, "rows": rows}


def bench_table3(args):
    """The Table 3 travelling wave (fixed ends) on the GPU, both schemes.

    For dX in {0.2, 0.1, 0.05} and a sweep of dT: tau = the paper's fit, raised
    by the stability guard where the fit is linearly unstable; solve to T = 0.5;
    G of section 3 against the analytic solution; GPU time of the solve.  Then,
    as in section 3, the D1Q5 plateau accuracy (its best G over the sweep,
    allowing 10 %) is matched by the largest-dT D1Q7 run at least as accurate,
    and the costs of the two runs are compared (the paper's Table 4 measured
    the same ratio on one CPU core)."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.lattice import Lattice, tau_fit

    dev = torch.device("cuda:0")
    T_end = 0.5
    lo, hi = inputs.table3_ends()
    runs = []
    for dX in (0.2, 0.1, 0.05):
        n = inputs.table3_sites(dX)
        X = np.arange(n) * dX
        rho0 = torch.tensor(inputs.table3_profile(X, 0.0), device=dev)
        exact = inputs.table3_profile(X, T_end)
        for q in (5, 7):
            for dT in (1e-6, 2e-6, 5e-6, 1e-5, 2e-5, 5e-5, 1e-4, 2e-4, 5e-4, 1e-3):
                steps = int(round(T_end / dT))
                if steps > 600_000 or steps < 50:
                    continue
                try:
                    lat = Lattice(n, q, "fp64", device=dev).set_physical(dX, dT, 0.0, guard="raise", rho_max=4.5)
                except Exception as e:
                    runs.append({"dX": dX, "q": q, "dT": dT, "error": str(e)})
                    continue
                # an untimed solve first: the first advance also sets up the
                # kernel's exchange area, host work that would sit between the events
                lat.set_fixed_ends(lo, hi).init_rho(rho0).advance(steps)
                lat.init_rho(rho0)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(lat.stream)
                lat.advance(steps)
                e1.record(lat.stream)
                rho = lat.rho()
                ms = e0.elapsed_time(e1)
                ok = bool(np.all(np.isfinite(rho)) and np.max(np.abs(rho)) < 1e3)
                G = float(np.sum(np.abs(rho - exact)) / np.sum(np.abs(exact))) if ok else None
                runs.append({"dX": dX, "q": q, "dT": dT, "tau": lat.coefficients()["tau"],
                             "tau_fit": tau_fit(q, dX, dT),
                             "steps": steps, "G": G, "gpu_ms": ms})
                print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
    matched = []
    for dX in (0.2, 0.1, 0.05):
        r5 = [r for r in runs if r["dX"] == dX and r["q"] == 5 and r.get("G")]
        r7 = [r for r in runs if r["dX"] == dX and r["q"] == 7 and r.get("G")]
        if not r5 or not r7:
            continue
        plateau = min(r["G"] for r in r5)
        a = max((r for r in r5 if r["G"] <= 1.1 * plateau), key=lambda r: r["dT"])
        cands = [r for r in r7 if r["G"] <= a["G"]]
        if not cands:
            continue
        b = max(cands, key=lambda r: r["dT"])
        matched.append({"dX": dX, "G_target": a["G"], "d1q5": {"dT": a["dT"], "tau": a["tau"], "G": a["G"],
                        "steps": a["steps"], "gpu_ms": a["gpu_ms"]},
                        "d1q7": {"dT": b["dT"], "tau": b["tau"], "G": b["G"], "steps": b["steps"],
                                 "gpu_ms": b["gpu_ms"]},
                        "step_ratio": a["steps"] / b["steps"], "gpu_time_ratio": a["gpu_ms"] / b["gpu_ms"],
                        "saving_pct": 100.0 * (1.0 - b["gpu_ms"] / a["gpu_ms"])})
    print(json.dumps({"workload": "table3_fixed_ends", "T_end": T_end, "runs": runs, "matched": matched}), flush=True)


def bench_profiles(args):
    """The Table 3 travelling wave at dX = 0.2 for both schemes (the comparison of
    the paper's Fig. 4): density profiles at several times against the analytic
    solution, with G and the largest pointwise error.  dT is each scheme's
    matched-accuracy step of the Table 3 study (D1Q5 1e-4, D1Q7 2e-4); tau is
    the paper's fit, raised by the stability guard where needed."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.lattice import Lattice

    dev = torch.device("cuda:0")
    dX = 0.2
    n = inputs.table3_sites(dX)
    X = np.arange(n) * dX
    lo, hi = inputs.table3_ends()
    times = [0.5, 1.0, 2.0, 4.0, 8.0]
    sample = list(range(0, n, 25))        # X = 0, 5, ..., 60
    out = {"workload": "profiles_table3_dx0.2", "dX": dX, "times": times, "X": [float(X[j]) for j in sample],
           "exact": {str(t): [float(v) for v in inputs.table3_profile(X[sample], t)] for t in times}, "schemes": {}}
    for q, dT in ((5, 1e-4), (7, 2e-4)):
        lat = Lattice(n, q, "fp64", device=dev).set_physical(dX, dT, 0.0, guard="raise", rho_max=4.5)
        lat.set_fixed_ends(lo, hi).init_rho(torch.tensor(inputs.table3_profile(X, 0.0), device=dev))
        done, rows = 0, []
        for t in times:
            steps = int(round(t / dT))
            lat.advance(steps - done)
            done = steps
            rho = lat.rho()
            exact = inputs.table3_profile(X, t)
            rows.append({"T": t, "steps": steps,
                         "G": float(np.sum(np.abs(rho - exact)) / np.sum(np.abs(exact))),
                         "max_abs_err": float(np.max(np.abs(rho - exact))),
                         "rho": [float(rho[j]) for j in sample]})
        out["schemes"]["D1Q%d" % q] = {"dT": dT, "tau": lat.coefficients()["tau"], "kernel": lat.kernel()["kernel"],
                                       "rows": rows}
    print(json.dumps(out), flush=True)


def bench_taumin(args):
    """Minimum stable tau on the Table 3 problem (the left panels of the
    paper's Figs. 1-3, section 3): for dX in {0.2, 0.1, 0.05}, both schemes and
    a sweep of dT, the smallest tau (to 0.005, by bisection) for which the
    fixed-end run to T = 0.5 stays bounded (finite and |rho| < 100; the solution
    lies in [0.6, 5.4]), with the library's stability guard off.  Reported
    beside the paper's fit, Eq. (general_tau_formula), and beside the lowest
    tau of the band the library's linear guard (rho_max = 4.5) accepts around
    the fit (None: no accepted tau up to 8)."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.lattice import Lattice, scheme_coefficients, stability_check, tau_fit

    dev = torch.device("cuda:0")
    T_end = 0.5
    lo_end, hi_end = inputs.table3_ends()
    tau_floor, tol = 0.92, 0.005
    out = []

    for dX in (0.2, 0.1, 0.05):
        n = inputs.table3_sites(dX)
        X = np.arange(n) * dX
        rho0 = torch.tensor(inputs.table3_profile(X, 0.0), device=dev)
        for q in (5, 7):
            for dT in (1e-6, 2e-6, 5e-6, 1e-5, 2e-5, 5e-5, 1e-4, 2e-4, 5e-4, 1e-3):
                steps = int(round(T_end / dT))
                if steps > 600_000 or steps < 50:
                    continue
                runs = [0]

                def stable(tau):
                    runs[0] += 1
                    lat = Lattice(n, q, "fp64", device=dev).set_physical(dX, dT, tau, guard="off")
                    lat.set_fixed_ends(lo_end, hi_end).init_rho(rho0).advance(steps)
                    rho = lat.rho()
                    lat.close()
                    return bool(np.all(np.isfinite(rho)) and np.max(np.abs(rho)) < 100.0)

                def guard_ok(tau):
                    _, E, G = scheme_coefficients(q, dX, dT, tau)
                    return stability_check(q, E, G, 1.0 / tau, dX, dT, 4.5)

                t0 = time.perf_counter()
                if stable(tau_floor):
                    tmin = None          # stable at the lowest tau the library accepts
                else:
                    lo, hi = tau_floor, max(1.0, tau_fit(q, dX, dT))
                    while not stable(hi) and hi < 12.0:
                        lo, hi = hi, hi + 0.5
                    if hi >= 12.0:
                        out.append({"dX": dX, "q": q, "dT": dT, "steps": steps, "error": "unstable up to tau = 12"})
                        continue
                    while hi - lo > tol:
                        mid = 0.5 * (lo + hi)
                        if stable(mid):
                            hi = mid
                        else:
                            lo = mid
                    tmin = hi
                # the guard's accepted taus need not extend upwards without
                # bound (at dX = 0.2 they end near 2), so search from the fit
                # in steps of 0.02 for the lowest accepted tau of that band,
                # then bisect the last step
                k_lo, k_hi = 46, 400                # tau = 0.02 k: 0.92 .. 8
                k = min(k_hi, max(k_lo, int(round(tau_fit(q, dX, dT) / 0.02))))
                gmin = None
                if guard_ok(0.02 * k):
                    while k > k_lo and guard_ok(0.02 * (k - 1)):
                        k -= 1
                else:
                    while k < k_hi and not guard_ok(0.02 * k):
                        k += 1
                    if not guard_ok(0.02 * k):
                        k = None
                if k is not None and k == k_lo:
                    gmin = tau_floor                # accepted down to the floor
                elif k is not None:
                    glo, ghi = 0.02 * (k - 1), 0.02 * k
                    while ghi - glo > tol:
                        mid = 0.5 * (glo + ghi)
                        if guard_ok(mid):
                            ghi = mid
                        else:
                            glo = mid
                    gmin = ghi
                out.append({"dX": dX, "q": q, "dT": dT, "steps": steps, "tau_min": tmin, "tau_fit": tau_fit(q, dX, dT),
                            "tau_guard": gmin, "runs": runs[0], "seconds": time.perf_counter() - t0})
                print(json.dumps(out[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"workload": "taumin_table3", "T_end": T_end, "tau_floor": tau_floor, "tol": tol, "scan": out}),
          flush=True)


def bench_lyapunov(args):
    """Largest Lyapunov exponent of the scheme's KS dynamics against the
    domain length L (the chaotic dynamics the paper names as its next subject,
    section 4).  D1Q7 FP64, dX = pi/16, dT = 1e-4, fitted tau; N in {112, 184,
    256, 512, 1024, 2048, 4096} (L = N dX, about 22 to 804); per L four pairs
    (reference and perturbed trajectory, 16 random modes of amplitude 0.1 with
    seeds 100 + 10 L-index + pair, perturbation 1e-8 times another seeded
    field), all in one ensemble.  Benettin renormalisation every unit of time
    to delta = 1e-8 on the GPU; lambda = sum of ln(d / delta) over T in
    [T0, T] / (T - T0), T0 = 200, T = --stats-t (1000).  Also the time-averaged
    energy spectrum of the references (one sample per unit time, T >= T0): its
    peak wavenumber and <rho^2>."""
    import numpy as np
    import torch

    from paper_1711_03540_amd.ensemble import Ensemble
    from paper_1711_03540_amd.inputs import random_modes_ic

    dev = torch.device("cuda:0")
    sizes_L = [112, 184, 256, 512, 1024, 2048, 4096]
    npair = 4
    dX, dT = math.pi / 16, 1e-4
    per = int(round(1.0 / dT))
    T0, T = 200, args.stats_t
    delta = 1e-8
    sizes, ref, pert, meta = [], [], [], []
    for li, n in enumerate(sizes_L):
        for p in range(npair):
            ref.append(len(sizes)); sizes.append(n)
            pert.append(len(sizes)); sizes.append(n)
            meta.append((li, n, p))
    ens = Ensemble(sizes, 7, "fp64", device=dev).set_physical(dX, dT, 0.0)
    for k, (li, n, p) in enumerate(meta):
        rho0 = random_modes_ic(n, n * dX, seed=100 + 10 * li + p)
        ens.init_rho(ref[k], rho0)
        ens.init_rho(pert[k], rho0 + 1e-8 * random_modes_ic(n, n * dX, seed=5000 + 10 * li + p, amplitude=1.0))
    acc = torch.zeros(len(meta), dtype=torch.float64, device=dev)
    spec = {n: torch.zeros(n // 2 + 1, dtype=torch.float64, device=dev) for n in sizes_L}
    rho2 = {n: 0.0 for n in sizes_L}
    buf = {n: torch.empty(n, dtype=torch.float64, device=dev) for n in sizes_L}
    samples = 0
    acc_T0 = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, T + 1):
        ens.advance(per)
        ens.renormalize(ref, pert, delta, acc)
        if t == T0:
            acc_T0 = acc.clone()
        if t > T0:
            for k, (li, n, p) in enumerate(meta):
                if p == 0:
                    r = ens.read_rho(ref[k], buf[n])
                    spec[n] += torch.abs(torch.fft.rfft(r) / n) ** 2
            samples += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lam = ((acc - acc_T0) / (T - T0)).cpu().numpy()
    out = []
    for li, n in enumerate(sizes_L):
        v = np.array([lam[k] for k, m in enumerate(meta) if m[0] == li])
        E = (spec[n] / samples).cpu().numpy()
        kap = 2 * np.pi * np.arange(E.size) / (n * dX)
        peak = int(np.argmax(E[1:]) + 1)
        out.append({"N": n, "L": n * dX, "lambda_pairs": v.tolist(), "lambda_mean": float(v.mean()),
                    "lambda_se": float(v.std(ddof=1) / np.sqrt(v.size)), "spectrum_peak_kappa": float(kap[peak]),
                    "rho2_ref0": float(2 * E[1:].sum() - (E[-1] if n % 2 == 0 else 0.0))})
        print(json.dumps(out[-1]), file=sys.stderr, flush=True)
    site_updates = float(sum(sizes)) * per * T
    print(json.dumps({"workload": "lyapunov_d1q7", "dX": dX, "dT": dT, "tau": ens.tau, "T0": T0, "T": T,
                      "delta": delta, "pairs_per_L": npair, "results": out, "wall_s": wall,
                      "glups_including_readouts": site_updates / wall / 1e9}), flush=True)


def bench_lyapunov_spectrum(args):
    """The 8 leading Lyapunov exponents of the scheme's KS dynamics for L = N dX,
    N in {112, 256, 512} (L about 22, 50, 100): D1Q7 FP64, dX = pi/16, dT = 1e-4,
    fitted tau; per L one reference trajectory (16 random modes of amplitude 0.1,
    seed 300 + L-index) and 8 perturbed copies (1e-8 times seeded fields), all in
    one ensemble; every unit of time the perturbations are orthonormalised (QR)
    and rescaled to delta = 1e-8 on the GPU; lambda_m = sum of ln(R_mm / delta)
    over T in [T0, T] / (T - T0), T0 = 200, T = --stats-t (1000).  Also the
    Kaplan-Yorke dimension where the 8 exponents bracket it."""
    import numpy as np
    import torch

    from paper_1711_03540_amd.ensemble import Ensemble
    from paper_1711_03540_amd.inputs import random_modes_ic

    dev = torch.device("cuda:0")
    sizes_L = [112, 256, 512]
    k = 8
    dX, dT = math.pi / 16, 1e-4
    per = int(round(1.0 / dT))
    T0, T = 200, args.stats_t
    delta = 1e-8
    sizes, ref, pert = [], [], []
    for li, n in enumerate(sizes_L):
        ref.append(len(sizes)); sizes.append(n)
        pert.append(list(range(len(sizes), len(sizes) + k))); sizes += [n] * k
    ens = Ensemble(sizes, 7, "fp64", device=dev).set_physical(dX, dT, 0.0)
    for li, n in enumerate(sizes_L):
        rho0 = random_modes_ic(n, n * dX, seed=300 + li)
        ens.init_rho(ref[li], rho0)
        for m in range(k):
            ens.init_rho(pert[li][m], rho0 + 1e-8 * random_modes_ic(n, n * dX, seed=7000 + 10 * li + m, amplitude=1.0))
    acc = torch.zeros(len(sizes_L) * k, dtype=torch.float64, device=dev)
    acc_T0 = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, T + 1):
        ens.advance(per)
        ens.orthonormalize(ref, pert, delta, acc)
        if t == T0:
            acc_T0 = acc.clone()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lam = ((acc - acc_T0) / (T - T0)).cpu().numpy().reshape(len(sizes_L), k)
    out = []
    for li, n in enumerate(sizes_L):
        l = lam[li]
        c = np.cumsum(l)
        j = int(np.max(np.nonzero(c >= 0)[0])) + 1 if c[0] >= 0 else 0
        dky = float(j + c[j - 1] / abs(l[j])) if 0 < j < k else None
        out.append({"N": n, "L": n * dX, "lambda": l.tolist(), "kaplan_yorke_dimension": dky})
        print(json.dumps(out[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"workload": "lyapunov_spectrum_d1q7", "dX": dX, "dT": dT, "tau": ens.tau, "T0": T0, "T": T,
                      "delta": delta, "k": k, "results": out, "wall_s": wall}), flush=True)


def bench_stats(args):
    """Reduced-precision error on long-time statistics: the D1Q7 N = 4096 lattice
    (L = 256 pi, dT = 1e-4, fitted tau, 16 random modes) run to T = 1000 in FP64,
    FP32 and split storage; time averages over T in [200, 1000] (one sample per
    unit time) of the energy spectrum E_m = <|rho_m|^2> (rho_m the discrete
    Fourier coefficient / N) and of <rho^2>, with standard errors from 8 blocks;
    plus the norm-wise error against FP64 at fixed times."""
    import numpy as np
    import torch

    from paper_1711_03540_amd import inputs
    from paper_1711_03540_amd.lattice import Lattice

    dev = torch.device("cuda:0")
    w = inputs.CFG_RESIDENT_Q7
    rho0 = torch.tensor(w.rho0(), device=dev)
    per_unit = int(round(1.0 / w.dT))
    t_lo, t_hi = 200, args.stats_t
    res = {}
    fixed = {}
    for prec in ("fp64", "fp32", "split"):
        lat = Lattice(w.n, 7, prec, device=dev).set_physical(w.dX, w.dT, 0.0).init_rho(rho0)
        out = torch.empty(w.n, dtype=torch.float64, device=dev)
        spec, r2 = [], []
        snaps = {}
        t0 = time.perf_counter()
        for t in range(1, t_hi + 1):
            lat.advance(per_unit)
            if t in (1, 10, 100):
                snaps[t] = lat.read_rho(out).clone()
            if t >= t_lo:
                lat.read_rho(out)
                f = torch.fft.rfft(out) / w.n
                spec.append((f.real ** 2 + f.imag ** 2).cpu().numpy())
                r2.append(float(torch.mean(out * out)))
        torch.cuda.synchronize()
        spec = np.array(spec)
        r2 = np.array(r2)
        nb = 8
        blocks = np.array_split(np.arange(len(r2)), nb)
        bm_s = np.array([spec[b].mean(axis=0) for b in blocks])
        bm_r = np.array([r2[b].mean() for b in blocks])
        res[prec] = {"E_m": spec.mean(axis=0), "E_m_se": bm_s.std(axis=0, ddof=1) / math.sqrt(nb),
                     "rho2": float(r2.mean()), "rho2_se": float(bm_r.std(ddof=1) / math.sqrt(nb)),
                     "seconds": time.perf_counter() - t0}
        fixed[prec] = snaps
        print("stats %s done in %.1f s" % (prec, res[prec]["seconds"]), file=sys.stderr, flush=True)
    ref = res["fp64"]
    kband = slice(1, 160)     # kappa = m / 128 < 1.25: the active band
    out = {"workload": "stats_d1q7_n4096", "T": [t_lo, t_hi], "samples": t_hi - t_lo + 1,
           "fp64": {"rho2": ref["rho2"], "rho2_se": ref["rho2_se"], "seconds": ref["seconds"]}}
    for prec in ("fp32", "split"):
        r = res[prec]
        z = (r["E_m"][kband] - ref["E_m"][kband]) / np.sqrt(r["E_m_se"][kband] ** 2 + ref["E_m_se"][kband] ** 2)
        out[prec] = {"rho2": r["rho2"], "rho2_se": r["rho2_se"],
                     "rho2_diff_in_se": (r["rho2"] - ref["rho2"]) / math.hypot(r["rho2_se"], ref["rho2_se"]),
                     "spectrum_max_abs_z": float(np.max(np.abs(z))), "spectrum_rms_z": float(np.sqrt(np.mean(z ** 2))),
                     "spectrum_max_rel_diff": float(np.max(np.abs(r["E_m"][kband] / ref["E_m"][kband] - 1))),
                     "fixed_time_rel_err_vs_fp64": {
                         "T=%d" % t: float(torch.max(torch.abs(fixed[prec][t] - fixed["fp64"][t])) /
                                           torch.max(torch.abs(fixed["fp64"][t]))) for t in (1, 10, 100)},
                     "seconds": r["seconds"]}
    print(json.dumps(out), flush=True)


def line(head: dict, steps: int, warmup: int, precision: str) -> dict:
    """The driver's JSON fields around one lattice result."""
    return {
        "metric": METRIC, "value": head["value"], "unit": "GLUPS", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": head["ms_per_solve"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "split": "f64+f32", "rho": "f64"}[precision],
        "data": "synthetic", "config": head["config"],
    }


def bench_all(args):
    """The headline lattice plus every other configuration, in one JSON line."""
    import torch

    from paper_1711_03540_amd import inputs

    torch.cuda.set_device(0)
    cpu = not args.no_cpu_baseline
    peaks = None if args.no_peaks else device_peaks()
    head = run_lattice(inputs.CFG_LARGE_Q7, args.precision, args.kernel or "tiled", args.steps, args.warmup,
                       args.tile_steps, args.autotune, plain=not args.no_plain, cpu=cpu, peaks=peaks)
    out = line(head, args.steps, args.warmup, args.precision)
    out.update({k: head[k] for k in ("latency_ms", "roofline", "autotuned", "s1_hbm_roofline_glups",
                                     "vs_s1_hbm_roofline") if k in head})
    if "plain_kernel" in head:
        out["plain_kernel"] = head["plain_kernel"]
    if "cpu_baseline" in head:
        out["cpu_baseline"] = head["cpu_baseline"]
        out["gpu_over_cpu"] = head["gpu_over_cpu"]
    out["peaks"] = peaks
    configs = {}
    # the large lattice in FP32 storage (the configuration names FP32 and
    # FP64), and in the rho-only state: at tau = 1 (this lattice's tau) the
    # collision leaves f = feq(rho), the densities are bitwise those of the
    # FP64 populations, and the state is one double per site
    w4 = inputs.CFG_LARGE_Q7
    for prec in ("fp32", "rho"):
        r = run_lattice(w4, prec, "tiled", max(5, args.steps // 2), 1, plain=not args.no_plain, cpu=False,
                        peaks=peaks)
        configs["%s_%s" % (w4.name, prec)] = r
    w0, w1 = inputs.CFG_SMALL_Q5, inputs.CFG_RESIDENT_Q7
    configs[w0.name] = run_lattice(w0, "fp64", "span", 100, 5, plain=not args.no_plain, cpu=cpu)
    configs[w1.name] = run_lattice(w1, "fp64", "span", 100, 2, plain=not args.no_plain, cpu=cpu)
    # the ensemble's tiling (sites per lane, steps per chunk, instance tiles
    # per workgroup window) picked by the autotuner for each storage
    ens64 = run_ensemble("fp64", args.instances, args.lb_steps, autotune=True, cpu=cpu)
    ens32 = run_ensemble("fp32", args.instances, args.lb_steps, autotune=True, cpu=False)
    # the split storage (rho in double, the non-equilibrium part in single) at
    # the library's default tiling
    enssp = run_ensemble("split", args.instances, args.lb_steps, cpu=False)
    configs[ens64["workload"]] = ens64
    configs[ens64["workload"] + "_fp32"] = ens32
    configs[ens64["workload"] + "_split"] = enssp
    srv = run_serve(2000.0, args.requests, args.budget_gib, serve_fp32=args.serve_fp32, cpu=cpu)
    configs[srv["workload"]] = srv
    rates = [float(r) for r in args.rates.split(",") if r]
    configs["serve_sweep"] = serve_sweep(rates, args.sweep_requests, args.budget_gib, args.serve_fp32)
    out["configs"] = configs
    # the targets, in one place: the one-step kernel's HBM fraction on the large
    # lattice; batched and served throughput over the plain one-instance kernel
    # at equal accuracy (bitwise-identical arithmetic); served p99 latency
    pk = head.get("plain_kernel", {})
    out["targets"] = {
        "s1_plain_hbm_frac": pk.get("hbm_frac"), "s1_plain_hbm_frac_target": TARGET_HBM_FRAC,
        "s1_plain_meets_target": pk.get("meets_target"),
        "tiled_over_plain": pk.get("speedup"),
        "ensemble_fp64_over_plain": ens64["speedup_vs_plain"],
        "served_glups": srv["value"], "served_over_plain_one_instance": srv["value"] / ens64["plain_one_instance_glups"],
        "served_p50_ms": srv["p50_ms"], "served_p99_ms": srv["p99_ms"],
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); a domain or an ensemble "
              "would shard across GPUs as described in the design notes, but no multi-GPU path is "
              "built." % args.gpus, file=sys.stderr)
        sys.exit(2)
    studies = {"table3": bench_table3, "stats": bench_stats, "profiles": bench_profiles,
               "lyapunov_spectrum": bench_lyapunov_spectrum, "taumin": bench_taumin, "lyapunov": bench_lyapunov}
    if args.workload in studies:
        studies[args.workload](args)
        return
    if args.workload == "all":
        bench_all(args)
        return
    cpu = not args.no_cpu_baseline
    if args.workload == "ensemble":
        print(json.dumps(run_ensemble(args.precision, args.instances, args.lb_steps, args.steps, args.warmup,
                                      args.chunk, args.segments, args.autotune, cpu=cpu)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args.rate, args.requests, args.budget_gib, args.chunk, args.round_steps,
                                   args.serve_fp32, cpu=cpu)), flush=True)
        return
    if args.workload == "serve_sweep":
        rates = [float(r) for r in args.rates.split(",") if r]
        print(json.dumps(serve_sweep(rates, args.sweep_requests, args.budget_gib, args.serve_fp32)), flush=True)
        return
    import torch

    from paper_1711_03540_amd import inputs
    torch.cuda.set_device(0)
    wname, default_kernel = WORKLOADS[args.workload]
    w = getattr(inputs, wname)
    kernel = args.kernel or default_kernel
    res = run_lattice(w, args.precision, kernel, args.steps, args.warmup, args.tile_steps,
                      args.autotune and args.kernel is None, plain=not args.no_plain, cpu=cpu)
    out = line(res, args.steps, args.warmup, args.precision)
    out.update({k: v for k, v in res.items() if k not in out})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
