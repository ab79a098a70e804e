"""Measured device peaks (libkslb_probe.so): HBM copy bandwidth and LDS read
bandwidth per compute unit and clock.  Argument marshalling only; the kernels
are in csrc/kslb_probe.hip.  They compute nothing of the method."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkslb_probe.so")
SIGNATURES = {
    "kslb_probe_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "kslb_probe_lds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
}
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkslb_probe.so not found at %s: build it first" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        _lib = lib
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError("%s failed (hipError %d)" % (what, rc))


def hbm_copy(nbytes: int = 4 << 30, reps: int = 10, device="cuda:0") -> dict:
    """Device-to-device copy of nbytes (well beyond the 256 MB last-level
    cache), timed with HIP events on the stream it runs on: 2 * nbytes moved per
    copy.  Returns the best and median rates in GB/s."""
    import numpy as np
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(device)
    lib = load()
    _check(lib.kslb_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream), "copy")
    stream.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _check(lib.kslb_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream), "copy")
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    if not torch.equal(dst[:1024], src[:1024]):
        raise RuntimeError("copy probe: wrong data")
    rates = [2 * nbytes / (m * 1e-3) / 1e9 for m in ms]
    out = {"bytes_per_copy": nbytes, "moved_per_copy": 2 * nbytes, "reps": reps,
           "best_gb_s": max(rates), "median_gb_s": float(np.median(rates)), "kernel": "k_probe_copy"}
    del src, dst
    return out


def lds_bandwidth(blocks_per_cu: int = 4, iters: int = 4000, device="cuda:0") -> dict:
    """LDS read bytes per clock per compute unit: blocks_per_cu workgroups of 256
    lanes per CU (four 32 KiB areas fit a CU's 160 KiB, so every workgroup is
    resident at once) each read their 32 KiB of LDS iters times with
    conflict-free 16-byte loads; the rate is all bytes over the launch's event
    time at the shader clock measured over the read loops (s_memtime against
    the 100 MHz constant clock), per CU."""
    import numpy as np
    import torch
    props = torch.cuda.get_device_properties(device)
    cus = props.multi_processor_count
    blocks = cus * blocks_per_cu
    out = torch.zeros(4 * blocks, dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream(device)
    lib = load()
    _check(lib.kslb_probe_lds(out.data_ptr(), blocks, 10, stream.cuda_stream), "lds")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    _check(lib.kslb_probe_lds(out.data_ptr(), blocks, iters, stream.cuda_stream), "lds")
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    v = out.view(blocks, 4).cpu().numpy().astype(np.float64)
    bytes_total = float(v[:, 0].sum())
    clk = float(np.median(v[:, 1]))
    ghz = float(np.median(v[:, 1] / v[:, 2])) * 0.1          # shader clocks per 10 ns tick
    # one round: every workgroup resident from the start; per CU, its share
    # of the bytes over the event time
    bpc_wall = bytes_total / (ms * 1e-3) / (ghz * 1e9) / cus
    return {"blocks": blocks, "iters": iters, "lds_bytes_read": bytes_total, "ms": ms,
            "shader_ghz": ghz, "bytes_per_clk_per_cu": bpc_wall,
            "bytes_per_clk_per_workgroup_loop": float(np.median(v[:, 0] / v[:, 1])),
            "kernel": "k_probe_lds"}
