"""Build libkslb.so and libkslb_probe.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkslb.so")
SOURCES = ["kslb_kernels.hip", "kslb_api.cpp", "kslb_params.cpp"]
# device-peak measurement kernels, a library of their own (not the method)
PROBE_LIB = os.path.join(HERE, "libkslb_probe.so")
PROBE_SOURCES = ["kslb_probe.hip"]

# -ffp-contract=off: only the explicit FMAs of the kernels are fused, so every
# kernel class rounds identically.  Packed FP32 instructions are disabled.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(lib: str, sources, verbose: bool, extra) -> None:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + list(extra or []) + ["-o", tmp] + [os.path.join(CSRC, s) for s in sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % os.path.basename(lib))
    os.replace(tmp, lib)


def build(verbose: bool = False, extra=None) -> str:
    """Compile libkslb.so and libkslb_probe.so next to this file (always rebuilds)."""
    _compile(LIB, SOURCES, verbose, extra)
    _compile(PROBE_LIB, PROBE_SOURCES, verbose, extra)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    print(LIB)
