"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the library's host-side parameter code (kslb_params.cpp) and the FP64
oracle with g++/gcc -fsanitize=address,undefined into a temporary directory,
runs a driver over each, and requires a clean exit (any report aborts).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(cmd, exe, tmp_path):
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if res.returncode != 0 and "asan" in (res.stderr or "").lower() and "cannot find" in res.stderr:
        pytest.skip("sanitizer runtime not available")
    assert res.returncode == 0, res.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-1000:], run.stderr[-3000:])
    return run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_parameter_code_is_sanitizer_clean(tmp_path):
    exe = str(tmp_path / "params_driver")
    cmd = ["g++", "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "paper_1711_03540_amd", "csrc"),
                                          os.path.join(HERE, "params_driver.cpp"),
                                          os.path.join(ROOT, "paper_1711_03540_amd", "csrc", "kslb_params.cpp"),
                                          "-o", exe]
    out = _build_and_run(cmd, exe, tmp_path)
    assert "params checks=" in out
    assert int(out.split("checks=")[1].split()[0]) > 50


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_sanitizer_clean(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c99", "-ffp-contract=off"] + SAN + [os.path.join(HERE, "oracle_driver.c"),
                                                            os.path.join(ROOT, "oracle", "ks_oracle.c"),
                                                            "-lm", "-o", exe]
    out = _build_and_run(cmd, exe, tmp_path)
    assert "oracle mass drift" in out and out.count("fixed-end G=") == 2
