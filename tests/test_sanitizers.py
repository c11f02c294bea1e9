"""Host code under the address and undefined-behaviour sanitizers (CPU only).

* The code plan behind gfbp_code_build (gfbp_plan.h: validation, field
  tables, column index, coefficient maps, visiting order, source chain, SUS
  levels and records), compiled with g++ into a host program that checks it on
  seeded random codes and malformed descriptions (tests/host_plan_check.cpp).
* The reference decoder (oracle/gfbp_oracle.c) and the workload encoder
  (workloads/_encoder.c), compiled with the sanitizers into a temporary
  directory and loaded, with the sanitizer runtime preloaded, by a child
  pytest that runs the whole CPU suite (this file aside).  Leak reports are
  off in the child (the Python interpreter keeps its own allocations to the
  end).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _tool(name):
    path = shutil.which(name)
    if not path:
        pytest.skip(f"{name} not available")
    return path


def test_code_plan_under_sanitizers(tmp_path):
    gxx = _tool("g++")
    exe = tmp_path / "plan_check"
    subprocess.check_call([gxx, "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                           os.path.join(ROOT, "tests", "host_plan_check.cpp")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe), "600"], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok 600"


def test_oracle_and_encoder_under_sanitizers(tmp_path):
    gcc = _tool("gcc")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan.so not found")
    sys.path.insert(0, ROOT)
    import oracle
    from paper_cs_0605069_amd import workloads

    oracle.build(out_dir=str(tmp_path), sanitize=True)
    workloads.build_native(out_dir=str(tmp_path), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, GFBP_SANITIZED_DIR=str(tmp_path),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", "tests",
           "--ignore=tests/test_sanitizers.py"]
    out = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, env=env, timeout=900)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "passed" in out.stdout
