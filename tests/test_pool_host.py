"""Serving-pool bookkeeping (lfsr_pool_*) on the CPU: the pool's own source is
built against a host-only model of the HIP runtime and of the solver entry
points (tests/pool_host), with AddressSanitizer and UBSan, and driven through
random admission / tick / poll sequences with device progress at random
points.  Covers arena accounting, slot reuse, graph re-capture and the
deferred destruction of replaced graphs, harvesting after each job's exact
iteration count, job isolation in a reused arena, pool destruction with
jobs in flight, and the error paths (every fifth seed makes one result copy or
one event query fail part-way: the pool must report LFSR_EDEVICE, keep each
job in exactly one of its lists, and never destroy a replaced graph whose
completion it could not confirm)."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2206_05047_amd" / "csrc"
HOST = ROOT / "tests" / "pool_host"


@pytest.fixture(scope="module")
def fuzz_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("pool_host")
    src = d / "lfsr_pool.cpp"  # the pool source, compiled as plain C++
    shutil.copy(CSRC / "lfsr_pool.hip", src)
    exe = d / "pool_fuzz"
    sanitize = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *sanitize,
           "-I", str(HOST), "-I", str(CSRC), "-I", str(ROOT / "include"),
           str(src), str(HOST / "mock_runtime.cpp"), str(HOST / "pool_fuzz.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_pool_bookkeeping_random_sequences(fuzz_exe):
    seeds = [str(s) for s in range(1, 401)]
    r = subprocess.run([str(fuzz_exe), *seeds], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "400 seeds ok" in r.stdout
