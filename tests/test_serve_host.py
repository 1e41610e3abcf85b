"""The serving stream's request loop on the CPU, through the library's real
host code.  lfsr_api, lfsr_pool and the kernel launchers of lfsr_kernels are
compiled for the host side only, with AddressSanitizer and UBSan, and linked
against a model of the HIP runtime (tests/serve_host/mock_hip.cpp: kernel
registration and launches checked and recorded, stream capture with HIP's
join rules, one FIFO of deferred device work).  The driver
(tests/serve_host/serve_replay.cpp) replays the request loop of
paper_2206_05047_amd/serve.py on the serving workload's 24 job types with
their real parameters: the seeded Poisson stream of 2000 jobs at 20 jobs/s,
32 slots, a 40 GiB arena, unsynchronised ticks with two outstanding, polls
and harvests."""
import os
import shutil
import struct
import subprocess
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2206_05047_amd" / "csrc"
HOST = ROOT / "tests" / "serve_host"
CXX = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def replay_exe(tmp_path_factory):
    if not os.path.exists(CXX) or shutil.which("nm") is None:
        pytest.skip("amdclang++ or nm not available")
    d = tmp_path_factory.mktemp("serve_host")
    # host side only; the sanitizers apply to host code
    common = ["-x", "hip", "--offload-host-only", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
              "-fno-omit-frame-pointer", "-I", str(ROOT / "include"),
              "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    objs = []
    srcs = [CSRC / f for f in ("lfsr_kernels.hip", "lfsr_api.hip", "lfsr_pool.hip")]
    srcs += [HOST / "mock_hip.cpp", HOST / "serve_replay.cpp"]
    for src in srcs:
        obj = d / (src.stem + ".o")
        r = subprocess.run([CXX, *common, "-c", str(src), "-o", str(obj)], capture_output=True, text=True,
                           timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        objs.append(str(obj))
    # the device code objects are not built: give their (unused) symbols a definition
    nm = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    names = sorted({ln.split()[-1] for ln in nm.splitlines() if "__hip_fatbin_" in ln})
    stub = d / "fatbin_stubs.c"
    stub.write_text("".join(f"char {n}[1];\n" for n in names))
    r = subprocess.run(["gcc", "-c", str(stub), "-o", str(d / "fatbin_stubs.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = d / "serve_replay"
    r = subprocess.run([CXX, "-fsanitize=address,undefined", "-o", str(exe), *objs, str(d / "fatbin_stubs.o")],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _inputs(tmp_path):
    from paper_2206_05047_amd import lfsr, serve, synth

    bounds = {}
    for z, hr in serve.SPATIAL:  # the disparity bounds serve.Workload derives from its scenes
        sc = synth.make_scene(synth.config("c3", sy=hr // z, sx=hr // z, zeta=z), seed=5 * 1000 + hr)
        bounds[hr] = max(float(np.abs(sc["disp"]).max()), 1e-3)
    blob = b"".join(bytes(lfsr.make_params(serve._cfg(a, n, z, hr), disp_bound=bounds[hr], storage=st))
                    for a, n, z, hr, st in serve.job_types())
    params = tmp_path / "params.bin"
    params.write_bytes(blob)
    t, k = serve.stream(2000, 20.0)
    stream = tmp_path / "stream.bin"
    stream.write_bytes(struct.pack("<i", len(t)) + b"".join(struct.pack("<di", float(a), int(b))
                                                              for a, b in zip(t, k)))
    return params, stream


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_serving_stream_replay_on_the_real_host_code(replay_exe, tmp_path, seed):
    params, stream = _inputs(tmp_path)
    r = subprocess.run([str(replay_exe), str(params), str(stream), "32", "40", "2", str(seed)],
                       capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "2000 jobs served" in r.stdout, r.stdout
