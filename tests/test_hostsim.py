"""The library's host code (runtime.hip, server.hip) built with g++ against a
stand-in HIP runtime (tests/hostsim) and run under AddressSanitizer + UBSan
and under ThreadSanitizer, on the CPU.

The stand-in runs each stream's work on a thread of its own, records work
under capture and replays it, and its launchers produce outputs of the real
kernels' shape (frontier entries, counts, offsets, picks, paths) from a
placeholder selection; the scenarios (tests/hostsim/driver.cpp) check the
library's results against that placeholder's definition and every server
result against the same request run alone. Failure injection covers a
failing request inside a batch, decreasing device-written segment offsets, an
impossible device step count, a request larger than an executor's memory,
cancellation and executors that cannot allocate. The partitioned
(out-of-memory) graph is checked against the same definition.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "hostsim")
CSRC = os.path.join(ROOT, "paper_2009_09103_amd", "csrc")
SOURCES = [os.path.join(CSRC, "runtime.hip"), os.path.join(CSRC, "server.hip"),
           os.path.join(SIM, "hip_sim.cpp"), os.path.join(SIM, "kernels_sim.cpp"), os.path.join(SIM, "driver.cpp")]
FLAGS = {
    "asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


def build(kind, outdir):
    exe = os.path.join(outdir, "driver_" + kind)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", SIM, "-x", "c++"] + SOURCES + FLAGS[kind] + \
        ["-o", exe]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert res.returncode == 0, res.stdout[-4000:]
    return exe


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("hostsim"))
    return {k: build(k, out) for k in FLAGS}


def run(exe, scenario, timeout=600):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:allocator_may_return_null=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    res = subprocess.run([exe, scenario], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         timeout=timeout, env=env)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok " + scenario), res.stdout[-6000:]


@pytest.mark.parametrize("scenario", ["runtime", "server", "failures", "streamed"])
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_code_under_sanitizers(drivers, kind, scenario):
    run(drivers[kind], scenario)


def test_served_request_shapes_on_a_2_26_vertex_graph(drivers):
    """8,192-seed sampling requests and 65,536-walker x 80-step walks on a
    graph of 2^26 vertices (16 MiB bitmaps per instance), under ASan."""
    run(drivers["asan"], "scale", timeout=900)
