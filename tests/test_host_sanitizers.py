"""The host planner (near-field adjacency, cluster and block trees) built with
a plain C++ compiler under AddressSanitizer and UndefinedBehaviorSanitizer
and run on several meshes (tests/host_planner_check.cpp): no sanitizer
report, and the invariants the GPU kernels rely on hold.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import cqm_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_05186_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    out = tmp_path_factory.mktemp("san")
    exe = str(out / "host_planner_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-D__align__(n)=__attribute__((aligned(n)))", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_planner_check.cpp"),
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "h2_tree.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe, out


@pytest.mark.parametrize("mesh,args", [
    ("icosahedron", ("8", "1.0", "2", "5")),
    ("sphere1280", ("32", "1.0", "4", "17")),
    ("ellipsoid320", ("16", "2.0", "3", "33")),
    ("ellipsoid1280", ("32", "0.5", "4", "65")),
])
def test_planner_clean_under_sanitizers(checker, mesh, args):
    exe, out = checker
    V, T = {"icosahedron": lambda: W.icosphere(0), "sphere1280": lambda: W.icosphere(3),
            "ellipsoid320": lambda: W.ellipsoid(2, (1.3, 0.8, 1.0)),
            "ellipsoid1280": lambda: W.ellipsoid(3, (0.6, 1.4, 1.0))}[mesh]()
    path = out / f"{mesh}.bin"
    with open(path, "wb") as f:
        f.write(np.array([len(V), len(T)], dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(V, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(T, dtype=np.int32).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(path), *args], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "planner ok" in r.stdout and "fails=0" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
