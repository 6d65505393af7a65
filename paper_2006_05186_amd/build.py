"""Build the HIP/C++ library libcqm.so for gfx950 in-tree.

Every source under csrc/ is compiled by hipcc (device code for gfx950 only) and
linked into paper_2006_05186_amd/lib/libcqm.so.  Packed FP32 instructions are
disabled for all device code.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib")
BUILD = os.path.join(HERE, "_build")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
         "-I" + os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
LIBNAME = "libcqm.so"
PROBENAME = "libcqm_probe.so"


# Per-file flags: the near-field entries (largest of every row, amplified by
# rho^-N in the time domain) and the double-layer operator are computed
# without fused multiply-adds.
FILE_FLAGS = {"k_near.hip": ["-ffp-contract=off"], "k_dlayer.hip": ["-ffp-contract=off"],
              "k_hsing.hip": ["-ffp-contract=off"]}


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    extra = FILE_FLAGS.get(os.path.basename(src), [])
    cmd = [HIPCC] + FLAGS + extra + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(SRC, f) for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    if verbose:
        for (_, err), s in zip(results, srcs):
            if err.strip():
                print(os.path.basename(s), err, file=sys.stderr)
    tmp = os.path.join(OUT, LIBNAME + ".tmp")
    # roctx: named stage ranges for rocprofv3 --marker-trace
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, os.path.join(OUT, LIBNAME))
    build_probe()
    return os.path.join(OUT, LIBNAME)


def build_probe():
    """The ALU throughput probe (probes/alu_rate.hip) as its own library,
    lib/libcqm_probe.so; bench.py --alu-probe loads it."""
    src = os.path.join(HERE, "probes", "alu_rate.hip")
    tmp = os.path.join(OUT, PROBENAME + ".tmp")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-shared", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"probe build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, os.path.join(OUT, PROBENAME))


if __name__ == "__main__":
    print(build(verbose=True))
