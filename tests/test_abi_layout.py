"""The ctypes mirrors of the C-ABI structures match include/cqm.h: a small
host program compiled against the header prints every field's offset and
size and each structure's size, and the binding must agree (a drift would corrupt
arguments without any error)."""
import os
import shutil
import subprocess

import pytest

from paper_2006_05186_amd import cqm as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INC = "/opt/rocm/include"

STRUCTS = {
    "cqm_options": C.cqm_options,
    "cqm_diag": C.cqm_diag,
    "cqm_server_opts": C.cqm_server_opts,
    "cqm_request": C.cqm_request,
    "cqm_server_stats_t": C.cqm_server_stats_t,
}


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC),
                    reason="needs g++ and the HIP runtime headers")
def test_ctypes_structures_match_the_header(tmp_path):
    lines = ["#include <cstdio>", "#include <cstddef>", '#include "cqm.h"', "int main() {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  std::printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  std::printf("{cname} {field} %zu %zu\\n", offsetof({cname}, {field}), '
                         f'sizeof((({cname}*)0)->{field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include",
                    f"-I{ROCM_INC}", str(src), "-o", str(exe)], check=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True,
                         timeout=30).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        cname, key, *vals = line.split()
        got[(cname, key)] = tuple(int(v) for v in vals)
    for cname, cls in STRUCTS.items():
        assert got[(cname, "size")] == (C.ctypes.sizeof(cls),), cname
        for field, _ in cls._fields_:
            desc = getattr(cls, field)
            assert got[(cname, field)] == (desc.offset, desc.size), (cname, field)
