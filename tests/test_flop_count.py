"""The pointwise flop counts behind bench.py's algorithmic FP64 flops are the
operation counts of the kernels' physics functions (sdm_physics.hpp),
counted by compiling that header on the host with a counting number type."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_point_flops_match_physics_source(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "count"
    subprocess.run(["g++", "-std=c++17", "-O0", "-I", os.path.join(ROOT, "tests", "flops"),
                    "-I", os.path.join(ROOT, "paper_2502_17805_amd", "csrc"),
                    os.path.join(ROOT, "tests", "flops", "count_physics_flops.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    n = {m.group(1): int(m.group(2)) for m in re.finditer(r"^(\w+)\s.*flops\(add\+mul\+div\+sqrt\)\s+(\d+)", out, re.M)}
    sys.path.insert(0, ROOT)
    import bench
    assert bench.PHYS_FLOPS == {k: n[k] for k in bench.PHYS_FLOPS}, out
