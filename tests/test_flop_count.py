"""The pointwise flop counts behind bench.py's algorithmic FP64 flops are the
operation counts of the FP64 oracle's physics functions
(oracle/sdmhd_oracle_point.inc), counted by compiling that source on the host
with a counting number type."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_point_flops_match_oracle_source(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "count"
    subprocess.run(["g++", "-std=c++17", "-O0", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "flops", "count_oracle_flops.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    n = {m.group(1): int(m.group(2)) for m in re.finditer(r"^(\w+)\s.*flops\(add\+mul\+div\+sqrt\)\s+(\d+)", out, re.M)}
    sys.path.insert(0, ROOT)
    import bench
    assert bench.PHYS_FLOPS == {k: n[k] for k in bench.PHYS_FLOPS}, out
