"""The algorithmic bytes behind bench.py's roofline are the sizes of the
arrays one RK stage must touch, each once: the FP64 state, the library's
stored geometry of a real shell mesh (positions, |J|, S^d/|J| at the solution
points, S^d at the flux points), the further Shu-Osher registers and the
output.  The average count of further registers comes from the oracle's
SSPRK(5,3) table, not from bench.py."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.fixture(scope="module")
def sd():
    from paper_2502_17805_amd import sdmhd
    return sdmhd


def test_further_registers_average_matches_the_scheme(oracle):
    """Stage i of the Shu-Osher form reads the current state u_(i-1) plus every
    other u_k with alpha_ik != 0; bench.py's default n_extra is their mean."""
    A, _, _ = oracle.ssprk53_table()
    extra = [sum(1 for k in range(i) if A[i, k] != 0 and k != i - 1) for i in range(1, 6)]
    assert extra == [0, 0, 1, 2, 3]
    assert bench.alg_bytes("stage", 6, 1) == pytest.approx(bench.alg_bytes("stage", 6, 1, n_extra=np.mean(extra)))


@pytest.mark.parametrize("p", [3, 5])
@pytest.mark.parametrize("n_extra", [0, 1, 2, 3, 1.2])
def test_stage_bytes_are_the_stored_arrays(sd, p, n_extra):
    m = sd.shell(2, 2, p)
    N3 = m.N ** 3
    geometry = sum(a.size for a in (m.x_sp, m.detJ, m.S_fp, m.Sj_sp)) // m.E
    state, registers = 9 * N3, 9 * N3 * (n_extra + 1)  # further registers and the output
    assert bench.alg_bytes("stage", m.N, m.E, n_extra) == pytest.approx(8 * m.E * (state + geometry + registers))


@pytest.mark.parametrize("fused", [True, False])
def test_volume_and_finish_split_the_stage(fused):
    for N in (4, 6):
        parts = bench.alg_bytes("volume", N, 10, fused=fused) + bench.alg_bytes("finish_stage", N, 10, fused=fused)
        assert parts == pytest.approx(bench.alg_bytes("stage", N, 10))
    assert bench.alg_bytes("finish_stage", 6, 10, fused=True) == 0


def test_p5_figure():
    """90,374.4 B per element-stage at p = 5 (418 B per solution point)."""
    assert bench.alg_bytes("stage", 6, 1) == pytest.approx(90374.4)
    assert bench.alg_bytes("stage", 6, 1) / 216 == pytest.approx(418.4, abs=0.05)
