"""A plain C program (tests/c/abi_step.c) advances the 48-element shell by
SSPRK(5,3) steps through the C ABI alone (sdm_shell_build, sdm_create,
sdm_mesh_bind, sdm_workspace_size, sdm_ssprk53_step; HIP runtime for the
device memory) and the result matches the oracle's SSPRK(5,3) steps
(paper, Sec. "Spectral Difference Method")."""
import os
import subprocess

import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "abi_step")


@pytest.mark.gpu
def test_c_caller_ssprk53_steps_match_oracle(oracle, tmp_path):
    from paper_2502_17805_amd import sdmhd as sd
    assert os.path.exists(EXE), "tests/c/abi_step is not built (run __graft_entry__.build())"
    Nz, Nr, p, steps = 2, 2, 5, 2
    om = oracle.Mesh.shell(p + 1, Nz, Nr)
    bg = inp.Background(3.0)
    Q = inp.shell_state(om.get("x_sp"), bg, 0)
    pr = inp.run_params(0, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, om.get("S_sp") / om.get("detJ_sp")[:, None, None, :], ch, 0.1)
    prm = sd.make_params(**pr)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        f.write(np.array([Nz, Nr, p, steps], dtype=np.int32).tobytes())
        f.write(bytes(prm))
        f.write(np.array([dt]).tobytes())
        f.write(np.ascontiguousarray(Q).tobytes())
    print(f"abi_step: shell 6x{Nz}^2x{Nr} p={p} {steps} steps dt={dt:.3e}", flush=True)
    r = subprocess.run([EXE, str(fin), str(fout)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = np.fromfile(fout, dtype=np.float64).reshape(Q.shape)
    po = oracle.make_params(**pr)
    want, scale = Q, None
    for _ in range(steps):
        _, ts = om.residual(po, want, with_scale=True)
        scale = ts if scale is None else np.maximum(scale, ts)
        want = om.step(po, want, dt)
    err = np.abs(got - want).max(axis=(0, 2)) / (np.abs(want).max(axis=(0, 2)) + dt * scale)
    assert (err <= 1e-12).all(), err
