"""Long runs of one seeded shell with diagnostics, in FP64 and FP32-mixed.

  python -m paper_2502_17805_amd.longrun --mesh 12,8 --p 5 --n-rho 3 --seed 1 \
      --steps 1000 --every 50 [--arith 0,1] [--cfl 0.1]

Prints one JSON line: for each arithmetic the diagnostics every `every` steps
(mass, total energy, volume-averaged kinetic and magnetic energy, max and L2
|div B|, max |psi|, NaN flag) and, when both arithmetics ran, the relative
difference of KE, E_B and max|div B| of the FP32-mixed run from the FP64 run
at each checkpoint.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as inp
from . import sdmhd as sd

DIAG_NAMES = ("volume", "mass", "energy", "KE", "E_B", "max_divB", "L2_divB", "max_psi", "nan")


def run(mesh, Q, pr, dt, steps, every, arith, label=""):
    import torch
    s = sd.Solver(mesh, arith=arith)
    prm = sd.make_params(**pr)
    s.set_state(torch.from_numpy(Q))
    rows = [[0, 0.0] + list(s.diagnostics(prm)[:9])]
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        s.step(prm, dt)
        if k % every == 0 or k == steps:
            d = s.diagnostics(prm)
            rows.append([k, k * dt] + list(d[:9]))
            print(f"# {label} arith={arith} step {k}: KE={d[3]:.6e} E_B={d[4]:.6e} max|divB|={d[5]:.3e} "
                  f"nan={d[8]:g} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
            if d[8] != 0:
                break
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mesh", default="12,8")
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--n-rho", type=float, default=3.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--arith", default="0,1")
    ap.add_argument("--cfl", type=float, default=0.1)
    a = ap.parse_args(argv)
    Nz, Nr = (int(x) for x in a.mesh.split(","))
    mesh = sd.shell(Nz, Nr, a.p)
    bg = inp.Background(a.n_rho)
    Q = inp.shell_state(mesh.x_sp, bg, a.seed)
    pr = inp.run_params(a.seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, mesh.Sj_sp, ch, a.cfl)
    label = f"shell 6x{Nz}x{Nz}x{Nr} p={a.p} N_rho={a.n_rho:g}"
    out = {"workload": f"{label}, seed {a.seed}, {a.steps} SSPRK(5,3) steps, CFL {a.cfl:g}",
           "elements": mesh.E, "dt": dt, "columns": ["step", "t", *DIAG_NAMES], "runs": {}}
    for ar in (int(x) for x in a.arith.split(",")):
        out["runs"]["fp64" if ar == 0 else "fp32-mixed"] = run(mesh, Q, pr, dt, a.steps, a.every, ar, label)
    r = out["runs"]
    if "fp64" in r and "fp32-mixed" in r:
        rel = []
        for x, y in zip(r["fp64"], r["fp32-mixed"]):
            rel.append([x[0]] + [abs(y[2 + i] - x[2 + i]) / abs(x[2 + i]) if x[2 + i] else None
                                 for i in (3, 4, 5)])
        out["mixed_vs_fp64_rel"] = {"columns": ["step", "KE", "E_B", "max_divB"], "rows": rel}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
