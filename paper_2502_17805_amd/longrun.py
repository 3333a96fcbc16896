"""Long runs of one seeded shell with diagnostics, in FP64 and FP32-mixed.

  python -m paper_2502_17805_amd.longrun --mesh 12,8 --p 5 --n-rho 3 --seed 1 \
      --steps 1000 --every 50 [--arith 0,1] [--cfl 0.1] [--profiles 8,16] [--setup solar]
      [--ch-every 100]

Prints one JSON line: for each arithmetic the diagnostics every `every` steps
(mass, total energy, volume-averaged kinetic and magnetic energy, max and L2
|div B|, max |psi|, NaN flag, the largest signal speed max(|u| + c_f) of the
state) and, when both arithmetics ran, the relative
difference of KE, E_B and max|div B| of the FP32-mixed run from the FP64 run
at each checkpoint.  With --profiles n_r,n_th it also reports, per
arithmetic, the poloidal and toroidal magnetic energies at each checkpoint
and the longitude-time averages of V_phi (differential rotation) and V_mer
(meridional flow) on n_r x n_th (r, theta) bins over the checkpoints after
the first (Sec. "Results").  --setup solar runs the solar benchmark's parameters
(section "Benchmark Problem Definition", in the units of inputs.py; N_rho 3
or 4) on its shell from the flux-balanced background of the section
"Initial Conditions".  Progress goes to stderr.
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


def run(mesh, Q, pr, dt, steps, every, arith, label="", bins=None, ch_every=0, depth=0.28, cfl=0.1):
    """ch_every > 0: every that many steps the GLM speed c_h is reset to the
    current maximum signal speed max(|u| + c_f) over the SPs, the damping to
    c_h / depth and dt to the CFL step of the current state (otherwise all
    three stay at their t = 0 values).  Returns the diagnostic rows (with
    c_h and dt appended when ch_every > 0) and the spherical profiles."""
    import torch
    s = sd.Solver(mesh, arith=arith)
    pr = dict(pr)
    prm = sd.make_params(**pr)
    s.set_state(torch.from_numpy(Q))
    rows = [[0, 0.0] + list(s.diagnostics(prm)[:9]) + [inp.glm_speed(Q)] + ([pr["c_h"], dt] if ch_every else [])]
    sph = {"E_Bpol": [], "E_Btor": []}
    acc = None

    def sample(k):
        nonlocal acc
        P = s.sph_profiles(bins)
        V = P[..., 0].sum()
        sph["E_Bpol"].append([k, P[..., 3].sum() / V])
        sph["E_Btor"].append([k, P[..., 4].sum() / V])
        if k > 0:
            acc = P[..., :3].copy() if acc is None else acc + P[..., :3]

    if bins is not None:
        sample(0)
    t0 = time.perf_counter()
    t = 0.0
    for k in range(1, steps + 1):
        s.step(prm, dt)
        t += dt
        if ch_every and k % ch_every == 0:
            q = s.state.cpu().numpy()
            if np.isfinite(q).all():
                ch = inp.glm_speed(q)
                pr.update(c_h=ch, glm_a=ch / depth)
                prm = sd.make_params(**pr)
                dt = inp.time_step(q, mesh.Sj_sp, ch, cfl)
        if k % every == 0 or k == steps:
            d = s.diagnostics(prm)
            q = s.state.cpu().numpy()
            sig = inp.glm_speed(q) if np.isfinite(q).all() else float("nan")
            rows.append([k, t] + list(d[:9]) + [sig] + ([pr["c_h"], dt] if ch_every else []))
            if bins is not None:
                sample(k)
            print(f"# {label} arith={arith} step {k}: KE={d[3]:.6e} E_B={d[4]:.6e} max|divB|={d[5]:.3e} "
                  f"nan={d[8]:g} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
            if d[8] != 0:
                break
    if bins is None:
        return rows, None
    if acc is not None:
        w = np.where(acc[..., 0] > 0, acc[..., 0], 1.0)
        sph["V_phi"] = (acc[..., 1] / w).tolist()
        sph["V_mer"] = (acc[..., 2] / w).tolist()
    return rows, sph


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
    ap.add_argument("--profiles", default="", metavar="N_R,N_TH",
                    help="also report spherical-component diagnostics on n_r x n_th (r, theta) bins")
    ap.add_argument("--damping", type=float, default=1.0,
                    help="GLM damping a = damping * c_h / (r_t - r_b) (default 1)")
    ap.add_argument("--ch-every", type=int, default=0,
                    help="reset c_h (and the GLM damping and dt) to the current state every that many steps")
    ap.add_argument("--setup", default="seeded", choices=("seeded", "solar"),
                    help="seeded: the polytrope with seeded transport coefficients and heat input; solar: "
                         "the solar benchmark's parameters on its flux-balanced background")
    a = ap.parse_args(argv)
    Nz, Nr = (int(x) for x in a.mesh.split(","))
    if a.setup == "solar":
        # the solar benchmark (N_rho = 3: first, 4: second) on its shell, from
        # the library's flux-balanced background plus the seeded perturbations
        sb = inp.solar_benchmark(a.n_rho)
        bgk = {k: sb[k] for k in ("GM", "Rgas", "gamma", "rb", "rt", "rho_b", "N_rho", "L", "kappa",
                                  "kr_scale", "kr_c0", "kr_c1", "kr_c2", "kr_omega_per_r")}
        bg = inp.Background(a.n_rho, rb=sb["rb"], rt=sb["rt"])
        mesh = sd.shell(Nz, Nr, a.p, bg.rb, bg.rt)
        Q = inp.shell_state(mesh.x_sp, bg, a.seed, profile=lambda r: sd.background_profile(r, **bgk))
        T_top = float(sd.background_profile(np.array([bg.rt]), **bgk)[2][0])
        pr = inp.solar_run_params(sb, T_top)
    else:
        mesh = sd.shell(Nz, Nr, a.p)
        bg = inp.Background(a.n_rho)
        Q = inp.shell_state(mesh.x_sp, bg, a.seed)
        pr = inp.run_params(a.seed, bg)
    ch = inp.glm_speed(Q)
    depth = (bg.rt - bg.rb) / a.damping
    pr.update(c_h=ch, glm_a=ch / depth)
    dt = inp.time_step(Q, mesh.Sj_sp, ch, a.cfl)
    label = f"{a.setup} shell 6x{Nz}x{Nz}x{Nr} p={a.p} N_rho={a.n_rho:g}"
    out = {"workload": f"{label}, seed {a.seed}, {a.steps} SSPRK(5,3) steps, CFL {a.cfl:g}"
                       + (f", GLM damping x{a.damping:g}" if a.damping != 1.0 else "")
                       + (f", c_h, damping and dt reset every {a.ch_every} steps" if a.ch_every else ""),
           "elements": mesh.E, "dt": dt,
           "columns": ["step", "t", *DIAG_NAMES, "max_signal"] + (["c_h", "dt"] if a.ch_every else []),
           "runs": {}}
    bins = None
    if a.profiles:
        n_r, n_th = (int(x) for x in a.profiles.split(","))
        bins = sd.sph_bins(mesh, n_r, n_th, bg.rb, bg.rt)
        out["profile_bins"] = {"n_r": n_r, "n_th": n_th, "r": [bg.rb, bg.rt], "theta": [0.0, float(np.pi)]}
    for ar in (int(x) for x in a.arith.split(",")):
        key = "fp64" if ar == 0 else "fp32-mixed"
        out["runs"][key], sph = run(mesh, Q, pr, dt, a.steps, a.every, ar, label, bins, a.ch_every, depth, a.cfl)
        if sph is not None:
            out.setdefault("spherical", {})[key] = sph
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
