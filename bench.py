"""Throughput benchmark of the spectral-difference GLM-MHD hot path on one MI355X.

One benchmark "step" is one full SSPRK(5,3) time step = five fused RK stages,
each a complete residual evaluation (traces, BR1 common solution, gradients,
fluxes, Riemann fluxes, divergence, sources) plus the Shu-Osher update, over
the whole synthetic shell.  Inputs (state, registers, metrics) are resident in
HBM before the timed region.

Workload (default): the 55,296-element cubed-sphere shell (6 x 24 x 24 x 16,
degree p = 5, 11.9M solution points x 9 FP64 variables), polytropic background
with N_rho = 5 plus seeded perturbations, rotation, viscosity/conduction/
resistivity, Powell and GLM terms, conducting heat-flux inner wall and
radial-field fixed-temperature outer wall.

Output: one JSON line (metric: DOF x RK-stage updates per second, FP64) with
the FP32-mixed figure beside it, the roofline of the dominant kernel (from HIP
events recorded around each launch in the timed region), and the FP64 CPU
oracle timed on this host on a bounded sample (one SSPRK step of the same
workload).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {  # name: (Nz, Nr, p, N_rho, seed)
    "shell_55296_p5": (24, 16, 5, 5.0, 2),
    "shell_6912_p5": (12, 8, 5, 3.0, 1),
    "shell_48_p5": (2, 2, 5, 3.0, 0),
    "shell_55296_p3": (24, 16, 3, 5.0, 2),
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def alg_bytes(kind, N, E, n_extra=1.2, fused=True):
    """Algorithmic HBM bytes of one launch: what the method itself must move,
    each once (state, RK registers, stored geometry), independent of the
    implementation's intermediate buffers (face traces, partial residuals,
    the partial stage output).

    stage:        8 [(R_in + 1) 9N^3 + 10N^3 + 9(N+1)N^2 + 3N^3] per element:
                  the state 9N^3, the n_extra further RK registers the
                  Shu-Osher combination reads (0, 0, 1, 2, 3 over the five
                  stages of SSPRK(5,3): 1.2 on average; R_in = 1 + n_extra)
                  and the stage output 9N^3, |J| and S^d/|J| at the SPs
                  10N^3, the metric S^d at the own-family flux points
                  9(N+1)N^2 and the SP positions 3N^3 (gravity), FP64.
    volume:       the state and the geometry; with the fused stage (both
                  arithmetics) the volume pass also reads the further
                  registers and writes the stage output, so all of the
                  stage's bytes.
    finish_stage: the rest: nothing with the fused stage (it moves only
                  intermediate data), else the further registers and the
                  output, 9N^3 each.
    """
    N2, N3 = N * N, N ** 3
    geo = 8 * (9 * N3 + 10 * N3 + 9 * (N + 1) * N2 + 3 * N3)
    rk = 8 * 9 * N3 * (n_extra + 1)
    per = {"volume": geo + (rk if fused else 0), "finish_stage": 0 if fused else rk, "stage": geo + rk}.get(kind)
    return None if per is None else per * E


# FP64 operations (+, -, *, /, sqrt) of one call of each pointwise physics
# function of the FP64 oracle (oracle/sdmhd_oracle_point.inc), counted on
# the host with an operation-counting number type
# (tests/flops/count_oracle_flops.cpp; tests/test_flop_count.py keeps them in
# step with the oracle source).  The kernels compute the same fluxes with
# fewer operations; the algorithmic count is the method's, as the oracle
# states it.
PHYS_FLOPS = {"inv_flux": 92, "visc_flux": 266, "rusanov": 356}


def alg_flops(N):
    """FP64 flops of one residual evaluation per element (Sec. "Spectral
    Difference Method"): the tensor contractions as multiply-adds (Q to the
    flux points of each family, the derivative of the flux-point polynomial
    at the SPs, the 27 gradient components to the flux points, the flux
    divergence, the chain rule), plus the pointwise physics as the oracle
    computes it: per interior flux point the inviscid and viscous fluxes
    through S^d and their difference (inv_flux + visc_flux + 9), per unique
    face point the Rusanov flux, both sides' viscous fluxes and the BR1
    average (rusanov + 2 visc_flux + 27), per SP the sources and the scaling
    by 1/|J| (67).  Wall faces are counted as interior faces; the RK update
    is not part of the residual."""
    N2, N3, NF = N * N, N ** 3, (N + 1) * N * N
    mac = 3 * 9 * NF * N + 3 * 9 * N3 * (N + 1) + 27 * 3 * NF * N + 3 * 9 * N3 * (N + 1) + 27 * 3 * N3
    f = PHYS_FLOPS
    interior = f["inv_flux"] + f["visc_flux"] + 9
    face = f["rusanov"] + 2 * f["visc_flux"] + 27
    point = interior * 3 * N2 * (N - 1) + face * 3 * N2 + 67 * N3
    return 2 * mac + point


def kernel_source_hash(root=ROOT):
    """Hash of the kernel sources with // comments removed and runs of
    whitespace collapsed, so that an edit of comments or layout alone does
    not invalidate counters taken on the code (the sources hold no string
    containing //)."""
    h = hashlib.sha256()
    for f in ("sdm_kernels.hip", "sdm_physics.hpp"):
        data = open(os.path.join(root, "paper_2502_17805_amd", "csrc", f), "rb").read()
        data = re.sub(rb"//[^\n]*", b"", data)
        h.update(re.sub(rb"\s+", b" ", data))
    return h.hexdigest()[:16]


def measured_traffic(kernel, config, arith):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        ent = d.get(f"{kernel}/{config}/{'fp64' if arith == 0 else 'mixed'}")
        if not ent or ent.get("source_hash") != kernel_source_hash():
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def _timed_steps(torch, s, prm, dt, steps):
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step(prm, dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), time.perf_counter() - t0


def run_gpu(sd, inp, cfg_name, arith, steps, warmup, mesh, Q, pr, dt, prof_steps=5):
    """Timed steps, then a few steps with the library's per-launch HIP events
    (per-kernel times)."""
    import torch
    s = sd.Solver(mesh, arith=arith)
    prm = sd.make_params(**pr)
    s.set_state(torch.from_numpy(Q))
    for _ in range(warmup):
        s.step(prm, dt)
    ms, wall = _timed_steps(torch, s, prm, dt, steps)
    s.profile(True)
    _timed_steps(torch, s, prm, dt, prof_steps)
    prof = s.profile_read()
    s.profile(False)
    d = s.diagnostics(prm)
    return {"ms": ms, "wall": wall, "prof": prof, "prof_steps": prof_steps, "diag": d}


def run_shard(sd, mesh, Q, pr, dt, steps, warmup):
    """One GPU's share of the shell split by cube patch (6 ways): patch 0 with
    its partition faces as import faces.  The halo buffers are filled once
    from an unsplit residual evaluation (a split run would refresh them
    between the launches of every stage); the timed work is the partition's
    own stages."""
    import torch
    sh = sd.make_shard(mesh, np.arange(mesh.E // 6))
    sf = sd.Solver(mesh)
    sf.residual(sd.make_params(**pr), torch.from_numpy(Q).cuda())
    iq, iv = sd.gather_imports(sh, *sf.trace_views())
    del sf
    s = sd.Solver(sh.mesh)
    prm = sd.make_params(import_q=iq, import_v=iv, **pr)
    s.set_state(torch.from_numpy(Q[sh.elems]))
    for _ in range(warmup):
        s.step(prm, dt)
    ms = _timed_steps(torch, s, prm, dt, steps)[0] / steps
    dof = sh.mesh.E * sh.mesh.N ** 3
    return {"workload": f"cube patch 0 of the same shell ({sh.mesh.E} elements, {len(sh.imports)} import faces), "
                        "FP64, halo buffers fixed", "elements": sh.mesh.E, "ms_per_step": ms,
            "value": dof * 5 / (ms * 1e-3), "unit": "DOF*RK-stage updates/s"}


def run_serving(n_requests, ariths):
    """The served ensemble: n_requests runs arriving as a Poisson process
    (mean gap 20 ms), shells 6 x {4,8,12}^2 x {3,4,8}, p in {3,5}, N_rho in
    {3,5}, 500 SSPRK(5,3) steps each, admitted by a 200 GB HBM budget and a
    cap of 32,768 resident elements, with continuous batching of their
    stages; completion-latency percentiles and aggregate DOF x RK-stage
    throughput per arithmetic."""
    from paper_2502_17805_amd import serve
    res = {}
    for arith in ariths:
        reqs = serve.poisson_requests(n_requests, 0.020, 500, arith=arith)
        results, st = serve.Server(budget_bytes=200e9, max_slots=64, max_elements=32768).run(reqs)
        res["fp64" if arith == 0 else "fp32_mixed"] = dict(
            requests=st["requests"], p50_latency_s=st["p50_latency_s"], p99_latency_s=st["p99_latency_s"],
            dof_stage_per_s=st["dof_stage_per_s"], makespan_s=st["makespan_s"], peak_active=st["peak_active"],
            nan_results=int(sum(r.diag[8] != 0 for r in results)))
    return res


def copy_rate(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (GB/s, bytes read + written) of a plain
    1 GiB copy: the practical HBM streaming rate the stage is compared to."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    return 2 * nbytes * reps / (ms * 1e-3) / 1e9


_SINGLE_CORE_CHILD = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as o
from paper_2502_17805_amd import inputs as inp
Nz, Nr, p, N_rho, seed = json.loads(sys.argv[2])
m = o.Mesh.shell(p + 1, Nz, Nr)
bg = inp.Background(N_rho)
Q = inp.shell_state(m.get("x_sp"), bg, seed)
pr = inp.run_params(seed, bg)
ch = inp.glm_speed(Q)
pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
t0 = time.perf_counter()
m.residual(o.make_params(**pr), Q)
t = time.perf_counter() - t0
print(json.dumps({"E": m.E, "seconds": t, "threads": o.threads()}))
"""


def cpu_single_core(Nz=12, Nr=8, p=5, N_rho=5.0, seed=3):
    """The oracle on one host core: one residual evaluation (the work of one
    RK stage) of the 6,912-element shell, in a child process started with
    OMP_NUM_THREADS=1 (the thread count is fixed when OpenMP starts)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _SINGLE_CORE_CHILD, ROOT, json.dumps([Nz, Nr, p, N_rho, seed])],
                       env=env, capture_output=True, text=True, timeout=300, check=True)
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["E"] * (p + 1) ** 3 / d["seconds"], "unit": "DOF*RK-stage updates/s",
            "cores": d["threads"], "kind": "oracle",
            "sample": f"one residual evaluation (one RK stage) of the {d['E']}-element p={p} shell, "
                      f"FP64 C oracle, {d['seconds']:.1f} s"}


def cpu_baseline(cfg, Q_fn, pr, dt):
    from oracle import oracle as o
    Nz, Nr, p, _, _ = cfg
    m = o.Mesh.shell(p + 1, Nz, Nr)
    Q = Q_fn(m.get("x_sp"))
    prm = o.make_params(**pr)
    t0 = time.perf_counter()
    m.step(prm, Q, dt)
    t = time.perf_counter() - t0
    dof = m.E * (p + 1) ** 3
    return {"value": dof * 5 / t, "unit": "DOF*RK-stage updates/s", "cores": o.threads(), "kind": "oracle",
            "sample": f"one SSPRK(5,3) step (5 stages) of the same {m.E}-element p={p} shell, "
                      f"FP64 C oracle, OpenMP over elements, {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="shell_55296_p5", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--cfl", type=float, default=0.1)
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="served-ensemble leg: that many Poisson-arriving runs of 500 steps (0: skip)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="BYTES",
                    help="first run a plain device copy of BYTES bytes (read BYTES, write BYTES) three "
                         "times, the reference that HBM byte counters are scaled by")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): sharding the shell "
              "across GPUs is not built in this library", file=sys.stderr)
        sys.exit(2)

    # the single-core oracle runs in a child process started before this
    # process touches the GPU
    single_core = None
    if not args.no_cpu_baseline:
        try:
            single_core = cpu_single_core()
        except Exception as ex:  # report, do not hide
            single_core = {"value": None, "error": repr(ex)}

    import torch
    from paper_2502_17805_amd import inputs as inp
    from paper_2502_17805_amd import sdmhd as sd

    if args.copy_calibration > 0:
        n = int(args.copy_calibration) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        print(f"# copy calibration: 3 x {8 * n} bytes read and written", file=sys.stderr, flush=True)

    cfg = CONFIGS[args.config]
    Nz, Nr, p, N_rho, seed = cfg
    N = p + 1
    t0 = time.perf_counter()
    mesh = sd.shell(Nz, Nr, p)
    t_mesh = time.perf_counter() - t0
    bg = inp.Background(N_rho)
    Q = inp.shell_state(mesh.x_sp, bg, seed)
    pr = inp.run_params(seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, mesh.Sj_sp, ch, args.cfl)
    dof = mesh.E * N ** 3
    print(f"# mesh {args.config}: E={mesh.E} DOF={dof} host build {t_mesh:.1f}s dt={dt:.3e}", file=sys.stderr,
          flush=True)

    res = {}
    for arith in ((0,) if args.no_mixed else (0, 1)):
        r = run_gpu(sd, inp, args.config, arith, args.steps, args.warmup, mesh, Q, pr, dt)
        res[arith] = r
        print(f"# arith={arith}: {r['ms'] / args.steps:.3f} ms/step; kernels {r['prof']}; "
              f"KE={r['diag'][3]:.3e} nan={r['diag'][8]}", file=sys.stderr, flush=True)

    r0 = res[0]
    ms, prof, diag = r0["ms"], r0["prof"], r0["diag"]
    stages = 5 * args.steps
    value = dof * stages / (ms * 1e-3)
    # roofline of the dominant kernel (largest summed time), from the HIP
    # events the library records around each launch on its stream.  Its bound is the
    # larger of the two algorithmic times: bytes at the HBM peak, FP64 flops
    # at the FP64 vector peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4
    # GHz = 78.6 TFLOP/s).
    dom = max(prof, key=lambda k: prof[k][0])
    avg_ms = prof[dom][0] / prof[dom][1]
    t = avg_ms * 1e-3
    bytes_launch = alg_bytes(dom, N, mesh.E)
    flops_launch = alg_flops(N) * mesh.E if dom == "volume" else 0
    traffic = measured_traffic(dom, args.config, 0)
    hbm_gbs = bytes_launch / t / 1e9 if bytes_launch else None
    tflops = flops_launch / t / 1e12
    alu_bound = flops_launch / (FP64_PEAK_TFLOPS * 1e12) > (bytes_launch or 0) / (HBM_PEAK_GBS * 1e9)
    if alu_bound:
        roof = {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / FP64_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None}
    roof.update({"traffic": traffic, "kernel": f"k_volume<{N}, double>" if dom == "volume" else dom,
                 "avg_launch_ms": avg_ms, "alg_bytes_per_launch": bytes_launch,
                 "alg_fp64_flops_per_launch": flops_launch, "alg_hbm_gbs": hbm_gbs,
                 "alg_hbm_frac": hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None,
                 "alg_fp64_tflops": tflops, "alg_fp64_frac": tflops / FP64_PEAK_TFLOPS,
                 "measured_hbm_gbs": traffic / t / 1e9 if traffic else None})
    # the whole stage (all kernels of one RK stage) against the same bounds
    t_stage = ms * 1e-3 / stages
    stage_roof = {"alg_bytes": alg_bytes("stage", N, mesh.E), "ms": t_stage * 1e3,
                  "hbm_frac": alg_bytes("stage", N, mesh.E) / t_stage / 1e9 / HBM_PEAK_GBS,
                  "fp64_frac": alg_flops(N) * mesh.E / t_stage / 1e12 / FP64_PEAK_TFLOPS}
    # measured HBM bytes of a stage (volume + finish pass, rocprofv3 counters
    # taken on the current kernel source), against the spec peak and against
    # the copy rate measured here
    tv, tf = measured_traffic("volume", args.config, 0), measured_traffic("finish_stage", args.config, 0)
    crate = copy_rate(torch)
    stage_roof["copy_gbs"] = crate
    if tv and tf:
        stage_roof.update({"measured_bytes": tv + tf,
                           "measured_hbm_frac": (tv + tf) / t_stage / 1e9 / HBM_PEAK_GBS,
                           "measured_copy_frac": (tv + tf) / t_stage / 1e9 / crate})
    out = {
        "metric": "SD-MHD DOF*RK-stage updates/s (FP64)",
        "value": value,
        "unit": "DOF*RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cubed-sphere shell 6x{Nz}x{Nz}x{Nr} = {mesh.E} elements, p={p}, "
                               f"{dof} solution points x 9 vars, N_rho={N_rho:g}, SSPRK(5,3) step = 5 stages",
                   "elements": mesh.E, "p": p, "dof": dof, "stages_per_step": 5, "parallelism": "single GPU"},
        "roofline": roof,
        "stage_roofline": stage_roof,
        "kernels_ms_per_step": {k: v[0] / r0["prof_steps"] for k, v in prof.items()},
        "variable_dof_value": 9 * value,
        "variable_dof_unit": "variable-DOF*RK-stage updates/s (9 variables per solution point)",
    }
    if 1 in res:
        r1 = res[1]
        ms1 = r1["ms"]
        out["mixed_fp32"] = {"value": dof * stages / (ms1 * 1e-3), "ms_per_step": ms1 / args.steps,
                             "kernels_ms_per_step": {k: v[0] / r1["prof_steps"]
                                                     for k, v in r1["prof"].items()},
                             "speedup_vs_fp64": ms / ms1}
    if args.serve_requests > 0:
        out["serving"] = run_serving(args.serve_requests, (0,) if args.no_mixed else (0, 1))
        for k, v in out["serving"].items():
            print(f"# serving {k}: p50 {v['p50_latency_s']:.2f} s, p99 {v['p99_latency_s']:.2f} s, "
                  f"{v['dof_stage_per_s']:.3e} DOF-stage/s", file=sys.stderr, flush=True)
    if not args.no_shard and args.config != "shell_48_p5":
        out["shard_6way"] = run_shard(sd, mesh, Q, pr, dt, min(args.steps, 20), args.warmup)
        print(f"# shard: {out['shard_6way']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(cfg, lambda x: inp.shell_state(x, bg, seed), pr, dt)
            out["cpu_baseline"]["single_core"] = single_core
        except Exception as ex:  # report, do not hide
            out["cpu_baseline"] = {"value": None, "error": repr(ex)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
