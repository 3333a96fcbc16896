"""Continuous-batching server for ensembles of independent SD-MHD runs on one GPU.

Requests (shell size, polynomial degree, density scale heights, seed, number of
SSPRK(5,3) steps, arithmetic) arrive over time.  A request is admitted as soon
as a slot is free and its device memory fits the HBM budget; its mesh, state
registers and workspace then stay resident on the device until it finishes.
Every scheduler iteration enqueues one SSPRK(5,3) step of each active run:
for each of the five stages, the stages of all active runs of one arithmetic
go into one sdm_batch_stage call, whose work lists cover every degree (the
degree groups of one call overlap on the device), so runs that arrive while
others are on the GPU join the same launches.  The host does not wait for
the GPU after each step: it stays at most `ahead` steps in front (events),
and learns that a run has finished, or has gone non-finite, by polling the
event after its diagnostics, which are copied to pinned host memory
asynchronously.  A run whose periodic diagnostics report NaN/Inf is evicted
(its result carries the flag).  A run's arithmetic is exactly that of a
single-run stage, so its result is bitwise the same alone and in any mix.
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import time

import numpy as np

from . import inputs as inp
from . import sdmhd as sd


@dataclasses.dataclass
class Request:
    rid: int
    Nz: int
    Nr: int
    p: int
    N_rho: float
    seed: int
    steps: int
    arith: int = 0
    arrival: float = 0.0  # seconds after the server starts

    @property
    def dof(self):
        return 6 * self.Nz * self.Nz * self.Nr * (self.p + 1) ** 3


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    steps: int
    dof: int
    diag: np.ndarray
    state: np.ndarray | None = None

    @property
    def latency(self):
        return self.done - self.arrival


class _MeshCache:
    """Host meshes and their device copies, shared by runs of equal shape."""

    def __init__(self, device):
        self.device = device
        self.host = {}
        self.dev = {}
        self.users = collections.Counter()

    def host_mesh(self, Nz, Nr, p):
        key = (Nz, Nr, p)
        if key not in self.host:
            self.host[key] = sd.shell(Nz, Nr, p)
        return self.host[key]

    def get(self, Nz, Nr, p):
        import torch
        key = (Nz, Nr, p)
        self.host_mesh(Nz, Nr, p)
        if key not in self.dev:
            m = self.host[key]
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)  # noqa: E731
            self.dev[key] = dict(x_sp=t(m.x_sp), detJ=t(m.detJ), S_fp=t(m.S_fp), Sj_sp=t(m.Sj_sp),
                                 nbr=t(m.nbr), n_face=t(m.n_face))
        self.users[key] += 1
        return self.host[key], self.dev[key]

    def release(self, Nz, Nr, p):
        key = (Nz, Nr, p)
        self.users[key] -= 1
        if self.users[key] == 0:
            del self.dev[key]  # device copy freed; the host mesh stays cached

    @staticmethod
    def device_bytes(Nz, Nr, p):
        E, N = 6 * Nz * Nz * Nr, p + 1
        N3, NF = N ** 3, (N + 1) * N * N
        return 8 * E * (3 * N3 + N3 + 9 * NF + 9 * N3 + 18 * N * N) + 4 * E * 6


def request_bytes(q: Request) -> int:
    """Device bytes a request holds while resident: four FP64 state
    registers, the workspace (face traces, viscous traces, partial residual
    in the arithmetic type), its mesh arrays (counted per request) and, in
    the mixed arithmetic, the FP32 geometry copies its context makes."""
    E, N = 6 * q.Nz * q.Nz * q.Nr, q.p + 1
    rs = 4 if q.arith else 8
    ws = rs * E * (6 * 9 * N * N + 6 * 7 * N * N + 9 * N ** 3) + 3 * 256
    mesh = _MeshCache.device_bytes(q.Nz, q.Nr, q.p)
    geo32 = 0
    if q.arith:
        N3, NF = N ** 3, (N + 1) * N * N
        geo32 = 4 * E * (3 * N3 + N3 + 9 * NF + 9 * N3 + 18 * N * N) + 5 * 256
    return 4 * 8 * 9 * q.dof + ws + mesh + geo32


def prepare(req: Request, mesh):
    """The request's input: seeded initial state, physical parameters and
    time step (synthesised on the host; a client would send them)."""
    bg = inp.Background(req.N_rho)
    Q = inp.shell_state(mesh.x_sp, bg, req.seed)
    pr = inp.run_params(req.seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    return Q, pr, inp.time_step(Q, mesh.Sj_sp, ch, 0.1)


class _Run:
    """One admitted request resident on the device."""

    def __init__(self, req: Request, cache: _MeshCache, device, t_admit, prepared=None):
        import torch
        self.req = req
        self.t_admit = t_admit
        mesh, dev = cache.get(req.Nz, req.Nr, req.p)
        self.mesh, self.devmesh = mesh, dev
        h = C.c_void_p()
        sd._check(sd._lib.sdm_create(device.index or 0, req.p, req.arith, C.byref(h)))
        self.ctx = h
        md = sd.MeshDesc(mesh.E, mesh.NB, dev["x_sp"].data_ptr(), dev["detJ"].data_ptr(), dev["S_fp"].data_ptr(),
                         dev["Sj_sp"].data_ptr(), dev["nbr"].data_ptr(), dev["n_face"].data_ptr())
        sd._check(sd._lib.sdm_mesh_bind(h, C.byref(md)))
        nb = C.c_size_t()
        sd._check(sd._lib.sdm_workspace_size(h, C.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        Q, pr, self.dt = prepared if prepared is not None else prepare(req, mesh)
        self.prm = sd.make_params(**pr)
        shp = (mesh.E, 9, mesh.N ** 3)
        self.regs = [torch.empty(shp, dtype=torch.float64, device=device) for _ in range(4)]
        self.regs[0].copy_(torch.from_numpy(Q))
        self.reg_ptrs = (C.c_void_p * 4)(*[r.data_ptr() for r in self.regs])
        self.steps_done = 0
        self.traces_valid = False
        self.bytes = request_bytes(req)
        # host side of the run's asynchronous diagnostics (pinned) and the
        # event after which they are valid
        self.diag_dev = torch.zeros(16, dtype=torch.float64, device=device)
        self.diag_host = torch.zeros(16, dtype=torch.float64).pin_memory()
        self.diag_event = None
        self.state_host = None

    def enqueue_diagnostics(self, stream, keep_state=False):
        """Diagnostics of register 0 into pinned host memory after the work
        enqueued so far; returns the event after which they are valid."""
        import torch
        sd._check(sd._lib.sdm_diagnostics(self.ctx, C.byref(self.prm), self.regs[0].data_ptr(),
                                          self.diag_dev.data_ptr(), self.ws.data_ptr(), stream))
        self.diag_host.copy_(self.diag_dev, non_blocking=True)
        if keep_state:
            self.state_host = torch.empty(self.regs[0].shape, dtype=torch.float64).pin_memory()
            self.state_host.copy_(self.regs[0], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self.diag_event = ev
        return ev

    def item(self, cur, inputs, beta, out):
        st = sd.Stage()
        st.n_in = len(inputs)
        for k, (idx, al) in enumerate(inputs):
            st.in_idx[k] = idx
            st.alpha[k] = al
        st.cur, st.out, st.beta = cur, out, beta
        st.traces_valid = 1 if self.traces_valid else 0
        self.traces_valid = True  # every stage leaves the traces of its output
        return sd.BatchItem(self.ctx.value, C.pointer(self.prm), self.reg_ptrs, 4, st, self.dt, self.ws.data_ptr())

    def close(self, cache):
        sd._lib.sdm_destroy(self.ctx)
        cache.release(self.req.Nz, self.req.Nr, self.req.p)


class Server:
    """Admission by slots and HBM budget; one batched SSPRK step per iteration,
    enqueued without waiting for the GPU."""

    def __init__(self, budget_bytes: float = 200e9, max_slots: int = 64, device: int = 0, max_blocks: int = 0,
                 keep_states=False, max_elements: int = 0, ahead: int = 2, check_every: int = 50):
        """keep_states: True (all), a set of request ids, or False: whose
        final states are copied back with their results.  max_elements > 0
        caps the elements resident at once (admission waits while the cap
        would be exceeded, except for a request that is alone): enough
        elements keep every CU busy, more only lengthen every resident
        request's latency.  ahead: steps the host may enqueue before the GPU
        has finished them.  check_every: steps between a run's NaN checks
        (0: only at the end)."""
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.max_elements = max_elements
        self.max_blocks = max_blocks
        self.keep_states = keep_states
        self.ahead = max(1, ahead)
        self.check_every = check_every
        self.cache = _MeshCache(self.device)
        nb = C.c_size_t()
        sd._check(sd._lib.sdm_batch_workspace_size(max_slots, C.byref(nb)))
        self.batch_ws_bytes = int(nb.value)
        self.batch_ws = torch.empty(self.batch_ws_bytes, dtype=torch.uint8, device=self.device)
        self.stats = {}

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _step_all(self, active):
        """Enqueue one SSPRK(5,3) step of every active run: per stage one
        batch call per arithmetic, over runs of any degree."""
        groups = collections.defaultdict(list)
        for r in active:
            groups[r.req.arith].append(r)
        stages = sd.ssp53_stages()
        for cur, inputs, beta, out in stages:
            for runs in groups.values():
                items = (sd.BatchItem * len(runs))(*[r.item(cur, inputs, beta, out) for r in runs])
                sd._check(sd._lib.sdm_batch_stage(items, len(runs), self.batch_ws.data_ptr(), self.batch_ws_bytes,
                                                  self.max_blocks, self._stream()))
        for r in active:
            r.steps_done += 1

    def run(self, requests, prepare_inputs: bool = True, inputs=None):
        """Serve the requests (arrival times relative to the start).  With
        prepare_inputs the requests' inputs and meshes are made on the host
        before the clock starts, so the latencies measure the GPU service.
        inputs: {rid: (Q, params dict, dt)} given instead of the seeded ones."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        prepared = dict(inputs or {})
        if prepare_inputs:
            for q in pending:
                if q.rid not in prepared:
                    prepared[q.rid] = prepare(q, self.cache.host_mesh(q.Nz, q.Nr, q.p))
        active, draining, results = [], [], []
        inflight = collections.deque()  # events of the steps enqueued and not yet waited for
        used, peak_used, peak_active, iters, queued_wait, evicted = 0, 0, 0, 0, 0, 0
        stream = self._stream()
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()

        def keep(r):
            return self.keep_states is True or (self.keep_states and r.req.rid in self.keep_states)

        while pending or active or draining:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now and len(active) + len(draining) < self.max_slots:
                q = pending[0]
                E_q = 6 * q.Nz * q.Nz * q.Nr
                resident = active + draining
                over_elems = self.max_elements > 0 and resident and \
                    sum(6 * r.req.Nz * r.req.Nz * r.req.Nr for r in resident) + E_q > self.max_elements
                if used + request_bytes(q) > self.budget or over_elems:
                    queued_wait += 1
                    break
                pending.popleft()
                r = _Run(q, self.cache, self.device, time.perf_counter() - t0, prepared.pop(q.rid, None))
                used += r.bytes
                active.append(r)
            peak_used = max(peak_used, used)
            peak_active = max(peak_active, len(active) + len(draining))
            # runs whose last diagnostics have arrived: done (or evicted)
            still = []
            for r in draining:
                if r.diag_event.query():
                    tnow = time.perf_counter() - t0
                    st = r.state_host.numpy().copy() if r.state_host is not None else None
                    results.append(Result(r.req.rid, r.req.arrival, r.t_admit, tnow, r.steps_done, r.req.dof,
                                          r.diag_host.numpy().copy(), st))
                    used -= r.bytes
                    r.close(self.cache)
                else:
                    still.append(r)
            draining = still
            # periodic NaN checks whose diagnostics have arrived
            for r in list(active):
                if r.diag_event is not None and r.diag_event.query():
                    if r.diag_host[8].item() != 0.0:
                        active.remove(r)
                        evicted += 1
                        r.enqueue_diagnostics(stream, keep(r))
                        draining.append(r)
                    r.diag_event = None if r in active else r.diag_event
            if not active:
                if draining:
                    time.sleep(0.0002)
                elif pending:
                    time.sleep(max(0.0, min(0.002, pending[0].arrival - (time.perf_counter() - t0))))
                continue
            self._step_all(active)
            iters += 1
            ev = torch.cuda.Event()
            ev.record()
            inflight.append(ev)
            if len(inflight) > self.ahead:
                inflight.popleft().synchronize()
            still = []
            for r in active:
                if r.steps_done >= r.req.steps:
                    r.enqueue_diagnostics(stream, keep(r))
                    draining.append(r)
                    continue
                if self.check_every and r.steps_done % self.check_every == 0 and r.diag_event is None:
                    r.enqueue_diagnostics(stream)
                still.append(r)
            active = still
        makespan = time.perf_counter() - t0
        lat = np.array([x.latency for x in results])
        work = sum(x.dof * 5 * x.steps for x in results)
        self.stats = dict(requests=len(results), makespan_s=makespan, iterations=iters,
                          p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else None,
                          p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else None,
                          dof_stage_per_s=work / makespan if makespan > 0 else None,
                          peak_active=peak_active, peak_bytes=peak_used, admissions_deferred=queued_wait,
                          evicted=evicted)
        return sorted(results, key=lambda x: x.rid), self.stats


def poisson_requests(n: int = 64, mean_gap_s: float = 0.020, steps: int = 500, seed: int = 7,
                     meshes=((4, 3), (8, 4), (12, 8)), degrees=(3, 5), n_rhos=(3.0, 5.0), arith: int = 0):
    """The served-ensemble workload: Poisson arrivals, mesh, degree and N_rho
    drawn uniformly, run seeds 1000 + request index."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(mean_gap_s)
        Nz, Nr = meshes[rng.integers(len(meshes))]
        out.append(Request(i, int(Nz), int(Nr), int(degrees[rng.integers(len(degrees))]),
                           float(n_rhos[rng.integers(len(n_rhos))]), 1000 + i, steps, arith, t))
    return out


def main(argv=None):
    """Serve the Poisson ensemble once and print one JSON line: latency
    percentiles, aggregate DOF x RK-stage throughput, admission figures, and
    the bitwise alone-vs-mixed check of the first `--identity` requests."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--arith", type=int, default=0)
    ap.add_argument("--mean-gap", type=float, default=0.020)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--identity", type=int, default=3)
    ap.add_argument("--max-elements", type=int, default=32768,
                    help="cap on resident elements (0: none); see Server")
    a = ap.parse_args(argv)
    reqs = poisson_requests(a.requests, a.mean_gap, a.steps, arith=a.arith)
    ids = set(range(min(a.identity, len(reqs))))
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_slots=a.slots, keep_states=ids, max_elements=a.max_elements)
    res, st = srv.run(reqs)
    same = []
    for i in sorted(ids):
        alone, _ = Server(max_slots=1, keep_states=True).run([dataclasses.replace(reqs[i], arrival=0.0)])
        same.append(bool(np.array_equal(alone[0].state, res[i].state)))
    out = dict(workload=f"{a.requests} requests, Poisson arrivals (mean gap {a.mean_gap * 1e3:g} ms), shells "
                        f"6x{{4,8,12}}^2x{{3,4,8}}, p in {{3,5}}, N_rho in {{3,5}}, {a.steps} SSPRK(5,3) steps each",
               arith="fp64" if a.arith == 0 else "fp32-mixed", budget_gb=a.budget_gb, slots=a.slots,
               max_elements=a.max_elements,
               nan_results=int(sum(r.diag[8] != 0 for r in res)), alone_vs_mix_bitwise=same, **st)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
