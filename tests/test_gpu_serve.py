"""Served ensembles: each run's result is bitwise the same alone, in a mix
of runs of different shell sizes and degrees (one batch call per stage over
all degrees), under forced queueing by a small HBM budget, and through the
single-run stage API; a run that goes non-finite is evicted; batched stages
match the oracle."""
import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_17805_amd import serve
    return serve


def _reqs(serve, steps=3):
    return [serve.Request(0, 2, 1, 5, 3.0, 1000, steps, 0, 0.0),
            serve.Request(1, 2, 2, 3, 5.0, 1001, steps + 1, 0, 0.0),
            serve.Request(2, 3, 1, 5, 5.0, 1002, steps, 0, 0.01),
            serve.Request(3, 2, 1, 3, 3.0, 1003, steps, 1, 0.0)]


def test_alone_equals_mix(srv):
    reqs = _reqs(srv)
    mix, st = srv.Server(max_slots=8, keep_states=True).run(reqs)
    assert st["peak_active"] >= 3
    for q in reqs:
        alone, _ = srv.Server(max_slots=1, keep_states=True).run([q])
        assert np.array_equal(alone[0].state, mix[q.rid].state), q.rid
        assert np.isfinite(mix[q.rid].diag[:8]).all() and mix[q.rid].diag[8] == 0.0


def test_forced_queueing_same_results(srv):
    import dataclasses
    reqs = [dataclasses.replace(q, arrival=0.0) for q in _reqs(srv)]
    budget = max(srv.request_bytes(q) for q in reqs) * 1.01  # the largest fits, not all together
    queued, st = srv.Server(budget_bytes=budget, max_slots=8, keep_states=True).run(reqs)
    assert st["admissions_deferred"] > 0 and st["peak_active"] < len(reqs)
    assert st["peak_bytes"] <= budget
    mix, _ = srv.Server(max_slots=8, keep_states=True).run(reqs)
    for q in reqs:
        assert np.array_equal(queued[q.rid].state, mix[q.rid].state)


def test_batched_equals_single_run_api(srv):
    import torch

    from paper_2502_17805_amd import inputs as inp
    from paper_2502_17805_amd import sdmhd as sd
    q = srv.Request(0, 2, 2, 5, 3.0, 1000, 3, 0, 0.0)
    res, _ = srv.Server(max_slots=2, keep_states=True, max_blocks=64).run([q])
    m = sd.shell(2, 2, 5)
    bg = inp.Background(3.0)
    Q = inp.shell_state(m.x_sp, bg, 1000)
    pr = inp.run_params(1000, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, m.Sj_sp, ch, 0.1)
    s = sd.Solver(m)
    s.set_state(torch.from_numpy(Q))
    prm = sd.make_params(**pr)
    for _ in range(3):
        s.step(prm, dt)
    assert np.array_equal(s.state.cpu().numpy(), res[0].state)


def _batch_step(sd, solvers, prms, dt, bws, nbytes, stream):
    """One SSPRK(5,3) step of several solvers through sdm_batch_stage."""
    import ctypes as C
    ptrs = [(C.c_void_p * 4)(*[r.data_ptr() for r in s.regs]) for s in solvers]
    for cur, inputs, beta, out in sd.ssp53_stages():
        items = (sd.BatchItem * len(solvers))()
        for k, s in enumerate(solvers):
            st = sd.Stage()
            st.n_in = len(inputs)
            for j, (idx, al) in enumerate(inputs):
                st.in_idx[j], st.alpha[j] = idx, al
            st.cur, st.out, st.beta, st.traces_valid = cur, out, beta, 0
            items[k] = sd.BatchItem(s._h.value, C.pointer(prms[k]), ptrs[k], 4, st, dt, s.ws.data_ptr())
        sd._check(sd._lib.sdm_batch_stage(items, len(solvers), bws.data_ptr(), nbytes, 0, stream))


def test_nan_run_does_not_touch_its_batch_neighbours(srv):
    """A run whose state is NaN, batched with a healthy one of another size:
    the healthy run is bitwise what it is alone; the bad one stays NaN."""
    import ctypes as C

    import torch

    from paper_2502_17805_amd import sdmhd as sd
    good_m, bad_m = sd.shell(2, 1, 5), sd.shell(3, 1, 5)
    bg = inp.Background(3.0)
    Qg, Qb = inp.shell_state(good_m.x_sp, bg, 3), inp.shell_state(bad_m.x_sp, bg, 4)
    Qb[2, 4, 17] = np.nan
    pr = inp.run_params(3, bg)
    pr.update(c_h=1.0, glm_a=3.0)
    dt = 1e-3
    nb = C.c_size_t()
    sd._check(sd._lib.sdm_batch_workspace_size(2, C.byref(nb)))
    bws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    prm = [sd.make_params(**pr), sd.make_params(**pr)]
    alone = sd.Solver(good_m)
    alone.set_state(Qg)
    mixed, bad = sd.Solver(good_m), sd.Solver(bad_m)
    mixed.set_state(Qg)
    bad.set_state(Qb)
    for _ in range(2):
        _batch_step(sd, [alone], prm[:1], dt, bws, nb.value, stream)
        _batch_step(sd, [mixed, bad], prm, dt, bws, nb.value, stream)
    torch.cuda.synchronize()
    assert torch.equal(alone.state, mixed.state)
    assert torch.isfinite(alone.state).all() and not torch.isfinite(bad.state).all()


def test_mixed_degree_batch_equals_alone(srv):
    """Runs of degree 3 and 5 (and two shell sizes) advanced together by
    sdm_batch_stage, whose degree groups overlap on the device: each run is
    bitwise what it is when batched alone."""
    import ctypes as C

    import torch

    from paper_2502_17805_amd import sdmhd as sd
    specs = ((2, 1, 3, 3.0, 11), (2, 2, 5, 5.0, 12), (3, 1, 3, 5.0, 13), (2, 1, 5, 3.0, 14))
    made = []
    for Nz, Nr, p, N_rho, seed in specs:
        m = sd.shell(Nz, Nr, p)
        bg = inp.Background(N_rho)
        Q = inp.shell_state(m.x_sp, bg, seed)
        pr = inp.run_params(seed, bg)
        ch = inp.glm_speed(Q)
        pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
        made.append((m, Q, sd.make_params(**pr), inp.time_step(Q, m.Sj_sp, ch, 0.1)))
    dt = min(x[3] for x in made)
    nb = C.c_size_t()
    sd._check(sd._lib.sdm_batch_workspace_size(len(made), C.byref(nb)))
    bws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    mixed = []
    for m, Q, _, _ in made:
        s = sd.Solver(m)
        s.set_state(Q)
        mixed.append(s)
    print(f"mixed-degree batch: {[x[:3] for x in specs]} dt={dt:.3e}", flush=True)
    for _ in range(3):
        _batch_step(sd, mixed, [x[2] for x in made], dt, bws, int(nb.value), stream)
    for k, (m, Q, prm, _) in enumerate(made):
        alone = sd.Solver(m)
        alone.set_state(Q)
        for _ in range(3):
            _batch_step(sd, [alone], [prm], dt, bws, int(nb.value), stream)
        torch.cuda.synchronize()
        assert torch.isfinite(alone.state).all()
        assert torch.equal(alone.state, mixed[k].state), specs[k]


def test_nan_run_is_evicted(srv):
    """A request whose input holds a NaN is evicted on its diagnostics flag
    before its last step; the healthy requests served beside it are bitwise
    what they are alone."""
    import dataclasses

    from paper_2502_17805_amd import sdmhd as sd
    reqs = [srv.Request(0, 2, 1, 5, 3.0, 2000, 40, 0, 0.0), srv.Request(1, 2, 1, 3, 5.0, 2001, 40, 0, 0.0),
            srv.Request(2, 2, 2, 5, 3.0, 2002, 40, 0, 0.0)]
    bad = reqs[1]
    m = sd.shell(bad.Nz, bad.Nr, bad.p)
    Q, pr, dt = srv.prepare(bad, m)
    Q = Q.copy()
    Q[3, 4, 7] = np.nan
    res, st = srv.Server(max_slots=4, keep_states=True, check_every=5).run(reqs, inputs={1: (Q, pr, dt)})
    assert st["evicted"] == 1
    assert res[1].diag[8] == 1.0 and res[1].steps < bad.steps
    for q in (reqs[0], reqs[2]):
        alone, _ = srv.Server(max_slots=1, keep_states=True).run([dataclasses.replace(q, arrival=0.0)])
        assert res[q.rid].diag[8] == 0.0 and res[q.rid].steps == q.steps
        assert np.array_equal(alone[0].state, res[q.rid].state), q.rid


@pytest.mark.parametrize("arith,tol", [(0, 1e-12), (1, 1e-5)])
def test_batched_stages_match_oracle(srv, oracle, arith, tol):
    """Three runs of different degrees, shell sizes and backgrounds advanced
    together by sdm_batch_stage: each run's state after two SSPRK(5,3) steps
    against the FP64 oracle's, within 1e-12 (FP64) or the mixed bound 1e-5
    (FP32-mixed) of max|u_v| + dt T_v.  The inputs are made from the
    oracle's meshes."""
    import ctypes as C

    import torch

    from paper_2502_17805_amd import sdmhd as sd
    runs = []
    for (Nz, Nr, p, N_rho, seed) in ((2, 1, 5, 3.0, 1000), (2, 2, 5, 5.0, 1001), (2, 2, 3, 3.0, 1002)):
        mo = oracle.Mesh.shell(p + 1, Nz, Nr)
        bg = inp.Background(N_rho)
        Q = inp.shell_state(mo.get("x_sp"), bg, seed)
        pr = inp.run_params(seed, bg)
        ch = inp.glm_speed(Q)
        pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
        s = sd.Solver(sd.shell(Nz, Nr, p), arith=arith)
        s.set_state(torch.from_numpy(Q))
        runs.append((s, sd.make_params(**pr), oracle.make_params(**pr), mo, Q))
    dt = 2e-3
    nb = C.c_size_t()
    sd._check(sd._lib.sdm_batch_workspace_size(len(runs), C.byref(nb)))
    bws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(2):
        _batch_step(sd, [r[0] for r in runs], [r[1] for r in runs], dt, bws, int(nb.value), stream)
    torch.cuda.synchronize()
    for s, _, po, mo, Q in runs:
        qo, scale = Q, None
        for _ in range(2):
            _, ts = mo.residual(po, qo, with_scale=True)
            scale = ts if scale is None else np.maximum(scale, ts)
            qo = mo.step(po, qo, dt)
        got = s.state.cpu().numpy()
        err = np.abs(got - qo).max(axis=(0, 2)) / (np.abs(qo).max(axis=(0, 2)) + dt * scale)
        assert (err <= tol).all(), err


def test_batches_from_two_host_threads(srv):
    """Two host threads each advance their own mixed-degree batch on their
    own stream at the same time (the library's streams and events for the
    extra degree groups are shared per device): every run is bitwise what
    the same calls give one after the other."""
    import ctypes as C
    import threading

    import torch

    from paper_2502_17805_amd import sdmhd as sd
    groups = (((2, 1, 3, 3.0, 21), (2, 1, 5, 5.0, 22)), ((2, 2, 3, 5.0, 23), (2, 1, 5, 3.0, 24)))

    def make(specs):
        solvers, prms, dts = [], [], []
        for Nz, Nr, p, N_rho, seed in specs:
            m = sd.shell(Nz, Nr, p)
            bg = inp.Background(N_rho)
            Q = inp.shell_state(m.x_sp, bg, seed)
            pr = inp.run_params(seed, bg)
            ch = inp.glm_speed(Q)
            pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
            s = sd.Solver(m)
            s.set_state(Q)
            solvers.append(s)
            prms.append(sd.make_params(**pr))
            dts.append(inp.time_step(Q, m.Sj_sp, ch, 0.1))
        nb = C.c_size_t()
        sd._check(sd._lib.sdm_batch_workspace_size(len(solvers), C.byref(nb)))
        bws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        return solvers, prms, min(dts), bws, int(nb.value)

    def advance(run, stream, errors):
        solvers, prms, dt, bws, nb = run
        try:
            with torch.cuda.stream(stream):
                for _ in range(3):
                    _batch_step(sd, solvers, prms, dt, bws, nb, C.c_void_p(stream.cuda_stream))
            stream.synchronize()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    print("two host threads, mixed-degree batches", flush=True)
    runs = [make(g) for g in groups]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in groups]
    errors = []
    threads = [threading.Thread(target=advance, args=(r, st, errors)) for r, st in zip(runs, streams)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for g, run in zip(groups, runs):
        ref = make(g)
        torch.cuda.synchronize()
        advance(ref, streams[0], errors)
        assert not errors, errors
        for a, b, spec in zip(run[0], ref[0], g):
            assert torch.isfinite(b.state).all()
            assert torch.equal(a.state, b.state), spec
