"""Served ensembles: each run's result is bitwise the same alone, in a mix
of runs of different shell sizes and degrees, under forced queueing by a small
HBM budget, and through the single-run stage API."""
import numpy as np
import pytest

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
