"""SSPRK(5,3) steps captured in a HIP graph (through torch's graph capture
on a side stream) and replayed: every replay, with eager steps and
synchronisations of the program in between, is bitwise the eager step.  The
step enqueues kernels only (no memset, copy or synchronisation), so both the
workspace step and the allocation-free one can be captured."""
import pytest

from paper_2502_17805_amd import inputs as inp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_17805_amd import sdmhd
    return sdmhd


@pytest.mark.parametrize("arith", [0, 1])
@pytest.mark.parametrize("noalloc", [False, True])
def test_graph_replays_equal_eager_steps(sd, arith, noalloc):
    import torch
    print(f"graph replay arith={arith} noalloc={noalloc}", flush=True)
    m = sd.shell(3, 2, 5)
    bg = inp.Background(5.0)
    Q = torch.from_numpy(inp.shell_state(m.x_sp, bg, 6))
    pr = inp.run_params(6, bg)
    ch = inp.glm_speed(Q.numpy())
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q.numpy(), m.Sj_sp, ch, 0.1)
    prm = sd.make_params(**pr)
    g_sv, ref = sd.Solver(m, arith=arith), sd.Solver(m, arith=arith)
    for s in (g_sv, ref):
        s.set_state(Q)
    step = (lambda s: s.step_noalloc(prm, dt)) if noalloc else (lambda s: s.step(prm, dt))
    step(g_sv)  # the workspace step then starts captures with valid traces
    step(ref)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            step(g_sv)
    torch.cuda.synchronize()
    for i in range(3):
        graph.replay()
        torch.cuda.synchronize()
        step(ref)
        torch.cuda.synchronize()
        assert torch.isfinite(ref.state).all()
        assert torch.equal(g_sv.state, ref.state), i
