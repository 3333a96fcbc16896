"""Overlapped stage schedule (sdm_set_overlap): the volume passes run chunk
by chunk (radial layers) while the finish passes of completed chunks run on
a second stream.  Every element's arithmetic is that of the plain schedule,
so whole SSPRK(5,3) steps must be bitwise equal to it."""
import numpy as np
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


def _inputs(mesh, N_rho, seed):
    bg = inp.Background(N_rho)
    Q = inp.shell_state(mesh.x_sp, bg, seed)
    pr = inp.run_params(seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    return Q, pr, inp.time_step(Q, mesh.Sj_sp, ch, 0.1)


def _steps(sd, mesh, Q, pr, dt, arith, min_chunk, n):
    import torch
    s = sd.Solver(mesh, arith=arith)
    k = s.set_overlap(min_chunk)
    prm = sd.make_params(**pr)
    s.set_state(torch.from_numpy(Q))
    for _ in range(n):
        s.step(prm, dt)
    torch.cuda.synchronize()
    return s.state.cpu(), k


@pytest.mark.parametrize("Nz,Nr,p,arith,min_chunk", [(4, 3, 5, 0, 1), (4, 3, 5, 1, 1), (8, 4, 3, 0, 100),
                                                      (12, 8, 5, 0, 2048), (12, 8, 5, 1, 700)])
def test_overlap_bitwise(sd, Nz, Nr, p, arith, min_chunk):
    import torch
    print(f"overlap shell 6x{Nz}^2x{Nr} p={p} arith={arith} min_chunk={min_chunk}", flush=True)
    mesh = sd.shell(Nz, Nr, p)
    Q, pr, dt = _inputs(mesh, 5.0, 3)
    ref, k0 = _steps(sd, mesh, Q, pr, dt, arith, 0, 3)
    got, k = _steps(sd, mesh, Q, pr, dt, arith, min_chunk, 3)
    assert k0 == 0 and k >= 2
    assert torch.isfinite(ref).all()
    assert torch.equal(got, ref)


def test_overlap_shard_bitwise(sd):
    """A partition with import faces (cube patch 0 of a shell)."""
    import torch
    full = sd.shell(8, 4, 5)
    Q, pr, dt = _inputs(full, 3.0, 4)
    sh = sd.make_shard(full, np.arange(full.E // 6))
    sf = sd.Solver(full)
    sf.residual(sd.make_params(**pr), torch.from_numpy(Q).cuda())
    iq, iv = sd.gather_imports(sh, *sf.trace_views())
    out = []
    for mc in (0, 64):
        s = sd.Solver(sh.mesh)
        k = s.set_overlap(mc)
        assert (k == 0) == (mc == 0)
        prm = sd.make_params(import_q=iq, import_v=iv, **pr)
        s.set_state(torch.from_numpy(Q[sh.elems]))
        for _ in range(2):
            s.step(prm, dt)
        torch.cuda.synchronize()
        out.append(s.state.cpu())
    assert torch.equal(out[0], out[1])


def test_overlap_toggle_and_rebind(sd):
    """Off again after set_overlap(0); a mesh too small for two chunks leaves
    it off; stages on another stream order correctly."""
    import torch
    mesh = sd.shell(2, 2, 5)
    Q, pr, dt = _inputs(mesh, 3.0, 5)
    s = sd.Solver(mesh)
    assert s.set_overlap(10 ** 6) == 0
    assert s.set_overlap(1) == 2
    assert s.set_overlap(0) == 0
    with pytest.raises(sd.SdmError):
        s.set_overlap(-1)
    ref, _ = _steps(sd, mesh, Q, pr, dt, 0, 0, 2)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        got, k = _steps(sd, mesh, Q, pr, dt, 0, 1, 2)
    assert k == 2 and torch.equal(got, ref)
