"""The allocation-free SSPRK(5,3) step (sdm_ssprk53_step_noalloc) against the
workspace one (sdm_ssprk53_step), through the C ABI: two calls in a row on
one device, the second on a smaller mesh (the static scratch keeps the first
call's traces, which the second must not use), in FP64 and FP32-mixed; then
the size limit of the scratch at its boundary.

The two entry points run the same kernels on the same inputs, so the results
must agree bitwise; the FP64 parity bar (1e-12 of the state plus dt times the
residual's term scale) is checked as well, as the parity tests state it."""
import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module")
def sd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_17805_amd import sdmhd
    return sdmhd


def _setup(sd, Nz, Nr, seed, arith):
    import torch
    m = sd.shell(Nz, Nr, 5)
    bg = inp.Background(3.0)
    Q = inp.shell_state(m.x_sp, bg, seed)
    pr = inp.run_params(seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, m.Sj_sp, ch, 0.1)
    s = sd.Solver(m, arith=arith)
    return s, sd.make_params(**pr), torch.from_numpy(Q).cuda(), dt


def _pair(sd, Nz, Nr, seed, arith, steps=2):
    """(workspace result, no-allocation result) after `steps` steps."""
    import torch
    s, prm, Q, dt = _setup(sd, Nz, Nr, seed, arith)
    regs = [torch.zeros_like(Q) for _ in range(4)]
    regs[0].copy_(Q)
    s.set_state(Q)
    for _ in range(steps):
        s.step(prm, dt)
        s.step_noalloc(prm, dt, regs=regs)
    torch.cuda.synchronize()
    return s.state.cpu().numpy(), regs[0].cpu().numpy(), dt


@pytest.mark.parametrize("arith", [0, 1])
def test_noalloc_step_equals_workspace_step_twice_shrinking(sd, arith):
    # first call: 6 x 3^2 x 2 = 108 elements; second: 6 x 2^2 x 1 = 24
    for Nz, Nr, seed in ((3, 2, 4), (2, 1, 5)):
        print(f"noalloc: shell 6x{Nz}^2x{Nr} p=5 arith={arith} seed={seed}", flush=True)
        a, b, dt = _pair(sd, Nz, Nr, seed, arith)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), np.abs(a - b).max()


def test_noalloc_matches_oracle_bar(sd, oracle):
    import torch
    # FP64 two steps of the 48-element shell against the oracle, at the bar
    # of the parity tests; the inputs are made from the oracle's mesh
    Nz, Nr, seed = 2, 2, 0
    om = oracle.Mesh.shell(6, Nz, Nr)
    bg = inp.Background(3.0)
    q0 = inp.shell_state(om.get("x_sp"), bg, seed)
    pr = inp.run_params(seed, bg)
    ch = inp.glm_speed(q0)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(q0, om.get("S_sp") / om.get("detJ_sp")[:, None, None, :], ch, 0.1)
    s = sd.Solver(sd.shell(Nz, Nr, 5))
    prm, po = sd.make_params(**pr), oracle.make_params(**pr)
    s.set_state(torch.from_numpy(q0))
    want, scale = q0, None
    for _ in range(2):
        s.step_noalloc(prm, dt)
        _, ts = om.residual(po, want, with_scale=True)
        scale = ts if scale is None else np.maximum(scale, ts)
        want = om.step(po, want, dt)
    torch.cuda.synchronize()
    got = s.state.cpu().numpy()
    err = np.abs(got - want).max(axis=(0, 2)) / (np.abs(want).max(axis=(0, 2)) + dt * scale)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("arith,E_ok", [(0, 2427), (1, 4854)])
def test_noalloc_scratch_limit(sd, arith, E_ok):
    import torch
    # boxes of exactly the largest element count the 64 MiB scratch holds, and
    # one more element (no periodic direction, so every factor of E is legal)
    per = 6 * (9 + 7) * 36 * (8 if arith == 0 else 4)
    assert E_ok * per <= SCRATCH_BYTES < (E_ok + 1) * per
    for E, ok in ((E_ok, True), (E_ok + 1, False)):
        ny = next(k for k in range(2, 10) if E % k == 0)
        nx = E // ny
        print(f"noalloc limit: box {nx}x{ny}x1 p=5 arith={arith} E={E}", flush=True)
        m = sd.box(nx, ny, 1, 5, L=(nx / 4.0, ny / 4.0, 0.25), periodic=0)
        s = sd.Solver(m, arith=arith)
        ghost = torch.zeros((m.NB, 9, 36), dtype=torch.float64, device="cuda")
        ghost[:, 0] = 1.0
        ghost[:, 4] = 2.5
        prm = sd.make_params(ghost=ghost, wall_kind=(1, 1))
        Q = torch.zeros((E, 9, 216), dtype=torch.float64, device="cuda")
        Q[:, 0] = 1.0
        Q[:, 4] = 2.5
        s.set_state(Q)
        if ok:
            regs = [Q.clone() for _ in range(4)]
            s.step(prm, 1e-3)
            s.step_noalloc(prm, 1e-3, regs=regs)
            torch.cuda.synchronize()
            assert torch.equal(s.state, regs[0])
            # a uniform state at rest with matching Dirichlet data stays put,
            # to the round-off of the residual arithmetic (FP32 in the mixed
            # context: about 1e-7 of the pressure per unit time)
            drift = (s.state - Q).abs().max().item()
            assert drift <= (1e-12 if arith == 0 else 1e-6), drift
        else:
            with pytest.raises(sd.SdmError, match="maximum is 67108864"):
                s.step_noalloc(prm, 1e-3)
