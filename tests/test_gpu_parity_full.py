"""GPU parity at the production sizes: the 6,912-element shell (all five
stages of the first step, and ten steps) and the 55,296-element shell that
the benchmark times (one fused stage, through the same stage entry point and
launch configuration), against the FP64 oracle over every element.

Criterion as in the small-shell parity tests: per variable, the maximum
difference of an RK stage output u is at most 1e-12 of max|u_v| + dt T_v,
T_v being the oracle's round-off scale of the residual.
"""
import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def sd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_17805_amd import sdmhd
    return sdmhd


def _setup(sd, oracle, Nz, Nr, p, N_rho, seed):
    ml = sd.shell(Nz, Nr, p)
    mo = oracle.Mesh.shell(p + 1, Nz, Nr)
    bg = inp.Background(N_rho)
    Q = inp.shell_state(ml.x_sp, bg, seed)
    pr = inp.run_params(seed, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    dt = inp.time_step(Q, ml.Sj_sp, ch, 0.1)
    return ml, mo, Q, pr, dt


@pytest.mark.parametrize("N_rho,seed", [(3.0, 1), (5.0, 2)])
def test_c2_first_step(sd, oracle, N_rho, seed):
    """6,912-element shell, p = 5: the state after one SSPRK(5,3) step."""
    ml, mo, Q, pr, dt = _setup(sd, oracle, 12, 8, 5, N_rho, seed)
    print(f"c2 first step N_rho={N_rho} seed={seed} E={ml.E}", flush=True)
    s = sd.Solver(ml)
    pg, po = sd.make_params(**pr), oracle.make_params(**pr)
    s.set_state(Q)
    s.step(pg, dt)
    qg = s.state.cpu().numpy()
    _, ts = mo.residual(po, Q, with_scale=True)
    qo = mo.step(po, Q, dt)
    err = np.abs(qg - qo).max(axis=(0, 2))
    scale = np.abs(qo).max(axis=(0, 2)) + dt * ts
    assert (err <= TOL * scale).all(), err / scale


@pytest.mark.parametrize("N_rho,seed", [(3.0, 1), (5.0, 2)])
def test_c2_step1_residual(sd, oracle, N_rho, seed):
    """6,912-element shell, p = 5: the step-1 residual itself, point by point
    against the oracle's, within 1e-12 of the term scale per variable."""
    import torch
    ml, mo, Q, pr, dt = _setup(sd, oracle, 12, 8, 5, N_rho, seed)
    print(f"c2 residual N_rho={N_rho} seed={seed} E={ml.E}", flush=True)
    s = sd.Solver(ml)
    Rg = s.residual(sd.make_params(**pr), torch.from_numpy(Q).cuda()).cpu().numpy()
    Ro, ts = mo.residual(oracle.make_params(**pr), Q, with_scale=True)
    err = np.abs(Rg - Ro).max(axis=(0, 2))
    assert (err <= TOL * ts).all(), err / ts


def test_c2_ten_steps(sd, oracle):
    """6,912-element shell, N_rho = 5: every one of ten steps."""
    ml, mo, Q, pr, dt = _setup(sd, oracle, 12, 8, 5, 5.0, 2)
    s = sd.Solver(ml)
    pg, po = sd.make_params(**pr), oracle.make_params(**pr)
    s.set_state(Q)
    qo = Q.copy()
    for step in range(10):
        print(f"c2 step {step}", flush=True)
        _, ts = mo.residual(po, qo, with_scale=True)
        s.step(pg, dt)
        qo = mo.step(po, qo, dt)
        qg = s.state.cpu().numpy()
        err = np.abs(qg - qo).max(axis=(0, 2))
        scale = np.abs(qo).max(axis=(0, 2)) + dt * ts
        assert (err <= TOL * scale).all(), (step, err / scale)


def test_c4_full_size_stage(sd, oracle):
    """55,296-element shell, p = 5 (the benchmark workload): the residual and
    the first fused stage u1 = u0 + b10 dt L(u0) in FP64 over every element,
    and the FP32-mixed residual arithmetic within 1e-5 of the same scale."""
    import torch
    ml, mo, Q, pr, dt = _setup(sd, oracle, 24, 16, 5, 5.0, 2)
    print(f"c4 full size E={ml.E}", flush=True)
    po = oracle.make_params(**pr)
    Ro, ts = mo.residual(po, Q, with_scale=True)
    # the residual itself, every element
    s = sd.Solver(ml)
    Rg = s.residual(sd.make_params(**pr), torch.from_numpy(Q).cuda()).cpu().numpy()
    err = np.abs(Rg - Ro).max(axis=(0, 2))
    assert (err <= TOL * ts).all(), err / ts
    del s, Rg
    _, b, _ = oracle.ssprk53_table()
    cur, inputs, beta, out = sd.ssp53_stages()[0]
    want = Q + dt * b[1, 0] * Ro
    scale = np.abs(want).max(axis=(0, 2)) + dt * ts
    for arith, tol in ((0, TOL), (1, 1e-5)):
        s = sd.Solver(ml, arith=arith)
        s.set_state(Q)
        s.stage(sd.make_params(**pr), cur, inputs, beta, out, dt)
        torch.cuda.synchronize()
        got = s.regs[out].cpu().numpy()
        err = np.abs(got - want).max(axis=(0, 2))
        assert np.isfinite(got).all()
        assert (err <= tol * scale).all(), (arith, err / scale)
        del s
