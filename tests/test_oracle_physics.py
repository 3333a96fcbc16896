"""Pointwise pins of the oracle's fluxes (paper, Sec. "MHD Governing Equations":
Eqs. energy, ideal gas, invF, visF, ssTensor, qFlux, entropy)."""
import numpy as np
import pytest

G53 = 5.0 / 3.0


def _state(rho, u, p, B, psi=0.0, g=G53):
    u, B = np.asarray(u, float), np.asarray(B, float)
    E = p / (g - 1) + 0.5 * rho * u @ u + 0.5 * B @ B + 0.5 * psi * psi
    return np.array([rho, *(rho * u), E, *B, psi])


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def _rotate_state(Rm, q):
    out = q.copy()
    out[1:4] = Rm @ q[1:4]
    out[5:8] = Rm @ q[5:8]
    return out


def _rotate_grad(Rm, q_grad):
    """G[v][j] -> rotated: vectors rotate in v, all rotate in j"""
    G = q_grad.reshape(9, 3) @ Rm.T
    G[1:4] = Rm @ G[1:4]
    G[5:8] = Rm @ G[5:8]
    return G.reshape(27)


def test_euler_limit(oracle):
    """B = psi = 0, c_h = 0: the textbook compressible Euler flux."""
    prm = oracle.make_params(c_h=0.0)
    rho, u, p = 1.3, np.array([0.2, -0.4, 0.1]), 0.7
    q = _state(rho, u, p, [0, 0, 0])
    n = np.array([0.3, -1.1, 0.6])
    Fi, _ = oracle.point_flux(prm, q, np.zeros(27), n)
    un = u @ n
    H = (q[4] + p) / rho
    want = np.array([rho * un, *(rho * u * un + p * n), rho * H * un, 0, 0, 0, 0])
    np.testing.assert_allclose(Fi, want, atol=1e-15)


def test_glm_and_magnetic_terms(oracle):
    """Known closed-form pieces: with u = 0 the induction flux is c_h psi n,
    the psi flux c_h B.n, the momentum flux (p + B^2/2) n - B (B.n)."""
    prm = oracle.make_params(c_h=0.8)
    B = np.array([0.3, 0.5, -0.2])
    q = _state(1.0, [0, 0, 0], 0.6, B, psi=0.05)
    n = np.array([0.0, 0.0, 2.0])
    Fi, _ = oracle.point_flux(prm, q, np.zeros(27), n)
    np.testing.assert_allclose(Fi[5:8], 0.8 * 0.05 * n, atol=1e-16)
    assert abs(Fi[8] - 0.8 * B @ n) < 1e-16
    np.testing.assert_allclose(Fi[1:4], (0.6 + 0.5 * B @ B) * n - B * (B @ n), atol=1e-15)
    assert abs(Fi[4] - 0.8 * 0.05 * (B @ n)) < 1e-16


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rotational_invariance(oracle, seed):
    """F_{Rn}(RQ, R grad) = R F_n(Q, grad) for inviscid and viscous fluxes."""
    prm = oracle.make_params(c_h=0.7, nu=0.3, kappa=0.2, eta=0.4, kr_scale=1.0, kr_c0=0.5)
    rng = np.random.default_rng(seed)
    q = _state(1.0 + rng.random(), rng.standard_normal(3) * 0.3, 1.0 + rng.random(),
               rng.standard_normal(3) * 0.5, psi=0.1 * rng.standard_normal())
    G = rng.standard_normal(27)
    n = rng.standard_normal(3)
    Rm = _rot(seed + 10)
    Fi, Fv = oracle.point_flux(prm, q, G, n, kr=0.3)
    Fi2, Fv2 = oracle.point_flux(prm, _rotate_state(Rm, q), _rotate_grad(Rm, G), Rm @ n, kr=0.3)
    for a, b in ((Fi, Fi2), (Fv, Fv2)):
        np.testing.assert_allclose(b[[0, 4, 8]], a[[0, 4, 8]], atol=1e-13)
        np.testing.assert_allclose(b[1:4], Rm @ a[1:4], atol=1e-13)
        np.testing.assert_allclose(b[5:8], Rm @ a[5:8], atol=1e-13)
    # linear in n
    Fi3, Fv3 = oracle.point_flux(prm, q, G, 2.5 * n, kr=0.3)
    np.testing.assert_allclose(Fi3, 2.5 * Fi, atol=1e-13)
    np.testing.assert_allclose(Fv3, 2.5 * Fv, atol=1e-13)


def test_viscous_closed_forms(oracle):
    """Simple shear u = (s y, 0, 0): tau_xy = mu s, work u.tau n; a uniform-
    pressure density gradient gives the entropy-diffusion heat flux; a
    uniform current J gives eta J x n and eta (B x J).n."""
    nu, kap, eta = 0.3, 0.2, 0.4
    prm = oracle.make_params(nu=nu, kappa=kap, eta=eta)
    rho, s, p = 1.2, 0.7, 0.9
    ux = 0.25
    q = _state(rho, [ux, 0, 0], p, [0, 0, 0])
    G = np.zeros((9, 3))
    G[1, 1] = rho * s                         # d(rho u)/dy
    G[4, 1] = rho * ux * s                     # dE/dy = rho u du/dy (p const)
    n = np.array([0.0, 1.0, 0.0])
    _, Fv = oracle.point_flux(prm, q, G.reshape(27), n)
    mu = rho * nu
    np.testing.assert_allclose(Fv[1:4], [mu * s, 0, 0], atol=1e-15)
    assert abs(Fv[4] - ux * mu * s) < 1e-15
    # heat: uniform p, drho/dz = c  => dS/dz = -cp c/rho, q_z = -kappa rho T dS/dz
    q2 = _state(rho, [0, 0, 0], p, [0, 0, 0])
    G2 = np.zeros((9, 3))
    c = 0.3
    G2[0, 2] = c
    G2[4, 2] = 0.0
    _, Fv2 = oracle.point_flux(prm, q2, G2.reshape(27), np.array([0, 0, 1.0]))
    cp = G53 / (G53 - 1)
    T = p / rho
    qz = -kap * rho * T * (-cp * c / rho)
    assert abs(Fv2[4] - (-qz)) < 1e-14
    # resistive: B = (0, x, 0) slope 1 => J = (0, 0, 1)
    B0 = np.array([0.2, 0.0, 0.1])
    q3 = _state(rho, [0, 0, 0], p, B0)
    G3 = np.zeros((9, 3))
    G3[6, 0] = 1.0
    G3[4, 0] = B0[1] * 1.0  # dE/dx from d(B^2/2)/dx with p const
    n3 = np.array([0.3, 0.4, -0.5])
    _, Fv3 = oracle.point_flux(prm, q3, G3.reshape(27), n3)
    J = np.array([0, 0, 1.0])
    np.testing.assert_allclose(Fv3[5:8], eta * np.cross(J, n3), atol=1e-15)
    assert abs(Fv3[4] - eta * np.cross(B0, J) @ n3) < 1e-15


def test_fast_speed_limits(oracle):
    prm = oracle.make_params()
    q = _state(1.3, [0, 0, 0], 0.8, [0, 0, 0])
    a = np.sqrt(G53 * 0.8 / 1.3)
    assert abs(oracle.point_cf(prm, q, [0, 0, 1.0]) - a) < 1e-15
    Bv = np.array([0.0, 0.6, 0.0])
    q0 = _state(2.0, [0, 0, 0], 0.0, Bv)
    # p -> 0: c_f = |B|/sqrt(rho) across B, 0 along B is the slow/Alfven branch: c_f stays |B|/sqrt(rho)
    assert abs(oracle.point_cf(prm, q0, [1.0, 0, 0]) - 0.6 / np.sqrt(2.0)) < 1e-15
    # along B with p > 0: c_f = max(a, b)
    q1 = _state(1.0, [0, 0, 0], 0.3, Bv)
    assert abs(oracle.point_cf(prm, q1, [0, 1.0, 0]) - max(np.sqrt(G53 * 0.3), 0.6)) < 1e-15


def test_rusanov_consistency_and_antisymmetry(oracle):
    prm = oracle.make_params(c_h=0.5)
    rng = np.random.default_rng(3)
    qL = _state(1.1, rng.standard_normal(3) * 0.2, 0.9, rng.standard_normal(3) * 0.3, 0.01)
    qR = _state(0.9, rng.standard_normal(3) * 0.2, 1.1, rng.standard_normal(3) * 0.3, -0.02)
    n = np.array([0.2, 0.9, -0.3])
    F = oracle.point_rusanov(prm, qL, qR, n)
    Fm = oracle.point_rusanov(prm, qR, qL, -n)
    np.testing.assert_array_equal(F, -Fm)  # bitwise: each face value is shared exactly
    Fi, _ = oracle.point_flux(prm, qL, np.zeros(27), n)
    np.testing.assert_allclose(oracle.point_rusanov(prm, qL, qL, n), Fi, atol=1e-15)


def test_wall_flux_invariants(oracle):
    """No mass flux through a wall; no resistive or inviscid energy flux
    through a perfectly conducting, adiabatic (q = 0) wall; the prescribed heat
    flux enters through a heat-flux wall."""
    prm = oracle.make_params(c_h=0.5, nu=0.1, kappa=0.1, eta=0.2, wall_mag=(0, 0), wall_th=(0, 0),
                             q_wall=(0.0, 0.0))
    rng = np.random.default_rng(5)
    q = _state(1.0, rng.standard_normal(3) * 0.3, 0.8, rng.standard_normal(3) * 0.4, 0.03)
    G = rng.standard_normal(27)
    n = np.array([0.1, -0.2, 1.5])
    F = oracle.point_wall_flux(prm, q, G, n, 1)
    assert abs(F[0]) < 1e-15
    assert abs(F[4]) < 1e-14
    nh = n / np.linalg.norm(n)
    # tangential momentum flux vanishes (stress-free, no inviscid shear)
    Ft = F[1:4] - (F[1:4] @ nh) * nh
    assert np.abs(Ft).max() < 1e-14
    prm2 = oracle.make_params(c_h=0.5, nu=0.1, kappa=0.1, eta=0.2, wall_th=(0, 0), q_wall=(2.0, 0.0))
    qs = _state(1.0, [0, 0, 0], 0.8, [0, 0, 0])
    F2 = oracle.point_wall_flux(prm2, qs, np.zeros(27), -n, 0)
    # outward energy flux = -q_inner |n| (energy enters at the inner wall)
    assert abs(F2[4] + 2.0 * np.linalg.norm(n)) < 1e-14
