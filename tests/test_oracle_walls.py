"""Pins of the oracle's wall treatments (paper, Sec. "Problem Formulation and
Boundary Conditions": impenetrable, stress-free walls; perfectly conducting
or radial-field magnetic walls; a prescribed heat flux or a fixed
temperature), with the cleaning field's wall condition of the readings.

Each wall kind has exact equilibria: uniform states that satisfy its
conditions. On a box periodic in x and y with walls at z = 0 (group 0) and
z = Lz (group 1), every flux of a uniform state is uniform, so its residual
is its source alone, to round-off, exactly when the walls accept the state;
the same state at the other kind of wall, or violating the condition, is
not an equilibrium. A fixed-temperature wall hotter than the gas must put
energy in, a colder one take it out, each at its own wall. At a wall point
the mirror state and the Rusanov flux give the reflection force of a flow
into the wall and the cleaning field's fluxes in closed form, and the
resistive fluxes follow the wall's electric condition. The last test plants a mistake into a copy of
the oracle source, one at a time, and checks that a pin fails for each.
"""
import os

import numpy as np
import pytest

G53 = 5.0 / 3.0
BASE = dict(c_h=0.6, glm_a=0.0, nu=0.02, kappa=0.02, eta=0.03, powell=1, wall_kind=(0, 0),
            wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.0, 0.0))


def _state(x, rho, u, p, B, psi=0.0):
    """Uniform conserved state on the SPs x [E][3][N^3]."""
    E, _, n3 = x.shape
    u, B = np.asarray(u, float), np.asarray(B, float)
    q = np.empty(9)
    q[0] = rho
    q[1:4] = rho * u
    q[4] = p / (G53 - 1) + 0.5 * rho * u @ u + 0.5 * B @ B + 0.5 * psi ** 2
    q[5:8] = B
    q[8] = psi
    return np.broadcast_to(q[None, :, None], (E, 9, n3)).copy()


def _box(oracle):
    return oracle.Mesh.box(4, 3, 3, 3, L=(1.0, 0.9, 0.8), periodic=3)


def _residual(oracle, m, Q, **kw):
    prm = dict(BASE)
    prm.update(kw)
    return m.residual(oracle.make_params(**prm), Q, with_scale=True)


def _rel(R, ts, want=None):
    """Largest |R - want| per variable over the residual's round-off scale
    (the largest over the variables: some variables' own fluxes vanish for
    these states, and their scale with them)."""
    d = R if want is None else R - np.asarray(want, float)[None, :, None]
    return np.abs(d).max(axis=(0, 2)) / ts.max()


def magnetic_walls_pin(oracle):
    """A uniform field at rest is an equilibrium of radial-field walls when it
    is normal to them (B passes) and of perfectly conducting walls when it is
    tangential (B_n = 0): residual zero to round-off. A normal field at
    conducting walls, or a tangential one at radial-field walls, is not."""
    m = _box(oracle)
    x = m.get("x_sp")
    for B0, accepts in (([0.0, 0.0, 0.3], 1), ([0.3, -0.2, 0.0], 0)):
        Q = _state(x, 1.1, [0.0, 0.0, 0.0], 0.7, B0)
        for mag in (0, 1):
            R, ts = _residual(oracle, m, Q, wall_mag=(mag, mag))
            rel = _rel(R, ts)
            if mag == accepts:
                assert (rel <= 1e-12).all(), (B0, mag, rel)
            else:
                assert rel.max() > 1e-6, (B0, mag, rel)


def impenetrable_stress_free_pin(oracle):
    """A uniform viscous flow along the walls is an equilibrium of
    impenetrable, stress-free walls (no slip condition, no gradient): zero
    residual. The same flow through the walls is not."""
    m = _box(oracle)
    x = m.get("x_sp")
    R, ts = _residual(oracle, m, _state(x, 1.1, [0.2, -0.1, 0.0], 0.7, [0.1, 0.05, 0.0]))
    assert (_rel(R, ts) <= 1e-12).all(), _rel(R, ts)
    R, ts = _residual(oracle, m, _state(x, 1.1, [0.0, 0.0, 0.2], 0.7, [0.1, 0.05, 0.0]))
    assert _rel(R, ts).max() > 1e-6


def cleaning_field_walls_pin(oracle):
    """A uniform cleaning field psi0 with B = 0 at rest: its flux c_h psi n is
    uniform, so where the walls accept it the residual is the damping source
    alone, dpsi/dt = -a psi0 and nothing else. A conducting wall reflects
    psi and accepts it; a radial-field wall holds psi = 0 and does not."""
    m = _box(oracle)
    x = m.get("x_sp")
    a, psi0 = 0.4, 0.05
    Q = _state(x, 1.1, [0.0, 0.0, 0.0], 0.7, [0.0, 0.0, 0.0], psi0)
    want = np.zeros(9)
    want[8] = -a * psi0
    R, ts = _residual(oracle, m, Q, glm_a=a, wall_mag=(0, 0))
    assert (_rel(R, ts, want) <= 1e-12).all(), _rel(R, ts, want)
    R, ts = _residual(oracle, m, Q, glm_a=a, wall_mag=(1, 1))
    assert _rel(R, ts, want).max() > 1e-6
    # at one wall point (c_h above every other signal speed, so it is the
    # Rusanov speed): a conducting wall passes the flux c_h psi0 n of B and
    # none of psi; a radial-field wall meets the reversed psi of its mirror
    # state, so B carries nothing and psi flows out at c_h |n| psi0
    ch, p = 2.0, 0.7
    n = np.array([0.2, 0.5, -1.1])
    q = np.zeros(9)
    q[0] = 1.1
    q[4] = p / (G53 - 1) + 0.5 * psi0 ** 2
    q[8] = psi0
    for mag in (0, 1):
        prm = oracle.make_params(c_h=ch, wall_mag=(mag, mag), wall_th=(0, 0), q_wall=(0.0, 0.0))
        F = oracle.point_wall_flux(prm, q, np.zeros(27), n, 0)
        want = np.zeros(9)
        want[1:4] = p * n
        if mag == 0:
            want[5:8] = ch * psi0 * n
        else:
            want[8] = ch * np.linalg.norm(n) * psi0
        assert np.abs(F - want).max() <= 1e-14 * np.abs(want).max(), (mag, F, want)


def _wall_layers(oracle, m, R):
    """Energy residual integrated (W^3 |J| quadrature) over the elements
    touching z = 0, over those touching z = Lz and over all, and the mass
    residual integrated over all."""
    x, wJ = m.get("x_sp"), m.get("W3detJ")
    e_int = (R[:, 4] * wJ).sum(axis=1)
    zc = x[:, 2].mean(axis=1)
    lo, hi = zc < zc.min() + 1e-9, zc > zc.max() - 1e-9
    return e_int[lo].sum(), e_int[hi].sum(), e_int.sum(), (R[:, 0] * wJ).sum()


def fixed_temperature_walls_pin(oracle):
    """Fixed-temperature walls: a uniform gas at rest at the wall temperature
    is an equilibrium (zero residual). A wall hotter than the gas heats the
    element layer next to it (its energy rate is positive), a colder wall
    cools its layer, each wall at its own temperature, and mass is
    conserved."""
    m = _box(oracle)
    x = m.get("x_sp")
    rho, p = 1.1, 0.77  # T = p / (rho R) = 0.7 with R = 1
    Q = _state(x, rho, [0.0, 0.0, 0.0], p, [0.0, 0.0, 0.0])
    R, ts = _residual(oracle, m, Q, wall_th=(1, 1), T_wall=(0.7, 0.7))
    assert (_rel(R, ts) <= 1e-12).all(), _rel(R, ts)
    R, ts = _residual(oracle, m, Q, wall_th=(1, 1), T_wall=(0.9, 0.5))  # hot bottom, cold top
    lo, hi, _, mass = _wall_layers(oracle, m, R)
    assert lo > 1e-6 and hi < -1e-6, (lo, hi)
    assert abs(mass) <= 1e-12 * ts[0] * m.E
    R, ts = _residual(oracle, m, Q, wall_th=(1, 1), T_wall=(0.5, 0.9))  # cold bottom, hot top
    lo, hi, _, _ = _wall_layers(oracle, m, R)
    assert lo < -1e-6 and hi > 1e-6, (lo, hi)


def wall_reflection_pin(oracle):
    """Inviscid, B = 0: a flow u_n n into a wall point meets its mirror state
    (normal momentum reversed), and the Rusanov flux gives no mass or energy
    flux and the normal momentum flux (rho u_n^2 + p + lambda rho u_n) n with
    lambda = |u_n| + sqrt(gamma p / rho), the fastest signal of either state."""
    prm = oracle.make_params(c_h=0.0, wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.0, 0.0))
    rho, p, un = 1.3, 0.9, 0.25
    n = np.array([0.3, -0.4, 1.2])
    nh = n / np.linalg.norm(n)
    q = np.zeros(9)
    q[0] = rho
    q[1:4] = rho * un * nh
    q[4] = p / (G53 - 1) + 0.5 * rho * un * un
    F = oracle.point_wall_flux(prm, q, np.zeros(27), n, 1)
    lam = abs(un) + np.sqrt(G53 * p / rho)
    want = np.zeros(9)
    want[1:4] = (rho * un * un + p + lam * rho * un) * n
    assert np.abs(F - want).max() <= 1e-14 * np.abs(want).max(), (F, want)


def wall_current_pin(oracle):
    """Resistive fluxes through a wall point at rest with a current J = curl B
    (from the interior gradient): a perfectly conducting wall has no
    tangential electric field, so no resistive flux of B or energy passes
    it (the fluxes do not depend on eta); at a radial-field wall the
    tangential current diffuses field through it: the resistive part of the
    B flux is -eta (J_t x n), J_t = J - (J.nh) nh."""
    n = np.array([0.1, -0.2, 1.3])
    nh = n / np.linalg.norm(n)
    q = np.zeros(9)
    q[0], p = 1.1, 0.7
    q[5:8] = [0.2, 0.1, 0.3]
    q[4] = p / (G53 - 1) + 0.5 * q[5:8] @ q[5:8]
    G = np.zeros(27)
    G[5 * 3 + 2] = 0.4   # dB_x/dz
    G[6 * 3 + 0] = -0.3  # dB_y/dx
    G[7 * 3 + 1] = 0.25  # dB_z/dy
    J = np.array([G[7 * 3 + 1] - G[6 * 3 + 2], G[5 * 3 + 2] - G[7 * 3 + 0], G[6 * 3 + 0] - G[5 * 3 + 1]])
    eta = 0.3
    for mag in (0, 1):
        F = {}
        for e in (0.0, eta):
            prm = oracle.make_params(c_h=2.0, eta=e, wall_mag=(mag, mag), wall_th=(0, 0), q_wall=(0.0, 0.0))
            F[e] = oracle.point_wall_flux(prm, q, G, n, 1)
        d = F[eta] - F[0.0]
        if mag == 0:
            assert np.abs(d).max() <= 1e-15, (mag, d)
        else:
            Jt = J - (J @ nh) * nh
            want = -eta * np.cross(Jt, n)
            assert np.abs(d[5:8] - want).max() <= 1e-15, (d[5:8], want)
            assert np.abs(want).max() > 1e-2


def fixed_temperature_wall_flux_pin(oracle):
    """Heat through a fixed-temperature wall point at rest (B = psi = 0), with
    interior gradients of E and rho: the heat flux of Eq. "qFlux",
    -kappa rho T grad S - kappa_r rho c_p grad T, taken at the wall
    temperature (p = rho R T_wall, S = c_v ln(p / rho^gamma)) is, since
    grad p = (gamma - 1) grad E at rest,
      q = -(kappa + gamma kappa_r) grad E + (kappa + kappa_r) c_p T_wall grad rho,
    and the outward energy flux through n is q . n."""
    R, g = 1.0, G53
    cp = g * R / (g - 1.0)
    kap, kr, Tw = 0.03, 0.05, 0.9
    rho, p = 1.1, 0.66  # interior T = 0.6, not the wall's
    n = np.array([0.2, -0.3, 1.1])
    q = np.zeros(9)
    q[0], q[4] = rho, p / (g - 1.0)
    G = np.zeros(27)
    gE, grho = np.array([0.3, -0.2, 0.5]), np.array([0.1, 0.4, -0.2])
    G[4 * 3:4 * 3 + 3] = gE
    G[0:3] = grho
    prm = oracle.make_params(kappa=kap, c_h=0.5, wall_th=(1, 1), T_wall=(Tw, Tw), wall_mag=(0, 0))
    F = oracle.point_wall_flux(prm, q, G, n, 1, kr)
    qvec = -(kap + g * kr) * gE + (kap + kr) * cp * Tw * grho
    want = qvec @ n
    assert abs(F[4] - want) <= 1e-14 * (np.abs(qvec).max() * np.abs(n).max()), (F[4], want)


def wall_traction_pin(oracle):
    """Viscous traction at a stress-free wall point at rest with an interior
    velocity gradient grad u = grad m / rho: only the normal traction
    t_nn = nh . tau . n of the stress tensor of Eq. "ssTensor"
    (tau = mu (grad u + grad u^T - 2/3 div u I), mu = rho nu) acts, so the
    momentum flux is p n - t_nn nh."""
    rho, p, nu = 1.2, 0.8, 0.07
    n = np.array([-0.4, 0.3, 0.9])
    nh = n / np.linalg.norm(n)
    q = np.zeros(9)
    q[0], q[4] = rho, p / (G53 - 1.0)
    A = np.array([[0.3, -0.1, 0.2], [0.15, -0.25, 0.05], [-0.2, 0.1, 0.4]])  # d m_i / d x_j
    G = np.zeros(27)
    for i in range(3):
        G[(1 + i) * 3:(1 + i) * 3 + 3] = A[i]
    gu = A / rho
    tau = rho * nu * (gu + gu.T - 2.0 / 3.0 * np.trace(gu) * np.eye(3))
    tnn = nh @ tau @ n
    prm = oracle.make_params(nu=nu, c_h=0.5, wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.0, 0.0))
    F = oracle.point_wall_flux(prm, q, G, n, 0)
    want = p * n - tnn * nh
    assert np.abs(F[1:4] - want).max() <= 1e-14 * np.abs(want).max(), (F[1:4], want)
    assert abs(tnn) > 1e-3


@pytest.mark.parametrize("pin", [magnetic_walls_pin, impenetrable_stress_free_pin, cleaning_field_walls_pin,
                                 fixed_temperature_walls_pin, wall_reflection_pin, wall_current_pin,
                                 fixed_temperature_wall_flux_pin, wall_traction_pin])
def test_wall_pins(oracle, pin):
    pin(oracle)


MUTANTS = [
    ("conducting and radial-field mirror states swapped",
     "qg[5 + i] = P->wall_mag[g] == 0 ? q[5 + i] - 2.0 * Bn * nh[i] : 2.0 * Bn * nh[i] - q[5 + i];",
     "qg[5 + i] = P->wall_mag[g] != 0 ? q[5 + i] - 2.0 * Bn * nh[i] : 2.0 * Bn * nh[i] - q[5 + i];",
     magnetic_walls_pin),
    ("no-slip common velocity", "uc[i] = u[i] - un * nh[i];", "uc[i] = 0.0 * u[i];",
     impenetrable_stress_free_pin),
    ("normal momentum not reversed in the mirror state", "qg[1 + i] = q[1 + i] - 2.0 * mn * nh[i];",
     "qg[1 + i] = q[1 + i];", wall_reflection_pin),
    ("cleaning field not reversed at a radial-field wall", "qg[8] = P->wall_mag[g] == 0 ? q[8] : -q[8];",
     "qg[8] = q[8];", cleaning_field_walls_pin),
    ("the other wall's temperature", "rho * P->Rgas * P->T_wall[g]", "rho * P->Rgas * P->T_wall[1 - g]",
     fixed_temperature_walls_pin),
    ("wall viscous state from the interior instead of the common state", "visc_state(qc, G, kr, P, &v);",
     "visc_state(q, G, kr, P, &v);", fixed_temperature_wall_flux_pin),
    ("normal traction projected on the unnormalised normal",
     "double tnn = tn[0] * nh[0] + tn[1] * nh[1] + tn[2] * nh[2];",
     "double tnn = tn[0] * n[0] + tn[1] * n[1] + tn[2] * n[2];", wall_traction_pin),
    ("conducting and radial-field wall currents swapped",
     "Jc[i] = P->wall_mag[g] == 0 ? Jn * nh[i] : v.J[i] - Jn * nh[i];",
     "Jc[i] = P->wall_mag[g] != 0 ? Jn * nh[i] : v.J[i] - Jn * nh[i];", wall_current_pin),
]


def test_planted_wall_mistakes_are_caught(oracle, tmp_path):
    src = oracle.source_text()
    for k, (what, find, repl, pin) in enumerate(MUTANTS):
        assert src.count(find) == 1, (what, src.count(find))
        path = oracle.build_variant(src.replace(find, repl), os.path.join(str(tmp_path), f"wall{k}.so"))
        prev = oracle.swap_library(path)
        try:
            with pytest.raises(AssertionError):
                pin(oracle)
        finally:
            oracle.swap_back(prev)
