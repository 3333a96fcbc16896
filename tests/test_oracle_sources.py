"""Closed-form pins of the oracle's source and radiative-diffusion terms
(paper, Sec. "MHD Governing Equations": the source vector of Eq. "M" with
the Coriolis force and the div-B (Powell) terms, and the heat flux of
Eq. "qFlux" with its radiative part -kappa_r rho C_p grad T).

Each pin compares the oracle's residual with the exact time derivative that
the PDE gives for a state the discretisation represents exactly (uniform or
low-degree polynomial fields on an affine box with exact Dirichlet ghosts),
or with a solution of the PDE (the inertial oscillation of a uniform flow).
The last test plants a sign or factor mistake into a copy of the oracle
source, one at a time, and checks that a pin fails for every one of them.
"""
import os

import numpy as np
import pytest

G53 = 5.0 / 3.0
CP = G53 / (G53 - 1.0)  # C_p with Rgas = 1


def _state(rho, u, p, B, psi=0.0):
    """Conserved state from primitive fields of shape [E][N^3] (scalars) and
    [E][3][N^3] (vectors)."""
    E, n3 = np.shape(rho)
    Q = np.empty((E, 9, n3))
    Q[:, 0] = rho
    Q[:, 1:4] = rho[:, None] * u
    Q[:, 4] = p / (G53 - 1) + 0.5 * rho * (u * u).sum(1) + 0.5 * (B * B).sum(1) + 0.5 * psi ** 2
    Q[:, 5:8] = B
    Q[:, 8] = psi
    return Q


def _const(x, c):
    return np.broadcast_to(np.asarray(c, float), x[:, 0].shape).copy()


def _vec(x, v):
    return np.broadcast_to(np.asarray(v, float)[None, :, None], x.shape).copy()


# ---------------------------------------------------------------------------
# Coriolis: -2 rho Omega z x u
# ---------------------------------------------------------------------------

def coriolis_uniform_pin(oracle):
    """A uniform state on a periodic box has zero flux divergence, so its
    residual is the source alone: the Coriolis force turns the momentum at
    rate 2 Omega (dm/dt = -2 Omega z x m) and does no work (dE/dt = 0)."""
    N = 4
    m = oracle.Mesh.box(N, 3, 3, 3, L=(1.0, 0.9, 0.8), periodic=7)
    x = m.get("x_sp")
    u0, B0 = np.array([0.3, -0.2, 0.1]), np.array([0.05, 0.1, -0.07])
    Q = _state(_const(x, 1.3), _vec(x, u0), _const(x, 0.8), _vec(x, B0))
    Om = 0.45
    R, ts = m.residual(oracle.make_params(Omega=Om, c_h=0.5, powell=1), Q, with_scale=True)
    mom = 1.3 * u0
    want = np.zeros(9)
    want[1:4] = -2.0 * Om * np.cross([0.0, 0.0, 1.0], mom)
    # round-off scale: the differentiated (uniform) fluxes plus the source
    err = np.abs(R - want[None, :, None]).max(axis=(0, 2))
    assert (err <= 1e-12 * ts).all(), (err, ts)


def coriolis_oscillation_pin(oracle):
    """Inertial oscillation: a uniform flow in the rotating frame keeps its
    speed and its direction turns clockwise (Omega > 0) at angular rate
    2 Omega; after SSPRK(5,3) steps to time t the momentum is the exact
    rotation by -2 Omega t, to the scheme's third-order time error."""
    N = 3
    m = oracle.Mesh.box(N, 3, 3, 3, periodic=7)
    x = m.get("x_sp")
    u0 = np.array([0.25, 0.1, 0.05])
    Q = _state(_const(x, 1.0), _vec(x, u0), _const(x, 0.6), _vec(x, [0.0, 0.0, 0.0]))
    Om, dt, n = 0.6, 0.02, 50
    prm = oracle.make_params(Omega=Om, c_h=0.5)
    for _ in range(n):
        Q = m.step(prm, Q, dt)
    th = -2.0 * Om * dt * n
    want = np.array([u0[0] * np.cos(th) - u0[1] * np.sin(th), u0[0] * np.sin(th) + u0[1] * np.cos(th), u0[2]])
    got = Q[:, 1:4].mean(axis=(0, 2))
    assert np.abs(Q[:, 1:4] - got[None, :, None]).max() < 1e-14  # stays uniform
    assert np.abs(got - want).max() < 1e-7, (got, want)


# ---------------------------------------------------------------------------
# Powell terms: -(div B) (B, u.B, u)
# ---------------------------------------------------------------------------

_A = np.array([[0.30, -0.12, 0.05], [0.07, -0.10, 0.20], [-0.15, 0.09, 0.25]])  # trace 0.45 (div B)
_B0 = np.array([0.2, -0.1, 0.3])
_U0 = np.array([0.2, -0.1, 0.15])


def _powell_case(oracle, powell):
    """Uniform rho, u, p, psi = 0 and a linear, divergent B = B0 + A x on an
    affine box with exact ghosts, inviscid: every flux is a polynomial the
    method differentiates exactly, so the residual is the exact dQ/dt."""
    N = 5
    m = oracle.Mesh.box(N, 2, 2, 2, L=(1.0, 0.8, 0.6), periodic=0)

    def st(X):
        B = _B0[None, :, None] + np.einsum("ij,ejq->eiq", _A, X)
        return _state(_const(X, 1.2), _vec(X, _U0), _const(X, 0.9), B), B

    x = m.get("x_sp")
    Q, B = st(x)
    gh, _ = st(m.get("x_bfp"))
    ch = 0.7
    R, ts = m.residual(oracle.make_params(c_h=ch, glm_a=0.3, powell=powell, wall_kind=(1, 1)), Q, gh,
                       with_scale=True)
    return R, B, ch, ts


def _powell_want(B, ch, powell):
    divB = np.trace(_A)
    u = _U0[None, :, None]
    gradB = _A  # dB_i/dx_j = A_ij
    J = np.array([gradB[2, 1] - gradB[1, 2], gradB[0, 2] - gradB[2, 0], gradB[1, 0] - gradB[0, 1]])
    lorentz = np.cross(J[None, :, None], B, axis=1)                      # (curl B) x B
    adv = np.einsum("j,ij->i", _U0, gradB)[None, :, None] * np.ones_like(B)  # (u . grad) B
    uB = (u * B).sum(1)
    want = np.zeros((B.shape[0], 9, B.shape[2]))
    want[:, 1:4] = lorentz
    want[:, 5:8] = -adv
    # magnetic energy changes by B . dB/dt, kinetic by u . dm/dt; Powell's
    # form leaves the pressure unchanged
    want[:, 4] = (u * lorentz).sum(1) - (B * adv).sum(1)
    want[:, 8] = -ch * divB
    if not powell:  # the conservative form keeps the div B terms
        want[:, 1:4] += B * divB
        want[:, 5:8] += u * divB
        want[:, 4] += uB * divB
    return want


@pytest.mark.parametrize("powell", [1, 0])
def test_powell_terms_linear_divergent_field(oracle, powell):
    powell_pin(oracle, powell)


def powell_pin(oracle, powell=1):
    R, B, ch, ts = _powell_case(oracle, powell)
    want = _powell_want(B, ch, powell)
    # round-off scale: the magnitude of the differentiated fluxes
    err = np.abs(R - want).max(axis=(0, 2))
    assert (err <= 1e-12 * ts).all(), (err, ts)


# ---------------------------------------------------------------------------
# radiative heat flux -kappa_r rho C_p grad T
# ---------------------------------------------------------------------------

_H = np.array([[0.20, 0.05, -0.03], [0.05, -0.10, 0.04], [-0.03, 0.04, 0.15]])  # trace 0.25
_GT = np.array([0.3, -0.2, 0.1])


def _kr_box(oracle, kr):
    """Gas at rest, B = 0, uniform rho, quadratic temperature
    T = T0 + g.x + x.H.x on an affine box with exact ghosts, kappa = nu =
    eta = 0: the heat equation gives dE/dt = div(kappa_r rho C_p grad T) and
    the momentum feels -grad p."""
    N = 5
    m = oracle.Mesh.box(N, 2, 2, 2, L=(1.0, 0.8, 0.6), periodic=0)
    rho0, T0 = 1.1, 0.9

    def st(X):
        T = T0 + np.einsum("j,ejq->eq", _GT, X) + np.einsum("eiq,ij,ejq->eq", X, _H, X)
        return _state(_const(X, rho0), _vec(X, [0.0, 0.0, 0.0]), rho0 * T, _vec(X, [0.0, 0.0, 0.0]))

    x = m.get("x_sp")
    prm = oracle.make_params(c_h=0.5, wall_kind=(1, 1), **kr)
    R, ts = m.residual(prm, st(x), st(m.get("x_bfp")), with_scale=True)
    gT = _GT[None, :, None] + 2.0 * np.einsum("ij,ejq->eiq", _H, x)
    return R, ts, x, rho0, gT


def kr_constant_pin(oracle):
    """Constant kappa_r: dE/dt = kappa_r rho C_p lap T = kappa_r rho C_p 2 tr H."""
    k = 0.04
    R, ts, x, rho0, gT = _kr_box(oracle, dict(kr_scale=2.0, kr_c0=k / 2.0))
    want_E = k * rho0 * CP * 2.0 * np.trace(_H)
    assert np.abs(R[:, 4] - want_E).max() <= 1e-12 * ts[4], (np.abs(R[:, 4] - want_E).max(), ts[4])
    want_m = -rho0 * gT  # -grad p with p = rho0 Rgas T
    assert np.abs(R[:, 1:4] - want_m).max() <= 1e-12 * ts[1:4].max()


def kr_quadratic_radius_pin(oracle):
    """kappa_r = s c2 (w r)^2 (the quadratic coefficient alone) is a
    polynomial of the position, so the method is exact again:
    dE/dt = rho C_p (kappa_r lap T + grad kappa_r . grad T) with
    grad kappa_r = 2 s c2 w^2 x.  This also fixes where kappa_r is taken: at
    the flux points, by interpolation from the solution points."""
    s, c2, w = 1.5, 0.2, 0.8
    R, ts, x, rho0, gT = _kr_box(oracle, dict(kr_scale=s, kr_c2=c2, kr_omega_per_r=w))
    r2 = (x * x).sum(1)
    kr = s * c2 * w * w * r2
    gkr = 2.0 * s * c2 * w * w * x
    want_E = rho0 * CP * (kr * 2.0 * np.trace(_H) + (gkr * gT).sum(1))
    assert np.abs(R[:, 4] - want_E).max() <= 1e-12 * ts[4], (np.abs(R[:, 4] - want_E).max(), ts[4])


def test_coriolis_turns_a_uniform_flow(oracle):
    coriolis_uniform_pin(oracle)


def test_coriolis_inertial_oscillation(oracle):
    coriolis_oscillation_pin(oracle)


def test_radiative_flux_constant_kappa_r(oracle):
    kr_constant_pin(oracle)


def test_radiative_flux_kappa_r_quadratic_in_radius(oracle):
    kr_quadratic_radius_pin(oracle)


def test_radiative_flux_kappa_r_of_radius_on_the_shell_converges(oracle):
    """kappa_r(r) = s (c0 + c1 w r) on the curved shell (not a polynomial of
    the position) with T = T0 + a r^2, gas at rest: the radiative part of the
    energy residual (the residual less that with kappa_r = 0) converges to
    div(kappa_r rho C_p grad T) = rho C_p (6 a kappa_r + 2 a s c1 w r) at the
    order p - 1 of the method's second derivatives (exact ghosts on both
    walls)."""
    s, c0, c1, w, a, rho0, T0 = 1.0, 0.01, 0.03, 1.3, 0.4, 1.0, 0.5
    errs = []
    for Nz in (2, 3, 4):
        m = oracle.Mesh.shell(6, Nz, Nz)

        def st(X):
            r2 = (X * X).sum(1)
            return _state(_const(X, rho0), _vec(X, [0.0, 0.0, 0.0]), rho0 * (T0 + a * r2), _vec(X, [0.0, 0.0, 0.0]))

        x = m.get("x_sp")
        r = np.sqrt((x * x).sum(1))
        gh = st(m.get("x_bfp"))
        R = m.residual(oracle.make_params(c_h=0.5, wall_kind=(1, 1), kr_scale=s, kr_c0=c0, kr_c1=c1,
                                          kr_omega_per_r=w), st(x), gh)
        R0 = m.residual(oracle.make_params(c_h=0.5, wall_kind=(1, 1)), st(x), gh)
        want = rho0 * CP * (6.0 * a * s * (c0 + c1 * w * r) + 2.0 * a * s * c1 * w * r)
        errs.append(np.abs(R[:, 4] - R0[:, 4] - want).max() / np.abs(want).max())
    order = np.log(errs[1] / errs[2]) / np.log(4.0 / 3.0)
    assert errs[2] < 1e-4 and order > 3.0, (errs, order)


# ---------------------------------------------------------------------------
# planted mistakes: each must make at least one pin fail
# ---------------------------------------------------------------------------

MUTANTS = [
    # (what is planted, text in the oracle source, replacement, pin)
    ("Coriolis sign", "2.0 * P->Omega * qq[2]", "-2.0 * P->Omega * qq[2]", coriolis_uniform_pin),
    ("Coriolis factor 2 dropped", "M[2] = rho * gv[1] - 2.0 * P->Omega", "M[2] = rho * gv[1] - 1.0 * P->Omega",
     coriolis_uniform_pin),
    ("Coriolis sign (both rows)", "M[1] = rho * gv[0] + 2.0 * P->Omega * qq[2]",
     "M[1] = rho * gv[0] - 2.0 * P->Omega * qq[2]", coriolis_oscillation_pin),
    ("Powell momentum sign", "- db * qq[5];", "+ db * qq[5];", powell_pin),
    ("Powell momentum dropped", "M[3] = rho * gv[2] - db * qq[7];", "M[3] = rho * gv[2];", powell_pin),
    ("Powell energy sign", "- db * uB;", "+ db * uB;", powell_pin),
    ("Powell induction sign", "M[5 + c] = -db * u[c];", "M[5 + c] = db * u[c];", powell_pin),
    ("radiative flux sign", "- kr * rho * cp * dT[j];", "+ kr * rho * cp * dT[j];", kr_constant_pin),
    ("radiative flux without C_p", "- kr * rho * cp * dT[j];", "- kr * rho * dT[j];", kr_constant_pin),
    ("kappa_r at the element centre, not interpolated",
     "for (int i = 0; i < N; ++i) kf += t->I[f][i] * kr[sp_on_line(N, d, a, b, i)];",
     "kf = kr[N3 / 2];", kr_quadratic_radius_pin),
    ("kappa_r quadratic coefficient squared radius dropped", "P->kr_c2 * w * w", "P->kr_c2 * w",
     kr_quadratic_radius_pin),
]


def test_planted_mistakes_are_caught(oracle, tmp_path):
    src = oracle.source_text()
    for k, (what, find, repl, pin) in enumerate(MUTANTS):
        assert src.count(find) == 1, (what, src.count(find))
        path = oracle.build_variant(src.replace(find, repl), os.path.join(str(tmp_path), f"mutant{k}.so"))
        prev = oracle.swap_library(path)
        try:
            with pytest.raises(AssertionError):
                pin(oracle)
        finally:
            oracle.swap_back(prev)
    # and the real oracle passes every pin used above
    for pin in {m[3] for m in MUTANTS}:
        pin(oracle)
