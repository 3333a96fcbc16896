"""Pins of the oracle's full residual: invariants the method fixes and exact
solutions it must converge to (paper, Sec. "Spectral Difference Method" and
Sec. "Problem Formulation and Boundary Conditions")."""
import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

G53 = 5.0 / 3.0


def _uniform(E, n3, rho, u, p, B, psi=0.0):
    u, B = np.asarray(u, float), np.asarray(B, float)
    st = np.array([rho, *(rho * u), p / (G53 - 1) + 0.5 * rho * u @ u + 0.5 * B @ B + 0.5 * psi ** 2, *B, psi])
    return np.tile(st[None, :, None], (E, 1, n3)).copy(), st


@pytest.mark.parametrize("N", [4, 6])
def test_free_stream_curved_shell(oracle, N):
    """A uniform state with equal Dirichlet ghosts is steady to round-off on
    the curved shell, viscous, resistive and GLM terms on (metric identities
    and face orientation codes)."""
    m = oracle.Mesh.shell(N, 2, 2)
    Q, st = _uniform(m.E, N ** 3, 1.3, [0.2, -0.1, 0.3], 0.7, [0.05, -0.02, 0.07], 0.01)
    g = np.tile(st[None, :, None], (m.NB, 1, N * N))
    prm = oracle.make_params(nu=1e-2, kappa=1e-2, eta=1e-2, c_h=1.0, powell=1, wall_kind=(1, 1))
    R, ts = m.residual(prm, Q, g, with_scale=True)
    assert (np.abs(R).max(axis=(0, 2)) <= 1e-13 * ts).all()


def test_polynomial_exactness_affine_box(oracle):
    """Passive density of degree p in x, y, z, uniform u, p, B (inviscid) on an
    affine box with exact ghosts: R = exact time derivative to round-off."""
    N = 5
    m = oracle.Mesh.box(N, 3, 2, 2, L=(1.0, 0.7, 0.5), periodic=0)
    x = m.get("x_sp")
    xb = m.get("x_bfp")
    u = np.array([0.3, -0.2, 0.15])
    B = np.array([0.1, 0.2, -0.05])
    p = 0.8

    def rho_f(X):
        return 1.0 + 0.1 * X[:, 0] ** 4 + 0.2 * X[:, 0] * X[:, 1] ** 2 * X[:, 2] - 0.1 * X[:, 2] ** 3 + 0.05 * X[:, 1]

    def grad_rho(X):
        return np.stack([0.4 * X[:, 0] ** 3 + 0.2 * X[:, 1] ** 2 * X[:, 2],
                         0.4 * X[:, 0] * X[:, 1] * X[:, 2] + 0.05,
                         0.2 * X[:, 0] * X[:, 1] ** 2 - 0.3 * X[:, 2] ** 2], axis=1)

    def state(X):
        r = rho_f(X)
        Q = np.empty((X.shape[0], 9, X.shape[2]))
        Q[:, 0] = r
        Q[:, 1:4] = r[:, None] * u[None, :, None]
        Q[:, 4] = p / (G53 - 1) + 0.5 * r * (u @ u) + 0.5 * B @ B
        Q[:, 5:8] = B[None, :, None]
        Q[:, 8] = 0.0
        return Q

    prm = oracle.make_params(c_h=0.5, wall_kind=(1, 1))
    R, ts = m.residual(prm, state(x), state(xb), with_scale=True)
    drho = -(grad_rho(x) * u[None, :, None]).sum(axis=1)
    want = np.zeros_like(R)
    want[:, 0] = drho
    want[:, 1:4] = u[None, :, None] * drho[:, None]
    want[:, 4] = 0.5 * (u @ u) * drho
    err = np.abs(R - want).max(axis=(0, 2))
    assert (err <= 1e-12 * ts).all(), (err, ts)


def _shell_setup(oracle, N=6, Nz=2, Nr=2, seed=0, N_rho=3.0):
    m = oracle.Mesh.shell(N, Nz, Nr)
    bg = inp.Background(N_rho)
    Q = inp.shell_state(m.get("x_sp"), bg, seed, u_amp=1e-2, b_amp=1e-2)
    return m, bg, Q


def test_mass_conservation_walls(oracle):
    m, bg, Q = _shell_setup(oracle)
    pr = inp.run_params(0, bg, nu=1e-3)
    pr.update(c_h=0.6, glm_a=2.0)
    prm = oracle.make_params(**pr)
    R = m.residual(prm, Q)
    w = m.get("W3detJ")
    dm = (w * R[:, 0]).sum()
    assert abs(dm) < 1e-14 * (w * np.abs(R[:, 0])).sum() * 100
    assert abs(dm) < 1e-15


def test_energy_conservation_closed_walls(oracle):
    """Conducting, adiabatic (q = 0), stress-free walls, no gravity, no GLM
    damping, Powell terms off: total energy is conserved to round-off even
    for a far-from-equilibrium state with all dissipative terms on."""
    m = oracle.Mesh.shell(6, 2, 2)
    Q = inp.smooth_random_state(m.get("x_sp"), 3)
    prm = oracle.make_params(nu=1e-2, kappa=1e-2, eta=1e-2, c_h=0.8, glm_a=0.0, Omega=0.3, powell=0,
                             wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.0, 0.0))
    R = m.residual(prm, Q)
    w = m.get("W3detJ")
    de = (w * R[:, 4]).sum()
    scale = (w * np.abs(R[:, 4])).sum()
    assert abs(de) < 1e-13 * scale
    # the same with a heat flux at the inner wall must not conserve energy
    prm2 = oracle.make_params(nu=1e-2, kappa=1e-2, eta=1e-2, c_h=0.8, glm_a=0.0, Omega=0.3, powell=0,
                              wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.1, 0.0))
    assert abs((w * m.residual(prm2, Q)[:, 4]).sum()) > 1e-3


def test_heat_flux_enters_at_rate_q_times_area(oracle):
    """At rest, B = 0, no gravity: d/dt total energy = q_inner x discrete
    inner-wall area (the paper's L through the bottom surface)."""
    N = 6
    m = oracle.Mesh.shell(N, 2, 2)
    Q, _ = _uniform(m.E, N ** 3, 1.0, [0, 0, 0], 0.5, [0, 0, 0])
    qin = 0.37
    prm = oracle.make_params(nu=1e-2, kappa=1e-2, eta=1e-2, c_h=0.5, wall_th=(0, 0), q_wall=(qin, 0.0))
    R = m.residual(prm, Q)
    w = m.get("W3detJ")
    _, _, _, _, W = oracle.tables(N)
    S = m.get("S_fp")
    faces = m.get("faces")
    area = 0.0
    for eL, fL, g, bi, _ in faces[faces[:, 2] == -1]:
        for b in range(N):
            for a in range(N):
                idx = a + N * (b + N * 0)
                area += W[a] * W[b] * np.linalg.norm(S[eL, 2, :, idx])
    assert abs(area - 4 * np.pi * 0.7 ** 2) / area < 1e-6
    np.testing.assert_allclose((w * R[:, 4]).sum(), qin * area, rtol=1e-12)


def _alfven(x, t, kdir, A=0.1, p0=0.1):
    kv = np.asarray(kdir, float)
    kh = kv / np.linalg.norm(kv)
    e1 = np.cross(kh, [0, 0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    xs = np.einsum("i,eiq->eq", kh, x)
    ph = 2 * np.pi * np.linalg.norm(kv) * (xs + t)  # Alfven speed 1 along -k
    b1, b2 = A * np.sin(ph), A * np.cos(ph)
    B = kh[None, :, None] + e1[None, :, None] * b1[:, None] + e2[None, :, None] * b2[:, None]
    u = e1[None, :, None] * b1[:, None] + e2[None, :, None] * b2[:, None]
    Q = np.empty((x.shape[0], 9, x.shape[2]))
    Q[:, 0] = 1.0
    Q[:, 1:4] = u
    Q[:, 4] = p0 / (G53 - 1) + 0.5 * (u * u).sum(1) + 0.5 * (B * B).sum(1)
    Q[:, 5:8] = B
    Q[:, 8] = 0.0
    return Q


def test_alfven_wave_residual_converges_at_order_p(oracle):
    """Exact nonlinear circularly polarised Alfven wave on a periodic box:
    the residual error falls like h^p (p = N-1 = 5)."""
    errs, hs = [], []
    for n in (3, 4, 6):
        m = oracle.Mesh.box(6, n, n, n, periodic=7)
        x = m.get("x_sp")
        Q = _alfven(x, 0.0, (1, 1, 0))
        eps = 1e-5
        dQ = (_alfven(x, eps, (1, 1, 0)) - _alfven(x, -eps, (1, 1, 0))) / (2 * eps)
        R = m.residual(oracle.make_params(c_h=1.0), Q)
        errs.append(np.abs(R - dQ)[:, [1, 2, 5, 6]].max())
        hs.append(1.0 / n)
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order > 4.5, (errs, order)
    assert errs[-1] < 5e-5


def test_viscous_and_resistive_decay_rates(oracle):
    """Shear wave u = A sin(2 pi y) x and B = (B0x, 0, B0z + e sin(2 pi y)):
    the residual gives nu d2u/dy2 and eta d2Bz/dy2 (closed forms, the linear
    viscous and resistive decay rates nu k^2, eta k^2), converging under
    refinement at order >= p - 1 (second derivatives through BR1)."""
    nu, eta, A, e = 0.05, 0.03, 0.1, 0.02
    k2 = (2 * np.pi) ** 2
    errs = []
    for n in (3, 6):
        m = oracle.Mesh.box(6, n, n, n, periodic=7)
        x = m.get("x_sp")
        s = np.sin(2 * np.pi * x[:, 1])
        Q = np.zeros((m.E, 9, 216))
        Q[:, 0] = 1.0
        Q[:, 1] = A * s
        Bz = 0.3 + e * s
        Q[:, 5] = 0.2
        Q[:, 7] = Bz
        Q[:, 4] = 1.0 / (G53 - 1) + 0.5 * (A * s) ** 2 + 0.5 * (0.04 + Bz ** 2)
        R = m.residual(oracle.make_params(nu=nu, eta=eta, c_h=0.5), Q)
        # x-momentum: no pressure or Lorentz force along x, so R = -nu k^2 u exactly
        errs.append((np.abs(R[:, 1] + nu * k2 * A * s).max() / (nu * k2 * A),
                     np.abs(R[:, 7] + eta * k2 * e * s).max() / (eta * k2 * e)))
    for c in range(2):
        assert errs[1][c] < 1e-3
        assert np.log(errs[0][c] / errs[1][c]) / np.log(2.0) > 3.5


def test_glm_divergence_wave_and_decay(oracle):
    """psi responds to div B at speed c_h (R_psi = -c_h div B - a psi), and
    with damping a > 0 the integral of (div B)^2 decays in time."""
    m = oracle.Mesh.box(6, 4, 4, 4, periodic=7)
    x = m.get("x_sp")
    Q = np.zeros((m.E, 9, 216))
    Q[:, 0] = 1.0
    eps = 0.01
    Q[:, 5] = 0.3 + eps * np.sin(2 * np.pi * x[:, 0])
    Q[:, 8] = 0.02
    Q[:, 4] = 1.0 / (G53 - 1) + 0.5 * (Q[:, 5] ** 2) + 0.5 * 0.02 ** 2
    ch, a = 0.9, 1.5
    prm = oracle.make_params(c_h=ch, glm_a=a)
    R = m.residual(prm, Q)
    want = -ch * eps * 2 * np.pi * np.cos(2 * np.pi * x[:, 0]) - a * 0.02
    assert np.abs(R[:, 8] - want).max() < 1e-3 * ch * eps * 2 * np.pi
    d0 = m.diagnostics(prm, Q)
    Q2 = Q
    for _ in range(60):
        Q2 = m.step(prm, Q2, 0.008)
    d1 = m.diagnostics(prm, Q2)
    assert d1[6] < 0.75 * d0[6]  # about exp(-a t / 2) for the damped GLM waves
    # without cleaning speed (u = 0, eta = 0) div B stays put up to the
    # small Rusanov dissipation of the trace jumps
    prm0 = oracle.make_params(c_h=0.0, glm_a=0.0)
    Q3 = m.step(prm0, Q, 0.004)
    assert abs(m.diagnostics(prm0, Q3)[6] - d0[6]) < 1e-4 * d0[6]  # only face dissipation acts


def test_spherical_symmetry_patches(oracle):
    """A spherically symmetric state at rest on the shell: the six cube
    patches are rotations of each other with identical local indexing, so the
    scalar residuals agree patch by patch and the momentum residual rotates."""
    m, bg, _ = _shell_setup(oracle, Nz=2, Nr=2)
    Q = inp.shell_state(m.get("x_sp"), bg, 0, u_amp=0.0, b_amp=0.0)
    pr = inp.run_params(0, bg, nu=1e-3, Omega=0.0)
    pr.update(c_h=0.5, glm_a=1.0)
    prm = oracle.make_params(**pr)
    R, ts = m.residual(prm, Q, with_scale=True)
    Rp = R.reshape(6, -1, 9, 216)
    rots = [np.eye(3),
            np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]]),
            np.array([[-1, 0, 0], [0, -1, 0], [0, 0, 1.0]]),
            np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 1.0]]),
            np.array([[0, 0, -1], [0, 1, 0], [1, 0, 0.0]]),
            np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0.0]])]
    for P in range(1, 6):
        for v in (0, 4, 8):
            assert np.abs(Rp[P, :, v] - Rp[0, :, v]).max() <= 1e-12 * ts[v]
        mom = np.einsum("ij,ejq->eiq", rots[P], Rp[0, :, 1:4])
        assert np.abs(Rp[P, :, 1:4] - mom).max() <= 1e-12 * ts[1:4].max()


def test_rotated_state_gives_rotated_residual(oracle):
    """A general (non-symmetric) state rotated by 90 degrees about z maps
    equatorial patch P to P+1 with identical local indexing; the residual
    must rotate with it (checks every inter-patch orientation code)."""
    N = 4
    m = oracle.Mesh.shell(N, 2, 1)
    x = m.get("x_sp")
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    Q0 = inp.smooth_random_state(x, 11)
    # the same smooth fields evaluated at the un-rotated positions, vectors rotated
    xr = np.einsum("ji,ejq->eiq", Rz, x)  # Rz^T x
    Q1 = inp.smooth_random_state(xr, 11)
    Q1[:, 1:4] = np.einsum("ij,ejq->eiq", Rz, Q1[:, 1:4])
    Q1[:, 5:8] = np.einsum("ij,ejq->eiq", Rz, Q1[:, 5:8])
    prm = oracle.make_params(nu=1e-2, kappa=1e-2, eta=1e-2, c_h=0.7, glm_a=0.5, powell=1, GM=1.0,
                             wall_mag=(0, 1), wall_th=(0, 1), q_wall=(0.1, 0), T_wall=(1.0, 0.8))
    R0, ts = m.residual(prm, Q0, with_scale=True)
    R1 = m.residual(prm, Q1)
    per = m.E // 6
    for P in range(4):
        Pn = (P + 1) % 4
        a = R0[P * per:(P + 1) * per]
        b = R1[Pn * per:(Pn + 1) * per]
        for v in (0, 4, 8):
            assert np.abs(b[:, v] - a[:, v]).max() <= 1e-12 * ts[v]
        for s in (slice(1, 4), slice(5, 8)):
            rot = np.einsum("ij,ejq->eiq", Rz, a[:, s])
            assert np.abs(b[:, s] - rot).max() <= 1e-12 * ts[s].max()


def test_hydrostatic_residual_converges(oracle):
    """The polytrope at rest is an exact equilibrium of the PDE; the discrete
    residual (exact Dirichlet ghosts) falls under refinement."""
    errs = []
    for Nz, Nr in ((1, 1), (2, 2)):
        m = oracle.Mesh.shell(6, Nz, Nr)
        bg = inp.Background(3.0)
        Q = inp.shell_state(m.get("x_sp"), bg, 0, u_amp=0.0, b_amp=0.0)
        gh = inp.shell_state(m.get("x_bfp"), bg, 0, u_amp=0.0, b_amp=0.0)
        prm = oracle.make_params(GM=1.0, c_h=0.5, wall_kind=(1, 1))
        R, ts = m.residual(prm, Q, gh, with_scale=True)
        errs.append(np.abs(R[:, 1:4]).max() / ts[1:4].max())
    assert errs[1] < errs[0] / 16 and errs[1] < 1e-5, errs
