"""Pins of the oracle's diagnostics (volume integrals with the Fejer weights
of the solution points times |J|, Sec. "Results"): closed forms for states
whose integrals are known exactly."""
import numpy as np

G53 = 5.0 / 3.0


def _state(x, rho, u, p, B, psi):
    """Q at points x [E][3][n] from fields given as functions of x."""
    E, _, n = x.shape
    r, U, P, Bv, ps = rho(x), u(x), p(x), B(x), psi(x)
    Q = np.zeros((E, 9, n))
    Q[:, 0] = r
    Q[:, 1:4] = r[:, None] * U
    Q[:, 4] = P / (G53 - 1) + 0.5 * r * (U * U).sum(1) + 0.5 * (Bv * Bv).sum(1) + 0.5 * ps ** 2
    Q[:, 5:8] = Bv
    Q[:, 8] = ps
    return Q


def test_uniform_state_integrals_on_box(oracle):
    """Uniform state on a box of known volume: volume, mass, energy, KE and
    E_B densities are the constants times the volume (or the constants);
    div B = 0; max|psi| = |psi|."""
    m = oracle.Mesh.box(5, 3, 3, 3, L=(1.0, 0.7, 0.5), periodic=7)
    x = m.get("x_sp")
    u0, B0 = np.array([0.3, -0.2, 0.1]), np.array([0.05, 0.1, -0.2])
    Q = _state(x, lambda x: np.full(x[:, 0].shape, 1.7), lambda x: np.broadcast_to(u0[None, :, None], x.shape),
               lambda x: np.full(x[:, 0].shape, 0.9), lambda x: np.broadcast_to(B0[None, :, None], x.shape),
               lambda x: np.full(x[:, 0].shape, -0.03))
    d = oracle.Mesh.diagnostics(m, oracle.make_params(), Q)
    V = 1.0 * 0.7 * 0.5
    assert abs(d[0] - V) <= 1e-14
    assert abs(d[1] - 1.7 * V) <= 1e-14
    assert abs(d[2] - Q[0, 4, 0] * V) <= 1e-14
    assert abs(d[3] - 0.5 * 1.7 * u0 @ u0) <= 1e-14
    assert abs(d[4] - 0.5 * B0 @ B0) <= 1e-15
    assert d[5] <= 1e-13 and d[6] <= 1e-13
    assert d[7] == 0.03 and d[8] == 0.0


def test_polynomial_integrals_and_divergence_on_affine_box(oracle):
    """Fields polynomial in x on an affine box: the Gauss-type quadrature on
    N points is exact to degree N-1 in each direction, so integrals of
    rho = 1 + x^2 y and of |B|^2/2 for B = (x, y, z) are exact; div B = 3
    exactly (Dirichlet ghosts with the exact field on every face)."""
    N = 5
    Lx, Ly, Lz = 1.0, 0.7, 0.5
    m = oracle.Mesh.box(N, 2, 2, 2, L=(Lx, Ly, Lz), periodic=0)
    x, xb = m.get("x_sp"), m.get("x_bfp")
    fields = (lambda x: 1.0 + x[:, 0] ** 2 * x[:, 1], lambda x: np.zeros(x.shape), lambda x: np.ones(x[:, 0].shape),
              lambda x: x.copy(), lambda x: np.zeros(x[:, 0].shape))
    Q, g = _state(x, *fields), _state(xb, *fields)
    d = oracle.Mesh.diagnostics(m, oracle.make_params(wall_kind=(1, 1)), Q, g)
    V = Lx * Ly * Lz
    mass = V + (Lx ** 3 / 3) * (Ly ** 2 / 2) * Lz
    EB = 0.5 * (Lx ** 3 * Ly * Lz + Lx * Ly ** 3 * Lz + Lx * Ly * Lz ** 3) / 3 / V
    assert abs(d[1] - mass) <= 1e-14
    assert abs(d[4] - EB) <= 1e-14
    assert abs(d[5] - 3.0) <= 1e-12 and abs(d[6] - 3.0) <= 1e-12
    assert d[3] == 0.0


def test_nan_flag(oracle):
    m = oracle.Mesh.box(3, 3, 3, 3, periodic=7)
    Q = np.zeros((m.E, 9, 27))
    Q[:, 0] = 1.0
    Q[:, 4] = 1.0
    assert oracle.Mesh.diagnostics(m, oracle.make_params(), Q)[8] == 0.0
    Q[5, 2, 7] = np.inf
    assert oracle.Mesh.diagnostics(m, oracle.make_params(), Q)[8] == 1.0


# --- spherical components (Sec. "Results": differential rotation, meridional
# flow, poloidal and toroidal magnetic energy) ---------------------------------

def _sph_frame(x):
    """r_hat, theta_hat, phi_hat at points x [E][3][n] (test-side construction)."""
    r = np.sqrt((x ** 2).sum(1))
    rc = np.sqrt(x[:, 0] ** 2 + x[:, 1] ** 2)
    rh = x / r[:, None]
    ph = np.stack([-x[:, 1] / rc, x[:, 0] / rc, np.zeros_like(rc)], 1)
    th = np.stack([x[:, 0] * x[:, 2] / (r * rc), x[:, 1] * x[:, 2] / (r * rc), -rc / r], 1)
    return rh, th, ph


def _flow_state(x, U, B):
    rho = 1.0 + 0.3 * np.sin(3 * x[:, 0]) * np.cos(2 * x[:, 2])
    return _state(x, lambda x: rho, lambda x: U, lambda x: np.full(rho.shape, 0.2), lambda x: B,
                  lambda x: np.zeros(rho.shape))


def test_sph_energy_split_sums_to_EB(oracle):
    """(B_r^2 + B_theta^2)/2 + B_phi^2/2 = |B|^2/2 pointwise, so the two volume
    averages add up to E_B of the diagnostics for any field."""
    m = oracle.Mesh.shell(6, 2, 2)
    x = m.get("x_sp")
    rng = np.random.default_rng(5)
    B = rng.normal(size=x.shape)
    U = rng.normal(size=x.shape) * 0.1
    Q = _flow_state(x, U, B)
    d = oracle.Mesh.diagnostics(m, oracle.make_params(), Q)
    P = m.sph_profiles(Q, 3, 5)
    V = P[..., 0].sum()
    assert abs(V - d[0]) <= 1e-13 * V
    assert abs((P[..., 3].sum() + P[..., 4].sum()) / V - d[4]) <= 1e-13 * d[4]


def test_sph_pure_fields(oracle):
    """A purely toroidal field has no poloidal energy and vice versa; the dipole
    of the initial condition is poloidal."""
    m = oracle.Mesh.shell(6, 2, 2)
    x = m.get("x_sp")
    rh, th, ph = _sph_frame(x)
    zero = np.zeros(x.shape)
    for B, tor in ((0.7 * ph, True), (0.4 * rh, False), (0.3 * th, False)):
        P = m.sph_profiles(_flow_state(x, zero, B), 2, 4)
        c2 = (B ** 2).sum(1).max() / 2
        if tor:
            assert np.abs(P[..., 3]).max() <= 1e-14 * P[..., 0].max()
            assert np.allclose(P[..., 4] / P[..., 0], c2, rtol=1e-13, atol=0)
        else:
            assert np.abs(P[..., 4]).max() <= 1e-14 * P[..., 0].max()
            assert np.allclose(P[..., 3] / P[..., 0], c2, rtol=1e-13, atol=0)
    r = np.sqrt((x ** 2).sum(1))
    zh = np.array([0.0, 0.0, 1.0])[None, :, None]
    dip = 1e-3 * (0.7 / r[:, None]) ** 3 * (3 * (rh * zh).sum(1, keepdims=True) * rh - zh)
    P = m.sph_profiles(_flow_state(x, zero, dip), 2, 4)
    assert np.abs(P[..., 4]).max() <= 1e-14 * np.abs(P[..., 3]).max()


def test_sph_flows(oracle):
    """Constant radial, polar and azimuthal flows: V_mer and V_phi bin averages
    are the constants exactly (the azimuthal direction counter-clockwise about
    +z); a solid-body rotation has no meridional flow and V_phi > 0."""
    m = oracle.Mesh.shell(6, 2, 2)
    x = m.get("x_sp")
    rh, th, ph = _sph_frame(x)
    zero = np.zeros(x.shape)
    for U, vm, vp in ((0.05 * rh, 0.05, 0.0), (-0.03 * th, 0.03, 0.0), (0.02 * ph, 0.0, 0.02),
                      (0.03 * rh + 0.04 * th, 0.05, 0.0)):
        P = m.sph_profiles(_flow_state(x, U, zero), 3, 4)
        assert np.allclose(P[..., 2] / P[..., 0], vm, rtol=1e-13, atol=1e-15)
        assert np.allclose(P[..., 1] / P[..., 0], vp, rtol=1e-13, atol=1e-15)
    Om = 0.12
    U = Om * np.stack([-x[:, 1], x[:, 0], np.zeros_like(x[:, 0])], 1)
    P = m.sph_profiles(_flow_state(x, U, zero), 3, 4)
    assert np.abs(P[..., 2]).max() <= 1e-14 * P[..., 0].max()
    assert (P[..., 1] > 0).all()


def test_sph_bin_volumes(oracle):
    """With the radial bins on the element layers (uniform in r) and the
    theta bins split at the equator (an element boundary for even N_z), the
    bins' summed weights are the volumes of the spherical-shell pieces, to
    the mesh's geometric accuracy."""
    m = oracle.Mesh.shell(6, 4, 3)
    Q = np.zeros((m.E, 9, 216))
    Q[:, 0] = 1.0
    Q[:, 4] = 1.0
    P = m.sph_profiles(Q, 3, 2)
    rs = 0.70 + np.arange(4) * (0.98 - 0.70) / 3
    for i in range(3):
        vol_half = 2 * np.pi / 3 * (rs[i + 1] ** 3 - rs[i] ** 3)
        assert abs(P[i, 0, 0] - vol_half) <= 1e-8 * vol_half
        assert abs(P[i, 1, 0] - vol_half) <= 1e-8 * vol_half
