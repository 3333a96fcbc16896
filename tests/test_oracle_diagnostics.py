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
