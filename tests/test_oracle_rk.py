"""Pins of the oracle's SSPRK(5,3) scheme (paper, Sec. "Spectral Difference
Method": five-stage, third-order strong-stability-preserving Runge-Kutta)."""
import numpy as np


def _butcher(a, b):
    A = np.zeros((6, 5))
    for i in range(1, 6):
        for k in range(i):
            A[i] += a[i, k] * A[k]
            A[i, k] += b[i, k]
    return A[:5], A[5]


def test_order_conditions_and_ssp_coefficient(oracle):
    a, b, c = oracle.ssprk53_table()
    np.testing.assert_allclose(a[1:].sum(axis=1), 1.0, atol=1e-15)   # consistency of the convex form
    assert (a >= 0).all() and (b >= 0).all()
    A, bb = _butcher(a, b)
    cc = A.sum(axis=1)
    np.testing.assert_allclose(cc, c, atol=1e-15)
    assert abs(bb.sum() - 1) < 1e-15
    assert abs(bb @ cc - 0.5) < 1e-15
    assert abs(bb @ cc ** 2 - 1 / 3) < 1e-15
    assert abs(bb @ A @ cc - 1 / 6) < 1e-15
    # 4th-order condition fails: the scheme is exactly third order
    assert abs(bb @ cc ** 3 - 0.25) > 1e-4
    r = min(a[i, k] / b[i, k] for i in range(6) for k in range(6) if b[i, k] > 0)
    assert abs(r - 2.6506) < 1e-4      # SSP coefficient of the optimal 5-stage 3rd-order scheme


def test_step_converges_at_third_order(oracle):
    """psi' = -a psi (uniform state, periodic box: the residual is exactly the
    GLM damping source); the one-step error of the oracle's full step against
    exp(-a t) over a fixed horizon falls like dt^3."""
    m = oracle.Mesh.box(3, 3, 3, 3, periodic=7)
    Q = np.zeros((m.E, 9, 27))
    Q[:, 0] = 1.0
    Q[:, 4] = 1.5 + 0.5 * 0.3 ** 2
    Q[:, 8] = 0.3
    a = 2.0
    prm = oracle.make_params(glm_a=a)
    errs = []
    for nstep in (4, 8, 16):
        dt = 1.0 / nstep
        q = Q.copy()
        for _ in range(nstep):
            q = m.step(prm, q, dt)
        errs.append(abs(q[0, 8, 0] - 0.3 * np.exp(-a)))
    o1 = np.log2(errs[0] / errs[1])
    o2 = np.log2(errs[1] / errs[2])
    assert 2.7 < o1 < 3.3 and 2.8 < o2 < 3.2, errs


def test_table_matches_derivation(oracle):
    """The oracle's compiled table equals the committed derivation."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "ssp_derive", os.path.join(os.path.dirname(__file__), "..", "oracle", "ssprk53_coefficients.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    a, b = mod.derive()
    A, B, _ = oracle.ssprk53_table()
    for (i, k), v in a.items():
        assert abs(A[i, k] - float(v)) <= 1e-16
    for (i, k), v in b.items():
        assert abs(B[i, k] - float(v)) <= 1e-16
