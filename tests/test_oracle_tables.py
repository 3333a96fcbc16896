"""Pins of the oracle's 1-D tables (paper, Sec. "Spectral Difference Method":
solution points, flux points, Lagrange bases h_i and l_i)."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sd_points.txt")


def _golden():
    out = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        kind, n, *vals = line.split()
        out[(kind, int(n))] = np.array([float(v) for v in vals])
    return out


@pytest.mark.parametrize("N", [4, 6])
def test_points_match_closed_forms(oracle, N):
    xs, xf, I, D, W = oracle.tables(N)
    g = _golden()
    np.testing.assert_allclose(xs, g[("xs", N)], atol=2e-16)
    np.testing.assert_allclose(xf, g[("xf", N)], atol=2e-16)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_points_textbook_and_symmetric(oracle, N):
    xs, xf, *_ = oracle.tables(N)
    # Legendre roots from numpy's own routine (independent of the oracle's Newton)
    r = np.sort(np.polynomial.legendre.legroots([0] * (N - 1) + [1])) if N > 1 else np.array([])
    np.testing.assert_allclose(xf[1:-1], 0.5 * (1 + r), atol=1e-15)
    assert xf[0] == 0.0 and xf[-1] == 1.0 and len(xf) == N + 1
    np.testing.assert_allclose(xs + xs[::-1], 1.0, atol=1e-15)
    np.testing.assert_allclose(xf + xf[::-1], 1.0, atol=1e-15)
    assert np.all(np.diff(xs) > 0) and np.all(np.diff(xf) > 0)


@pytest.mark.parametrize("N", [3, 4, 6, 8])
def test_interpolation_and_derivative_exactness(oracle, N):
    xs, xf, I, D, W = oracle.tables(N)
    # I reproduces every polynomial of degree <= N-1 at the flux points
    for k in range(N):
        np.testing.assert_allclose(I @ xs ** k, xf ** k, atol=1e-13)
    # D differentiates every polynomial of degree <= N (sampled at the flux points)
    for k in range(N + 1):
        exact = k * xs ** (k - 1) if k else np.zeros(N)
        np.testing.assert_allclose(D @ xf ** k, exact, atol=1e-11 * max(1, k))
    np.testing.assert_allclose(I.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)
    # the degree-N+1 monomial is NOT differentiated exactly (the pin is tight)
    k = N + 1
    assert np.abs(D @ xf ** k - k * xs ** (k - 1)).max() > 1e-6


@pytest.mark.parametrize("N", [3, 4, 6, 8])
def test_quadrature_weights(oracle, N):
    xs, xf, I, D, W = oracle.tables(N)
    assert abs(W.sum() - 1.0) < 1e-15
    for k in range(N):  # exact for degree <= N-1
        assert abs(W @ xs ** k - 1.0 / (k + 1)) < 1e-14
    # discrete fundamental theorem: sum_i W_i (D F)_i = F_N - F_0 for any F
    rng = np.random.default_rng(N)
    for _ in range(5):
        F = rng.standard_normal(N + 1)
        assert abs(W @ (D @ F) - (F[-1] - F[0])) < 1e-12
