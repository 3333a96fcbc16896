"""Pins of the oracle's initial background (Sec. "Initial Conditions"): the
polytrope's defining properties, hydrostatic balance and the heat flux of
the flux-balanced profile, checked by finite differences and quadrature of
the oracle's output (none of them re-evaluates the oracle's own formulas)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import background as ob

BASE = dict(GM=1.0, Rgas=1.0, gamma=5.0 / 3.0, rb=0.70, rt=0.98, rho_b=1.0)


def _fd(f, r, h):
    """Fourth-order central difference of f at r."""
    return (f(r - 2 * h) - 8 * f(r - h) + 8 * f(r + h) - f(r + 2 * h)) / (12 * h)


@pytest.mark.parametrize("N_rho", [3.0, 5.0])
def test_polytrope_defining_properties(N_rho):
    """rho(r_b) = rho_b, ln(rho_b / rho_t) = N_rho, ideal gas, and dp/dr = -rho g."""
    rho, p, T = ob.polytrope(np.array([0.70, 0.98]), N_rho=N_rho, **BASE)
    assert rho[0] == pytest.approx(1.0, rel=1e-15)
    assert np.log(rho[0] / rho[1]) == pytest.approx(N_rho, rel=1e-13)
    np.testing.assert_allclose(p, rho * T, rtol=1e-15)
    r = np.linspace(0.71, 0.97, 9)
    dpdr = _fd(lambda x: ob.polytrope(x, N_rho=N_rho, **BASE)[1], r, 2e-4)
    rho_r = ob.polytrope(r, N_rho=N_rho, **BASE)[0]
    np.testing.assert_allclose(dpdr, -rho_r / r ** 2, rtol=1e-8)


def test_polytrope_is_isentropic():
    r = np.linspace(0.70, 0.98, 11)
    rho, p, _ = ob.polytrope(r, N_rho=3.0, **BASE)
    S = ob.entropy(rho, p, 5.0 / 3.0, 1.0)
    assert np.ptp(S) < 1e-13 * 2.5


def test_no_flux_gives_the_polytrope():
    """L = 0 and kappa_r = 0: no entropy gradient, so the hydrostatic density
    equation must return the adiabatic polytrope (with the printed exponent
    +gamma S / C_p it would not, since S_b != 0)."""
    r = np.linspace(0.70, 0.98, 29)
    rho, p, T, S = ob.flux_balanced(r, N_rho=3.0, L=0.0, kappa=1e-5, kr=lambda x: 0.0 * x, **BASE)
    r0, p0, T0 = ob.polytrope(r, N_rho=3.0, **BASE)
    assert abs(S[0]) > 0.1
    np.testing.assert_allclose(rho, r0, rtol=1e-11)
    np.testing.assert_allclose(p, p0, rtol=1e-11)
    np.testing.assert_allclose(T, T0, rtol=1e-11)


def _kr(x):
    return 2e-6 * (1.5 - 1.2 * x)


@pytest.mark.parametrize("L,kr", [(2e-7, None), (1e-6, None), (1e-6, _kr)])
def test_flux_balanced_is_hydrostatic(L, kr):
    """dp/dr = -rho GM / r^2 of the returned profile (4th-order differences of
    its pressure), and the ideal-gas law."""
    kr = kr or (lambda x: 0.0 * x)
    kw = dict(N_rho=3.0, L=L, kappa=1e-5, kr=kr, **BASE)
    r = np.linspace(0.72, 0.96, 13)
    h = 2e-3
    pts = np.concatenate([r + k * h for k in (-2, -1, 1, 2)])
    rho_all, p_all, T_all, _ = ob.flux_balanced(np.concatenate([r, pts]), **kw)
    n = len(r)
    P = {k: p_all[n + i * n:n + (i + 1) * n] for i, k in enumerate((-2, -1, 1, 2))}
    dpdr = (P[-2] - 8 * P[-1] + 8 * P[1] - P[2]) / (12 * h)
    np.testing.assert_allclose(dpdr, -rho_all[:n] / r ** 2, rtol=2e-8)
    np.testing.assert_allclose(p_all, rho_all * T_all, rtol=1e-15)


def test_flux_balanced_carries_the_luminosity_outward():
    """kappa_r = 0: the entropy-diffusion flux through the polytrope,
    -kappa rho0 T0 dS/dr with dS/dr differenced from the returned profile's
    entropy, times 4 pi r^2 is L at every radius; the entropy falls outward."""
    L, kappa = 1e-6, 1e-5
    kw = dict(N_rho=3.0, L=L, kappa=kappa, kr=lambda x: 0.0 * x, **BASE)
    r = np.linspace(0.72, 0.96, 7)
    h = 5e-4
    ks = (-2, -1, 1, 2)
    rho, p, _, _ = ob.flux_balanced(np.concatenate([r + k * h for k in ks]), **kw)
    S = ob.entropy(rho, p, 5.0 / 3.0, 1.0).reshape(4, -1)
    dS = (S[0] - 8 * S[1] + 8 * S[2] - S[3]) / (12 * h)
    assert (dS < 0).all()
    rho0, _, T0 = ob.polytrope(r, N_rho=3.0, **BASE)
    np.testing.assert_allclose(-kappa * rho0 * T0 * dS * 4 * np.pi * r ** 2, L, rtol=1e-8)


def test_flux_balanced_entropy_is_the_integral_of_its_gradient():
    """S(r) of the returned profile = S_b + quadrature of the entropy
    gradient (radiative term included)."""
    kw = dict(N_rho=3.0, L=5e-7, kappa=1e-5, kr=_kr, **BASE)
    r = np.array([0.70, 0.77, 0.85, 0.98])
    rho, p, _, S = ob.flux_balanced(r, **kw)
    np.testing.assert_allclose(S, ob.entropy(rho, p, 5.0 / 3.0, 1.0), rtol=1e-13, atol=1e-13)
    r0, p0, _ = ob.polytrope(0.70, N_rho=3.0, **BASE)
    S_b = ob.entropy(r0, p0, 5.0 / 3.0, 1.0)
    for x, s in zip(r, S):
        integral = quad(lambda y: float(ob.entropy_gradient(y, N_rho=3.0, L=5e-7, kappa=1e-5, kr=_kr, **BASE)),
                        0.70, x, epsabs=1e-14, epsrel=1e-13)[0]
        assert s == pytest.approx(S_b + integral, rel=1e-11, abs=1e-12)


def test_radiative_flux_stabilises_the_bottom():
    """When the polytrope's radiative flux at r_b equals the luminosity
    (kappa_r rho C_p |dT/dr| = L / (4 pi r_b^2)), the entropy gradient
    vanishes there and turns negative above, where kappa_r falls."""
    kw = dict(N_rho=3.0, **BASE)
    L, kappa = 1e-6, 1e-5
    rb = 0.70
    rho_b = ob.polytrope(rb, **kw)[0]
    k_b = L / (4 * np.pi * rb ** 2) / (rho_b * 2.5 * (1.0 / (2.5 * rb ** 2)))

    def kr(x):
        return k_b * (rb / np.asarray(x)) ** 8

    g = ob.entropy_gradient(np.array([rb, 0.8, 0.9]), L=L, kappa=kappa, kr=kr, **kw)
    assert abs(g[0]) < 1e-9 * abs(g[1])
    assert g[1] < 0 and g[2] < g[1]
