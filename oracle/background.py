"""Initial background profiles of the section "Initial Conditions"
(TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library).  Plain FP64 numpy/scipy, independent of the library's host code.

Two profiles, both functions of radius only with U = 0:

* the adiabatic polytrope (Eq. "polytrop eqns" with T_b from N_rho), and
* the almost flux-balanced profile the paper builds from it: an entropy
  gradient from the bottom heat-flux condition (Eqs. "qfluxIC", "dSdr"),
  integrated from the bottom entropy S_b, and a new density from the
  hydrostatic density equation (Eq. "densityprofile"), then p and T.

Readings where the printed equations are inconsistent or silent (each is
pinned by a test in tests/test_oracle_background.py):

* Heat-flux sign.  Eq. "qFlux" defines q = -kappa rho T grad S -
  kappa_r rho C_p grad T and the luminosity leaves the shell outward, so
  dS/dr = -(q_r + kappa_r rho C_p dT/dr) / (kappa rho T).  The printed Eq.
  "dSdr" has no leading minus; with it the entropy term would carry heat
  inward.
* Flux density.  "The total heat flux ... is constant through each radial
  layer": q_r(r) = L / (4 pi r^2), which is the printed L / (4 pi r_b^2) at
  the bottom boundary.
* Density equation.  With S = C_p ln(p^(1/gamma) / rho) (Eq. "entropy"),
  p = rho^gamma exp(gamma S / C_p); hydrostatic balance dp/dr = -rho g then
  gives d rho/dr = -(rho / C_p) dS/dr - (g / gamma) rho^(2 - gamma)
  exp(-gamma S / C_p).  The printed exponent is +gamma S / C_p, which does not
  satisfy hydrostatic balance unless S = 0.
* The entropy gradient is evaluated on the polytrope (rho, T, dT/dr of Eq.
  "polytrop eqns"), as the text says; S_b is the polytrope's entropy at r_b
  and rho(r_b) = rho_b.
* g = GM / r^2; the radiative diffusivity kappa_r(r) is a caller function.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp


def _cp(gamma, Rgas):
    return gamma * Rgas / (gamma - 1.0)


def polytrope(r, GM, Rgas, gamma, rb, rt, rho_b, N_rho):
    """(rho, p, T) of Eq. "polytrop eqns" at radii r, with
    T_b = (Phi_t - Phi_b) / (C_p (1 - exp(-(gamma - 1) N_rho))), Phi = -GM / r,
    p_b = rho_b R T_b."""
    r = np.asarray(r, dtype=np.float64)
    cp = _cp(gamma, Rgas)
    phi_b, phi_t = -GM / rb, -GM / rt
    T_b = (phi_t - phi_b) / (cp * (1.0 - np.exp(-(gamma - 1.0) * N_rho)))
    p_b = rho_b * Rgas * T_b
    z = 1.0 - (-GM / r - phi_b) / (cp * T_b)
    return rho_b * z ** (1.0 / (gamma - 1.0)), p_b * z ** (gamma / (gamma - 1.0)), T_b * z


def entropy(rho, p, gamma, Rgas):
    """Specific entropy S = C_p ln(p^(1/gamma) / rho) (Eq. "entropy")."""
    return _cp(gamma, Rgas) * np.log(np.asarray(p) ** (1.0 / gamma) / np.asarray(rho))


def entropy_gradient(r, GM, Rgas, gamma, rb, rt, rho_b, N_rho, L, kappa, kr):
    """dS/dr from the flux condition on the polytrope (readings above):
    -(L / (4 pi r^2) + kappa_r rho C_p dT/dr) / (kappa rho T)."""
    r = np.asarray(r, dtype=np.float64)
    cp = _cp(gamma, Rgas)
    rho, _, T = polytrope(r, GM, Rgas, gamma, rb, rt, rho_b, N_rho)
    # dT/dr of the polytrope: T_b dz/dr with dz/dr = -(dPhi/dr) / (C_p T_b)
    dTdr = -GM / (cp * r * r)
    q = L / (4.0 * np.pi * r * r)
    return -(q + kr(r) * rho * cp * dTdr) / (kappa * rho * T)


def flux_balanced(r_eval, GM, Rgas, gamma, rb, rt, rho_b, N_rho, L, kappa, kr, rtol=1e-13):
    """(rho, p, T, S) of the flux-balanced profile at radii r_eval in [rb, rt]:
    S and rho integrated together from (S_b, rho_b) at r_b with scipy's
    DOP853 at relative tolerance rtol."""
    r_eval = np.asarray(r_eval, dtype=np.float64)
    cp = _cp(gamma, Rgas)
    rho0_b, p0_b, _ = polytrope(rb, GM, Rgas, gamma, rb, rt, rho_b, N_rho)
    S_b = float(entropy(rho0_b, p0_b, gamma, Rgas))

    def rhs(r, y):
        S, rho = y
        dS = float(entropy_gradient(r, GM, Rgas, gamma, rb, rt, rho_b, N_rho, L, kappa, kr))
        g = GM / (r * r)
        drho = -(rho / cp) * dS - (g / gamma) * rho ** (2.0 - gamma) * np.exp(-gamma * S / cp)
        return [dS, drho]

    ru, inv = np.unique(r_eval, return_inverse=True)
    if ru[0] < rb or ru[-1] > rt:
        raise ValueError("radii outside [rb, rt]")
    sol = solve_ivp(rhs, (rb, rt), [S_b, rho_b], method="DOP853", rtol=rtol,
                    atol=[1e-14 * cp, 1e-16 * rho_b], t_eval=ru)
    if not sol.success:
        raise RuntimeError(sol.message)
    S = sol.y[0][inv].reshape(r_eval.shape)
    rho = sol.y[1][inv].reshape(r_eval.shape)
    p = rho ** gamma * np.exp(gamma * S / cp)
    return rho, p, p / (rho * Rgas), S
