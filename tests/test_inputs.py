"""Pins of the synthetic input generator (the paper's polytropic background,
Sec. "Initial Conditions"), by the properties that define it."""
import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp


def test_polytrope_density_contrast_and_balance():
    for N_rho in (3.0, 4.0, 5.0):
        bg = inp.Background(N_rho)
        rho_b = bg.profile(bg.rb)[0]
        rho_t = bg.profile(bg.rt)[0]
        assert abs(rho_b - 1.0) < 1e-15
        assert abs(np.log(rho_b / rho_t) - N_rho) < 1e-12           # N_rho = ln(rho_b / rho_t)
        r = np.linspace(bg.rb, bg.rt, 101)[1:-1]
        h = 1e-6
        rho, p, T = bg.profile(r)
        dpdr = (bg.profile(r + h)[1] - bg.profile(r - h)[1]) / (2 * h)
        np.testing.assert_allclose(dpdr, -rho * bg.GM / r ** 2, rtol=1e-7)   # dp/dr = -rho g
        np.testing.assert_allclose(p, rho * bg.Rgas * T, rtol=1e-14)          # ideal gas
        np.testing.assert_allclose(p / rho ** bg.gamma, p[0] / rho[0] ** bg.gamma, rtol=1e-12)  # adiabatic


def test_shell_state_is_seeded_and_divergence_free_dipole():
    x = np.random.default_rng(0).uniform(0.5, 0.6, size=(4, 3, 27)) * np.sign(
        np.random.default_rng(1).standard_normal((4, 3, 27)))
    bg = inp.Background(3.0)
    a = inp.shell_state(x, bg, 5)
    b = inp.shell_state(x, bg, 5)
    c = inp.shell_state(x, bg, 6)
    np.testing.assert_array_equal(a, b)
    assert np.abs(a[:, 1:4] - c[:, 1:4]).max() > 0
    # the dipole seed field is divergence free (finite differences at one point)
    x0 = np.array([0.3, -0.5, 0.6])
    h = 1e-5

    def Bf(p):
        return inp.shell_state(p.reshape(1, 3, 1), bg, 0, u_amp=0.0)[0, 5:8, 0]
    div = sum((Bf(x0 + h * e) - Bf(x0 - h * e))[i] / (2 * h) for i, e in enumerate(np.eye(3)))
    assert abs(div) < 1e-8


def test_radius_is_permutation_symmetric():
    x = np.random.default_rng(2).standard_normal((5, 3, 8))
    r1 = inp.radius(x)
    r2 = inp.radius(x[:, [2, 0, 1]] * np.array([-1, 1, -1])[None, :, None])
    np.testing.assert_array_equal(r1, r2)


def test_solar_benchmark_units():
    """The solar table in model units: the dimensionless groups of the table
    are kept (Omega r_t / v0, nu / (r_t v0), the ratio r_b / r_t, C_p / R),
    and the kappa_r prefactor makes the polytrope's radiative flux equal to
    the luminosity's flux density at r_b."""
    t = inp.SOLAR_TABLE
    sb = inp.solar_benchmark(3.0)
    GM = t["G"] * t["M"]
    v0 = np.sqrt(GM / t["r_t"])
    assert sb["rb"] == pytest.approx(t["r_b"] / t["r_t"], rel=1e-15)
    assert sb["Omega"] == pytest.approx(t["Omega"] * t["r_t"] / v0, rel=1e-14)
    assert sb["nu"] / sb["eta"] == pytest.approx(t["nu"] / t["eta"], rel=1e-14)
    assert sb["kappa"] == pytest.approx(t["kappa"] / (t["r_t"] * v0), rel=1e-14)
    assert t["Cp"] / t["R"] == pytest.approx(sb["gamma"] / (sb["gamma"] - 1.0), rel=1e-14)
    # luminosity in units rho_b v0^3 r_t^2
    assert sb["L"] * t["rho"] * v0 ** 3 * t["r_t"] ** 2 == pytest.approx(t["L"], rel=1e-14)
    # kappa_r(r_b) rho_b C_p |dT0/dr|(r_b) = L / (4 pi r_b^2), dT0/dr = -GM / (C_p r^2)
    rb, w = sb["rb"], sb["rb"] * sb["kr_omega_per_r"]
    kr_b = sb["kr_scale"] * (sb["kr_c0"] + sb["kr_c1"] * w + sb["kr_c2"] * w * w)
    cp = sb["gamma"] / (sb["gamma"] - 1.0)
    assert kr_b * 1.0 * cp * (1.0 / (cp * rb * rb)) == pytest.approx(sb["q_inner"], rel=1e-13)
    assert sb["q_inner"] == pytest.approx(sb["L"] / (4 * np.pi * rb * rb), rel=1e-15)
    # w = r * 1e-10 / cm: at the top of the shell w = 6.61
    assert sb["kr_omega_per_r"] == pytest.approx(6.61, rel=1e-15)
