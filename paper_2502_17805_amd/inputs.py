"""Seeded synthetic inputs for the shell runs (no spectral-difference arithmetic).

This module only draws random numbers and evaluates closed-form initial data at
positions it is given; it is shared by the product driver, the benchmark and
the tests so that the oracle and the HIP library see identical inputs.

* Background: the adiabatic polytrope in hydrostatic balance of the paper's
  section "Initial Conditions" (profiles of p, rho, T in terms of the potential
  Phi = -GM/r, with T_b fixed by the number of density scale heights N_rho so
  that rho_t / rho_b = exp(-N_rho)).
* Perturbations (synthetic, seeded): velocity 1e-4 * U(-1,1) per component per
  point times sin(pi (r - r_b)/(r_t - r_b)); a dipole seed field
  1e-3 (r_b/r)^3 (3 (z.r) r - z); psi = 0.
* Run parameters: nondimensional units GM = R = 1, gamma = 5/3; kinematic
  viscosity, thermal and magnetic diffusivities from seeded Prandtl and magnetic
  Prandtl numbers in [0.5, 4].
* Solar benchmark parameters: the dimensional parameter table of the section
  "Benchmark Problem Definition" expressed in the same units (length r_t,
  velocity sqrt(GM / r_t), density rho_b, R = 1); the profile of the initial
  state is then computed by the library (the flux-balanced background).
"""
from __future__ import annotations

import dataclasses

import numpy as np

GAMMA = 5.0 / 3.0


@dataclasses.dataclass
class Background:
    """Polytrope of the section "Initial Conditions" in nondimensional units."""
    N_rho: float
    rb: float = 0.70
    rt: float = 0.98
    GM: float = 1.0
    Rgas: float = 1.0
    gamma: float = GAMMA
    rho_b: float = 1.0

    @property
    def cp(self):
        return self.gamma * self.Rgas / (self.gamma - 1.0)

    @property
    def T_b(self):
        phi_b, phi_t = -self.GM / self.rb, -self.GM / self.rt
        return (phi_t - phi_b) / (self.cp * (1.0 - np.exp(-(self.gamma - 1.0) * self.N_rho)))

    @property
    def p_b(self):
        return self.rho_b * self.Rgas * self.T_b

    def profile(self, r):
        """(rho, p, T) at radius r."""
        r = np.asarray(r, dtype=np.float64)
        z = 1.0 - (-self.GM / r + self.GM / self.rb) / (self.cp * self.T_b)
        g1 = self.gamma - 1.0
        return (self.rho_b * z ** (1.0 / g1), self.p_b * z ** (self.gamma / g1), self.T_b * z)

    @property
    def T_t(self):
        return float(self.profile(self.rt)[2])


def radius(x: np.ndarray) -> np.ndarray:
    """|x| over axis 1, squares summed in ascending order so that positions
    related by a signed permutation of the axes get bit-identical radii."""
    return np.sqrt(np.sort(x * x, axis=1).sum(axis=1))


def shell_state(x_sp: np.ndarray, bg: Background, seed: int, u_amp=1e-4, b_amp=1e-3, profile=None) -> np.ndarray:
    """Conserved state Q [E][9][N^3] (rho, rho u, E, B, psi) at positions x_sp [E][3][N^3];
    profile(r) -> (rho, p, ...) replaces the polytrope of bg when given."""
    x = np.asarray(x_sp, dtype=np.float64)
    E, _, n3 = x.shape
    r = radius(x)
    rho, p = (profile or bg.profile)(r)[:2]
    rng = np.random.Generator(np.random.PCG64(seed))
    u = u_amp * rng.uniform(-1.0, 1.0, size=(E, 3, n3))
    u *= np.sin(np.pi * (r - bg.rb) / (bg.rt - bg.rb))[:, None, :]
    rhat = x / r[:, None, :]
    cz = rhat[:, 2, :]
    B = b_amp * (bg.rb / r)[:, None, :] ** 3 * (3.0 * cz[:, None, :] * rhat - np.array([0.0, 0.0, 1.0])[None, :, None])
    Q = np.empty((E, 9, n3))
    Q[:, 0] = rho
    Q[:, 1:4] = rho[:, None, :] * u
    Q[:, 4] = p / (bg.gamma - 1.0) + 0.5 * rho * (u * u).sum(axis=1) + 0.5 * (B * B).sum(axis=1)
    Q[:, 5:8] = B
    Q[:, 8] = 0.0
    return Q


def smooth_random_state(x_sp: np.ndarray, seed: int, gamma=GAMMA) -> np.ndarray:
    """A smooth, far-from-equilibrium state (random low Fourier modes)."""
    x = np.asarray(x_sp, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    E, _, n3 = x.shape

    def field(amp):
        k = rng.integers(-2, 3, size=(3, 3)).astype(float)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = rng.uniform(-1, 1, size=3)
        s = np.zeros((E, n3))
        for m in range(3):
            s += a[m] * np.sin(np.pi * np.einsum("d,edq->eq", k[m], x) + ph[m])
        return amp * s

    rho = 1.0 + field(0.2)
    u = np.stack([field(0.3) for _ in range(3)], axis=1)
    p = 1.0 + field(0.2)
    B = np.stack([field(0.4) for _ in range(3)], axis=1)
    psi = field(0.05)
    Q = np.empty((E, 9, n3))
    Q[:, 0] = rho
    Q[:, 1:4] = rho[:, None, :] * u
    Q[:, 4] = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(axis=1) + 0.5 * (B * B).sum(axis=1) + 0.5 * psi * psi
    Q[:, 5:8] = B
    Q[:, 8] = psi
    return Q


def run_params(seed: int, bg: Background, nu=2.0e-5, Omega=0.12, q_inner=1.0e-4) -> dict:
    """Physical parameters of one synthetic dynamo run (seeded Pr, Pm in [0.5, 4])."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    Pr, Pm = rng.uniform(0.5, 4.0, size=2)
    return dict(gamma=bg.gamma, Rgas=bg.Rgas, GM=bg.GM, Omega=Omega, nu=nu, kappa=nu / Pr,
                eta=nu / Pm, kr_scale=0.0, kr_c0=0.0, kr_c1=0.0, kr_c2=0.0, kr_omega_per_r=0.0,
                powell=1, wall_kind=(0, 0), wall_mag=(0, 1), wall_th=(0, 1),
                q_wall=(q_inner, 0.0), T_wall=(bg.T_b, bg.T_t))


def glm_speed(Q: np.ndarray, gamma=GAMMA) -> float:
    """c_h = max over points of |u| + sqrt(a^2 + b^2) (largest signal speed of Q)."""
    rho = Q[:, 0]
    u2 = (Q[:, 1:4] ** 2).sum(axis=1) / rho ** 2
    b2 = (Q[:, 5:8] ** 2).sum(axis=1)
    p = (gamma - 1.0) * (Q[:, 4] - 0.5 * rho * u2 - 0.5 * b2 - 0.5 * Q[:, 8] ** 2)
    return float(np.max(np.sqrt(u2) + np.sqrt(gamma * p / rho + b2 / rho)))


def time_step(Q: np.ndarray, Sj_sp: np.ndarray, c_h: float, cfl: float, gamma=GAMMA) -> float:
    """dt = cfl / max over points of lambda * sum_d |S^d / J| (lambda incl. c_h);
    Sj_sp [E][3][3][N^3] holds S^d / |J| at the solution points."""
    rho = Q[:, 0]
    u2 = (Q[:, 1:4] ** 2).sum(axis=1) / rho ** 2
    b2 = (Q[:, 5:8] ** 2).sum(axis=1)
    p = (gamma - 1.0) * (Q[:, 4] - 0.5 * rho * u2 - 0.5 * b2 - 0.5 * Q[:, 8] ** 2)
    lam = np.maximum(np.sqrt(u2) + np.sqrt(gamma * p / rho + b2 / rho), c_h)
    inv_h = np.sqrt((Sj_sp ** 2).sum(axis=2)).sum(axis=1)
    return float(cfl / np.max(lam * inv_h))


# Dimensional parameters of the solar benchmark (section "Benchmark Problem
# Definition", table "Solar Benchmark Parameters", cgs units) and the
# coefficients of its radiative diffusivity kappa_r = lambda (c0 + c1 w +
# c2 w^2), w = r 1e-10 / cm.
SOLAR_TABLE = dict(r_t=6.61e10, r_b=4.87e10, M=1.98891e33, Omega=8.1e-5, rho=0.21, G=6.67e-8, R=1.4e8,
                   kappa=6.0e13, nu=6.0e13, gamma=5.0 / 3.0, eta=1.2e13, L=3.846e36, Cp=3.5e8,
                   c0=1.5600975e8, c1=-4.5631718e7, c2=3.3370368e6)


def solar_benchmark(N_rho: float = 3.0) -> dict:
    """The solar benchmark in the units of this module: length r_t, velocity
    v0 = sqrt(G M / r_t), time r_t / v0, density rho_b (the table's density),
    gas constant 1 (C_p / R = 2.5 as in the table, i.e. gamma = 5/3);
    diffusivities in units of r_t v0, the luminosity in rho_b v0^3 r_t^2.
    N_rho = 3 is the first benchmark, 4 the second.  The prefactor lambda of
    kappa_r is not given in the paper; it is set so that the polytrope's
    radiative flux kappa_r rho C_p |dT/dr| carries the whole luminosity at
    r_b: lambda = L / (4 pi rho_b G M c(r_b)), c = c0 + c1 w + c2 w^2 in units
    of r_t v0 (with dT/dr = -G M / (C_p r^2) it is independent of r_b).
    Returns the background parameters (for the library's background profile)
    and the run's transport coefficients, rotation and bottom heat flux."""
    t = SOLAR_TABLE
    GMc = t["G"] * t["M"]
    v0 = np.sqrt(GMc / t["r_t"])
    t0 = t["r_t"] / v0
    D = t["r_t"] * v0
    L = t["L"] / (t["rho"] * v0 ** 3 * t["r_t"] ** 2)
    rb = t["r_b"] / t["r_t"]
    w_per_r = t["r_t"] * 1e-10
    c = (t["c0"] / D, t["c1"] / D, t["c2"] / D)
    wb = rb * w_per_r
    lam = L / (4.0 * np.pi * 1.0 * 1.0 * (c[0] + c[1] * wb + c[2] * wb * wb))
    return dict(GM=1.0, Rgas=1.0, gamma=t["gamma"], rb=rb, rt=1.0, rho_b=1.0, N_rho=float(N_rho), L=L,
                kappa=t["kappa"] / D, nu=t["nu"] / D, eta=t["eta"] / D, Omega=t["Omega"] * t0,
                kr_scale=lam, kr_c0=c[0], kr_c1=c[1], kr_c2=c[2], kr_omega_per_r=w_per_r,
                q_inner=L / (4.0 * np.pi * rb * rb))


def solar_run_params(sb: dict, T_top: float) -> dict:
    """Run parameters of the solar benchmark: stress-free impenetrable walls,
    perfectly conducting bottom with the heat flux L / (4 pi r_b^2), perfectly
    radial field at the top held at temperature T_top (section "Problem
    Formulation and Boundary Conditions"), Powell terms on."""
    return dict(gamma=sb["gamma"], Rgas=sb["Rgas"], GM=sb["GM"], Omega=sb["Omega"], nu=sb["nu"],
                kappa=sb["kappa"], eta=sb["eta"], kr_scale=sb["kr_scale"], kr_c0=sb["kr_c0"],
                kr_c1=sb["kr_c1"], kr_c2=sb["kr_c2"], kr_omega_per_r=sb["kr_omega_per_r"], powell=1,
                wall_kind=(0, 0), wall_mag=(0, 1), wall_th=(0, 1), q_wall=(sb["q_inner"], 0.0),
                T_wall=(0.0, T_top))
