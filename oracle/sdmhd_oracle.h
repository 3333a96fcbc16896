/*
 * sdmhd_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the spectral-difference (SD)
 * residual and SSPRK(5,3) step for viscous, resistive GLM-MHD on a mapped
 * hexahedral mesh (cubed-sphere shell or box), written from the paper
 * (arXiv 2502.17805: sections "MHD Governing Equations", "Meshing",
 * "Spectral Difference Method", "Initial Conditions", "Problem Formulation
 * and Boundary Conditions", "Results").
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the HIP
 * library; the two meet only through the documented array layouts.
 *
 * What pins each part against the paper and the mathematics, not against
 * itself (tests/test_oracle_*.py):
 *   or_tables           closed-form points, textbook Legendre roots,
 *                       exactness of I, D, W on monomials, symmetry
 *   mesh builders       volume -> closed form, Jacobian positive, discrete
 *                       GCL, metric = cofactors of the Jacobian, watertight
 *                       faces with negated normals, boundary nodes on spheres
 *   point fluxes        Euler limit, GLM/magnetic terms, rotational
 *                       invariance, viscous closed forms, fast-speed limits,
 *                       Rusanov consistency and exact antisymmetry
 *   or_residual         free stream on the curved shell, polynomial
 *                       exactness on an affine box, mass and energy
 *                       conservation, heat input = q x wall area, Alfven
 *                       wave convergence at order p, viscous and resistive
 *                       decay rates, GLM divergence wave, spherical
 *                       symmetry, rotation equivariance, hydrostatic
 *                       convergence; the sources and the radiative flux by
 *                       closed forms: Coriolis turning of a uniform flow
 *                       and its inertial oscillation, the exact residual of
 *                       a linear divergent B with and without the Powell
 *                       terms, div(kappa_r rho C_p grad T) for quadratic T
 *                       with constant and radius-squared kappa_r (exact) and
 *                       radius-linear kappa_r on the shell (order p - 1);
 *                       planted sign and factor mistakes in those terms
 *                       fail these pins
 *   or_ssprk53_*        order conditions, SSP coefficient, third-order
 *                       convergence, table = independent derivation
 *   or_diagnostics      exact integrals of uniform and polynomial states,
 *                       div B of a linear field, NaN flag
 *   or_sph_profiles     poloidal + toroidal = E_B of or_diagnostics, purely
 *                       toroidal / radial / dipole fields, constant radial,
 *                       polar and azimuthal flows, bin volumes = shell
 *                       volumes of the bins
 *   wall treatments     (tests/test_oracle_walls.py) the exact equilibria
 *                       of each wall kind: a uniform field normal to
 *                       radial-field walls and tangential to conducting
 *                       ones, a uniform flow along impenetrable stress-free
 *                       walls, a uniform cleaning field at conducting walls,
 *                       a gas at the wall temperature at fixed-temperature
 *                       walls (zero residual; the other kind of wall or the
 *                       violated condition gives none); hotter / colder
 *                       walls heat / cool their own layer; the reflection
 *                       force of a flow into a wall, the cleaning field's
 *                       wall fluxes, the heat flux through a fixed-
 *                       temperature wall and the normal traction at a
 *                       stress-free wall in closed form; no resistive flux
 *                       through a conducting wall, -eta J_t x n through a
 *                       radial-field one; each with a planted mistake it
 *                       catches.  Also zero mass flux, zero tangential
 *                       stress, zero energy flux through a conducting
 *                       adiabatic wall and the prescribed heat input.
 */
#ifndef SDMHD_ORACLE_H
#define SDMHD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NMAX 8 /* max solution points per direction */

typedef struct or_mesh or_mesh;

/* Physical and boundary parameters (nondimensional).  Wall group 0 is the
 * zeta=0 boundary (inner shell radius), group 1 the zeta=1 boundary (outer
 * radius); any other boundary face is always Dirichlet (ghost buffer). */
typedef struct {
  double gamma, Rgas, GM, Omega, nu, kappa, eta;
  double kr_scale, kr_c0, kr_c1, kr_c2, kr_omega_per_r;
  double c_h, glm_a;
  int32_t powell;
  int32_t wall_kind[2]; /* 0 physical wall, 1 Dirichlet ghost buffer       */
  int32_t wall_mag[2];  /* 0 perfectly conducting, 1 perfectly radial      */
  int32_t wall_th[2];   /* 0 prescribed heat flux, 1 fixed temperature     */
  double q_wall[2];     /* outward-radial heat-flux density at the wall    */
  double T_wall[2];     /* wall temperature for fixed-temperature walls    */
} or_params;

/* 1-D tables: xs[N], xf[N+1], I[(N+1)*N] (row f), D[N*(N+1)] (row i),
 * W[N].  Returns 0 on success. */
int or_tables(int N, double* xs, double* xf, double* I, double* D, double* W);

/* Mesh construction.  Shell: 6 patches x Nz x Nz x Nr elements, element
 * index e = ((P*Nr + k)*Nz + j)*Nz + i.  Box: nx*ny*nz elements of a
 * (possibly warped) box, e = (k*ny + j)*nx + i; periodic bit d of
 * `periodic` makes direction d periodic (at least 3 elements there). */
or_mesh* or_shell_new(int N, int Nz, int Nr, double rb, double rt);
or_mesh* or_box_new(int N, int nx, int ny, int nz, double Lx, double Ly,
                    double Lz, int periodic, double warp);
void or_mesh_free(or_mesh* m);

/* Sizes: [0]=E, [1]=unique faces, [2]=boundary faces, [3]=N */
void or_mesh_sizes(const or_mesh* m, int64_t* out4);

/* Copy a named mesh array into `out` (caller sized).  Names:
 *  "x_sp"   [E][3][N^3]          "detJ_sp" [E][N^3]
 *  "S_sp"   [E][3 d][3 x][N^3]   "S_fp"    [E][3 d][3 x][(N+1)N^2]
 *  "faces"  [F][5] int32 (eL,fL,eR,fR,orient), boundary: eR=-1-group,
 *           fR = boundary-face index
 *  "x_bfp"  [NB][3][N^2] physical coordinates of boundary-face points
 *  "W3detJ" [E][N^3]  quadrature weight * detJ
 * Returns 0, or -1 for an unknown name. */
int or_mesh_get(const or_mesh* m, const char* name, void* out);

/* R = dQ/dt at the solution points for state Q ([E][9][N^3]).  `ghost`
 * ([NB][9][N^2], may be NULL when no Dirichlet face exists) gives the
 * outside state on Dirichlet faces.  `term_scale` (9 doubles, may be NULL)
 * receives, per variable, max over points of the round-off scale
 * sum_f |D_if| A(f) / |detJ| + |source|, where A(f) is |flux| at interior
 * flux points and the summed magnitude of the common-flux inputs on faces.  `divB` ([E][N^3], may be NULL) receives div B at the SPs.
 * Returns 0, or -1 if a Dirichlet face is met with ghost == NULL. */
int or_residual(const or_mesh* m, const or_params* p, const double* Q,
                const double* ghost, double* R, double* term_scale,
                double* divB);

/* Shu-Osher coefficients of the SSPRK(5,3) scheme: alpha[6*6], beta[6*6]
 * (row i = stage i, 1..5), c[5] stage times. */
void or_ssprk53_table(double* alpha, double* beta, double* c);

/* One SSPRK(5,3) step in place (static ghost data). */
int or_ssprk53_step(const or_mesh* m, const or_params* p, double* Q,
                    const double* ghost, double dt);

/* One stage in Shu-Osher form: out = sum_k a[k]*U[k] + dt*sum_k b[k]*L[k]
 * for n terms (plain array arithmetic, used by the Python driver). */
void or_combine(int64_t n_dof, int nterm, const double* const* U,
                const double* a, const double* const* L, const double* b,
                double dt, double* out);

/* Diagnostics: out[16] = {volume, mass, total energy, KE density, E_B
 * density, max|divB|, L2(divB), max|psi|, nan flag, 0...}. */
int or_diagnostics(const or_mesh* m, const or_params* p, const double* Q,
                   const double* ghost, double* out);

/* Spherical-component diagnostics (Sec. "Results"): per (r, theta) bin of
 * n_r x n_th uniform bins (r in [rb, rt], theta in [0, pi]) the sums over
 * the SPs in the bin of w, w V_phi, w V_mer, w (B_r^2 + B_theta^2)/2 and
 * w B_phi^2/2 (w = quadrature weight x |J|) into out[n_r][n_th][5].
 * Returns 0, or -1 for bad bin counts. */
int or_sph_profiles(const or_mesh* m, const double* Q, double rb, double rt, int n_r, int n_th,
                    double* out);

/* Pointwise functions: inviscid and viscous flux through n for state q and
 * gradient G[v*3+j]; Rusanov common flux; fast speed along the unit nh;
 * total wall flux of wall group 0/1. */
void or_point_flux(const double* q, const double* G, double kr, const double* n,
                   const or_params* p, double* Finv, double* Fvis);
void or_point_rusanov(const double* qL, const double* qR, const double* n,
                      const or_params* p, double* F);
double or_point_cf(const double* q, const double* nh, const or_params* p);
void or_point_wall_flux(const double* q, const double* G, double kr,
                        const double* n, int group, const or_params* p, double* F);

/* Number of OpenMP threads the oracle uses (1 if built without OpenMP). */
int or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
