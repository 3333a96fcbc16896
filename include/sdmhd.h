/*
 * sdmhd.h -- C ABI of the MI355X (gfx950) spectral-difference GLM-MHD library.
 *
 * The library advances the compressible, viscous, resistive MHD equations
 * with a generalised-Lagrange-multiplier cleaning field psi (9 conserved
 * variables Q = rho, rho u, E, B, psi; paper arXiv 2502.17805, Sec. "MHD
 * Governing Equations", Eq. "General Form1") on hexahedral elements of a
 * mapped cubed-sphere shell (Sec. "Meshing") with the spectral-difference
 * method of Sec. "Spectral Difference Method" and the SSPRK(5,3) integrator
 * named there.  Device work is hand-written HIP; every pointer marked
 * "device" must be device memory of the context's GPU, allocated and owned
 * by the caller (the library never frees it and allocates no device memory
 * except its static constant tables, the static trace scratch of
 * sdm_ssprk53_step_noalloc and, for a mixed-arithmetic context, the FP32
 * geometry copies sdm_mesh_bind makes).  Calls that take a stream only
 * enqueue work on it; results are valid after the stream is synchronised.
 *
 * Layouts (all row-major, last index fastest):
 *   N      = p + 1 solution points per direction; N3 = N^3; NF = (N+1) N^2
 *   point  (a, b, c) -> a + N b + N^2 c   (a along xi, b along eta, c along zeta)
 *   Q, R   [E][9][N3]   variable order rho, rho u_x, rho u_y, rho u_z, E,
 *                       B_x, B_y, B_z, psi (FP64)
 *   x_sp   [E][3][N3]   physical solution-point coordinates (FP64)
 *   detJ   [E][N3]      Jacobian determinant at the solution points (FP64)
 *   Sj_sp  [E][3 d][3 x][N3]  S^d_x / |J| at the solution points: the
 *                       chain-rule factors d xi_d / d x (FP64)
 *   S_fp   [E][3 d][3 x][NF]  metric vector S^d = |J| grad(xi_d) at the
 *                       family-d flux points; family d stores its flux-point
 *                       index along axis d (d = 0: f + (N+1)(b + N c);
 *                       d = 1: a + N (f + (N+1) c); d = 2: a + N (b + N f))
 *   nbr    [E][6]       int32 per element face (0/1: xi = 0/1, 2/3: eta,
 *                       4/5: zeta).  Interior: (e' << 6) | (f' << 3) | o,
 *                       neighbour element e', its face f', orientation o.
 *                       Boundary: -(1 + group + 4 * bface), group 0 = zeta=0
 *                       wall (inner sphere), 1 = zeta=1 wall (outer sphere),
 *                       2 = other (always Dirichlet), 3 = import face (the
 *                       neighbour belongs to another partition of the
 *                       mesh: its trace and viscous flux come from the
 *                       import buffers of sdm_params); bface numbers the
 *                       boundary faces in (element, face) order.
 *   face-local point (a, b): the two axes other than the face normal, in
 *   increasing axis order; orientation o = 4 swap + 2 flip_b + flip_a maps
 *   it to the neighbour's point: (p, q) = swap ? (b, a) : (a, b);
 *   a' = flip_a ? N-1-p : p; b' = flip_b ? N-1-q : q.
 *   n_face [E][6][3][N^2]  outward face normal at every face point: the
 *                       symmetric (S_own - S_neighbour)/2 of the two sides'
 *                       outward metric vectors (exact negatives across the
 *                       face); S_own on boundary faces (FP64)
 *   ghost  [n_bfaces][9][N^2]  outside state on Dirichlet faces (device).
 *   import_q [n_bfaces][9][N^2], import_v [n_bfaces][7][N^2]  on import faces:
 *                       the neighbour's Q trace and its viscous normal flux
 *                       (components 1..7 of the BR1 viscous flux through the
 *                       symmetric normal, as the neighbour's own workspace
 *                       holds them), already in this face's point order, in
 *                       the residual arithmetic type (FP64, or FP32 for a
 *                       mixed context); rows of other faces are not read.
 *
 * Errors: every call returns an sdm_status; nothing is thrown across the
 * ABI.  SDM_EINVAL: bad sizes, NULL pointers, unsupported p; SDM_EHIP: a HIP
 * runtime error (text in sdm_last_error()).  NaN/Inf in the state is not an
 * API error: sdm_diagnostics reports it.
 */
#ifndef SDMHD_H
#define SDMHD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SDM_OK = 0,
  SDM_EINVAL = -1,
  SDM_ENOMEM = -2,
  SDM_EHIP = -3,
  SDM_ESTATE = -4,
  SDM_EUNSUPPORTED = -5
} sdm_status;

typedef struct sdm_ctx sdm_ctx;

/* Message for the last non-OK status returned on this thread. */
const char* sdm_last_error(void);

/* Library version string. */
const char* sdm_version(void);

/* ---------------- host-side mesh construction (no GPU needed) ---------- */

/* Element and boundary-face counts of the cubed-sphere shell with Nz x Nz
 * elements per cube face and Nr radial layers (Sec. "Meshing":
 * N_cells = 6 N_r N_z^2).  n_bfaces = 12 Nz^2. */
sdm_status sdm_shell_sizes(int Nz, int Nr, int64_t* n_elem, int64_t* n_bfaces);

/* Build the shell of degree p between radii rb < rt into caller HOST
 * buffers sized from sdm_shell_sizes (layouts above); Sj_sp receives the
 * chain-rule factors S^d/|J| at the solution points.  Element index
 * e = ((P Nr + k) Nz + j) Nz + i for cube patch P (+x,+y,-x,-y,+z,-z),
 * radial layer k (inner to outer), and equiangular indices (i, j).
 * The element map is the degree-N isoparametric interpolant of the exact
 * shell through the (N+1)^3 flux-point nodes; metrics use the invariant
 * curl form (paper, Sec. "Spectral Difference Method": transfinite map P,
 * Jacobi matrix J, transformed system Eq. "G.E. comp").  Uses all host
 * threads (OpenMP). */
sdm_status sdm_shell_build(int Nz, int Nr, int p, double rb, double rt, double* x_sp,
                           double* detJ, double* S_fp, double* Sj_sp, int32_t* nbr,
                           double* n_face);

/* The same for an nx x ny x nz box [0,Lx]x[0,Ly]x[0,Lz] (element index
 * e = (k ny + j) nx + i), periodic in direction d if bit d of `periodic` is
 * set (needs >= 3 elements there), node positions displaced by the smooth
 * periodic warp  w sin(2 pi x/Lx) sin(2 pi y/Ly) sin(2 pi z/Lz) (L_d each).
 * Boundary faces at z = 0 / z = Lz are groups 0 / 1, others group 2.
 * n_bfaces is returned through *n_bfaces (may be NULL). */
sdm_status sdm_box_sizes(int nx, int ny, int nz, int periodic, int64_t* n_elem,
                         int64_t* n_bfaces);
sdm_status sdm_box_build(int nx, int ny, int nz, double Lx, double Ly, double Lz,
                         int periodic, double warp, int p, double* x_sp, double* detJ,
                         double* S_fp, double* Sj_sp, int32_t* nbr, double* n_face);

/* 1-D tables of the method for N = p+1 (host): solution points xs[N],
 * flux points xf[N+1], interpolation I[(N+1)][N] (SP basis at FPs),
 * derivative D[N][N+1] (FP basis derivative at SPs), weights W[N]. */
sdm_status sdm_tables(int p, double* xs, double* xf, double* I, double* D, double* W);

/* ---------------- device context ------------------------------------- */

/* A context: the spectral-difference operators of degree p on one device
 * (Sec. "Spectral Difference Method": N = p + 1 Chebyshev-Gauss solution
 * points and N + 1 Legendre-Gauss flux points with both end points per
 * direction, the Lagrange bases h_i on the former and l_i on the latter).
 * arith: 0 = FP64 throughout; 1 = mixed (FP32 residual arithmetic, FP64
 * state, RK accumulation and diagnostics; the residual reads an FP32 copy of
 * the geometry, see sdm_mesh_bind).  p in 1..6 (the FP64
 * volume kernel of p = 7 would exceed the 160 KB of LDS).  Uploads the 1-D
 * tables to the device's constant memory once per device; *out is owned by
 * the caller and released with sdm_destroy.  SDM_EUNSUPPORTED for p outside
 * 1..6, SDM_EINVAL for a bad arith or device. */
sdm_status sdm_create(int device, int p, int arith, sdm_ctx** out);
sdm_status sdm_destroy(sdm_ctx* ctx);

/* Borrowed DEVICE arrays of one mesh (layouts above; Sec. "Meshing": the
 * cubed-sphere shell of hexahedra, and Sec. "Spectral Difference Method":
 * the Jacobian |J| and metric terms of the element map, with which the
 * equations are solved in the transformed form of Eq. "G.E. comp"); they
 * must outlive every call that uses them.  sdm_mesh_bind copies the
 * neighbour table to the host once to check every code decodes into range
 * (SDM_EINVAL otherwise) and stores the pointers.  With arith 1 it also
 * allocates, on the context's device, FP32 copies (rounded to nearest) of
 * x_sp, detJ, S_fp, Sj_sp and n_face, 22.9 KB per element at p = 5, which the
 * FP32 residual kernels read instead (the values they would round on use, at
 * half the bytes); the context owns them until sdm_destroy or the next bind,
 * so rebind after changing those arrays.  Synchronous, on the null stream
 * (writes to the arrays on other non-blocking streams must be complete
 * first); SDM_EHIP if the allocation fails. */
typedef struct {
  int64_t n_elem;
  int64_t n_bfaces;
  const double* x_sp;
  const double* detJ;
  const double* S_fp;
  const double* Sj_sp;
  const int32_t* nbr;
  const double* n_face;
} sdm_mesh;
sdm_status sdm_mesh_bind(sdm_ctx* ctx, const sdm_mesh* mesh);

/* Physical and boundary parameters (nondimensional).
 *  mu = rho nu, lambda = -2/3 mu (Eq. "ssTensor"); heat flux
 *  q = -kappa rho T grad S - kappa_r rho c_p grad T (Eq. "qFlux") with
 *  kappa_r(r) = kr_scale (kr_c0 + kr_c1 w + kr_c2 w^2), w = r kr_omega_per_r;
 *  GLM speed c_h and damping a (source -a psi); powell != 0 enables the
 *  div-B source terms of Eq. "M".  Walls (group 0 inner, 1 outer):
 *  wall_kind 0 = physical wall, 1 = Dirichlet ghost buffer; wall_mag 0 =
 *  perfectly conducting, 1 = perfectly radial field; wall_th 0 = prescribed
 *  outward-radial heat-flux density q_wall, 1 = fixed temperature T_wall
 *  (Sec. "Problem Formulation and Boundary Conditions"). */
typedef struct {
  double gamma, Rgas, GM, Omega, nu, kappa, eta;
  double kr_scale, kr_c0, kr_c1, kr_c2, kr_omega_per_r;
  double c_h, glm_a;
  int32_t powell;
  int32_t wall_kind[2];
  int32_t wall_mag[2];
  int32_t wall_th[2];
  double q_wall[2];
  double T_wall[2];
  const double* ghost;    /* device [n_bfaces][9][N^2] or NULL */
  const void* import_q;   /* device [n_bfaces][9][N^2] or NULL (needed with import faces) */
  const void* import_v;   /* device [n_bfaces][7][N^2] or NULL (needed with import faces) */
} sdm_params;

/* Bytes of scratch (face traces of Q and of the viscous normal flux, the
 * data the common solution and common viscous flux of Sec. "Spectral
 * Difference Method" exchange between face neighbours, and the partial
 * residual) one call needs; the caller allocates it (device, 256-byte
 * aligned) and passes it as `ws`. */
sdm_status sdm_workspace_size(const sdm_ctx* ctx, size_t* bytes);

/* Device addresses, inside workspace `ws`, of the face traces a partition
 * sends to its neighbours (the halo of a mesh split over several GPUs; the
 * receiving side passes them, orientation-mapped to its face points, as
 * import_q / import_v): q_traces [E][6][9][N^2] = Q at the six faces of
 * every element, of the state the next stage takes (written by each stage
 * and by sdm_residual for its Q); v_traces [E][6][7][N^2] = the element's
 * own viscous normal flux at its faces from the last residual evaluation.
 * Residual arithmetic type.  Views only: nothing is copied. */
sdm_status sdm_workspace_traces(const sdm_ctx* ctx, void* ws, void** q_traces, void** v_traces);

/* R = dQ/dt at the solution points (device Q, R, layout [E][9][N3]): the
 * spectral-difference residual of Sec. "Spectral Difference Method" (the
 * procedure paragraph: Q and its gradient reconstructed at the flux points,
 * common solution and common fluxes on the element faces, the flux
 * divergence at the solution points) for the equations of Sec. "MHD
 * Governing Equations" in the transformed form of Eq. "G.E. comp", i.e.
 * R = -(div of the flux)/|J| + M with the sources of Eq. "M"; the boundary
 * treatment of Sec. "Problem Formulation and Boundary Conditions".  `ws` is
 * the caller's workspace of sdm_workspace_size bytes. */
sdm_status sdm_residual(sdm_ctx* ctx, const sdm_params* prm, const double* Q, double* R,
                        void* ws, void* stream);

/* One explicit Runge-Kutta stage in Shu-Osher form (Sec. "Spectral
 * Difference Method": the time integrator is a strong-stability-preserving
 * Runge-Kutta scheme, whose stages are convex combinations of forward-Euler
 * steps), fused into the last pass of the residual:
 *   regs[out] = sum_k alpha[k] regs[in[k]] + beta dt R(regs[cur])
 * regs: n_regs device state buffers ([E][9][N3] FP64); out may equal cur or
 * an input (each element reads before it writes).  The SSPRK(5,3) step of
 * the paper is five such stages.  Every stage leaves the face traces of
 * regs[out] in `ws`; traces_valid != 0 tells the next call that `ws` holds
 * the traces of its regs[cur] (it then skips recomputing them); pass 0
 * whenever the state was changed by anything else. */
typedef struct {
  int32_t n_in;
  int32_t in_idx[4];
  double alpha[4];
  int32_t cur;
  int32_t out;
  double beta;
  int32_t traces_valid;
} sdm_stage;
sdm_status sdm_rk_stage(sdm_ctx* ctx, const sdm_params* prm, double* const* regs, int n_regs,
                        const sdm_stage* stage, double dt, void* ws, void* stream);

/* The SSPRK(5,3) scheme of Sec. "Spectral Difference Method" (five stages,
 * third order, optimal SSP coefficient 2.6506) as five sdm_stage records on
 * four registers: u0 in regs[0] (A), u1 in B, u2 in C, u3 and u4 in D, the
 * step's result back in A.  The Shu-Osher form of stages 4 and 5 also takes
 * the residuals of u0 and u1; they are folded into the weights of u0, u1,
 * u2 by L(u0) = (u1 - u0)/(beta10 dt), L(u1) = (u2 - u1)/(beta21 dt), which
 * holds because stages 1 and 2 are single forward-Euler steps, so every
 * stage takes one residual.  out[5] (host) receives the records (stage 1
 * has traces_valid = 0, the others 1: each takes the previous one's
 * output); c[5] (host, may be NULL) the time of each stage's input state in
 * units of dt (0, beta10, ...), for callers whose boundary data depend on
 * time.  No GPU needed. */
sdm_status sdm_ssprk53_stages(sdm_stage* out, double* c);

/* One SSPRK(5,3) step of the state in regs[0]: the five stages of
 * sdm_ssprk53_stages in order on regs[0..3] (device, [E][9][N3] FP64 each;
 * regs[1..3] are overwritten).  traces_valid != 0 declares that `ws` holds
 * the face traces of regs[0] (left there by the previous step); afterwards
 * it does.  Same errors as sdm_rk_stage. */
sdm_status sdm_ssprk53_step(sdm_ctx* ctx, const sdm_params* prm, double* const* regs, double dt,
                            int traces_valid, void* ws, void* stream);

/* sdm_ssprk53_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same five stages on regs[0..3] (device, caller-owned,
 * [E][9][N3] FP64 each; regs[1..3] are overwritten), bitwise the same
 * result, with no workspace argument.  The face traces the stages exchange
 * live in a library-owned static device array of 64 MiB per device (held
 * from the first sdm_create on that device until the process ends), so a
 * mesh may need at most 64 MiB of them: E (6 (9 + 7) N^2) x 8 bytes in FP64,
 * x 4 in FP32-mixed (2,427 elements at p = 5 in FP64, 4,854 in
 * FP32-mixed); a larger mesh returns SDM_EINVAL with the limit in the
 * message.  The first stage always recomputes the traces of regs[0] (no
 * traces_valid).  Stage and step calls, no-allocation or not, allocate
 * nothing, and this one frees nothing.  All contexts on one device share the one array:
 * calls that may overlap on one device (different streams, or other
 * threads) race and must be serialised by the caller; a call on one stream
 * after another completes is safe. */
sdm_status sdm_ssprk53_step_noalloc(sdm_ctx* ctx, const sdm_params* prm, double* const* regs, double dt,
                                    void* stream);

/* The two halves of sdm_rk_stage, for a mesh split over several GPUs: the
 * volume half (face traces of regs[cur] unless traces_valid, then every
 * element's residual except the neighbour half of the viscous flux; it
 * reads import_q and leaves this partition's viscous face fluxes in `ws`,
 * see sdm_workspace_traces) and the finish half (the neighbour half, read
 * from import_v on import faces, and the Shu-Osher update; it leaves the
 * new state's face traces in `ws`).  The volume half already forms the
 * Shu-Osher combination (FP64) with that partial residual and writes it to
 * regs[out], and the finish half subtracts beta dt times the neighbour half
 * in place.  Between the halves regs[out] is therefore not a state.  A split run exchanges the Q traces
 * before the volume half and the viscous fluxes between the halves.  Same
 * arguments as sdm_rk_stage; volume followed by finish equals sdm_rk_stage
 * bitwise. */
sdm_status sdm_rk_stage_volume(sdm_ctx* ctx, const sdm_params* prm, double* const* regs, int n_regs,
                               const sdm_stage* stage, double dt, void* ws, void* stream);
sdm_status sdm_rk_stage_finish(sdm_ctx* ctx, const sdm_params* prm, double* const* regs, int n_regs,
                               const sdm_stage* stage, double dt, void* ws, void* stream);

/* Diagnostics of state Q into DEVICE out[16] (FP64): volume, mass, total
 * energy, volume-averaged KE = (1/V) int rho|u|^2/2, E_B = (1/V) int
 * |B|^2/2 (Sec. "Results"), max|div B|, L2 norm of div B (div B from the
 * gradient of Sec. "Spectral Difference Method", the quantity the GLM
 * cleaning of Sec. "MHD Governing Equations" drives to zero), max|psi|,
 * NaN/Inf flag (1.0 if any), zeros after.  Quadrature: the weights of the
 * solution points times |J|.  Deterministic (fixed reduction order). */
sdm_status sdm_diagnostics(sdm_ctx* ctx, const sdm_params* prm, const double* Q, double* out,
                           void* ws, void* stream);

/* ---------------- batched stages of independent runs ------------------ */

/* One item of a batch: a run with its own context (bound mesh), parameters,
 * registers and workspace, and the stage it takes next. */
typedef struct {
  sdm_ctx* ctx;
  const sdm_params* prm;
  double* const* regs;
  int32_t n_regs;
  sdm_stage stage;
  double dt;
  void* ws;
} sdm_batch_item;

/* ---------------- initial background ----------------------------------- */

/* Radial profiles of the initial state (Sec. "Initial Conditions"; U = 0,
 * hydrostatic).  flux_balanced = 0: the polytrope of Eq. "polytrop eqns",
 * T_b = (Phi_t - Phi_b) / (C_p (1 - exp(-(gamma - 1) N_rho))), Phi = -GM/r,
 * p_b = rho_b Rgas T_b, C_p = gamma Rgas / (gamma - 1).  flux_balanced = 1:
 * the almost flux-balanced profile built from it: the entropy gradient that
 * makes the entropy-diffusion and radiative fluxes through the polytrope
 * carry the luminosity L outward through every layer,
 *   dS/dr = -(L / (4 pi r^2) + kappa_r rho0 C_p dT0/dr) / (kappa rho0 T0),
 * integrated from the polytrope's entropy S_b at r_b, and the hydrostatic
 * density d rho/dr = -(rho / C_p) dS/dr - (g / gamma) rho^(2 - gamma)
 * exp(-gamma S / C_p) from rho(r_b) = rho_b (Eqs. "qfluxIC", "dSdr",
 * "densityprofile", with the signs that make Eq. "qFlux" and hydrostatic
 * balance hold); then p = rho^gamma exp(gamma S / C_p), T = p / (rho Rgas).
 * kappa_r(r) = kr_scale (kr_c0 + kr_c1 w + kr_c2 w^2), w = r kr_omega_per_r.
 * Solved by classical RK4 on 2^14 uniform steps with cubic Hermite
 * interpolation between them (fourth order; host only, no GPU). */
typedef struct {
  double GM, Rgas, gamma;
  double rb, rt;
  double rho_b, N_rho;
  double L;      /* luminosity through every layer */
  double kappa;  /* thermal diffusivity (entropy diffusion) */
  double kr_scale, kr_c0, kr_c1, kr_c2, kr_omega_per_r;
  int32_t flux_balanced;
} sdm_background;

/* rho, p, T (host [n]) at the host radii r[n] in [rb, rt].  SDM_EINVAL for
 * bad parameters, a radius outside the shell, or a flux-balanced density
 * that reaches zero before r_t (no hydrostatic profile for that L). */
sdm_status sdm_background_profile(const sdm_background* bg, int64_t n, const double* r, double* rho, double* p,
                                  double* T);

/* ---------------- spherical-component diagnostics ---------------------- */

/* The paper reports the differential rotation (longitude-time average of
 * V_phi), the meridional flow (that of V_mer = sqrt(V_r^2 + V_theta^2)) and
 * the poloidal / toroidal magnetic energies (B_r^2 + B_theta^2 and B_phi^2
 * over 8 pi; 1/2 in the rationalized units of this library) (Sec.
 * "Results").  The longitude average is taken per (r, theta) bin: n_r x n_th
 * uniform bins, r in [rb, rt], theta = atan2(sqrt(x^2 + y^2), z) in [0, pi];
 * solution point x lies in bin (ir, it) = (floor((|x| - rb)/(rt - rb) n_r),
 * floor(theta/pi n_th)), clamped to the ranges.
 *
 * sdm_sph_bins (HOST, no GPU): groups the n_elem (p+1)^3 solution points of
 * a mesh (x_sp: host [n_elem][3][(p+1)^3], as built by sdm_shell_build) by
 * bin.  order (host, int32 [n_elem (p+1)^3]) receives the global SP indices
 * e (p+1)^3 + sp bin by bin, ascending within a bin; offsets (host, int64
 * [n_r n_th + 1]) the bin ranges, bin b = ir n_th + it.  SDM_EINVAL for bad
 * sizes or more than 2^31 points.
 *
 * sdm_sph_profiles (DEVICE): for state Q ([E][9][N^3] FP64) of ctx's bound
 * mesh and DEVICE copies of order / offsets (n_bins = n_r n_th), writes
 * DEVICE out[n_bins][5]: the sums over the bin's SPs of w, w V_phi, w V_mer,
 * w (B_r^2 + B_theta^2)/2 and w B_phi^2/2, w = quadrature weight x |J|
 * (divide by the first for bin averages; sum over bins and divide by the
 * volume for the energies).  On the polar axis phi_hat = (0, 1, 0).  FP64 in
 * either arithmetic; bitwise reproducible (fixed summation order).  Time
 * averages are the caller's (sum the outputs of several states). */
sdm_status sdm_sph_bins(int64_t n_elem, int p, const double* x_sp, double rb, double rt, int n_r, int n_th,
                        int32_t* order, int64_t* offsets);
sdm_status sdm_sph_profiles(sdm_ctx* ctx, const double* Q, const int32_t* order, const int64_t* offsets,
                            int n_bins, double* out, void* stream);

/* Bytes of DEVICE scratch sdm_batch_stage needs for n_items runs (the work
 * lists of the batch); 256-byte aligned. */
sdm_status sdm_batch_workspace_size(int n_items, size_t* bytes);

/* Serving (continuous batching of independent runs; not part of the paper's
 * method): advance n_items runs by one fused RK stage each (the stage of
 * sdm_rk_stage, Sec. "Spectral Difference Method").  The runs may differ in
 * mesh, degree and parameters; they must share the arithmetic and the
 * device.  The library builds a device work list per degree: the runs'
 * stage descriptors and element offsets, copied (staged through
 * library-owned pinned host memory) into batch_ws on `stream`.  Each degree
 * group then takes three launches over the concatenated elements of its
 * runs, one workgroup per element (trace pass for items without valid
 * traces, volume pass, finish pass); a pass with more than max_blocks
 * elements (0: no limit) is issued as consecutive launches of at most
 * max_blocks workgroups.  The first degree group runs on `stream`, the
 * others on library-owned streams (default priority, created once per
 * device) that start after the work-list copy and that `stream` waits for:
 * the groups overlap on the device, and work enqueued on `stream`
 * afterwards sees every run's stage done (calls from several host threads
 * take turns enqueueing on those streams).  Every run gets exactly the
 * arithmetic of sdm_rk_stage on its own: results are bitwise identical
 * alone and in any batch.  batch_ws must not be reused by another call
 * before this one's work on `stream` has been enqueued (the next call on
 * the same stream is safe). */
sdm_status sdm_batch_stage(const sdm_batch_item* items, int n_items, void* batch_ws,
                           size_t batch_ws_bytes, int max_blocks, void* stream);

/* Per-kernel timing for benchmarks.  While enabled, every launch the
 * context makes is bracketed by two HIP events recorded on the call's
 * stream.  sdm_profile_read waits for them, then returns per kernel kind
 * (0 trace pass, 1 volume pass, 2 diagnostics volume pass, 3 residual
 * finish, 4 stage finish) the summed milliseconds ms[8] and launch counts
 * count[8], and forgets the recorded launches.  Enabling again clears. */
sdm_status sdm_profile_enable(sdm_ctx* ctx, int enable);
sdm_status sdm_profile_read(sdm_ctx* ctx, double* ms, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif
