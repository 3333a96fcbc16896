// sdm_physics.hpp -- pointwise GLM-MHD physics for the gfx950 kernels
// (paper arXiv 2502.17805, Sec. "MHD Governing Equations" and Sec. "Problem
// Formulation and Boundary Conditions").  Templated on the arithmetic type T
// (double, or float for the mixed-precision residual).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdm {

// Physical parameters as seen by the kernels (converted to T).
template <typename T>
struct Phys {
  T gm1;       // gamma - 1
  T gamma;
  T Rgas;
  T cp;        // gamma R / (gamma - 1)
  T inv_R, inv_gamma, inv_gm1;
  T GM, Omega, nu, kappa, eta;
  T kr_scale, kr_c0, kr_c1, kr_c2, kr_w;
  T c_h, glm_a;
  T q_wall[2], T_wall[2];
  int32_t powell;
  int32_t wall_kind[2], wall_mag[2], wall_th[2];
};

// 1/x: the hardware reciprocal refined by Newton steps (FP64: two, from
// its 2^-23 start to within an ulp of the rounded quotient; FP32: the
// instruction is already within 1 ulp).  Shorter dependency chain than the
// full IEEE division sequence; differs from it only in the last bit.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// sqrt(x) for x >= 0 (FP64: the hardware reciprocal square root y, one
// coupled Newton step on g = x y and h = y / 2, then one correction of g
// by h (x - g^2): within an ulp of the rounded root, against the two
// corrections and the range scaling of the IEEE sequence.  Arguments below
// 1e-290, where the scaling would matter, give 0; negative arguments and NaN
// give NaN.  FP32: the hardware square root, within 1 ulp.)
__device__ __forceinline__ double sqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  return x >= 1e-290 ? g : (x >= 0.0 ? 0.0 : g);
}
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// value of a two-wall parameter for wall group g (a select, so the
// parameter block stays in registers)
template <typename X>
__device__ __forceinline__ X wsel(int g, const X (&a)[2]) {
  return g == 0 ? a[0] : a[1];
}

// variables: 0 rho, 1-3 rho u, 4 E, 5-7 B, 8 psi ; gradients G[v*3 + j]

template <typename T>
__device__ __forceinline__ T pressure(const T* q, const Phys<T>& P) {
  const T ir = recip(q[0]);
  const T m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const T b2 = q[5] * q[5] + q[6] * q[6] + q[7] * q[7];
  return P.gm1 * (q[4] - T(0.5) * m2 * ir - T(0.5) * b2 - T(0.5) * q[8] * q[8]);
}

// Inviscid flux through the (unnormalised) direction n (Eq. "invF"; the
// GLM energy term is c_h psi B.n, e = E - psi^2/2).  Every term is linear in
// n, so F(-n) = -F(n) exactly.
template <typename T>
__device__ __forceinline__ void flux_inviscid(const T* q, const T n[3], const Phys<T>& P, T F[9]) {
  const T ir = recip(q[0]);
  const T u0 = q[1] * ir, u1 = q[2] * ir, u2 = q[3] * ir;
  const T b2 = q[5] * q[5] + q[6] * q[6] + q[7] * q[7];
  const T pm = T(0.5) * b2;
  const T p = P.gm1 * (q[4] - T(0.5) * (q[1] * u0 + q[2] * u1 + q[3] * u2) - pm - T(0.5) * q[8] * q[8]);
  const T un = u0 * n[0] + u1 * n[1] + u2 * n[2];
  const T Bn = q[5] * n[0] + q[6] * n[1] + q[7] * n[2];
  const T uB = u0 * q[5] + u1 * q[6] + u2 * q[7];
  const T pt = p + pm;
  const T e = q[4] - T(0.5) * q[8] * q[8];
  F[0] = q[0] * un;
  F[1] = q[1] * un + pt * n[0] - q[5] * Bn;
  F[2] = q[2] * un + pt * n[1] - q[6] * Bn;
  F[3] = q[3] * un + pt * n[2] - q[7] * Bn;
  F[4] = un * (e + pt) - Bn * uB + P.c_h * q[8] * Bn;
  F[5] = un * q[5] - Bn * u0 + P.c_h * q[8] * n[0];
  F[6] = un * q[6] - Bn * u1 + P.c_h * q[8] * n[1];
  F[7] = un * q[7] - Bn * u2 + P.c_h * q[8] * n[2];
  F[8] = P.c_h * Bn;
}

// Primitive derivatives needed by the viscous flux.
template <typename T>
struct ViscLocal {
  T u[3], B[3];
  T tau[3][3];  // shear stress (Eq. "ssTensor", lambda = -2/3 mu, mu = rho nu)
  T qh[3];      // heat flux (Eq. "qFlux", grad S from Eq. "entropy")
  T J[3];       // current curl B
};

template <typename T>
__device__ __forceinline__ void viscous_local(const T* q, const T* G, T kr, const Phys<T>& P,
                                              ViscLocal<T>& v) {
  const T rho = q[0], ir = recip(rho);
  v.u[0] = q[1] * ir; v.u[1] = q[2] * ir; v.u[2] = q[3] * ir;
  v.B[0] = q[5]; v.B[1] = q[6]; v.B[2] = q[7];
  const T p = pressure(q, P);
  const T Tt = p * ir * P.inv_R;
  const T uu = v.u[0] * v.u[0] + v.u[1] * v.u[1] + v.u[2] * v.u[2];
  T du[3][3];
  T dp[3], drho[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    drho[j] = G[j];
#pragma unroll
    for (int i = 0; i < 3; ++i) du[i][j] = (G[(1 + i) * 3 + j] - v.u[i] * drho[j]) * ir;
    const T um = v.u[0] * G[3 + j] + v.u[1] * G[6 + j] + v.u[2] * G[9 + j];
    const T bb = v.B[0] * G[15 + j] + v.B[1] * G[18 + j] + v.B[2] * G[21 + j];
    dp[j] = P.gm1 * (G[12 + j] - um + T(0.5) * uu * drho[j] - bb - q[8] * G[24 + j]);
  }
  const T mu = rho * P.nu;
  const T lam = T(-2.0 / 3.0) * mu * (du[0][0] + du[1][1] + du[2][2]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) v.tau[i][j] = mu * (du[i][j] + du[j][i]) + (i == j ? lam : T(0));
  const T ip = recip(p);
  const T irR = ir * P.inv_R;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T dS = P.cp * (dp[j] * ip * P.inv_gamma - drho[j] * ir);
    const T dT = (dp[j] - P.Rgas * Tt * drho[j]) * irR;
    v.qh[j] = -P.kappa * rho * Tt * dS - kr * rho * P.cp * dT;
  }
  v.J[0] = G[21 + 1] - G[18 + 2];
  v.J[1] = G[15 + 2] - G[21 + 0];
  v.J[2] = G[18 + 0] - G[15 + 1];
}

// Viscous flux through n (Eq. "visF"; the induction row is the antisymmetric
// tensor eta (dB_i/dx_j - dB_j/dx_i), whose flux through n is eta J x n).
// Only the 7 non-zero components (1..7) are produced: Fv[0..6].
template <typename T>
__device__ __forceinline__ void flux_viscous7(const ViscLocal<T>& v, const T n[3], const Phys<T>& P,
                                              T Fv[7]) {
  T tn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) tn[i] = v.tau[i][0] * n[0] + v.tau[i][1] * n[1] + v.tau[i][2] * n[2];
  const T bxj0 = v.B[1] * v.J[2] - v.B[2] * v.J[1];
  const T bxj1 = v.B[2] * v.J[0] - v.B[0] * v.J[2];
  const T bxj2 = v.B[0] * v.J[1] - v.B[1] * v.J[0];
  Fv[0] = tn[0];
  Fv[1] = tn[1];
  Fv[2] = tn[2];
  Fv[3] = (v.u[0] * tn[0] + v.u[1] * tn[1] + v.u[2] * tn[2]) -
          (v.qh[0] * n[0] + v.qh[1] * n[1] + v.qh[2] * n[2]) +
          P.eta * (bxj0 * n[0] + bxj1 * n[1] + bxj2 * n[2]);
  Fv[4] = P.eta * (v.J[1] * n[2] - v.J[2] * n[1]);
  Fv[5] = P.eta * (v.J[2] * n[0] - v.J[0] * n[2]);
  Fv[6] = P.eta * (v.J[0] * n[1] - v.J[1] * n[0]);
}

// ---- fused fluxes of the interior and face flux points --------------------
// The inviscid and viscous fluxes of one state share 1/rho, u, p and T, and
// only their component along n is needed, so the gradients are projected on
// n before they are combined.  The heat flux through n uses Eq. "qFlux" with
// grad S from Eq. "entropy" and the ideal gas p = rho R T, c_p/(gamma R) =
// 1/(gamma - 1):  -kappa rho T grad S - kappa_r rho c_p grad T
//   = -(kappa + gamma kappa_r)/(gamma - 1) grad p + (kappa + kappa_r) c_p T grad rho.

template <typename T>
struct PointState {
  T ir, u[3], uu, pm, p, Tt;
};

template <typename T>
__device__ __forceinline__ void point_state(const T* q, const Phys<T>& P, PointState<T>& s) {
  s.ir = recip(q[0]);
  s.u[0] = q[1] * s.ir; s.u[1] = q[2] * s.ir; s.u[2] = q[3] * s.ir;
  s.uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
  s.pm = T(0.5) * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
  s.p = P.gm1 * (q[4] - T(0.5) * (q[1] * s.u[0] + q[2] * s.u[1] + q[3] * s.u[2]) - s.pm - T(0.5) * q[8] * q[8]);
  s.Tt = s.p * s.ir * P.inv_R;
}

// flux_inviscid from a point state (same formulas)
template <typename T>
__device__ __forceinline__ void flux_inviscid_s(const T* q, const PointState<T>& s, const T n[3], const Phys<T>& P,
                                                T F[9]) {
  const T un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
  const T Bn = q[5] * n[0] + q[6] * n[1] + q[7] * n[2];
  const T uB = s.u[0] * q[5] + s.u[1] * q[6] + s.u[2] * q[7];
  const T pt = s.p + s.pm;
  const T e = q[4] - T(0.5) * q[8] * q[8];
  F[0] = q[0] * un;
  F[1] = q[1] * un + pt * n[0] - q[5] * Bn;
  F[2] = q[2] * un + pt * n[1] - q[6] * Bn;
  F[3] = q[3] * un + pt * n[2] - q[7] * Bn;
  F[4] = un * (e + pt) - Bn * uB + P.c_h * q[8] * Bn;
  F[5] = un * q[5] - Bn * s.u[0] + P.c_h * q[8] * n[0];
  F[6] = un * q[6] - Bn * s.u[1] + P.c_h * q[8] * n[1];
  F[7] = un * q[7] - Bn * s.u[2] + P.c_h * q[8] * n[2];
  F[8] = P.c_h * Bn;
}

// Components 1..7 of the viscous flux through n (Eq. "visF"; the same
// quantities as viscous_local + flux_viscous7): Fv[0..2] = tau n, Fv[3] =
// u.(tau n) - q.n + eta (B x J).n, Fv[4..6] = eta J x n.
template <typename T>
__device__ __forceinline__ void flux_viscous_n(const T* q, const T* G, T kr, const PointState<T>& s, const T n[3],
                                               const Phys<T>& P, T Fv[7]) {
  const T grn = G[0] * n[0] + G[1] * n[1] + G[2] * n[2];
  T gmn[3], gBn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gmn[i] = G[(1 + i) * 3] * n[0] + G[(1 + i) * 3 + 1] * n[1] + G[(1 + i) * 3 + 2] * n[2];
    gBn[i] = G[(5 + i) * 3] * n[0] + G[(5 + i) * 3 + 1] * n[1] + G[(5 + i) * 3 + 2] * n[2];
  }
  const T gEn = G[12] * n[0] + G[13] * n[1] + G[14] * n[2];
  const T gpn = G[24] * n[0] + G[25] * n[1] + G[26] * n[2];
  // velocity gradient du_ij = (d m_i/dx_j - u_i d rho/dx_j) / rho
  T du[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) du[i][j] = (G[(1 + i) * 3 + j] - s.u[i] * G[j]) * s.ir;
  const T mu = q[0] * P.nu;
  const T lam = T(-2.0 / 3.0) * mu * (du[0][0] + du[1][1] + du[2][2]);
  T tn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    tn[i] = mu * ((du[i][0] + du[0][i]) * n[0] + (du[i][1] + du[1][i]) * n[1] + (du[i][2] + du[2][i]) * n[2]) +
            lam * n[i];
  // grad p . n (from the conserved gradients) and the heat flux through n
  const T dpn = P.gm1 * (gEn - (s.u[0] * gmn[0] + s.u[1] * gmn[1] + s.u[2] * gmn[2]) + T(0.5) * s.uu * grn -
                         (q[5] * gBn[0] + q[6] * gBn[1] + q[7] * gBn[2]) - q[8] * gpn);
  const T qn = -(P.kappa + P.gamma * kr) * P.inv_gm1 * dpn + (P.kappa + kr) * P.cp * s.Tt * grn;
  const T J0 = G[21 + 1] - G[18 + 2], J1 = G[15 + 2] - G[21 + 0], J2 = G[18 + 0] - G[15 + 1];
  const T bxjn = (q[6] * J2 - q[7] * J1) * n[0] + (q[7] * J0 - q[5] * J2) * n[1] + (q[5] * J1 - q[6] * J0) * n[2];
  Fv[0] = tn[0];
  Fv[1] = tn[1];
  Fv[2] = tn[2];
  Fv[3] = (s.u[0] * tn[0] + s.u[1] * tn[1] + s.u[2] * tn[2]) - qn + P.eta * bxjn;
  Fv[4] = P.eta * (J1 * n[2] - J2 * n[1]);
  Fv[5] = P.eta * (J2 * n[0] - J0 * n[2]);
  Fv[6] = P.eta * (J0 * n[1] - J1 * n[0]);
}

// fast magnetosonic speed along the unit direction nh
template <typename T>
__device__ __forceinline__ T fast_speed(const T* q, const T nh[3], const Phys<T>& P) {
  const T ir = recip(q[0]);
  const T a2 = P.gamma * pressure(q, P) * ir;
  const T b2 = (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]) * ir;
  const T Bn = q[5] * nh[0] + q[6] * nh[1] + q[7] * nh[2];
  const T s = a2 + b2;
  T disc = s * s - T(4) * a2 * Bn * Bn * ir;
  disc = disc > T(0) ? disc : T(0);
  return sqrt_fast(T(0.5) * (s + sqrt_fast(disc)));
}

// Rusanov flux from `own` to `oth` through the unnormalised normal n pointing
// out of `own`.  Written symmetrically so that the other side, calling it
// with the arguments swapped and -n, gets exactly the negated value.
template <typename T>
__device__ __forceinline__ void rusanov(const T* own, const T* oth, const T n[3], const Phys<T>& P,
                                        T F[9]) {
  const T nn = sqrt_fast(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  const T inn = recip(nn);
  const T nh[3] = {n[0] * inn, n[1] * inn, n[2] * inn};
  const T s1 = fabs((own[1] * nh[0] + own[2] * nh[1] + own[3] * nh[2]) * recip(own[0])) + fast_speed(own, nh, P);
  const T s2 = fabs((oth[1] * nh[0] + oth[2] * nh[1] + oth[3] * nh[2]) * recip(oth[0])) + fast_speed(oth, nh, P);
  T lam = s1 > s2 ? s1 : s2;
  lam = lam > P.c_h ? lam : P.c_h;
  T F1[9], F2[9];
  flux_inviscid(own, n, P, F1);
  flux_inviscid(oth, n, P, F2);
  const T dis = T(0.5) * lam * nn;
#pragma unroll
  for (int v = 0; v < 9; ++v) F[v] = T(0.5) * (F1[v] + F2[v]) - dis * (oth[v] - own[v]);
}

// ---- walls (nh: outward unit normal of the domain) ------------------------

// Common solution for the gradients: tangential velocity only
// (impenetrable), B tangential (conducting) or normal (radial), pressure
// kept (heat-flux wall) or rho R T_wall (fixed temperature); psi reflected
// at a conducting wall, zero at a radial-field wall.
template <typename T>
__device__ __forceinline__ void wall_common(const T* q, const T nh[3], int g, const Phys<T>& P, T* qc) {
  const T rho = q[0], ir = recip(rho);
  const T un = (q[1] * nh[0] + q[2] * nh[1] + q[3] * nh[2]) * ir;
  const T Bn = q[5] * nh[0] + q[6] * nh[1] + q[7] * nh[2];
  const bool cond = wsel(g, P.wall_mag) == 0;
  const T p = wsel(g, P.wall_th) == 0 ? pressure(q, P) : rho * P.Rgas * wsel(g, P.T_wall);
  T uc[3], Bc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    uc[i] = q[1 + i] * ir - un * nh[i];
    Bc[i] = cond ? q[5 + i] - Bn * nh[i] : Bn * nh[i];
  }
  const T psi = cond ? q[8] : T(0);
  qc[0] = rho;
#pragma unroll
  for (int i = 0; i < 3; ++i) { qc[1 + i] = rho * uc[i]; qc[5 + i] = Bc[i]; }
  qc[8] = psi;
  qc[4] = p / P.gm1 + T(0.5) * rho * (uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]) +
          T(0.5) * (Bc[0] * Bc[0] + Bc[1] * Bc[1] + Bc[2] * Bc[2]) + T(0.5) * psi * psi;
}

// Mirror state for the wall Rusanov flux.
template <typename T>
__device__ __forceinline__ void wall_mirror(const T* q, const T nh[3], int g, const Phys<T>& P, T* qg) {
  const T mn = q[1] * nh[0] + q[2] * nh[1] + q[3] * nh[2];
  const T Bn = q[5] * nh[0] + q[6] * nh[1] + q[7] * nh[2];
  const bool cond = wsel(g, P.wall_mag) == 0;
  qg[0] = q[0];
  qg[4] = q[4];
  qg[8] = cond ? q[8] : -q[8];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    qg[1 + i] = q[1 + i] - T(2) * mn * nh[i];
    qg[5 + i] = cond ? q[5 + i] - T(2) * Bn * nh[i] : T(2) * Bn * nh[i] - q[5 + i];
  }
}

// Viscous part of the wall flux, from the viscous locals v evaluated with
// the wall's common state and the interior gradient.  Stress-free: only the
// normal traction; no work term; heat flux prescribed (q.n = q_wall * (-1
// inner, +1 outer) |n|) or computed at a fixed-T wall; current reduced to J_r
// (conducting) or J - J_r (radial).  Subtracted from F (F = F_inv - F_vis).
template <typename T>
__device__ __forceinline__ void wall_viscous_sub(const ViscLocal<T>& v, const T n[3], const T nh[3], T nn,
                                                 int g, const Phys<T>& P, T F[9]) {
  T tn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) tn[i] = v.tau[i][0] * n[0] + v.tau[i][1] * n[1] + v.tau[i][2] * n[2];
  const T tnn = tn[0] * nh[0] + tn[1] * nh[1] + tn[2] * nh[2];
  const T qn = wsel(g, P.wall_th) == 0 ? wsel(g, P.q_wall) * (g == 0 ? T(-1) : T(1)) * nn
                                       : v.qh[0] * n[0] + v.qh[1] * n[1] + v.qh[2] * n[2];
  const T Jn = v.J[0] * nh[0] + v.J[1] * nh[1] + v.J[2] * nh[2];
  const bool cond = wsel(g, P.wall_mag) == 0;
  T Jc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Jc[i] = cond ? Jn * nh[i] : v.J[i] - Jn * nh[i];
  const T bxj0 = v.B[1] * Jc[2] - v.B[2] * Jc[1];
  const T bxj1 = v.B[2] * Jc[0] - v.B[0] * Jc[2];
  const T bxj2 = v.B[0] * Jc[1] - v.B[1] * Jc[0];
#pragma unroll
  for (int i = 0; i < 3; ++i) F[1 + i] -= tnn * nh[i];
  F[4] -= -qn + P.eta * (bxj0 * n[0] + bxj1 * n[1] + bxj2 * n[2]);
  F[5] -= P.eta * (Jc[1] * n[2] - Jc[2] * n[1]);
  F[6] -= P.eta * (Jc[2] * n[0] - Jc[0] * n[2]);
  F[7] -= P.eta * (Jc[0] * n[1] - Jc[1] * n[0]);
}

template <typename T>
__device__ __forceinline__ T kappa_r(const T x[3], const Phys<T>& P) {
  const T w = sqrt_fast(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) * P.kr_w;
  return P.kr_scale * (P.kr_c0 + P.kr_c1 * w + P.kr_c2 * w * w);
}

}  // namespace sdm
