// Operation count of the pointwise physics of the gfx950 kernels
// (sdm_physics.hpp), compiled on the host with a counting number type: every
// +, -, *, / and sqrt of one call of each function is counted once (a fused
// multiply-add of the device code is two).  The benchmark's algorithmic flop
// count uses these numbers; tests/test_flop_count.py checks that they match.
#include <cmath>
#include <cstdio>
#include <cstdint>
#define __device__
#define __forceinline__ inline
#define __host__
static long g_add = 0, g_mul = 0, g_div = 0, g_sqrt = 0, g_cmp = 0;
namespace sdm {
struct CD {
  double v;
  CD() : v(0) {}
  CD(double x) : v(x) {}
};
inline CD operator+(CD a, CD b) { ++g_add; return CD(a.v + b.v); }
inline CD operator-(CD a, CD b) { ++g_add; return CD(a.v - b.v); }
inline CD operator-(CD a) { return CD(-a.v); }
inline CD operator*(CD a, CD b) { ++g_mul; return CD(a.v * b.v); }
inline CD operator/(CD a, CD b) { ++g_div; return CD(a.v / b.v); }
inline CD& operator+=(CD& a, CD b) { ++g_add; a.v += b.v; return a; }
inline CD& operator-=(CD& a, CD b) { ++g_add; a.v -= b.v; return a; }
inline CD& operator*=(CD& a, CD b) { ++g_mul; a.v *= b.v; return a; }
inline bool operator<(CD a, CD b) { ++g_cmp; return a.v < b.v; }
inline bool operator>(CD a, CD b) { ++g_cmp; return a.v > b.v; }
inline bool operator!=(CD a, CD b) { return a.v != b.v; }
inline bool operator==(CD a, CD b) { return a.v == b.v; }
inline CD sqrt(CD a) { ++g_sqrt; return CD(std::sqrt(a.v)); }
inline CD fabs(CD a) { return CD(std::fabs(a.v)); }
inline CD fmax(CD a, CD b) { ++g_cmp; return CD(std::fmax(a.v, b.v)); }
inline CD max(CD a, CD b) { ++g_cmp; return CD(std::fmax(a.v, b.v)); }
inline CD recip(CD a) { ++g_div; return CD(1.0 / a.v); }
}  // namespace sdm
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#include "sdm_physics.hpp"

using namespace sdm;
static void reset() { g_add = g_mul = g_div = g_sqrt = g_cmp = 0; }
static void report(const char* what) {
  printf("%-22s add %3ld mul %3ld div %2ld sqrt %2ld cmp %2ld  flops(add+mul+div+sqrt) %4ld\n", what, g_add, g_mul, g_div,
         g_sqrt, g_cmp, g_add + g_mul + g_div + g_sqrt);
}
int main() {
  Phys<CD> P;
  P.gm1 = 2.0 / 3; P.gamma = 5.0 / 3; P.Rgas = 1; P.cp = 2.5; P.inv_R = 1; P.inv_gamma = 0.6;
  P.nu = 1e-5; P.kappa = 1e-5; P.eta = 1e-5; P.c_h = 1; P.powell = 1;
  CD q[9] = {1.0, 0.01, 0.02, 0.03, 2.0, 0.001, 0.002, 0.003, 0.0}, q2[9], G[27], n[3] = {0.3, 0.4, 0.5}, F[9], Fv[7];
  for (int i = 0; i < 9; ++i) q2[i] = CD(q[i].v * 1.01);
  for (int i = 0; i < 27; ++i) G[i] = CD(0.01 * (i + 1));
  ViscLocal<CD> vl;
  reset(); flux_inviscid(q, n, P, F); report("flux_inviscid");
  reset(); viscous_local(q, G, CD(0.0), P, vl); report("viscous_local");
  reset(); flux_viscous7(vl, n, P, Fv); report("flux_viscous7");
  reset(); rusanov(q, q2, n, P, F); report("rusanov");
  return 0;
}
