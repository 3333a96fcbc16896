// Operation count of the oracle's pointwise physics (oracle/sdmhd_oracle_point.inc:
// the inviscid flux, the viscous flux and the Rusanov flux of Sec. "MHD
// Governing Equations" and Sec. "Spectral Difference Method"), compiled on
// the host with a counting number type: every +, -, *, / and sqrt of one
// call is counted once.  These counts define the benchmark's algorithmic
// FP64 flops per flux point (tests/test_flop_count.py keeps bench.py's
// table equal to them), independent of how the kernels compute the fluxes.
#include <cmath>
#include <cstdint>
#include <cstdio>

static long g_add = 0, g_mul = 0, g_div = 0, g_sqrt = 0, g_cmp = 0;
namespace cnt {
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
inline CD sqrt(CD a) { ++g_sqrt; return CD(std::sqrt(a.v)); }
inline CD fabs(CD a) { return CD(std::fabs(a.v)); }
}  // namespace cnt
using cnt::CD;

extern "C" {
#include "sdmhd_oracle.h"
}
#define NV 9
#define OR_REAL CD
#include "sdmhd_oracle_point.inc"

static void reset() { g_add = g_mul = g_div = g_sqrt = g_cmp = 0; }
static void report(const char* what) {
  printf("%-12s add %3ld mul %3ld div %2ld sqrt %2ld cmp %2ld  flops(add+mul+div+sqrt) %4ld\n", what, g_add, g_mul,
         g_div, g_sqrt, g_cmp, g_add + g_mul + g_div + g_sqrt);
}

int main() {
  or_params P = {};
  P.gamma = 5.0 / 3.0;
  P.Rgas = 1.0;
  P.nu = 1e-5;
  P.kappa = 1e-5;
  P.eta = 1e-5;
  P.c_h = 1.0;
  CD q[9] = {1.0, 0.01, 0.02, 0.03, 2.0, 0.001, 0.002, 0.003, 0.0}, q2[9], G[27], n[3] = {0.3, 0.4, 0.5}, F[9];
  for (int i = 0; i < 9; ++i) q2[i] = CD(q[i].v * 1.01);
  for (int i = 0; i < 27; ++i) G[i] = CD(0.01 * (i + 1));
  reset(); inv_flux(q, n, &P, F); report("inv_flux");
  reset(); visc_flux(q, G, CD(0.0), n, &P, F); report("visc_flux");
  reset(); rusanov(q, q2, n, &P, F); report("rusanov");
  return 0;
}
