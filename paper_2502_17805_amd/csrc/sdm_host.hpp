// sdm_host.hpp -- host-side setup of the spectral-difference library.
#pragma once
#include <cstdint>
#include <vector>

namespace sdm {

// 1-D operators of the method for N solution points per direction
// (paper, Sec. "Spectral Difference Method": Chebyshev-Gauss solution
// points, Legendre flux points with both end points, bases h_i and l_i).
struct Tables1D {
  int N = 0;
  std::vector<double> xs;   // [N]       solution points
  std::vector<double> xf;   // [N+1]     flux points
  std::vector<double> I;    // [N+1][N]  h_i(xf_f)
  std::vector<double> D;    // [N][N+1]  l_f'(xs_i)
  std::vector<double> L;    // [N][N+1]  l_f(xs_i)
  std::vector<double> Dff;  // [N+1][N+1] l_f'(xf_g)
  std::vector<double> DI;   // [N][N]    h_j'(xs_i) = (D I)_ij
  std::vector<double> W;    // [N]       integral of h_i over [0,1]
};

Tables1D make_tables(int N);

int shell_build(int Nz, int Nr, int p, double rb, double rt, double* x_sp, double* detJ,
                double* S_fp, double* S_sp, int32_t* nbr, double* n_face);
int box_build(int nx, int ny, int nz, double Lx, double Ly, double Lz, int periodic, double warp,
              int p, double* x_sp, double* detJ, double* S_fp, double* S_sp, int32_t* nbr, double* n_face);

// Solution points grouped by (r, theta) bin: bin of SP g (= e N^3 + sp) from
// its position; order[] lists the SPs bin by bin (ascending g within a bin),
// offsets[b] .. offsets[b + 1] is bin b's range.
void sph_bins(int64_t E, int N, const double* x_sp, double rb, double rt, int n_r, int n_th, int32_t* order,
              int64_t* offsets);

// One explicit Runge-Kutta stage in Shu-Osher form on numbered state
// registers: regs[out] = sum_k alpha[k] regs[in_idx[k]] + beta dt R(regs[cur]).
struct ShuOsherStage {
  int cur, n_in, in_idx[4];
  double alpha[4];
  int out;
  double beta;
};

// The SSPRK(5,3) scheme named in Sec. "Spectral Difference Method" as five
// such stages on four registers (u0 in register 0, the step's result back in
// register 0), and c[5]: the time, in units of dt, of the state each stage
// takes the residual of.
void ssprk53_stages(ShuOsherStage st[5], double c[5]);

// Initial background of Sec. "Initial Conditions": the polytrope, or the
// almost flux-balanced profile (entropy gradient from the outward heat flux
// L / (4 pi r^2) through the polytrope, hydrostatic density from it).
struct Background {
  double GM, Rgas, gamma, rb, rt, rho_b, N_rho, L, kappa;
  double kr_scale, kr_c0, kr_c1, kr_c2, kr_w;
  int flux_balanced;
};
// (rho, p, T) at n radii in [rb, rt].  Nonzero: 1 bad parameters, 2 a radius
// outside the shell, 3 the density of the flux-balanced profile reaches zero.
int background_profile(const Background& b, int64_t n, const double* r, double* rho, double* p, double* T);

}  // namespace sdm
