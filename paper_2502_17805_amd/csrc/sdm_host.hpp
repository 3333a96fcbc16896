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

// Element chunks for the overlapped stage schedule: breadth-first levels over
// interior faces, seeded by the elements with a face in boundary group 0 (the
// inner wall of a shell, whose levels are then its radial layers) and, for
// pieces without such a face, by their lowest element.  order[E] lists the
// elements level by level (ascending within a level); chunk k covers
// order[lo[k] .. lo[k + 1]), whole levels of at least min_chunk elements (a
// short last chunk joins the previous one); dep[k] >= k is the last chunk
// holding a face neighbour of an element of chunk k.  Nonzero on bad sizes.
int element_chunks(int64_t E, const int32_t* nbr, int64_t min_chunk, int32_t* order, std::vector<int64_t>& lo,
                   std::vector<int32_t>& dep);

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
