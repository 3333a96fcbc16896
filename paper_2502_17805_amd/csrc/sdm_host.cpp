// sdm_host.cpp -- host-side setup of the spectral-difference library:
// 1-D tables, cubed-sphere / box meshes, face connectivity and the metric
// terms of the transformed equations (paper arXiv 2502.17805, Sec. "Meshing"
// and Sec. "Spectral Difference Method").  Runs once per mesh, on the CPU.
#include "sdm_host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <unordered_map>
#include <utility>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace sdm {

using ld = long double;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// 1-D tables
// ---------------------------------------------------------------------------

namespace {

// Roots of the Legendre polynomial P_m on (-1, 1), ascending.  Newton on the
// three-term recurrence, started from the asymptotic estimate of each root.
std::vector<ld> legendre_zeros(int m) {
  std::vector<ld> z(m);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int k = 1; k <= m; ++k) {
    ld x = -std::cos(pi * (k - 0.25L) / (m + 0.5L));  // k-th smallest
    for (int it = 0; it < 60; ++it) {
      ld pm1 = 1, p = x;  // P_0, P_1
      for (int n = 2; n <= m; ++n) {
        ld pn = ((2 * n - 1) * x * p - (n - 1) * pm1) / n;
        pm1 = p;
        p = pn;
      }
      if (m == 1) { p = x; pm1 = 1; }
      ld dp = m * (x * p - pm1) / (x * x - 1);
      ld step = p / dp;
      x -= step;
      if (std::fabs(step) < 1e-21L) break;
    }
    z[k - 1] = x;
  }
  return z;
}

// Lagrange basis j over `nodes` and its derivative at x (x not a node for
// the derivative form used here: l'_j(x) = l_j(x) sum_{k != j} 1/(x - x_k)).
ld lagrange(const std::vector<ld>& nodes, int j, ld x) {
  ld v = 1;
  for (size_t k = 0; k < nodes.size(); ++k)
    if ((int)k != j) v *= (x - nodes[k]) / (nodes[j] - nodes[k]);
  return v;
}
ld lagrange_deriv(const std::vector<ld>& nodes, int j, ld x) {
  for (size_t k = 0; k < nodes.size(); ++k)
    if (std::fabs(x - nodes[k]) < 1e-30L) {
      // x is node k: differentiation-matrix entry
      if ((int)k != j) {
        ld wj = 1, wk = 1;
        for (size_t m = 0; m < nodes.size(); ++m) {
          if ((int)m != j) wj *= nodes[j] - nodes[m];
          if (m != k) wk *= nodes[k] - nodes[m];
        }
        return (wk / wj) / (nodes[k] - nodes[j]);
      }
      ld s = 0;
      for (size_t m = 0; m < nodes.size(); ++m)
        if ((int)m != j) s += 1 / (nodes[j] - nodes[m]);
      return s;
    }
  ld s = 0;
  for (size_t k = 0; k < nodes.size(); ++k)
    if ((int)k != j) s += 1 / (x - nodes[k]);
  return lagrange(nodes, j, x) * s;
}

}  // namespace

Tables1D make_tables(int N) {
  Tables1D t;
  t.N = N;
  const ld pi = 3.141592653589793238462643383279502884L;
  std::vector<ld> xs(N), xf(N + 1);
  for (int n = 1; n <= N; ++n) xs[n - 1] = (1 - std::cos((2 * n - 1) * pi / (2 * N))) / 2;
  std::vector<ld> z = legendre_zeros(N - 1);
  xf[0] = 0;
  for (int k = 0; k < N - 1; ++k) xf[k + 1] = (1 + z[k]) / 2;
  xf[N] = 1;
  t.xs.assign(xs.begin(), xs.end());
  t.xf.assign(xf.begin(), xf.end());
  t.I.resize((N + 1) * N);
  t.D.resize(N * (N + 1));
  t.L.resize(N * (N + 1));
  t.Dff.resize((N + 1) * (N + 1));
  t.DI.resize(N * N);
  for (int f = 0; f <= N; ++f)
    for (int i = 0; i < N; ++i) t.I[f * N + i] = (double)lagrange(xs, i, xf[f]);
  for (int i = 0; i < N; ++i)
    for (int f = 0; f <= N; ++f) {
      t.D[i * (N + 1) + f] = (double)lagrange_deriv(xf, f, xs[i]);
      t.L[i * (N + 1) + f] = (double)lagrange(xf, f, xs[i]);
    }
  for (int g = 0; g <= N; ++g)
    for (int f = 0; f <= N; ++f) t.Dff[g * (N + 1) + f] = (double)lagrange_deriv(xf, f, xf[g]);
  // derivative of the solution polynomial itself at the SPs: (D I)_ij = h_j'(xs_i)
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) t.DI[i * N + j] = (double)lagrange_deriv(xs, j, xs[i]);
  // weights W_i = integral of h_i over [0,1]: solve the moment equations
  // sum_i W_i xs_i^k = 1/(k+1), k < N, by Gaussian elimination (long double)
  std::vector<ld> A(N * (N + 1));
  for (int k = 0; k < N; ++k) {
    for (int i = 0; i < N; ++i) A[k * (N + 1) + i] = std::pow(xs[i], (ld)k);
    A[k * (N + 1) + N] = 1.0L / (k + 1);
  }
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(A[r * (N + 1) + c]) > std::fabs(A[piv * (N + 1) + c])) piv = r;
    for (int q = 0; q <= N; ++q) std::swap(A[c * (N + 1) + q], A[piv * (N + 1) + q]);
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      ld fct = A[r * (N + 1) + c] / A[c * (N + 1) + c];
      for (int q = c; q <= N; ++q) A[r * (N + 1) + q] -= fct * A[c * (N + 1) + q];
    }
  }
  t.W.resize(N);
  for (int i = 0; i < N; ++i) t.W[i] = (double)(A[i * (N + 1) + N] / A[i * (N + 1) + i]);
  return t;
}

// ---------------------------------------------------------------------------
// Geometry of one element
// ---------------------------------------------------------------------------

namespace {

// Small dense operator applied along one axis of an (n0, n1, n2) block.
struct Block3 {
  int n[3];
  std::vector<double> v;
  Block3(int a, int b, int c) : n{a, b, c}, v((size_t)a * b * c, 0.0) {}
  double& at(int i, int j, int k) { return v[i + n[0] * (j + n[1] * k)]; }
  double at(int i, int j, int k) const { return v[i + n[0] * (j + n[1] * k)]; }
};

// out = M applied along `axis` (M has `rows` rows and n[axis] columns)
Block3 along(const Block3& in, int axis, const double* M, int rows) {
  int m[3] = {in.n[0], in.n[1], in.n[2]};
  m[axis] = rows;
  Block3 out(m[0], m[1], m[2]);
  const int cols = in.n[axis];
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        int idx[3] = {i, j, k};
        const int r = idx[axis];
        double acc = 0.0;
        for (int c = 0; c < cols; ++c) {
          idx[axis] = c;
          acc += M[r * cols + c] * in.at(idx[0], idx[1], idx[2]);
        }
        out.at(i, j, k) = acc;
      }
  return out;
}

enum Op { KEEP, VAL, DER };  // keep node index / value at SPs / derivative at SPs

Block3 sample(const Tables1D& t, const Block3& nodes, Op o0, Op o1, Op o2) {
  Block3 cur = nodes;
  const Op ops[3] = {o0, o1, o2};
  for (int ax = 0; ax < 3; ++ax) {
    if (ops[ax] == KEEP) continue;
    cur = along(cur, ax, ops[ax] == VAL ? t.L.data() : t.D.data(), t.N);
  }
  return cur;
}

// Metric data of one element from the map nodes X[c] (c = x, y, z) on the
// (N+1)^3 flux-point tensor grid.
void element_geometry(const Tables1D& t, const Block3 Xabs[3], double* x_sp, double* detJ,
                      double* S_fp, double* S_sp) {
  const int N = t.N, NP = N + 1, N3 = N * N * N, NF = NP * N * N;
  // The metric terms, the map derivatives and |J| are invariant under a
  // translation of the element (the discrete curl of a discrete gradient of
  // a tensor-product polynomial vanishes), so they are formed from node
  // positions relative to the element's first node: coordinates of size h
  // instead of 1 keep their round-off proportional to the terms (h^2).
  Block3 X[3] = {Xabs[0], Xabs[1], Xabs[2]};
  for (int c = 0; c < 3; ++c) {
    const double o = Xabs[c].v[0];
    for (double& v : X[c].v) v -= o;
  }
  // derivatives of the map at the nodes
  Block3 dX[3][3] = {{X[0], X[0], X[0]}, {X[0], X[0], X[0]}, {X[0], X[0], X[0]}};  // [axis][comp]
  for (int ax = 0; ax < 3; ++ax)
    for (int c = 0; c < 3; ++c) dX[ax][c] = along(X[c], ax, t.Dff.data(), NP);
  // invariant curl form: S^i_n = d_k W_j - d_j W_k, (i,j,k) cyclic, with
  // W_a = (X_l dX_m/dxi_a - X_m dX_l/dxi_a)/2, (n,m,l) cyclic
  for (int n = 0; n < 3; ++n) {
    const int mm = (n + 1) % 3, l = (n + 2) % 3;
    Block3 W[3] = {X[0], X[0], X[0]};
    for (int a = 0; a < 3; ++a)
      for (size_t q = 0; q < W[a].v.size(); ++q)
        W[a].v[q] = 0.5 * (X[l].v[q] * dX[a][mm].v[q] - X[mm].v[q] * dX[a][l].v[q]);
    for (int i = 0; i < 3; ++i) {
      const int j = (i + 1) % 3, k = (i + 2) % 3;
      Op pa[3] = {VAL, VAL, VAL}, pb[3] = {VAL, VAL, VAL};
      pa[i] = pb[i] = KEEP;  // family i keeps its flux-point index
      pa[k] = DER;           // d_k W_j
      pb[j] = DER;           // d_j W_k
      Block3 A = sample(t, W[j], pa[0], pa[1], pa[2]);
      Block3 B = sample(t, W[k], pb[0], pb[1], pb[2]);
      double* out = S_fp + (i * 3 + n) * NF;
      for (int q = 0; q < NF; ++q) out[q] = A.v[q] - B.v[q];
      if (S_sp) {
        pa[i] = pb[i] = VAL;
        Block3 As = sample(t, W[j], pa[0], pa[1], pa[2]);
        Block3 Bs = sample(t, W[k], pb[0], pb[1], pb[2]);
        double* os = S_sp + (i * 3 + n) * N3;
        for (int q = 0; q < N3; ++q) os[q] = As.v[q] - Bs.v[q];
      }
    }
  }
  // positions and Jacobian determinant at the solution points
  Block3 J[3][3] = {{X[0], X[0], X[0]}, {X[0], X[0], X[0]}, {X[0], X[0], X[0]}};  // J[c][axis]
  for (int c = 0; c < 3; ++c) {
    Block3 p = sample(t, Xabs[c], VAL, VAL, VAL);
    std::memcpy(x_sp + c * N3, p.v.data(), sizeof(double) * N3);
    J[c][0] = sample(t, X[c], DER, VAL, VAL);
    J[c][1] = sample(t, X[c], VAL, DER, VAL);
    J[c][2] = sample(t, X[c], VAL, VAL, DER);
  }
  for (int q = 0; q < N3; ++q) {
    const double a = J[0][0].v[q], b = J[0][1].v[q], c = J[0][2].v[q];
    const double d = J[1][0].v[q], e = J[1][1].v[q], f = J[1][2].v[q];
    const double g = J[2][0].v[q], h = J[2][1].v[q], k = J[2][2].v[q];
    detJ[q] = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  }
  // the chain-rule factors S^d/|J| at the solution points
  if (S_sp)
    for (int r = 0; r < 9; ++r)
      for (int q = 0; q < N3; ++q) S_sp[r * N3 + q] /= detJ[q];
}

// ---------------------------------------------------------------------------
// Connectivity from integer corner keys
// ---------------------------------------------------------------------------

using Key = std::array<int32_t, 4>;
struct FaceKey {
  std::array<Key, 4> c;  // sorted corner keys
  bool operator==(const FaceKey& o) const { return c == o.c; }
};
struct FaceKeyHash {
  size_t operator()(const FaceKey& k) const {
    size_t h = 1469598103934665603ull;
    for (const Key& q : k.c)
      for (int32_t v : q) h = (h ^ (uint32_t)v) * 1099511628211ull;
    return h;
  }
};

// element corner (bit 0: xi, bit 1: eta, bit 2: zeta) at face-local corner (a,b)
int corner_of(int face, int a, int b) {
  const int ax = face >> 1, side = face & 1;
  int bits[3];
  bits[ax] = side;
  const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
  bits[o1] = a;
  bits[o2] = b;
  return bits[0] | (bits[1] << 1) | (bits[2] << 2);
}

void map_point(int o, int n, int a, int b, int& a2, int& b2) {
  int p = a, q = b;
  if (o & 4) std::swap(p, q);
  a2 = (o & 1) ? n - 1 - p : p;
  b2 = (o & 2) ? n - 1 - q : q;
}

// keys[e][8] -> nbr[e][6]; returns false on a non-manifold key set
bool connect(int64_t E, const std::vector<Key>& keys, int32_t* nbr) {
  std::unordered_map<FaceKey, int64_t, FaceKeyHash> open;
  open.reserve((size_t)E * 4);
  std::vector<int32_t> out((size_t)E * 6, INT32_MIN);
  auto face_keys = [&](int64_t e, int f) {
    FaceKey k;
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) k.c[a + 2 * b] = keys[e * 8 + corner_of(f, a, b)];
    std::sort(k.c.begin(), k.c.end());
    return k;
  };
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      FaceKey k = face_keys(e, f);
      auto it = open.find(k);
      if (it == open.end()) {
        open.emplace(k, e * 6 + f);
        continue;
      }
      const int64_t e2 = it->second / 6;
      const int f2 = (int)(it->second % 6);
      open.erase(it);
      // orientation from (e,f) to (e2,f2) and back, matched on corner keys
      int o12 = -1, o21 = -1;
      for (int o = 0; o < 8; ++o) {
        bool fw = true, bw = true;
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a) {
            int a2, b2;
            map_point(o, 2, a, b, a2, b2);
            fw = fw && keys[e * 8 + corner_of(f, a, b)] == keys[e2 * 8 + corner_of(f2, a2, b2)];
            bw = bw && keys[e2 * 8 + corner_of(f2, a, b)] == keys[e * 8 + corner_of(f, a2, b2)];
          }
        if (fw && o12 < 0) o12 = o;
        if (bw && o21 < 0) o21 = o;
      }
      if (o12 < 0 || o21 < 0 || out[e * 6 + f] != INT32_MIN || out[e2 * 6 + f2] != INT32_MIN)
        return false;
      out[e * 6 + f] = (int32_t)((e2 << 6) | (f2 << 3) | o12);
      out[e2 * 6 + f2] = (int32_t)((e << 6) | (f << 3) | o21);
    }
  int64_t nb = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f)
      if (out[e * 6 + f] == INT32_MIN) {
        const int group = f == 4 ? 0 : (f == 5 ? 1 : 2);
        out[e * 6 + f] = (int32_t)(-(1 + group + 4 * nb));
        ++nb;
      }
  std::memcpy(nbr, out.data(), sizeof(int32_t) * out.size());
  return true;
}

// cube-patch frame: the reference point (1, a, b) of patch P in 3-D
inline void patch_frame(int P, double one, double a, double b, double v[3]) {
  static const int perm[6][3] = {{0, 1, 2}, {1, 0, 2}, {0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {2, 1, 0}};
  // components: which slot receives (one, a, b), and the signs
  static const double sgn[6][3] = {{1, 1, 1}, {1, -1, 1}, {-1, -1, 1},
                                   {-1, 1, 1}, {1, 1, -1}, {-1, 1, 1}};
  double src[3] = {one, a, b};
  for (int s = 0; s < 3; ++s) v[perm[P][s]] = sgn[P][s] * src[s];
}

// tan(-pi/4 + s (pi/2)/Nz), exactly +-1 on the patch edges
inline double edge_tan(double s, int Nz) {
  if (s == 0.0) return -1.0;
  if (s == (double)Nz) return 1.0;
  return std::tan(-kPi / 4 + s * (kPi / 2) / Nz);
}

}  // namespace

// ---------------------------------------------------------------------------
// Public builders
// ---------------------------------------------------------------------------

// Symmetric outward normal at every element face point: n = (S_own - S_nbr)/2
// with S_out = +-S^d at the face (sign by the face side); on boundary faces
// n = S_own.  The two sides of an interior face get exact negatives.
static void face_normals(int N, int64_t E, const double* S_fp, const int32_t* nbr, double* n_face) {
  const int N2 = N * N, NF = (N + 1) * N2;
  auto fp_of = [N](int d, int f, int a, int b) {
    return d == 0 ? f + (N + 1) * (a + N * b) : (d == 1 ? a + N * (f + (N + 1) * b) : a + N * (b + N * f));
  };
  auto s_out = [&](int64_t e, int face, int a, int b, int c) {
    const int d = face >> 1, side = face & 1;
    const double v = S_fp[((e * 3 + d) * 3 + c) * NF + fp_of(d, side ? N : 0, a, b)];
    return side ? v : -v;
  };
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      const int32_t code = nbr[e * 6 + f];
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a)
          for (int c = 0; c < 3; ++c) {
            double v = s_out(e, f, a, b, c);
            if (code >= 0) {
              int a2, b2;
              map_point(code & 7, N, a, b, a2, b2);
              v = 0.5 * (v - s_out(code >> 6, (code >> 3) & 7, a2, b2, c));
            }
            n_face[((e * 6 + f) * 3 + c) * N2 + a + N * b] = v;
          }
    }
}

static int run_geometry(const Tables1D& t, int64_t E, const std::function<void(int64_t, Block3*)>& nodes,
                        double* x_sp, double* detJ, double* S_fp, double* S_sp) {
  const int N = t.N, NP = N + 1, N3 = N * N * N, NF = NP * N * N;
#pragma omp parallel for schedule(dynamic, 32)
  for (int64_t e = 0; e < E; ++e) {
    Block3 X[3] = {Block3(NP, NP, NP), Block3(NP, NP, NP), Block3(NP, NP, NP)};
    nodes(e, X);
    element_geometry(t, X, x_sp + e * 3 * N3, detJ + e * N3, S_fp + e * 9 * NF,
                     S_sp ? S_sp + e * 9 * N3 : nullptr);
  }
  return 0;
}

int shell_build(int Nz, int Nr, int p, double rb, double rt, double* x_sp, double* detJ,
                double* S_fp, double* S_sp, int32_t* nbr, double* n_face) {
  const Tables1D t = make_tables(p + 1);
  const int NP = p + 2;
  const int64_t E = 6LL * Nr * Nz * Nz;
  auto decode = [=](int64_t e, int& P, int& k, int& j, int& i) {
    i = (int)(e % Nz);
    j = (int)((e / Nz) % Nz);
    k = (int)((e / ((int64_t)Nz * Nz)) % Nr);
    P = (int)(e / ((int64_t)Nz * Nz * Nr));
  };
  std::vector<Key> keys((size_t)E * 8);
  for (int64_t e = 0; e < E; ++e) {
    int P, k, j, i;
    decode(e, P, k, j, i);
    for (int c = 0; c < 8; ++c) {
      const int ci = c & 1, cj = (c >> 1) & 1, ck = (c >> 2) & 1;
      double v[3];
      patch_frame(P, (double)Nz, (double)(2 * (i + ci) - Nz), (double)(2 * (j + cj) - Nz), v);
      keys[e * 8 + c] = {(int32_t)std::lround(v[0]), (int32_t)std::lround(v[1]),
                         (int32_t)std::lround(v[2]), k + ck};
    }
  }
  if (!connect(E, keys, nbr)) return -1;
  auto nodes = [&](int64_t e, Block3* X) {
    int P, k, j, i;
    decode(e, P, k, j, i);
    for (int c = 0; c < NP; ++c) {
      const double r = rb + (k + t.xf[c]) * (rt - rb) / Nr;
      for (int b = 0; b < NP; ++b) {
        const double tb = edge_tan(j + t.xf[b], Nz);
        for (int a = 0; a < NP; ++a) {
          const double ta = edge_tan(i + t.xf[a], Nz);
          double v[3];
          patch_frame(P, 1.0, ta, tb, v);
          const double s = r / std::sqrt(1.0 + ta * ta + tb * tb);  // patch-local order
          for (int q = 0; q < 3; ++q) X[q].at(a, b, c) = s * v[q];
        }
      }
    }
  };
  run_geometry(t, E, nodes, x_sp, detJ, S_fp, S_sp);
  if (n_face) face_normals(p + 1, E, S_fp, nbr, n_face);
  return 0;
}

int box_build(int nx, int ny, int nz, double Lx, double Ly, double Lz, int periodic, double warp,
              int p, double* x_sp, double* detJ, double* S_fp, double* S_sp, int32_t* nbr, double* n_face) {
  const Tables1D t = make_tables(p + 1);
  const int NP = p + 2;
  const int n[3] = {nx, ny, nz};
  const double L[3] = {Lx, Ly, Lz};
  const int64_t E = (int64_t)nx * ny * nz;
  std::vector<Key> keys((size_t)E * 8);
  for (int64_t e = 0; e < E; ++e) {
    const int idx[3] = {(int)(e % nx), (int)((e / nx) % ny), (int)(e / ((int64_t)nx * ny))};
    for (int c = 0; c < 8; ++c) {
      Key k{0, 0, 0, 0};
      for (int d = 0; d < 3; ++d) {
        const int v = idx[d] + ((c >> d) & 1);
        k[d] = ((periodic >> d) & 1) ? v % n[d] : v;
      }
      keys[e * 8 + c] = k;
    }
  }
  if (!connect(E, keys, nbr)) return -1;
  auto nodes = [&](int64_t e, Block3* X) {
    const int idx[3] = {(int)(e % nx), (int)((e / nx) % ny), (int)(e / ((int64_t)nx * ny))};
    for (int c = 0; c < NP; ++c)
      for (int b = 0; b < NP; ++b)
        for (int a = 0; a < NP; ++a) {
          const int ab[3] = {a, b, c};
          double y[3];
          for (int d = 0; d < 3; ++d) y[d] = (idx[d] + t.xf[ab[d]]) * L[d] / n[d];
          const double s = warp * std::sin(2 * kPi * y[0] / Lx) * std::sin(2 * kPi * y[1] / Ly) *
                           std::sin(2 * kPi * y[2] / Lz);
          for (int d = 0; d < 3; ++d) X[d].at(a, b, c) = y[d] + s * L[d];
        }
  };
  run_geometry(t, E, nodes, x_sp, detJ, S_fp, S_sp);
  if (n_face) face_normals(p + 1, E, S_fp, nbr, n_face);
  return 0;
}

void sph_bins(int64_t E, int N, const double* x_sp, double rb, double rt, int n_r, int n_th, int32_t* order,
              int64_t* offsets) {
  const int64_t N3 = (int64_t)N * N * N, n = E * N3, nb = (int64_t)n_r * n_th;
  std::vector<int32_t> bin(n);
  for (int64_t g = 0; g < n; ++g) {
    const int64_t e = g / N3, q = g % N3;
    const double x = x_sp[(e * 3 + 0) * N3 + q], y = x_sp[(e * 3 + 1) * N3 + q], z = x_sp[(e * 3 + 2) * N3 + q];
    const double r = std::sqrt(x * x + y * y + z * z), th = std::atan2(std::sqrt(x * x + y * y), z);
    int ir = (int)std::floor((r - rb) / (rt - rb) * n_r), it = (int)std::floor(th / kPi * n_th);
    ir = std::min(std::max(ir, 0), n_r - 1);
    it = std::min(std::max(it, 0), n_th - 1);
    bin[g] = ir * n_th + it;
  }
  // counting sort, stable in g
  std::fill(offsets, offsets + nb + 1, 0);
  for (int64_t g = 0; g < n; ++g) ++offsets[bin[g] + 1];
  for (int64_t b = 0; b < nb; ++b) offsets[b + 1] += offsets[b];
  std::vector<int64_t> next(offsets, offsets + nb);
  for (int64_t g = 0; g < n; ++g) order[next[bin[g]]++] = (int32_t)g;
}


// ---------------------------------------------------------------------------
// SSPRK(5,3) (Sec. "Spectral Difference Method": the time integrator is the
// five-stage, third-order strong-stability-preserving Runge-Kutta scheme)
// ---------------------------------------------------------------------------
// Shu-Osher coefficients u(i) = sum_k a_ik u(k) + dt b_ik L(u(k)) of the
// optimal scheme (SSP coefficient 2.6506): the published 14-digit values,
// with the b entries corrected by a minimal-norm Newton step (< 4e-10) so
// that the four third-order conditions hold in double precision.
static const double kSspA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0, 0, 0, 0, 0, 0},
    {0, 1.0, 0, 0, 0, 0},
    {0.56656131914032997754, 0, 0.43343868085967002246, 0, 0, 0},
    {0.09299483444412999511, 0.000020903696200000000053, 0, 0.90698426185967000489, 0, 0},
    {0.0073613226092000003456, 0.20127980325145000684, 0.0018295538968200000286, 0,
     0.78952932024252999279, 0}};
static const double kSspB[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.37726891519897837344, 0, 0, 0, 0, 0},
    {0, 0.37726891516114840825, 0, 0, 0, 0},
    {0, 0, 0.16352294101188272956, 0, 0, 0},
    {0.00071997350394151505236, 0, 0, 0.3421769684090429351, 0, 0},
    {0.0027771984070493497694, 0.000015679038088402258468, 0, 0, 0.29786487003033598351, 0}};

void ssprk53_stages(ShuOsherStage st[5], double c[5]) {
  const double(*a)[6] = kSspA;
  const double(*b)[6] = kSspB;
  // Stages 4 and 5 also need the residuals of u0 and u1.  Stages 1 and 2
  // have a single input of weight 1 (u1 = u0 + b10 dt L(u0), u2 = u1 +
  // b21 dt L(u1)), so those residuals are (u1 - u0)/(b10 dt) and
  // (u2 - u1)/(b21 dt): folding them into the weights of u0, u1, u2 leaves
  // one residual per stage and four registers (A = u0, B = u1, C = u2,
  // D = u3 then u4; the step's result replaces u0 in A).
  const double r0 = b[4][0] / b[1][0], s0 = b[5][0] / b[1][0], s1 = b[5][1] / b[2][1];
  enum { A = 0, B = 1, C = 2, D = 3 };
  auto set = [&](ShuOsherStage& x, int cur, std::initializer_list<std::pair<int, double>> in, double beta, int out) {
    x.cur = cur;
    x.n_in = 0;
    for (const auto& p : in) {
      x.in_idx[x.n_in] = p.first;
      x.alpha[x.n_in] = p.second;
      ++x.n_in;
    }
    for (int k = x.n_in; k < 4; ++k) {
      x.in_idx[k] = 0;
      x.alpha[k] = 0.0;
    }
    x.beta = beta;
    x.out = out;
  };
  set(st[0], A, {{A, a[1][0]}}, b[1][0], B);
  set(st[1], B, {{B, a[2][1]}}, b[2][1], C);
  set(st[2], C, {{A, a[3][0]}, {C, a[3][2]}}, b[3][2], D);
  set(st[3], D, {{A, a[4][0] - r0}, {B, a[4][1] + r0}, {D, a[4][3]}}, b[4][3], D);
  set(st[4], D, {{A, a[5][0] - s0}, {B, a[5][1] + s0 - s1}, {C, a[5][2] + s1}, {D, a[5][4]}}, b[5][4], A);
  // stage times from the equivalent Butcher rows: row i of the Butcher
  // matrix is sum_k a_ik (row k) + b_ik e_k, and c_i is its sum
  double Bt[6][5] = {{0}};
  for (int i = 1; i < 6; ++i)
    for (int k = 0; k < i; ++k) {
      for (int j = 0; j < 5; ++j) Bt[i][j] += a[i][k] * Bt[k][j];
      Bt[i][k] += b[i][k];
    }
  for (int i = 0; i < 5; ++i) {
    double s = 0.0;
    for (int j = 0; j < 5; ++j) s += Bt[i][j];
    c[i] = s;
  }
}

}  // namespace sdm

namespace sdm {

}  // namespace sdm

// ---------------------------------------------------------------------------
// initial background (Sec. "Initial Conditions")
// ---------------------------------------------------------------------------
namespace sdm {

namespace {

struct BgEval {
  const Background& b;
  double cp, T_b, p_b;
  explicit BgEval(const Background& bg) : b(bg) {
    cp = b.gamma * b.Rgas / (b.gamma - 1.0);
    T_b = (b.GM / b.rb - b.GM / b.rt) / (cp * (1.0 - std::exp(-(b.gamma - 1.0) * b.N_rho)));
    p_b = b.rho_b * b.Rgas * T_b;
  }
  // the polytrope: z = 1 - (Phi - Phi_b) / (C_p T_b), Phi = -GM / r
  double z(double r) const { return 1.0 - (b.GM / b.rb - b.GM / r) / (cp * T_b); }
  double kappa_r(double r) const {
    const double w = r * b.kr_w;
    return b.kr_scale * (b.kr_c0 + b.kr_c1 * w + b.kr_c2 * w * w);
  }
  // dS/dr from the outward heat flux L / (4 pi r^2) carried by entropy
  // diffusion and radiation through the polytrope
  double dSdr(double r) const {
    const double zz = z(r);
    const double rho0 = b.rho_b * std::pow(zz, 1.0 / (b.gamma - 1.0)), T0 = T_b * zz;
    const double dT0 = -b.GM / (cp * r * r);
    const double q = b.L / (4.0 * kPi * r * r);
    return -(q + kappa_r(r) * rho0 * cp * dT0) / (b.kappa * rho0 * T0);
  }
  // (S, rho)' of the hydrostatic profile with entropy S: p = rho^gamma exp(gamma S / C_p)
  void rhs(double r, const double y[2], double f[2]) const {
    const double s = dSdr(r);
    f[0] = s;
    f[1] = -(y[1] / cp) * s - (b.GM / (r * r) / b.gamma) * std::pow(y[1], 2.0 - b.gamma) *
                                  std::exp(-b.gamma * y[0] / cp);
  }
};

}  // namespace

int background_profile(const Background& b, int64_t n, const double* r, double* rho, double* p, double* T) {
  if (!(b.gamma > 1.0) || !(b.Rgas > 0.0) || !(b.GM > 0.0) || !(b.rb > 0.0) || !(b.rt > b.rb) ||
      !(b.rho_b > 0.0) || !(b.N_rho > 0.0) || n < 0)
    return 1;
  const double span = b.rt - b.rb;
  for (int64_t i = 0; i < n; ++i)
    if (!(r[i] >= b.rb - 1e-12 * span && r[i] <= b.rt + 1e-12 * span)) return 2;
  const BgEval ev(b);
  if (!b.flux_balanced) {
    for (int64_t i = 0; i < n; ++i) {
      const double zz = ev.z(r[i]);
      rho[i] = b.rho_b * std::pow(zz, 1.0 / (b.gamma - 1.0));
      p[i] = ev.p_b * std::pow(zz, b.gamma / (b.gamma - 1.0));
      T[i] = ev.T_b * zz;
    }
    return 0;
  }
  if (!(b.kappa > 0.0)) return 1;
  // classical RK4 on a uniform grid, then cubic Hermite interpolation with
  // the exact derivatives at the nodes (both fourth order, h = span / 2^14)
  const int M = 1 << 14;
  const double h = span / M;
  std::vector<double> Y(2 * (M + 1)), F(2 * (M + 1));
  Y[0] = ev.cp * std::log(std::pow(ev.p_b, 1.0 / b.gamma) / b.rho_b);  // S_b of the polytrope
  Y[1] = b.rho_b;
  ev.rhs(b.rb, &Y[0], &F[0]);
  for (int k = 0; k < M; ++k) {
    const double r0 = b.rb + k * h;
    const double* y = &Y[2 * k];
    double k1[2], k2[2], k3[2], k4[2], t[2];
    for (int c = 0; c < 2; ++c) k1[c] = F[2 * k + c];
    for (int c = 0; c < 2; ++c) t[c] = y[c] + 0.5 * h * k1[c];
    ev.rhs(r0 + 0.5 * h, t, k2);
    for (int c = 0; c < 2; ++c) t[c] = y[c] + 0.5 * h * k2[c];
    ev.rhs(r0 + 0.5 * h, t, k3);
    for (int c = 0; c < 2; ++c) t[c] = y[c] + h * k3[c];
    ev.rhs(r0 + h, t, k4);
    for (int c = 0; c < 2; ++c) Y[2 * (k + 1) + c] = y[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    if (!(Y[2 * (k + 1) + 1] > 0.0) || !std::isfinite(Y[2 * (k + 1)])) return 3;  // no hydrostatic profile
    ev.rhs(r0 + h, &Y[2 * (k + 1)], &F[2 * (k + 1)]);
  }
  for (int64_t i = 0; i < n; ++i) {
    const double x = std::min(std::max(r[i], b.rb), b.rt);
    int k = (int)std::floor((x - b.rb) / h);
    k = std::min(std::max(k, 0), M - 1);
    const double s = (x - (b.rb + k * h)) / h;
    const double h00 = (1.0 + 2.0 * s) * (1.0 - s) * (1.0 - s), h10 = s * (1.0 - s) * (1.0 - s);
    const double h01 = s * s * (3.0 - 2.0 * s), h11 = s * s * (s - 1.0);
    double y[2];
    for (int c = 0; c < 2; ++c)
      y[c] = h00 * Y[2 * k + c] + h10 * h * F[2 * k + c] + h01 * Y[2 * (k + 1) + c] + h11 * h * F[2 * (k + 1) + c];
    rho[i] = y[1];
    p[i] = std::pow(y[1], b.gamma) * std::exp(b.gamma * y[0] / ev.cp);
    T[i] = p[i] / (y[1] * b.Rgas);
  }
  return 0;
}

}  // namespace sdm
