/*
 * sdmhd_oracle.c -- TEST INFRASTRUCTURE ONLY (see sdmhd_oracle.h).
 *
 * Plain FP64 loops, one step of the paper's procedure at a time:
 *   1-D point sets and Lagrange bases   (Sec. Spectral Difference Method:
 *                                         solution/flux points, bases h_i, l_i)
 *   cubed-sphere shell mesh             (Sec. Meshing)
 *   element map, Jacobian, transformed  (Sec. Spectral Difference Method:
 *   equations                            mapping P, Jacobi matrix J, Eq. G.E. comp)
 *   fluxes and sources                  (Sec. MHD Governing Equations:
 *                                         Eqs. energy, ideal gas, M, invF, visF,
 *                                         ssTensor, qFlux, entropy)
 *   BR1 common solution, Rusanov common (Sec. Spectral Difference Method,
 *   flux, divergence                     last paragraphs)
 *   SSPRK(5,3)                          (same section; coefficients: the
 *                                         optimal five-stage third-order SSP
 *                                         scheme, see or_ssprk53_table)
 *   wall conditions                     (Sec. Problem Formulation and
 *                                         Boundary Conditions)
 *   KE / E_B diagnostics                (Sec. Results)
 * Where the paper is silent the readings used are stated next to the code.
 * Compile with -ffp-contract=off (no fused multiply-add) and no fast-math.
 */
#include "sdmhd_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 9  /* conserved variables rho, rho*u(3), E, B(3), psi */
#define NG 27 /* gradient components dQ_v/dx_j, index v*3+j */

/* ------------------------------------------------------------------ */
/* 1-D tables (Sec. Spectral Difference Method)                        */
/* ------------------------------------------------------------------ */

typedef struct {
  int N;
  double xs[OR_NMAX], xf[OR_NMAX + 1];
  double I[OR_NMAX + 1][OR_NMAX];     /* I[f][i]  = h_i(xf_f)            */
  double D[OR_NMAX][OR_NMAX + 1];     /* D[i][f]  = l_f'(xs_i)           */
  double L[OR_NMAX][OR_NMAX + 1];     /* L[i][f]  = l_f(xs_i)            */
  double Dn[OR_NMAX + 1][OR_NMAX + 1]; /* Dn[g][f] = l_f'(xf_g)           */
  double W[OR_NMAX];                  /* W[i] = integral over [0,1] of h_i */
} tab_t;

/* Legendre polynomial P_M and its derivative at t (three-term recurrence). */
static void legendre(int M, long double t, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = t;
  if (M == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 2; k <= M; ++k) {
    long double p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / k;
    p0 = p1; p1 = p2;
  }
  *P = p1;
  *dP = M * (t * p1 - p0) / (t * t - 1.0L);
}

/* Ascending roots of P_M on (-1,1) by Newton iteration in extended precision. */
static void legendre_roots(int M, long double* r) {
  for (int k = 0; k < M; ++k) {
    long double t = cosl(3.14159265358979323846264338327950288L * (k + 0.75L) / (M + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre(M, t, &P, &dP);
      long double dt = P / dP;
      t -= dt;
      if (fabsl(dt) < 1e-19L) break;
    }
    r[M - 1 - k] = t; /* cos(...) decreases with k */
  }
}

/* Lagrange basis on nodes x[0..n-1]: value of basis j at X. */
static long double lag(const long double* x, int n, int j, long double X) {
  long double v = 1.0L;
  for (int s = 0; s < n; ++s)
    if (s != j) v *= (X - x[s]) / (x[j] - x[s]);
  return v;
}
/* derivative of basis j at X */
static long double dlag(const long double* x, int n, int j, long double X) {
  long double sum = 0.0L;
  for (int m = 0; m < n; ++m) {
    if (m == j) continue;
    long double term = 1.0L / (x[j] - x[m]);
    for (int s = 0; s < n; ++s)
      if (s != j && s != m) term *= (X - x[s]) / (x[j] - x[s]);
    sum += term;
  }
  return sum;
}

static int build_tab(int N, tab_t* t) {
  if (N < 2 || N > OR_NMAX) return -1;
  const long double PI = 3.14159265358979323846264338327950288L;
  long double xs[OR_NMAX], xf[OR_NMAX + 1], roots[OR_NMAX];
  memset(t, 0, sizeof(*t));
  t->N = N;
  /* Chebyshev-Gauss solution points X_s,n = (1 - cos((2n-1)pi/(2N)))/2, n=1..N */
  for (int n = 0; n < N; ++n) xs[n] = 0.5L * (1.0L - cosl((2.0L * n + 1.0L) * PI / (2.0L * N)));
  /* Flux points: the end points 0 and 1 plus the N-1 roots of the Legendre
   * polynomial of degree N-1 mapped to [0,1] -- N+1 points in all (the
   * count the (N+1)-point flux polynomial of the section requires). */
  legendre_roots(N - 1, roots);
  xf[0] = 0.0L;
  for (int k = 0; k < N - 1; ++k) xf[k + 1] = 0.5L * (1.0L + roots[k]);
  xf[N] = 1.0L;
  for (int n = 0; n < N; ++n) t->xs[n] = (double)xs[n];
  for (int f = 0; f <= N; ++f) t->xf[f] = (double)xf[f];
  for (int f = 0; f <= N; ++f)
    for (int i = 0; i < N; ++i) t->I[f][i] = (double)lag(xs, N, i, xf[f]);
  for (int i = 0; i < N; ++i)
    for (int f = 0; f <= N; ++f) {
      t->D[i][f] = (double)dlag(xf, N + 1, f, xs[i]);
      t->L[i][f] = (double)lag(xf, N + 1, f, xs[i]);
    }
  for (int g = 0; g <= N; ++g)
    for (int f = 0; f <= N; ++f) t->Dn[g][f] = (double)dlag(xf, N + 1, f, xf[g]);
  /* W_i = integral of h_i over [0,1]; 8-point Gauss-Legendre is exact for
   * the degree N-1 <= 7 integrand. */
  long double gr[8];
  legendre_roots(8, gr);
  for (int i = 0; i < N; ++i) {
    long double s = 0.0L;
    for (int q = 0; q < 8; ++q) {
      long double P, dP;
      legendre(8, gr[q], &P, &dP);
      long double w = 2.0L / ((1.0L - gr[q] * gr[q]) * dP * dP);
      s += 0.5L * w * lag(xs, N, i, 0.5L * (1.0L + gr[q]));
    }
    t->W[i] = (double)s;
  }
  return 0;
}

int or_tables(int N, double* xs, double* xf, double* I, double* D, double* W) {
  tab_t t;
  if (build_tab(N, &t)) return -1;
  for (int i = 0; i < N; ++i) xs[i] = t.xs[i];
  for (int f = 0; f <= N; ++f) xf[f] = t.xf[f];
  for (int f = 0; f <= N; ++f)
    for (int i = 0; i < N; ++i) I[f * N + i] = t.I[f][i];
  for (int i = 0; i < N; ++i)
    for (int f = 0; f <= N; ++f) D[i * (N + 1) + f] = t.D[i][f];
  for (int i = 0; i < N; ++i) W[i] = t.W[i];
  return 0;
}

/* ------------------------------------------------------------------ */
/* Mesh                                                                */
/* ------------------------------------------------------------------ */

struct or_mesh {
  int N;
  int64_t E, F, NB;
  tab_t t;
  double* xn;   /* [E][3][(N+1)^3] map nodes at the flux-point tensor grid  */
  double* xsp;  /* [E][3][N^3]                                              */
  double* detJ; /* [E][N^3]                                                 */
  double* Ssp;  /* [E][3][3][N^3]   S^d_x = |J| (J^-1)_{d x} at SPs         */
  double* Sfp;  /* [E][3][3][(N+1)N^2] S^d at the family-d flux points      */
  int32_t* faces; /* [F][5] */
  int32_t* nbr;   /* [E][6][3]: (e', f', orient) or (-1-group, bface, 0)    */
  int32_t* bface_ef; /* [NB][2] (e, f) of each boundary face                */
};

/* index helpers (i fastest) */
#define SP(N, a, b, c) ((a) + (N) * ((b) + (N) * (c)))
/* family-d flux point with flux index f along d and SP indices (a,b) on the
 * two remaining axes in increasing order */
static int fp_index(int N, int d, int f, int a, int b) {
  if (d == 0) return f + (N + 1) * (a + N * b);
  if (d == 1) return a + N * (f + (N + 1) * b);
  return a + N * (b + N * f);
}
/* solution point at position i along the family-d line (a,b) */
static int sp_on_line(int N, int d, int a, int b, int i) {
  if (d == 0) return SP(N, i, a, b);
  if (d == 1) return SP(N, a, i, b);
  return SP(N, a, b, i);
}

/* Apply a 1-D matrix M (rows x n_axis, row-major) along `axis` of the 3-D
 * array `in` with extents n[3] (axis 0 fastest). */
static void apply1d(const double* in, const int n[3], int axis, const double* M,
                    int rows, double* out) {
  int m[3] = {n[0], n[1], n[2]};
  m[axis] = rows;
  for (int c = 0; c < m[2]; ++c)
    for (int b = 0; b < m[1]; ++b)
      for (int a = 0; a < m[0]; ++a) {
        int o[3] = {a, b, c};
        double s = 0.0;
        for (int k = 0; k < n[axis]; ++k) {
          int ii[3] = {a, b, c};
          ii[axis] = k;
          s += M[o[axis] * n[axis] + k] * in[ii[0] + n[0] * (ii[1] + n[1] * ii[2])];
        }
        out[a + m[0] * (b + m[1] * c)] = s;
      }
}

/* Evaluate a field given on the (N+1)^3 map nodes: per axis choose identity
 * (keep the node index), L (value at SPs) or Dsp (derivative at SPs). */
enum { OP_ID = 0, OP_L = 1, OP_D = 2 };
static void eval_nodes(const tab_t* t, const double* w, const int op[3], double* out) {
  const int N = t->N, NP = N + 1;
  double Lm[OR_NMAX * (OR_NMAX + 1)], Dm[OR_NMAX * (OR_NMAX + 1)];
  for (int i = 0; i < N; ++i)
    for (int f = 0; f < NP; ++f) { Lm[i * NP + f] = t->L[i][f]; Dm[i * NP + f] = t->D[i][f]; }
  double b1[(OR_NMAX + 1) * (OR_NMAX + 1) * (OR_NMAX + 1)];
  double b2[(OR_NMAX + 1) * (OR_NMAX + 1) * (OR_NMAX + 1)];
  int n[3] = {NP, NP, NP};
  const double* cur = w;
  double* bufs[2] = {b1, b2};
  int which = 0;
  for (int ax = 0; ax < 3; ++ax) {
    if (op[ax] == OP_ID) continue;
    const double* M = op[ax] == OP_L ? Lm : Dm;
    apply1d(cur, n, ax, M, N, bufs[which]);
    n[ax] = N;
    cur = bufs[which];
    which ^= 1;
  }
  memcpy(out, cur, sizeof(double) * n[0] * n[1] * n[2]);
}

/* Patch frames of the cubed sphere: (1,a,b) on the reference face is sent
 * to R_P(1,a,b); all six are right-handed in (xi,eta,zeta). */
static void patch_vec(int P, double one, double a, double b, double* v) {
  switch (P) {
    case 0: v[0] = one; v[1] = a; v[2] = b; break;      /* +x */
    case 1: v[0] = -a; v[1] = one; v[2] = b; break;     /* +y */
    case 2: v[0] = -one; v[1] = -a; v[2] = b; break;    /* -x */
    case 3: v[0] = a; v[1] = -one; v[2] = b; break;     /* -y */
    case 4: v[0] = -b; v[1] = a; v[2] = one; break;     /* +z */
    default: v[0] = b; v[1] = a; v[2] = -one; break;    /* -z */
  }
}

/* tan of the equiangular coordinate -pi/4 + s*(pi/2)/Nz for s in [0, Nz];
 * the patch edges s = 0, Nz give exactly -1, +1 */
static double equiangular_tan(double s, int Nz) {
  const double PI = 3.14159265358979323846;
  if (s == 0.0) return -1.0;
  if (s == (double)Nz) return 1.0;
  return tan(-PI / 4 + s * (PI / 2) / Nz);
}

typedef struct { int32_t k[4][4]; int32_t e, f; } facerec;

static int key_cmp4(const int32_t* a, const int32_t* b) {
  for (int i = 0; i < 4; ++i) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}
static int facerec_cmp(const void* pa, const void* pb) {
  const facerec* a = (const facerec*)pa;
  const facerec* b = (const facerec*)pb;
  for (int i = 0; i < 4; ++i) {
    int c = key_cmp4(a->k[i], b->k[i]);
    if (c) return c;
  }
  if (a->e != b->e) return a->e < b->e ? -1 : 1;
  return a->f - b->f;
}
/* element corner index (cx + 2cy + 4cz) of face f at face-local corner (a,b) */
static int face_corner(int f, int a, int b) {
  int d = f / 2, s = f % 2;
  if (d == 0) return s + 2 * a + 4 * b;
  if (d == 1) return a + 2 * s + 4 * b;
  return a + 2 * b + 4 * s;
}
/* orientation code o = 4*swap + 2*flip_b + flip_a: face-local (a,b) on one
 * side becomes (a2,b2) on the other */
static void orient_map(int o, int n, int a, int b, int* a2, int* b2) {
  int p = (o & 4) ? b : a, q = (o & 4) ? a : b;
  *a2 = (o & 1) ? n - 1 - p : p;
  *b2 = (o & 2) ? n - 1 - q : q;
}

static void sort4(int32_t k[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (key_cmp4(k[j], k[i]) < 0) {
        int32_t tmp[4];
        memcpy(tmp, k[i], sizeof tmp); memcpy(k[i], k[j], sizeof tmp); memcpy(k[j], tmp, sizeof tmp);
      }
}

/* Build faces/neighbours from integer corner keys ckey[E][8][4]. */
static int build_faces(or_mesh* m, const int32_t* ckey) {
  const int64_t E = m->E;
  facerec* r = (facerec*)malloc(sizeof(facerec) * E * 6);
  if (!r) return -1;
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      facerec* x = &r[e * 6 + f];
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a)
          memcpy(x->k[a + 2 * b], &ckey[(e * 8 + face_corner(f, a, b)) * 4], 4 * sizeof(int32_t));
      sort4(x->k);
      x->e = (int32_t)e; x->f = f;
    }
  qsort(r, E * 6, sizeof(facerec), facerec_cmp);
  m->nbr = (int32_t*)malloc(sizeof(int32_t) * E * 18);
  for (int64_t i = 0; i < E * 18; ++i) m->nbr[i] = 0;
  int8_t* matched = (int8_t*)calloc(E * 6, 1);
  int32_t* fl = (int32_t*)malloc(sizeof(int32_t) * 5 * E * 6);
  int64_t nf = 0;
  for (int64_t i = 0; i < E * 6; ) {
    int64_t j = i + 1;
    while (j < E * 6 && memcmp(r[j].k, r[i].k, sizeof r[i].k) == 0) ++j;
    if (j - i == 2) {
      int eL = r[i].e, fL = r[i].f, eR = r[i + 1].e, fR = r[i + 1].f;
      int found = -1;
      for (int o = 0; o < 8 && found < 0; ++o) {
        int ok = 1;
        for (int b = 0; b < 2 && ok; ++b)
          for (int a = 0; a < 2 && ok; ++a) {
            int a2, b2;
            orient_map(o, 2, a, b, &a2, &b2);
            if (key_cmp4(&ckey[((int64_t)eL * 8 + face_corner(fL, a, b)) * 4],
                         &ckey[((int64_t)eR * 8 + face_corner(fR, a2, b2)) * 4]) != 0) ok = 0;
          }
        if (ok) found = o;
      }
      if (found < 0) { free(r); free(matched); free(fl); return -2; }
      /* inverse orientation: R's (a,b) -> L's */
      int inv = -1;
      for (int o = 0; o < 8 && inv < 0; ++o) {
        int ok = 1;
        for (int b = 0; b < 2 && ok; ++b)
          for (int a = 0; a < 2 && ok; ++a) {
            int a2, b2, a3, b3;
            orient_map(found, 2, a, b, &a2, &b2);
            orient_map(o, 2, a2, b2, &a3, &b3);
            if (a3 != a || b3 != b) ok = 0;
          }
        if (ok) inv = o;
      }
      int32_t* F = &fl[nf * 5];
      F[0] = eL; F[1] = fL; F[2] = eR; F[3] = fR; F[4] = found;
      ++nf;
      int32_t* nl = &m->nbr[((int64_t)eL * 6 + fL) * 3];
      nl[0] = eR; nl[1] = fR; nl[2] = found;
      int32_t* nr = &m->nbr[((int64_t)eR * 6 + fR) * 3];
      nr[0] = eL; nr[1] = fL; nr[2] = inv;
      matched[(int64_t)eL * 6 + fL] = matched[(int64_t)eR * 6 + fR] = 1;
    } else if (j - i > 2) {
      free(r); free(matched); free(fl); return -3;
    }
    i = j;
  }
  /* boundary faces, numbered in (element, face) order */
  int64_t nb = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f)
      if (!matched[e * 6 + f]) ++nb;
  m->NB = nb;
  m->bface_ef = (int32_t*)malloc(sizeof(int32_t) * 2 * (nb > 0 ? nb : 1));
  nb = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f)
      if (!matched[e * 6 + f]) {
        int group = f == 4 ? 0 : (f == 5 ? 1 : 2);
        int32_t* nl = &m->nbr[(e * 6 + f) * 3];
        nl[0] = -1 - group; nl[1] = (int32_t)nb; nl[2] = 0;
        int32_t* F = &fl[nf * 5];
        F[0] = (int32_t)e; F[1] = f; F[2] = -1 - group; F[3] = (int32_t)nb; F[4] = 0;
        m->bface_ef[nb * 2] = (int32_t)e; m->bface_ef[nb * 2 + 1] = f;
        ++nf; ++nb;
      }
  m->F = nf;
  m->faces = (int32_t*)realloc(fl, sizeof(int32_t) * 5 * nf);
  free(r); free(matched);
  return 0;
}

/* Metrics of one element from its map nodes (isoparametric map of degree N
 * through the (N+1)^3 flux-point tensor nodes; curl form of the metric
 * terms |J| J^-1, so that sum_d d/dxi_d S^d = 0 holds for the discrete
 * operators; Sec. Spectral Difference Method, Jacobi matrix and
 * Eq. G.E. comp). */
static void element_metrics(or_mesh* m, int64_t e) {
  const tab_t* t = &m->t;
  const int N = t->N, NP = N + 1, N3 = N * N * N, NPn = NP * NP * NP, NF = NP * N * N;
  const double* Xa = &m->xn[e * 3 * NPn];
  /* The metric terms, the map derivatives and |J| do not change when the
   * element is translated (the discrete curl of a discrete gradient is zero
   * for tensor-product polynomials), so they are formed from the node
   * positions relative to the element's first node: with coordinates of
   * size h instead of 1 their round-off scales like the terms themselves. */
  double* X = (double*)malloc(sizeof(double) * 3 * NPn);
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < NPn; ++q) X[c * NPn + q] = Xa[c * NPn + q] - Xa[c * NPn];
  double Dn[(OR_NMAX + 1) * (OR_NMAX + 1)];
  for (int g = 0; g < NP; ++g)
    for (int f = 0; f < NP; ++f) Dn[g * NP + f] = t->Dn[g][f];
  /* derivatives of the map at the nodes: dX[k][comp] */
  double* dX = (double*)malloc(sizeof(double) * 9 * NPn);
  int n3[3] = {NP, NP, NP};
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) apply1d(&X[c * NPn], n3, k, Dn, NP, &dX[(k * 3 + c) * NPn]);
  double* Wn = (double*)malloc(sizeof(double) * NPn);
  double* tmp = (double*)malloc(sizeof(double) * NPn);
  for (int n = 0; n < 3; ++n) {
    int mm = (n + 1) % 3, l = (n + 2) % 3;
    /* W^n_k = (X_l dX_m/dxi_k - X_m dX_l/dxi_k)/2 at the nodes, k = 0,1,2
     * (invariant curl form: unchanged under signed permutations of the
     * coordinates, so rotated meshes get exactly rotated metrics) */
    double* Wk[3];
    for (int k = 0; k < 3; ++k) {
      Wk[k] = (double*)malloc(sizeof(double) * NPn);
      for (int q = 0; q < NPn; ++q)
        Wk[k][q] = 0.5 * (X[l * NPn + q] * dX[(k * 3 + mm) * NPn + q] -
                          X[mm * NPn + q] * dX[(k * 3 + l) * NPn + q]);
    }
    for (int i = 0; i < 3; ++i) {
      int j = (i + 1) % 3, k = (i + 2) % 3;
      /* S^i_n = d/dxi_k W^n_j - d/dxi_j W^n_k at family-i flux points */
      int opA[3], opB[3];
      for (int ax = 0; ax < 3; ++ax) { opA[ax] = OP_L; opB[ax] = OP_L; }
      opA[i] = OP_ID; opB[i] = OP_ID;
      opA[k] = OP_D; opB[j] = OP_D;
      double* outF = &m->Sfp[((e * 3 + i) * 3 + n) * NF];
      eval_nodes(t, Wk[j], opA, tmp);
      double* t2 = (double*)malloc(sizeof(double) * NPn);
      eval_nodes(t, Wk[k], opB, t2);
      for (int q = 0; q < NF; ++q) outF[q] = tmp[q] - t2[q];
      /* and at the solution points */
      opA[i] = OP_L; opB[i] = OP_L;
      double* outS = &m->Ssp[((e * 3 + i) * 3 + n) * N3];
      eval_nodes(t, Wk[j], opA, tmp);
      eval_nodes(t, Wk[k], opB, t2);
      for (int q = 0; q < N3; ++q) outS[q] = tmp[q] - t2[q];
      free(t2);
    }
    for (int k = 0; k < 3; ++k) free(Wk[k]);
  }
  /* positions and Jacobian determinant at the solution points */
  int opL[3] = {OP_L, OP_L, OP_L};
  for (int c = 0; c < 3; ++c) eval_nodes(t, &Xa[c * NPn], opL, &m->xsp[(e * 3 + c) * N3]);
  double* Jm = (double*)malloc(sizeof(double) * 9 * N3); /* Jm[c][k] = dx_c/dxi_k */
  for (int k = 0; k < 3; ++k) {
    int op[3] = {OP_L, OP_L, OP_L};
    op[k] = OP_D;
    for (int c = 0; c < 3; ++c) eval_nodes(t, &X[c * NPn], op, &Jm[(c * 3 + k) * N3]);
  }
  for (int q = 0; q < N3; ++q) {
    double a[3][3];
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < 3; ++k) a[c][k] = Jm[(c * 3 + k) * N3 + q];
    m->detJ[e * N3 + q] = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                          a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                          a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  }
  free(Jm); free(dX); free(Wn); free(tmp); free(X);
}

static or_mesh* mesh_alloc(int N, int64_t E) {
  or_mesh* m = (or_mesh*)calloc(1, sizeof(or_mesh));
  if (!m) return NULL;
  if (build_tab(N, &m->t)) { free(m); return NULL; }
  m->N = N; m->E = E;
  const int NP = N + 1;
  m->xn = (double*)malloc(sizeof(double) * E * 3 * NP * NP * NP);
  m->xsp = (double*)malloc(sizeof(double) * E * 3 * N * N * N);
  m->detJ = (double*)malloc(sizeof(double) * E * N * N * N);
  m->Ssp = (double*)malloc(sizeof(double) * E * 9 * N * N * N);
  m->Sfp = (double*)malloc(sizeof(double) * E * 9 * NP * N * N);
  if (!m->xn || !m->xsp || !m->detJ || !m->Ssp || !m->Sfp) { or_mesh_free(m); return NULL; }
  return m;
}

static int mesh_finish(or_mesh* m, const int32_t* ckey) {
  if (build_faces(m, ckey)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t e = 0; e < m->E; ++e) element_metrics(m, e);
  return 0;
}

or_mesh* or_shell_new(int N, int Nz, int Nr, double rb, double rt) {
  if (Nz < 1 || Nr < 1 || !(rt > rb) || !(rb > 0)) return NULL;
  const int64_t E = 6LL * Nz * Nz * Nr;
  or_mesh* m = mesh_alloc(N, E);
  if (!m) return NULL;
  const int NP = N + 1, NPn = NP * NP * NP;
  const double PI = 3.14159265358979323846;
  int32_t* ckey = (int32_t*)malloc(sizeof(int32_t) * E * 32);
  for (int P = 0; P < 6; ++P)
    for (int k = 0; k < Nr; ++k)
      for (int j = 0; j < Nz; ++j)
        for (int i = 0; i < Nz; ++i) {
          int64_t e = (((int64_t)P * Nr + k) * Nz + j) * Nz + i;
          /* Sec. Meshing: equiangular alpha, beta on each cube face; radial
           * layers uniform in r (the map is then linear in zeta) */
          for (int c = 0; c < NP; ++c)
            for (int b = 0; b < NP; ++b)
              for (int a = 0; a < NP; ++a) {
                double ta = equiangular_tan(i + m->t.xf[a], Nz);
                double tb = equiangular_tan(j + m->t.xf[b], Nz);
                double r = rb + (k + m->t.xf[c]) * (rt - rb) / Nr;
                double v[3];
                patch_vec(P, 1.0, ta, tb, v);
                /* summed in patch-local order so that points shared by two
                 * patches get bit-identical coordinates */
                double nv = sqrt(1.0 + ta * ta + tb * tb);
                for (int q = 0; q < 3; ++q)
                  m->xn[(e * 3 + q) * NPn + a + NP * (b + NP * c)] = r * v[q] / nv;
              }
          /* integer corner keys: cube-surface lattice point and radial layer */
          for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
              for (int cx = 0; cx < 2; ++cx) {
                double v[3];
                patch_vec(P, (double)Nz, (double)(2 * (i + cx) - Nz), (double)(2 * (j + cy) - Nz), v);
                int32_t* K = &ckey[(e * 8 + cx + 2 * cy + 4 * cz) * 4];
                K[0] = (int32_t)lround(v[0]); K[1] = (int32_t)lround(v[1]);
                K[2] = (int32_t)lround(v[2]); K[3] = k + cz;
              }
        }
  int rc = mesh_finish(m, ckey);
  free(ckey);
  if (rc) { or_mesh_free(m); return NULL; }
  return m;
}

or_mesh* or_box_new(int N, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                    int periodic, double warp) {
  int n[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || ((periodic >> d) & 1 && n[d] < 3)) return NULL; /* keys need 3 */
  const int64_t E = (int64_t)nx * ny * nz;
  or_mesh* m = mesh_alloc(N, E);
  if (!m) return NULL;
  const int NP = N + 1, NPn = NP * NP * NP;
  const double PI = 3.14159265358979323846;
  double Lv[3] = {Lx, Ly, Lz};
  int32_t* ckey = (int32_t*)malloc(sizeof(int32_t) * E * 32);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t e = ((int64_t)k * ny + j) * nx + i;
        int ijk[3] = {i, j, k};
        for (int c = 0; c < NP; ++c)
          for (int b = 0; b < NP; ++b)
            for (int a = 0; a < NP; ++a) {
              int ab[3] = {a, b, c};
              double X[3];
              for (int d = 0; d < 3; ++d) X[d] = (ijk[d] + m->t.xf[ab[d]]) * Lv[d] / n[d];
              /* smooth periodic warp of the whole box (curvilinear test meshes) */
              double s = warp * sin(2 * PI * X[0] / Lx) * sin(2 * PI * X[1] / Ly) * sin(2 * PI * X[2] / Lz);
              for (int d = 0; d < 3; ++d)
                m->xn[(e * 3 + d) * NPn + a + NP * (b + NP * c)] = X[d] + s * Lv[d];
            }
        for (int cz = 0; cz < 2; ++cz)
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              int cc[3] = {i + cx, j + cy, k + cz};
              int32_t* K = &ckey[(e * 8 + cx + 2 * cy + 4 * cz) * 4];
              for (int d = 0; d < 3; ++d) K[d] = ((periodic >> d) & 1) ? cc[d] % n[d] : cc[d];
              K[3] = 0;
            }
      }
  int rc = mesh_finish(m, ckey);
  free(ckey);
  if (rc) { or_mesh_free(m); return NULL; }
  return m;
}

void or_mesh_free(or_mesh* m) {
  if (!m) return;
  free(m->xn); free(m->xsp); free(m->detJ); free(m->Ssp); free(m->Sfp);
  free(m->faces); free(m->nbr); free(m->bface_ef);
  free(m);
}

void or_mesh_sizes(const or_mesh* m, int64_t* o) {
  o[0] = m->E; o[1] = m->F; o[2] = m->NB; o[3] = m->N;
}

int or_mesh_get(const or_mesh* m, const char* name, void* out) {
  const int N = m->N, NP = N + 1, N3 = N * N * N, NF = NP * N * N, NPn = NP * NP * NP;
  const int64_t E = m->E;
  if (!strcmp(name, "x_sp")) { memcpy(out, m->xsp, sizeof(double) * E * 3 * N3); return 0; }
  if (!strcmp(name, "detJ_sp")) { memcpy(out, m->detJ, sizeof(double) * E * N3); return 0; }
  if (!strcmp(name, "S_sp")) { memcpy(out, m->Ssp, sizeof(double) * E * 9 * N3); return 0; }
  if (!strcmp(name, "S_fp")) { memcpy(out, m->Sfp, sizeof(double) * E * 9 * NF); return 0; }
  if (!strcmp(name, "faces")) { memcpy(out, m->faces, sizeof(int32_t) * 5 * m->F); return 0; }
  if (!strcmp(name, "nbr")) { memcpy(out, m->nbr, sizeof(int32_t) * 18 * E); return 0; }
  if (!strcmp(name, "W3detJ")) {
    double* o = (double*)out;
    for (int64_t e = 0; e < E; ++e)
      for (int c = 0; c < N; ++c)
        for (int b = 0; b < N; ++b)
          for (int a = 0; a < N; ++a) {
            int q = SP(N, a, b, c);
            o[e * N3 + q] = m->t.W[a] * m->t.W[b] * m->t.W[c] * m->detJ[e * N3 + q];
          }
    return 0;
  }
  if (!strcmp(name, "x_bfp")) {
    double* o = (double*)out;
    double* tmp = (double*)malloc(sizeof(double) * NPn);
    for (int64_t bi = 0; bi < m->NB; ++bi) {
      int64_t e = m->bface_ef[bi * 2];
      int f = m->bface_ef[bi * 2 + 1], d = f / 2, s = f % 2;
      int op[3] = {OP_L, OP_L, OP_L};
      op[d] = OP_ID;
      for (int c = 0; c < 3; ++c) {
        eval_nodes(&m->t, &m->xn[(e * 3 + c) * NPn], op, tmp);
        for (int b = 0; b < N; ++b)
          for (int a = 0; a < N; ++a)
            o[(bi * 3 + c) * N * N + a + N * b] = tmp[fp_index(N, d, s ? N : 0, a, b)];
      }
    }
    free(tmp);
    return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* Pointwise physics (Sec. MHD Governing Equations)                    */
/* ------------------------------------------------------------------ */

#include "sdmhd_oracle_point.inc"

/* ------------------------------------------------------------------ */
/* Wall and Dirichlet faces (Sec. Problem Formulation and Boundary       */
/* Conditions).  nh is the outward unit normal of the domain.           */
/* ------------------------------------------------------------------ */

/* common solution at a wall: tangential velocity (impenetrable), B_r = 0
 * (conducting) or B purely normal (radial), pressure kept (heat-flux wall)
 * or set from the wall temperature (fixed-temperature wall) */
static void wall_common(const double* q, const double* nh, int g, const or_params* P, double* qc) {
  double rho = q[0];
  double u[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
  double un = u[0] * nh[0] + u[1] * nh[1] + u[2] * nh[2];
  double Bn = q[5] * nh[0] + q[6] * nh[1] + q[7] * nh[2];
  double uc[3], Bc[3];
  for (int i = 0; i < 3; ++i) {
    uc[i] = u[i] - un * nh[i];
    Bc[i] = P->wall_mag[g] == 0 ? q[5 + i] - Bn * nh[i] : Bn * nh[i];
  }
  double p = P->wall_th[g] == 0 ? pressure(q, P) : rho * P->Rgas * P->T_wall[g];
  qc[0] = rho;
  for (int i = 0; i < 3; ++i) { qc[1 + i] = rho * uc[i]; qc[5 + i] = Bc[i]; }
  /* cleaning field: reflected at a conducting wall (B_n = 0 is imposed
   * there), held at zero at a radial-field wall (B_n passes freely, so the
   * GLM pair needs its condition on psi) */
  qc[8] = P->wall_mag[g] == 0 ? q[8] : 0.0;
  qc[4] = p / (P->gamma - 1.0) + 0.5 * rho * (uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]) +
          0.5 * (Bc[0] * Bc[0] + Bc[1] * Bc[1] + Bc[2] * Bc[2]) + 0.5 * qc[8] * qc[8];
}

/* mirror state for the wall Rusanov flux: normal momentum reversed, B
 * mirrored (conducting) or anti-mirrored with psi reversed (radial); rho and
 * E unchanged (|u|, |B|, psi^2 are preserved) */
static void wall_ghost(const double* q, const double* nh, int g, const or_params* P, double* qg) {
  double mn = q[1] * nh[0] + q[2] * nh[1] + q[3] * nh[2];
  double Bn = q[5] * nh[0] + q[6] * nh[1] + q[7] * nh[2];
  qg[0] = q[0]; qg[4] = q[4];
  qg[8] = P->wall_mag[g] == 0 ? q[8] : -q[8];
  for (int i = 0; i < 3; ++i) {
    qg[1 + i] = q[1 + i] - 2.0 * mn * nh[i];
    qg[5 + i] = P->wall_mag[g] == 0 ? q[5 + i] - 2.0 * Bn * nh[i] : 2.0 * Bn * nh[i] - q[5 + i];
  }
}

/* total common flux (outward, through the unnormalised outward normal n) at
 * a wall point with interior state q and interior gradient G */
static void wall_flux(const double* q, const double* G, double kr, const double* n, int g,
                      const or_params* P, double* F) {
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
  double qg[NV], qc[NV], Fi[NV];
  wall_ghost(q, nh, g, P, qg);
  rusanov(q, qg, n, P, Fi);
  wall_common(q, nh, g, P, qc);
  visc_t v;
  visc_state(qc, G, kr, P, &v);
  double tn[3];
  for (int i = 0; i < 3; ++i) tn[i] = v.tau[i][0] * n[0] + v.tau[i][1] * n[1] + v.tau[i][2] * n[2];
  /* stress-free: only the normal traction survives; it does no work on the
   * tangential wall velocity */
  double tnn = tn[0] * nh[0] + tn[1] * nh[1] + tn[2] * nh[2];
  double Fv[NV];
  Fv[0] = 0.0; Fv[8] = 0.0;
  for (int i = 0; i < 3; ++i) Fv[1 + i] = tnn * nh[i];
  /* heat: prescribed outward-radial flux density, or computed at fixed T */
  double qn;
  if (P->wall_th[g] == 0) qn = P->q_wall[g] * (g == 0 ? -1.0 : 1.0) * nn;
  else qn = v.q[0] * n[0] + v.q[1] * n[1] + v.q[2] * n[2];
  /* current: conducting wall keeps only J_r; radial-field wall drops J_r */
  double Jn = v.J[0] * nh[0] + v.J[1] * nh[1] + v.J[2] * nh[2];
  double Jc[3];
  for (int i = 0; i < 3; ++i) Jc[i] = P->wall_mag[g] == 0 ? Jn * nh[i] : v.J[i] - Jn * nh[i];
  double BxJ[3] = {v.B[1] * Jc[2] - v.B[2] * Jc[1], v.B[2] * Jc[0] - v.B[0] * Jc[2],
                   v.B[0] * Jc[1] - v.B[1] * Jc[0]};
  Fv[4] = -qn + P->eta * (BxJ[0] * n[0] + BxJ[1] * n[1] + BxJ[2] * n[2]);
  Fv[5] = P->eta * (Jc[1] * n[2] - Jc[2] * n[1]);
  Fv[6] = P->eta * (Jc[2] * n[0] - Jc[0] * n[2]);
  Fv[7] = P->eta * (Jc[0] * n[1] - Jc[1] * n[0]);
  for (int k = 0; k < NV; ++k) F[k] = Fi[k] - Fv[k];
}

/* ------------------------------------------------------------------ */
/* Residual                                                            */
/* ------------------------------------------------------------------ */

static double kr_at(const double* x, const or_params* P) {
  if (P->kr_scale == 0.0) return 0.0;
  double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double w = r * P->kr_omega_per_r;
  return P->kr_scale * (P->kr_c0 + P->kr_c1 * w + P->kr_c2 * w * w);
}

/* outward unnormalised normal of face f at face-local point (a,b) */
static void face_normal(const or_mesh* m, int64_t e, int f, int a, int b, double* n) {
  const int N = m->N, NF = (N + 1) * N * N;
  int d = f / 2, s = f % 2;
  int idx = fp_index(N, d, s ? N : 0, a, b);
  for (int c = 0; c < 3; ++c) {
    double v = m->Sfp[((e * 3 + d) * 3 + c) * NF + idx];
    n[c] = s ? v : -v;
  }
}

/* Magnitude of the inputs of a common flux (for the round-off scale of the
 * residual): |F(qL).n| + |F(qR).n| + lambda|n|(|qL| + |qR|) + |viscous|, halved. */
static void face_abs(const double* qL, const double* qR, const double* FvL, const double* FvR,
                     const double* n, const or_params* P, double* FA) {
  double FL[NV], FR[NV];
  inv_flux(qL, n, P, FL);
  inv_flux(qR, n, P, FR);
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
  double lam = fabs((qL[1] * nh[0] + qL[2] * nh[1] + qL[3] * nh[2]) / qL[0]) + fast_speed(qL, nh, P);
  double lr = fabs((qR[1] * nh[0] + qR[2] * nh[1] + qR[3] * nh[2]) / qR[0]) + fast_speed(qR, nh, P);
  if (lr > lam) lam = lr;
  if (P->c_h > lam) lam = P->c_h;
  for (int v = 0; v < NV; ++v)
    FA[v] = 0.5 * (fabs(FL[v]) + fabs(FR[v]) + lam * nn * (fabs(qL[v]) + fabs(qR[v])) +
                   fabs(FvL[v]) + fabs(FvR[v]));
}

static int boundary_kind(const or_params* P, int group) {
  if (group >= 2) return 1;
  return P->wall_kind[group];
}

int or_residual(const or_mesh* m, const or_params* P, const double* Q, const double* ghost,
                double* R, double* term_scale, double* divB_out) {
  const int N = m->N, NP = N + 1, N2 = N * N, N3 = N2 * N, NF = NP * N2;
  const int64_t E = m->E;
  const tab_t* t = &m->t;
  for (int64_t fi = 0; fi < m->F; ++fi) {
    const int32_t* fc = &m->faces[fi * 5];
    if (fc[2] < 0 && boundary_kind(P, -1 - fc[2]) == 1 && !ghost) return -1;
  }
  double* Qtr = (double*)malloc(sizeof(double) * E * 6 * NV * N2);
  double* Qc = (double*)malloc(sizeof(double) * E * 6 * NV * N2);
  double* Gtr = (double*)malloc(sizeof(double) * E * 6 * NG * N2);
  double* Ktr = (double*)malloc(sizeof(double) * E * 6 * N2);
  double* Ft = (double*)malloc(sizeof(double) * E * 3 * NV * NF);
  double* Fh = (double*)malloc(sizeof(double) * E * 6 * NV * N2);
  double* Fa = (double*)malloc(sizeof(double) * E * 6 * NV * N2); /* magnitude of the face-flux inputs */
  double* dB = (double*)malloc(sizeof(double) * E * N3);
  double tsc[NV] = {0};

  /* 1. traces of Q on the element faces (interpolation to the end flux points) */
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int d = f / 2, fe = (f % 2) ? N : 0;
      for (int v = 0; v < NV; ++v)
        for (int b = 0; b < N; ++b)
          for (int a = 0; a < N; ++a) {
            double s = 0.0;
            for (int i = 0; i < N; ++i) s += t->I[fe][i] * Q[(e * NV + v) * N3 + sp_on_line(N, d, a, b, i)];
            Qtr[((e * 6 + f) * NV + v) * N2 + a + N * b] = s;
          }
    }

  /* 2. BR1 common solution on every face: the average of the two traces;
   *    wall or Dirichlet state on boundary faces */
#pragma omp parallel for schedule(static)
  for (int64_t fi = 0; fi < m->F; ++fi) {
    const int32_t* fc = &m->faces[fi * 5];
    int64_t eL = fc[0];
    int fL = fc[1];
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        double qL[NV], qc[NV];
        for (int v = 0; v < NV; ++v) qL[v] = Qtr[((eL * 6 + fL) * NV + v) * N2 + a + N * b];
        if (fc[2] >= 0) {
          int64_t eR = fc[2];
          int fR = fc[3], a2, b2;
          orient_map(fc[4], N, a, b, &a2, &b2);
          for (int v = 0; v < NV; ++v) {
            double qR = Qtr[((eR * 6 + fR) * NV + v) * N2 + a2 + N * b2];
            qc[v] = 0.5 * (qL[v] + qR);
            Qc[((eR * 6 + fR) * NV + v) * N2 + a2 + N * b2] = qc[v];
          }
        } else {
          int g = -1 - fc[2];
          if (boundary_kind(P, g) == 1) {
            for (int v = 0; v < NV; ++v)
              qc[v] = 0.5 * (qL[v] + ghost[((int64_t)fc[3] * NV + v) * N2 + a + N * b]);
          } else {
            double n[3];
            face_normal(m, eL, fL, a, b, n);
            double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            double nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
            wall_common(qL, nh, g, P, qc);
          }
        }
        for (int v = 0; v < NV; ++v) Qc[((eL * 6 + fL) * NV + v) * N2 + a + N * b] = qc[v];
      }
  }

  /* 3. gradients at the solution points (derivative of the flux-point
   *    polynomial whose end values are the common solution), chain rule to
   *    physical space; interpolation of Q and grad Q to every family of flux
   *    points; the total flux S^d . (F_inv - F_vis) at interior flux points */
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t e = 0; e < E; ++e) {
    double* dQ = (double*)malloc(sizeof(double) * 3 * NV * N3); /* [d][v][sp] */
    double* G = (double*)malloc(sizeof(double) * NG * N3);      /* [v*3+j][sp] */
    double* kr = (double*)malloc(sizeof(double) * N3);
    const double* Qe = &Q[e * NV * N3];
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < NV; ++v)
        for (int b = 0; b < N; ++b)
          for (int a = 0; a < N; ++a) {
            double qh[OR_NMAX + 1];
            for (int f = 0; f <= N; ++f) {
              if (f == 0) qh[f] = Qc[((e * 6 + 2 * d) * NV + v) * N2 + a + N * b];
              else if (f == N) qh[f] = Qc[((e * 6 + 2 * d + 1) * NV + v) * N2 + a + N * b];
              else {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += t->I[f][i] * Qe[v * N3 + sp_on_line(N, d, a, b, i)];
                qh[f] = s;
              }
            }
            for (int i = 0; i < N; ++i) {
              double s = 0.0;
              for (int f = 0; f <= N; ++f) s += t->D[i][f] * qh[f];
              dQ[(d * NV + v) * N3 + sp_on_line(N, d, a, b, i)] = s;
            }
          }
    for (int q = 0; q < N3; ++q) {
      double J = m->detJ[e * N3 + q];
      for (int v = 0; v < NV; ++v)
        for (int j = 0; j < 3; ++j) {
          double s = 0.0;
          for (int d = 0; d < 3; ++d) s += m->Ssp[((e * 3 + d) * 3 + j) * N3 + q] / J * dQ[(d * NV + v) * N3 + q];
          G[(v * 3 + j) * N3 + q] = s;
        }
      dB[e * N3 + q] = G[(5 * 3 + 0) * N3 + q] + G[(6 * 3 + 1) * N3 + q] + G[(7 * 3 + 2) * N3 + q];
      double x[3] = {m->xsp[(e * 3 + 0) * N3 + q], m->xsp[(e * 3 + 1) * N3 + q], m->xsp[(e * 3 + 2) * N3 + q]};
      kr[q] = kr_at(x, P);
    }
    /* per family d, per line: interpolate to the N+1 flux points */
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a)
          for (int f = 0; f <= N; ++f) {
            double qf[NV], gf[NG], kf = 0.0;
            for (int v = 0; v < NV; ++v) {
              double s = 0.0;
              for (int i = 0; i < N; ++i) s += t->I[f][i] * Qe[v * N3 + sp_on_line(N, d, a, b, i)];
              qf[v] = s;
            }
            for (int k = 0; k < NG; ++k) {
              double s = 0.0;
              for (int i = 0; i < N; ++i) s += t->I[f][i] * G[k * N3 + sp_on_line(N, d, a, b, i)];
              gf[k] = s;
            }
            for (int i = 0; i < N; ++i) kf += t->I[f][i] * kr[sp_on_line(N, d, a, b, i)];
            if (f == 0 || f == N) {
              int face = 2 * d + (f == N);
              for (int k = 0; k < NG; ++k) Gtr[((e * 6 + face) * NG + k) * N2 + a + N * b] = gf[k];
              Ktr[(e * 6 + face) * N2 + a + N * b] = kf;
              continue;
            }
            int idx = fp_index(N, d, f, a, b);
            double n[3];
            for (int c = 0; c < 3; ++c) n[c] = m->Sfp[((e * 3 + d) * 3 + c) * NF + idx];
            double Fi[NV], Fv[NV];
            inv_flux(qf, n, P, Fi);
            visc_flux(qf, gf, kf, n, P, Fv);
            for (int v = 0; v < NV; ++v) Ft[((e * 3 + d) * NV + v) * NF + idx] = Fi[v] - Fv[v];
          }
    free(dQ); free(G); free(kr);
  }

  /* 4. common flux on every face: Rusanov for the inviscid part on the
   *    symmetric face normal, BR1 average of the two sides' viscous fluxes;
   *    wall and Dirichlet fluxes on boundary faces */
#pragma omp parallel for schedule(static)
  for (int64_t fi = 0; fi < m->F; ++fi) {
    const int32_t* fc = &m->faces[fi * 5];
    int64_t eL = fc[0];
    int fL = fc[1];
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        double qL[NV], gL[NG], nL[3], F[NV];
        for (int v = 0; v < NV; ++v) qL[v] = Qtr[((eL * 6 + fL) * NV + v) * N2 + a + N * b];
        for (int k = 0; k < NG; ++k) gL[k] = Gtr[((eL * 6 + fL) * NG + k) * N2 + a + N * b];
        double kL = Ktr[(eL * 6 + fL) * N2 + a + N * b];
        face_normal(m, eL, fL, a, b, nL);
        if (fc[2] >= 0) {
          int64_t eR = fc[2];
          int fR = fc[3], a2, b2;
          orient_map(fc[4], N, a, b, &a2, &b2);
          double qR[NV], gR[NG], nR[3], n[3];
          for (int v = 0; v < NV; ++v) qR[v] = Qtr[((eR * 6 + fR) * NV + v) * N2 + a2 + N * b2];
          for (int k = 0; k < NG; ++k) gR[k] = Gtr[((eR * 6 + fR) * NG + k) * N2 + a2 + N * b2];
          double kR = Ktr[(eR * 6 + fR) * N2 + a2 + N * b2];
          face_normal(m, eR, fR, a2, b2, nR);
          for (int c = 0; c < 3; ++c) n[c] = 0.5 * (nL[c] - nR[c]);
          double Fr[NV], FvL[NV], FvR[NV], FA[NV];
          rusanov(qL, qR, n, P, Fr);
          visc_flux(qL, gL, kL, n, P, FvL);
          visc_flux(qR, gR, kR, n, P, FvR);
          face_abs(qL, qR, FvL, FvR, n, P, FA);
          for (int v = 0; v < NV; ++v) {
            F[v] = Fr[v] - 0.5 * (FvL[v] + FvR[v]);
            Fh[((eR * 6 + fR) * NV + v) * N2 + a2 + N * b2] = -F[v];
            Fa[((eR * 6 + fR) * NV + v) * N2 + a2 + N * b2] = FA[v];
            Fa[((eL * 6 + fL) * NV + v) * N2 + a + N * b] = FA[v];
          }
        } else {
          int g = -1 - fc[2];
          if (boundary_kind(P, g) == 1) {
            double qg[NV], Fr[NV], FvL[NV], FvG[NV];
            for (int v = 0; v < NV; ++v) qg[v] = ghost[((int64_t)fc[3] * NV + v) * N2 + a + N * b];
            double FA[NV];
            rusanov(qL, qg, nL, P, Fr);
            visc_flux(qL, gL, kL, nL, P, FvL);
            visc_flux(qg, gL, kL, nL, P, FvG);
            face_abs(qL, qg, FvL, FvG, nL, P, FA);
            for (int v = 0; v < NV; ++v) {
              F[v] = Fr[v] - 0.5 * (FvL[v] + FvG[v]);
              Fa[((eL * 6 + fL) * NV + v) * N2 + a + N * b] = FA[v];
            }
          } else {
            double qg[NV], nh[3], FA[NV], Fz[NV] = {0};
            double nn = sqrt(nL[0] * nL[0] + nL[1] * nL[1] + nL[2] * nL[2]);
            for (int c = 0; c < 3; ++c) nh[c] = nL[c] / nn;
            wall_flux(qL, gL, kL, nL, g, P, F);
            wall_ghost(qL, nh, g, P, qg);
            face_abs(qL, qg, F, Fz, nL, P, FA);
            for (int v = 0; v < NV; ++v) Fa[((eL * 6 + fL) * NV + v) * N2 + a + N * b] = FA[v];
          }
        }
        for (int v = 0; v < NV; ++v) Fh[((eL * 6 + fL) * NV + v) * N2 + a + N * b] = F[v];
      }
  }

  /* 5. divergence of the flux polynomials (end values = common flux with
   *    the sign of the family's direction), sources, R = -div/|J| + M */
  double tsc_all[NV] = {0};
#pragma omp parallel
  {
    double tl[NV] = {0};
#pragma omp for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
      double* div = (double*)calloc(NV * N3, sizeof(double));
      double* adiv = (double*)calloc(NV * N3, sizeof(double));
      for (int d = 0; d < 3; ++d)
        for (int v = 0; v < NV; ++v)
          for (int b = 0; b < N; ++b)
            for (int a = 0; a < N; ++a) {
              double fl[OR_NMAX + 1], fa[OR_NMAX + 1];
              for (int f = 0; f <= N; ++f) {
                if (f == 0) {
                  fl[f] = -Fh[((e * 6 + 2 * d) * NV + v) * N2 + a + N * b];
                  fa[f] = Fa[((e * 6 + 2 * d) * NV + v) * N2 + a + N * b];
                } else if (f == N) {
                  fl[f] = Fh[((e * 6 + 2 * d + 1) * NV + v) * N2 + a + N * b];
                  fa[f] = Fa[((e * 6 + 2 * d + 1) * NV + v) * N2 + a + N * b];
                } else {
                  fl[f] = Ft[((e * 3 + d) * NV + v) * NF + fp_index(N, d, f, a, b)];
                  fa[f] = fabs(fl[f]);
                }
              }
              for (int i = 0; i < N; ++i) {
                int q = sp_on_line(N, d, a, b, i);
                for (int f = 0; f <= N; ++f) {
                  div[v * N3 + q] += t->D[i][f] * fl[f];
                  adiv[v * N3 + q] += fabs(t->D[i][f]) * fa[f];
                }
              }
            }
      for (int q = 0; q < N3; ++q) {
        double J = m->detJ[e * N3 + q];
        double qq[NV];
        for (int v = 0; v < NV; ++v) qq[v] = Q[(e * NV + v) * N3 + q];
        double x[3] = {m->xsp[(e * 3 + 0) * N3 + q], m->xsp[(e * 3 + 1) * N3 + q], m->xsp[(e * 3 + 2) * N3 + q]};
        /* sources (Eq. M): gravity g = -GM x/|x|^3, Coriolis -2 rho Omega z x u,
         * Powell-type terms with the discrete div B, GLM damping -a psi */
        double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        double r3 = r2 * sqrt(r2);
        double gv[3] = {0, 0, 0};
        if (P->GM != 0.0)
          for (int c = 0; c < 3; ++c) gv[c] = -P->GM * x[c] / r3;
        double rho = qq[0], u[3] = {qq[1] / rho, qq[2] / rho, qq[3] / rho};
        double db = P->powell ? dB[e * N3 + q] : 0.0;
        double uB = u[0] * qq[5] + u[1] * qq[6] + u[2] * qq[7];
        double M[NV];
        M[0] = 0.0;
        M[1] = rho * gv[0] + 2.0 * P->Omega * qq[2] - db * qq[5];
        M[2] = rho * gv[1] - 2.0 * P->Omega * qq[1] - db * qq[6];
        M[3] = rho * gv[2] - db * qq[7];
        M[4] = qq[1] * gv[0] + qq[2] * gv[1] + qq[3] * gv[2] - db * uB;
        for (int c = 0; c < 3; ++c) M[5 + c] = -db * u[c];
        M[8] = -P->glm_a * qq[8];
        for (int v = 0; v < NV; ++v) {
          R[(e * NV + v) * N3 + q] = -div[v * N3 + q] / J + M[v];
          double sc = adiv[v * N3 + q] / fabs(J) + fabs(M[v]);
          if (sc > tl[v]) tl[v] = sc;
        }
      }
      free(div); free(adiv);
    }
#pragma omp critical
    for (int v = 0; v < NV; ++v)
      if (tl[v] > tsc_all[v]) tsc_all[v] = tl[v];
  }
  for (int v = 0; v < NV; ++v) tsc[v] = tsc_all[v];
  if (term_scale) memcpy(term_scale, tsc, sizeof tsc);
  if (divB_out) memcpy(divB_out, dB, sizeof(double) * E * N3);
  free(Qtr); free(Qc); free(Gtr); free(Ktr); free(Ft); free(Fh); free(Fa); free(dB);
  return 0;
}

/* ------------------------------------------------------------------ */
/* SSPRK(5,3)                                                          */
/* ------------------------------------------------------------------ */

/* Shu-Osher form u(i) = sum_k alpha_ik u(k) + dt beta_ik L(u(k)) of the
 * optimal five-stage, third-order strong-stability-preserving Runge-Kutta
 * scheme (SSP coefficient 2.6506...).  The published 14-digit values of
 * this scheme were corrected by a minimal-norm Newton step on the beta
 * entries so that the four third-order conditions hold to double
 * precision (oracle/ssprk53_coefficients.py derives and checks them). */
static const double SSP_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0, 0, 0, 0, 0, 0},
    {0, 1.0, 0, 0, 0, 0},
    {0.56656131914032997754, 0, 0.43343868085967002246, 0, 0, 0},
    {0.09299483444412999511, 0.000020903696200000000053, 0, 0.90698426185967000489, 0, 0},
    {0.0073613226092000003456, 0.20127980325145000684, 0.0018295538968200000286, 0,
     0.78952932024252999279, 0}};
static const double SSP_B[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.37726891519897837344, 0, 0, 0, 0, 0},
    {0, 0.37726891516114840825, 0, 0, 0, 0},
    {0, 0, 0.16352294101188272956, 0, 0, 0},
    {0.00071997350394151505236, 0, 0, 0.3421769684090429351, 0, 0},
    {0.0027771984070493497694, 0.000015679038088402258468, 0, 0, 0.29786487003033598351, 0}};

void or_ssprk53_table(double* alpha, double* beta, double* c) {
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 6; ++k) { alpha[i * 6 + k] = SSP_A[i][k]; beta[i * 6 + k] = SSP_B[i][k]; }
  /* stage times: c_i of stage value u(i), from the Butcher form */
  double A[6][5] = {{0}};
  for (int i = 1; i < 6; ++i)
    for (int k = 0; k < i; ++k) {
      for (int j = 0; j < 5; ++j) A[i][j] += SSP_A[i][k] * A[k][j];
      A[i][k] += SSP_B[i][k];
    }
  for (int i = 0; i < 5; ++i) {
    double s = 0.0;
    for (int j = 0; j < 5; ++j) s += A[i][j];
    c[i] = s;
  }
}

void or_combine(int64_t n, int nterm, const double* const* U, const double* a,
                const double* const* L, const double* b, double dt, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = 0; k < nterm; ++k) {
      if (a[k] != 0.0) s += a[k] * U[k][i];
      if (b[k] != 0.0) s += dt * b[k] * L[k][i];
    }
    out[i] = s;
  }
}

int or_ssprk53_step(const or_mesh* m, const or_params* P, double* Q, const double* ghost, double dt) {
  const int64_t n = m->E * NV * (int64_t)m->N * m->N * m->N;
  double* U[6];
  double* L[5];
  U[0] = Q;
  for (int i = 1; i < 6; ++i) U[i] = (double*)malloc(sizeof(double) * n);
  for (int i = 0; i < 5; ++i) L[i] = (double*)malloc(sizeof(double) * n);
  int rc = 0;
  for (int i = 1; i <= 5 && !rc; ++i) {
    rc = or_residual(m, P, U[i - 1], ghost, L[i - 1], NULL, NULL);
    if (rc) break;
    double a[5], b[5];
    for (int k = 0; k < i; ++k) { a[k] = SSP_A[i][k]; b[k] = SSP_B[i][k]; }
    or_combine(n, i, (const double* const*)U, a, (const double* const*)L, b, dt, U[i]);
  }
  if (!rc) memcpy(Q, U[5], sizeof(double) * n);
  for (int i = 1; i < 6; ++i) free(U[i]);
  for (int i = 0; i < 5; ++i) free(L[i]);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Diagnostics (Sec. Results: volume-averaged KE and E_B)              */
/* ------------------------------------------------------------------ */

int or_diagnostics(const or_mesh* m, const or_params* P, const double* Q, const double* ghost,
                   double* out) {
  const int N = m->N, N3 = N * N * N;
  const int64_t E = m->E;
  double* R = (double*)malloc(sizeof(double) * E * NV * N3);
  double* dB = (double*)malloc(sizeof(double) * E * N3);
  int rc = or_residual(m, P, Q, ghost, R, NULL, dB);
  free(R);
  if (rc) { free(dB); return rc; }
  double vol = 0, mass = 0, en = 0, ke = 0, eb = 0, mx = 0, l2 = 0, mpsi = 0;
  int nan = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int c = 0; c < N; ++c)
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a) {
          int q = SP(N, a, b, c);
          double w = m->t.W[a] * m->t.W[b] * m->t.W[c] * m->detJ[e * N3 + q];
          const double* s = &Q[e * NV * N3 + q];
          double rho = s[0];
          double m2 = s[N3] * s[N3] + s[2 * N3] * s[2 * N3] + s[3 * N3] * s[3 * N3];
          double b2 = s[5 * N3] * s[5 * N3] + s[6 * N3] * s[6 * N3] + s[7 * N3] * s[7 * N3];
          vol += w; mass += w * rho; en += w * s[4 * N3];
          ke += w * 0.5 * m2 / rho; eb += w * 0.5 * b2;
          double db = dB[e * N3 + q];
          if (fabs(db) > mx) mx = fabs(db);
          l2 += w * db * db;
          if (fabs(s[8 * N3]) > mpsi) mpsi = fabs(s[8 * N3]);
          for (int v = 0; v < NV; ++v)
            if (!isfinite(s[v * N3])) nan = 1;
        }
  for (int i = 0; i < 16; ++i) out[i] = 0.0;
  out[0] = vol; out[1] = mass; out[2] = en; out[3] = ke / vol; out[4] = eb / vol;
  out[5] = mx; out[6] = sqrt(l2 / vol); out[7] = mpsi; out[8] = nan ? 1.0 : 0.0;
  free(dB);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Spherical components (Sec. Results)                                  */
/* ------------------------------------------------------------------ */

/* The paper reports the differential rotation as the longitude (and time)
 * average of V_phi, the meridional flow as that of V_mer = sqrt(V_r^2 +
 * V_theta^2), and the magnetic energy split into poloidal (B_r^2 + B_theta^2)
 * and toroidal (B_phi^2) parts.  Readings: rationalized units (the
 * factor 1/(8 pi) becomes 1/2, as for E_B); the longitude average over a
 * bin of uniform (r, theta) bins, r in [rb, rt], theta in [0, pi], is the
 * volume-weighted mean of the SPs the bin holds; a bin holds SP x when
 * floor((|x| - rb) / (rt - rb) * n_r) and floor(theta / pi * n_th) (clamped
 * to the range) are its indices, theta = atan2(sqrt(x^2 + y^2), z).  On the
 * polar axis (x = y = 0) phi_hat = (0, 1, 0) and theta_hat = (1, 0, 0) sign z.
 * out[(ir * n_th + it) * 5 + k]: k = 0 sum of w, 1 sum of w V_phi, 2 sum of
 * w V_mer, 3 sum of w (B_r^2 + B_theta^2)/2, 4 sum of w B_phi^2/2, with w =
 * W_a W_b W_c |J| at the SP. */
static void sph_basis(const double x[3], double rh[3], double th[3], double ph[3], double* r,
                      double* theta) {
  const double rc = sqrt(x[0] * x[0] + x[1] * x[1]);
  *r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  *theta = atan2(rc, x[2]);
  for (int c = 0; c < 3; ++c) rh[c] = x[c] / *r;
  if (rc > 0.0) {
    ph[0] = -x[1] / rc; ph[1] = x[0] / rc; ph[2] = 0.0;
    /* theta_hat = phi_hat x r_hat */
    th[0] = ph[1] * rh[2] - ph[2] * rh[1];
    th[1] = ph[2] * rh[0] - ph[0] * rh[2];
    th[2] = ph[0] * rh[1] - ph[1] * rh[0];
  } else {
    ph[0] = 0.0; ph[1] = 1.0; ph[2] = 0.0;
    th[0] = x[2] >= 0.0 ? 1.0 : -1.0; th[1] = 0.0; th[2] = 0.0;
  }
}

int or_sph_profiles(const or_mesh* m, const double* Q, double rb, double rt, int n_r, int n_th,
                    double* out) {
  if (n_r < 1 || n_th < 1 || !(rt > rb)) return -1;
  const int N = m->N, N3 = N * N * N;
  const double pi = 3.14159265358979323846;
  for (int64_t i = 0; i < (int64_t)n_r * n_th * 5; ++i) out[i] = 0.0;
  for (int64_t e = 0; e < m->E; ++e)
    for (int c = 0; c < N; ++c)
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a) {
          const int q = SP(N, a, b, c);
          const double w = m->t.W[a] * m->t.W[b] * m->t.W[c] * m->detJ[e * N3 + q];
          const double x[3] = {m->xsp[(e * 3 + 0) * N3 + q], m->xsp[(e * 3 + 1) * N3 + q],
                               m->xsp[(e * 3 + 2) * N3 + q]};
          double rh[3], th[3], ph[3], r, theta;
          sph_basis(x, rh, th, ph, &r, &theta);
          int ir = (int)floor((r - rb) / (rt - rb) * n_r);
          int it = (int)floor(theta / pi * n_th);
          ir = ir < 0 ? 0 : (ir >= n_r ? n_r - 1 : ir);
          it = it < 0 ? 0 : (it >= n_th ? n_th - 1 : it);
          const double* s = &Q[e * NV * N3 + q];
          const double u[3] = {s[N3] / s[0], s[2 * N3] / s[0], s[3 * N3] / s[0]};
          const double B[3] = {s[5 * N3], s[6 * N3], s[7 * N3]};
          double ur = 0, ut = 0, up = 0, br = 0, bt = 0, bp = 0;
          for (int k = 0; k < 3; ++k) {
            ur += u[k] * rh[k]; ut += u[k] * th[k]; up += u[k] * ph[k];
            br += B[k] * rh[k]; bt += B[k] * th[k]; bp += B[k] * ph[k];
          }
          double* o = &out[((int64_t)ir * n_th + it) * 5];
          o[0] += w;
          o[1] += w * up;
          o[2] += w * sqrt(ur * ur + ut * ut);
          o[3] += w * 0.5 * (br * br + bt * bt);
          o[4] += w * 0.5 * bp * bp;
        }
  return 0;
}

int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Pointwise entry points (for the pointwise tests)                    */
/* ------------------------------------------------------------------ */

void or_point_flux(const double* q, const double* G, double kr, const double* n,
                   const or_params* P, double* Finv, double* Fvis) {
  inv_flux(q, n, P, Finv);
  visc_flux(q, G, kr, n, P, Fvis);
}

void or_point_rusanov(const double* qL, const double* qR, const double* n, const or_params* P,
                      double* F) {
  rusanov(qL, qR, n, P, F);
}

double or_point_cf(const double* q, const double* nh, const or_params* P) {
  return fast_speed(q, nh, P);
}

void or_point_wall_flux(const double* q, const double* G, double kr, const double* n, int group,
                        const or_params* P, double* F) {
  wall_flux(q, G, kr, n, group, P, F);
}
