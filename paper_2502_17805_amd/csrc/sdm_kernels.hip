// sdm_kernels.hip -- gfx950 kernels of the spectral-difference GLM-MHD
// residual and fused Runge-Kutta stage (paper arXiv 2502.17805, Sec.
// "Spectral Difference Method"), and the C ABI declared in include/sdmhd.h.
//
// One stage = two launches (k_volume, k_finish), one workgroup per element;
// k_traces runs only before a run's first stage:
//   k_traces  Q at the two end flux points of every line = the element's face
//             traces (afterwards each stage's k_finish writes them)
//   k_volume  BR1 common solution from the own and neighbour traces, gradient
//             at the solution points (chain rule with S^d/|J|), interpolation
//             of Q and grad Q to each flux-point family, total flux at the
//             interior flux points, Rusanov + own half of the BR1 viscous flux
//             at the face points (wall / Dirichlet fluxes complete), flux
//             divergence, sources -> partial residual (without the neighbour
//             half of the viscous flux), or, in a stage, the FP64 Shu-Osher
//             combination with it written to the output register; writes
//             this side's viscous normal flux for the neighbour
//   k_finish  adds the neighbour half of the BR1 viscous flux: stores R, or
//             corrects the stage output in place; in a stage it writes the
//             new state's face traces for the next stage.
// The face coupling uses the per-element neighbour/orientation table; each
// interior face is evaluated by both of its elements, with the symmetric face
// normal n = (S_own - S_other)/2 so the two values are exact negatives.
// Faces whose neighbour lives in another partition of a split mesh (import
// faces) take the neighbour's trace and viscous flux from caller buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sdmhd.h"
#include "sdm_host.hpp"
#include "sdm_physics.hpp"

namespace sdm {

constexpr int kNMax = 8;

// ---------------------------------------------------------------------------
// constant tables (one set per N, FP64 and FP32 copies)
// ---------------------------------------------------------------------------
template <typename T>
struct DevTab {
  T I[kNMax + 1][kNMax];   // SP basis at FPs
  T D[kNMax][kNMax + 1];   // FP-basis derivative at SPs
  T DI[kNMax][kNMax];      // derivative of the SP polynomial at SPs
  T W[kNMax];              // quadrature weights
};
__constant__ DevTab<double> c_tab_d[kNMax + 1];
__constant__ DevTab<float> c_tab_f[kNMax + 1];

// Scratch of the allocation-free SSPRK(5,3) step: the face traces of Q and of
// the viscous normal flux that the stages exchange between face neighbours.
// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it takes the device address from
// hipGetSymbolAddress (sdm_create, once per device) and uses that.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

template <typename T>
__device__ __forceinline__ const DevTab<T>& tab(int N);
template <>
__device__ __forceinline__ const DevTab<double>& tab<double>(int N) { return c_tab_d[N]; }
template <>
__device__ __forceinline__ const DevTab<float>& tab<float>(int N) { return c_tab_f[N]; }

// ---------------------------------------------------------------------------
// per-run descriptor (kernel argument for one run, device array for batches)
// ---------------------------------------------------------------------------
struct RunDesc {
  int32_t N;           // solution points per direction (p + 1)
  int64_t E;
  int64_t n_bfaces;
  const double* x_sp;
  const double* detJ;
  const double* S_fp;
  const double* Sj_sp;
  const int32_t* nbr;
  const double* n_face;
  // FP32 copies of the five geometry arrays (mixed arithmetic; made by
  // sdm_mesh_bind), read by the FP32 kernels in place of the FP64 ones
  const float* x_sp_f;
  const float* detJ_f;
  const float* S_fp_f;
  const float* Sj_sp_f;
  const float* n_face_f;
  const double* ghost;
  const void* imp_q;   // [n_bfaces][9][N2]  T  neighbour traces on import faces
  const void* imp_v;   // [n_bfaces][7][N2]  T  neighbour viscous normal fluxes
  const double* Q;     // state whose residual is taken
  void* Qtr;           // [E][6][9][N2]  T
  void* Vtr;           // [E][6][7][N2]  T
  void* Rp;            // [E][9][N3]     T
  double* R;           // residual output (residual mode)
  const double* in[4]; // stage inputs
  double alpha[4];
  int32_t n_in;
  int32_t write_traces;
  int32_t fuse;        // stage: k_volume writes sum alpha u + beta dt (R
                       // without the neighbour viscous half) to `out` and
                       // k_finish subtracts that half; residual: k_volume
                       // writes Rp, k_finish adds the half and writes R
  double* out;         // stage output
  double beta_dt;
  Phys<double> P;
};

// One launch: a single run (many == nullptr), or the work list of a batch of
// runs of one degree: their descriptors and element offsets (prefix[k] =
// elements of runs 0 .. k-1), one element per workgroup.
struct Launch {
  RunDesc one;                  // used when many == nullptr
  const RunDesc* many;          // batched runs (device)
  const int64_t* prefix;        // [n_run + 1] element offsets of the runs (device)
  int32_t n_run;
  int64_t n_work;               // work items end here (one element each)
  int64_t w0;                   // first work item of this launch (one per workgroup)
};

// Device-side view of one run's descriptor with every array pointer in the
// global address space, so that element data moves with global (not flat)
// loads and stores and LDS waits never wait on them.
#define GBL __attribute__((address_space(1)))

template <typename T>
struct Run {
  int64_t e;  // element index within the run
  // geometry in the residual arithmetic (FP32-mixed reads FP32 copies); the
  // diagnostics' quadrature takes |J| in FP64 in either arithmetic
  const GBL T* x_sp;
  const GBL T* detJ;
  const GBL T* S_fp;
  const GBL T* Sj_sp;
  const GBL int32_t* nbr;
  const GBL T* n_face;
  const GBL double* detJ64;
  const GBL double* ghost;
  const GBL T* imp_q;
  const GBL T* imp_v;
  const GBL double* Q;
  GBL T* Qtr;
  GBL T* Vtr;
  GBL T* Rp;
  GBL double* R;
  const GBL double* in[4];
  double alpha[4];
  int32_t n_in;
  int32_t write_traces;
  int32_t fuse;
  GBL double* out;
  double beta_dt;
  // the physical parameters stay in the descriptor (the kernels copy them
  // to LDS with vector loads, so that they take no scalar registers); the
  // two values needed before that copy is visible are kept here
  const Phys<double>* P;
  int32_t wall_kind[2];
  bool kr_on;
};

// Phys<double> -> Phys<T> by lane: the 23 real parameters then the 7 int32
// selectors (tid >= 29 copies nothing)
template <typename T>
__device__ __forceinline__ void copy_phys(const Phys<double>* src, Phys<T>* dst, int tid) {
  constexpr int NR = 23, NS = 7;
  static_assert(offsetof(Phys<T>, powell) == NR * sizeof(T) && offsetof(Phys<double>, powell) == NR * sizeof(double),
                "real parameters first");
  static_assert(sizeof(Phys<T>) >= NR * sizeof(T) + NS * sizeof(int32_t), "selectors after them");
  if (tid < NR) {
    reinterpret_cast<T*>(dst)[tid] = (T)reinterpret_cast<const double*>(src)[tid];
  } else if (tid < NR + NS) {
    reinterpret_cast<int32_t*>(&dst->powell)[tid - NR] = reinterpret_cast<const int32_t*>(&src->powell)[tid - NR];
  }
}

template <typename T, typename S>
__device__ __forceinline__ void fill_run(Run<T>& r, S& d) {
  if constexpr (sizeof(T) == 8) {
    r.x_sp = (const GBL T*)d.x_sp;
    r.detJ = (const GBL T*)d.detJ;
    r.S_fp = (const GBL T*)d.S_fp;
    r.Sj_sp = (const GBL T*)d.Sj_sp;
    r.n_face = (const GBL T*)d.n_face;
  } else {
    r.x_sp = (const GBL T*)d.x_sp_f;
    r.detJ = (const GBL T*)d.detJ_f;
    r.S_fp = (const GBL T*)d.S_fp_f;
    r.Sj_sp = (const GBL T*)d.Sj_sp_f;
    r.n_face = (const GBL T*)d.n_face_f;
  }
  r.detJ64 = (const GBL double*)d.detJ;
  r.nbr = (const GBL int32_t*)d.nbr;
  r.ghost = (const GBL double*)d.ghost;
  r.imp_q = (const GBL T*)d.imp_q;
  r.imp_v = (const GBL T*)d.imp_v;
  r.Q = (const GBL double*)d.Q;
  r.Qtr = (GBL T*)d.Qtr;
  r.Vtr = (GBL T*)d.Vtr;
  r.Rp = (GBL T*)d.Rp;
  r.R = (GBL double*)d.R;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r.in[k] = (const GBL double*)d.in[k];
    r.alpha[k] = d.alpha[k];
  }
  r.n_in = d.n_in;
  r.write_traces = d.write_traces;
  r.fuse = d.fuse;
  r.out = (GBL double*)d.out;
  r.beta_dt = d.beta_dt;
  r.P = (const Phys<double>*)&d.P;
  r.wall_kind[0] = d.P.wall_kind[0];
  r.wall_kind[1] = d.P.wall_kind[1];
  r.kr_on = d.P.kr_scale != 0.0;
}

// the run and element of work item w (batched: the last run whose element
// offset is <= w, by binary search over the prefix table)
template <typename T>
__device__ __forceinline__ Run<T> view(const Launch& L, int64_t w) {
  Run<T> r;
  if (L.many == nullptr) {
    fill_run(r, L.one);
    r.e = w;
    return r;
  }
  const GBL int64_t* pre = (const GBL int64_t*)L.prefix;
  int lo = 0, hi = L.n_run - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= w) lo = mid; else hi = mid - 1;
  }
  fill_run(r, ((const GBL RunDesc*)L.many)[lo]);
  r.e = w - pre[lo];
  return r;
}

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ int sp_line(int d, int p, int q, int i) {
  return d == 0 ? i + N * (p + N * q) : (d == 1 ? p + N * (i + N * q) : p + N * (q + N * i));
}
template <int N>
__device__ __forceinline__ int fp_fam(int d, int f, int p, int q) {
  return d == 0 ? f + (N + 1) * (p + N * q) : (d == 1 ? p + N * (f + (N + 1) * q) : p + N * (q + N * f));
}
template <int N>
__device__ __forceinline__ void omap(int o, int a, int b, int& a2, int& b2) {
  const int p = (o & 4) ? b : a, q = (o & 4) ? a : b;
  a2 = (o & 1) ? N - 1 - p : p;
  b2 = (o & 2) ? N - 1 - q : q;
}

template <int N>
constexpr int block_threads() {
  return ((N * N * N + 63) / 64) * 64 < 64 ? 64 : ((N * N * N + 63) / 64) * 64;
}
// k_finish: at least one lane per face point, so that the neighbours'
// viscous fluxes travel with the element's own loads (p = 3: 128 lanes for
// 96 face points, k_finish 0.224 -> 0.199 ms FP64, 0.158 -> 0.134 ms
// FP32-mixed on 55,296 elements; the volume pass keeps one lane per SP)
template <int N>
constexpr int finish_threads() {
  return block_threads<N>() >= 6 * N * N ? block_threads<N>() : ((6 * N * N + 63) / 64) * 64;
}

// Face point (face, ab) handled by lane t of k_volume's face passes, which
// read the N point rows of the line through each face point.  For N = 6 the
// lanes are arranged so that the 16 lanes LDS serves together read rows in
// 16 distinct bank groups: each direction gets a slot of 80 lanes, the two
// opposite faces of a direction alternate (they read the same rows, which
// LDS broadcasts), and the points of the y faces run in 4 x 2 tiles (the
// row stride 6 of their lines would otherwise repeat bank groups).  Other N
// use the plain order.  Returns false for lanes without a face point.
template <int N>
constexpr int face_lanes() {
  return N == 6 ? 240 : 6 * N * N;
}
template <int N>
__device__ __forceinline__ bool face_lane(int t, int& face, int& ab) {
  if constexpr (N == 6) {
    const int d = t / 80, r = t % 80;
    if (d >= 3 || r >= 72) return false;
    const int k = r >> 1;
    face = 2 * d + (r & 1);
    int a, b;
    if (d == 1) {
      const int blk = k >> 3, j = k & 7;
      a = blk < 3 ? (j & 3) : 4 + (j & 1);
      b = blk < 3 ? 2 * blk + (j >> 2) : (blk == 3 ? (j >> 1) : 4 + (j >> 1));
    } else {
      a = k % 6;
      b = k / 6;
    }
    ab = a + 6 * b;
    return true;
  } else {
    if (t >= 6 * N * N) return false;
    face = t / (N * N);
    ab = t % (N * N);
    return true;
  }
}

// ---------------------------------------------------------------------------
// interpolation of the solution-point fields to one flux point
// ---------------------------------------------------------------------------
// k_volume keeps Q and grad_x Q of its element in LDS point by point: row sp
// of `RS` values holds Q (0..8), then the gradient (9 + 3 v + c: component c
// of variable v), then padding; a point's 36 fields are contiguous, so one
// 16-byte LDS read fetches two of them.  RS = 38 doubles (a row is 19
// 16-byte units, so 16 consecutive rows start in 16 distinct bank groups)
// or 36 floats.
template <typename T>
constexpr int row_stride() {
  return sizeof(T) == 8 ? 38 : 36;
}

// Q and grad_x Q at one flux point from the point rows: one pass over the
// line's N solution points accumulating all 36 fields (the first point's
// products start the sums); w[i * ws] are the interpolation weights;
// optionally the radiative diffusivity sampled at the SPs and interpolated
// the same way.  In FP64 the row reads are software-pipelined by half rows:
// the second half of row i and the first half of row i + 1 are requested
// while the previous half is accumulated, so LDS latency overlaps arithmetic
// with no more registers than one row.
template <typename T>
struct RowVec;
template <>
struct RowVec<double> {
  using V = double2;
  static constexpr int W = 2;
};
template <>
struct RowVec<float> {
  using V = float4;
  static constexpr int W = 4;
};

template <typename T, int K>
__device__ __forceinline__ void lds_vecs(const T* p, typename RowVec<T>::V a[K]) {
  const typename RowVec<T>::V* v = reinterpret_cast<const typename RowVec<T>::V*>(p);
#pragma unroll
  for (int j = 0; j < K; ++j) a[j] = v[j];
}

__device__ __forceinline__ void vec_elems(const double2& v, double x[2]) {
  x[0] = v.x;
  x[1] = v.y;
}
__device__ __forceinline__ void vec_elems(const float4& v, float x[4]) {
  x[0] = v.x;
  x[1] = v.y;
  x[2] = v.z;
  x[3] = v.w;
}

// acc[base + ...] (=|+=) w * a, for the K vectors of a half row
template <typename T, int K, bool FIRST>
__device__ __forceinline__ void acc_vecs(T* acc, int base, T w, const typename RowVec<T>::V a[K]) {
  constexpr int W = RowVec<T>::W;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    T x[W];
    vec_elems(a[j], x);
#pragma unroll
    for (int c = 0; c < W; ++c) {
      if (FIRST) acc[base + j * W + c] = w * x[c];
      else acc[base + j * W + c] += w * x[c];
    }
  }
}

template <int N, typename T>
__device__ __forceinline__ T interp_rows(const T* sR, const T* w, int ws, int s0, int st, T qf[9], T gf[27],
                                         bool use_kr, const Run<T>& R, const Phys<T>& P) {
  constexpr int N3 = N * N * N;
  constexpr int RS = row_stride<T>();
  constexpr int W = RowVec<T>::W, NV = 36 / W, H0 = (NV + 1) / 2, H1 = NV - H0;
  using V = typename RowVec<T>::V;
  T acc[36];
  if constexpr (N <= 3 || sizeof(T) == 4) {
    // plain row loop: for short lines (the pipelined form spills registers
    // there) and in FP32, whose four waves per SIMD already hide the latency
    // (measured 1 % faster)
    V a[NV];
    lds_vecs<T, NV>(sR + s0 * RS, a);
    acc_vecs<T, NV, true>(acc, 0, w[0], a);
#pragma unroll 1
    for (int i = 1; i < N; ++i) {
      lds_vecs<T, NV>(sR + (s0 + i * st) * RS, a);
      acc_vecs<T, NV, false>(acc, 0, w[i * ws], a);
    }
  } else {
    V a0[H0], a1[H1];
    // row 0; the weight of the next row is requested with its first half
    T wc = w[0];
    lds_vecs<T, H0>(sR + s0 * RS, a0);
    lds_vecs<T, H1>(sR + s0 * RS + H0 * W, a1);
    acc_vecs<T, H0, true>(acc, 0, wc, a0);
    T wn = w[ws];
    lds_vecs<T, H0>(sR + (s0 + st) * RS, a0);
    acc_vecs<T, H1, true>(acc, H0 * W, wc, a1);
    // rows 1 .. N-2: the next row's first half is requested before this
    // row's second half is accumulated
#pragma unroll 1
    for (int i = 1; i < N - 1; ++i) {
      wc = wn;
      lds_vecs<T, H1>(sR + (s0 + i * st) * RS + H0 * W, a1);
      acc_vecs<T, H0, false>(acc, 0, wc, a0);
      wn = w[(i + 1) * ws];
      lds_vecs<T, H0>(sR + (s0 + (i + 1) * st) * RS, a0);
      acc_vecs<T, H1, false>(acc, H0 * W, wc, a1);
    }
    // row N-1
    wc = wn;
    lds_vecs<T, H1>(sR + (s0 + (N - 1) * st) * RS + H0 * W, a1);
    acc_vecs<T, H0, false>(acc, 0, wc, a0);
    acc_vecs<T, H1, false>(acc, H0 * W, wc, a1);
  }
#pragma unroll
  for (int v = 0; v < 9; ++v) qf[v] = acc[v];
#pragma unroll
  for (int k = 0; k < 27; ++k) gf[k] = acc[9 + k];
  T kf = T(0);
  if (use_kr) {
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
      const int sidx = s0 + i * st;
      const T x[3] = {(T)R.x_sp[(R.e * 3 + 0) * N3 + sidx], (T)R.x_sp[(R.e * 3 + 1) * N3 + sidx],
                      (T)R.x_sp[(R.e * 3 + 2) * N3 + sidx]};
      kf += w[i * ws] * kappa_r(x, P);
    }
  }
  return kf;
}

// Outward normal at face point ab of face f.
template <int N, typename T>
__device__ __forceinline__ void load_normal(const Run<T>& R, int f, int ab, T n[3]) {
  constexpr int N2 = N * N;
  const GBL T* nf = R.n_face + (R.e * 6 + f) * 3 * N2 + ab;
  n[0] = (T)nf[0];
  n[1] = (T)nf[N2];
  n[2] = (T)nf[2 * N2];
}

// Outside state at face point ab: the neighbour's stored trace
// (orientation-mapped), the caller's trace on import faces, the ghost state
// on Dirichlet faces; nothing on walls (their state is built from the own one).
template <int N, typename T>
__device__ __forceinline__ void load_outside_state(const Run<T>& R, int ab, int32_t code, T q[9]) {
  constexpr int N2 = N * N;
  // one source pointer, then one block of loads
  const GBL T* tn = nullptr;
  const GBL double* gh = nullptr;
  if (code >= 0) {
    const int64_t en = code >> 6;
    const int fn = (code >> 3) & 7, o = code & 7;
    int a2, b2;
    omap<N>(o, ab % N, ab / N, a2, b2);
    tn = R.Qtr + (en * 6 + fn) * 9 * N2 + a2 + N * b2;
  } else {
    const int c2 = -code - 1, g = c2 & 3;
    const int64_t bf = c2 >> 2;
    if (g == 3) tn = R.imp_q + bf * 9 * N2 + ab;
    else if (g == 2 || wsel(g, R.wall_kind) == 1) gh = R.ghost + bf * 9 * N2 + ab;
  }
  if constexpr (sizeof(T) == 8) {
    if (gh) tn = (const GBL T*)gh;  // the ghost state is FP64 like the traces
  }
  if (tn) {
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = tn[v * N2];
  } else if (sizeof(T) != 8 && gh) {
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = (T)gh[v * N2];
  } else {
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = T(0);
  }
}

template <int N, typename T>
__device__ __forceinline__ void load_outside(const Run<T>& R, int f, int ab, int32_t code, T q[9], T n[3]) {
  load_normal<N>(R, f, ab, n);
  load_outside_state<N>(R, ab, code, q);
}

// ---------------------------------------------------------------------------
// the basis tables a thread indexes by its own point (not uniformly across
// the wave) are staged once per workgroup in LDS: I [N+1][N], D [N][N+1]
// ---------------------------------------------------------------------------
template <int N, typename T>
__device__ __forceinline__ void stage_tables(T* sI, T* sD, int tid, int nthreads) {
  const DevTab<T>& tb = tab<T>(N);
  for (int i = tid; i < (N + 1) * N; i += nthreads) {
    sI[i] = tb.I[i / N][i % N];
    sD[i] = tb.D[i / (N + 1)][i % (N + 1)];
  }
}

// ---------------------------------------------------------------------------
// LDS of one element, per pass: the kernels below take a base pointer into a
// workgroup buffer, so that a single-element launch and a batched launch (one
// buffer holding one element of degree 5 or several of a lower degree) run
// the same code.  Offsets are 16-byte aligned.
// ---------------------------------------------------------------------------
constexpr size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

template <int N, typename T>
struct TraceLds {
  static constexpr int N3 = N * N * N;
  static constexpr size_t oQ = 0, oI = al16(oQ + sizeof(T) * 9 * N3), oD = al16(oI + sizeof(T) * (N + 1) * N);
  static constexpr size_t bytes = al16(oD + sizeof(T) * N * (N + 1));
};

// ---------------------------------------------------------------------------
// k_traces: face traces of Q (used before a run's first stage)
// ---------------------------------------------------------------------------
// tid: this thread's index within the element (>= the element's thread
// count for threads without work, which still reach every barrier)
template <int N, typename T>
__device__ __forceinline__ void traces_body(const Run<T>& R, int tid, char* lds) {
  constexpr int N2 = N * N, N3 = N2 * N, BS = block_threads<N>();
  using Ly = TraceLds<N, T>;
  T* sQ = reinterpret_cast<T*>(lds + Ly::oQ);
  T* sI = reinterpret_cast<T*>(lds + Ly::oI);
  T* sD = reinterpret_cast<T*>(lds + Ly::oD);
  stage_tables<N>(sI, sD, tid, BS);
  const GBL double* Qe = R.Q + R.e * 9 * N3;
  for (int i = tid; i < 9 * N3; i += BS) sQ[i] = (T)Qe[i];
  __syncthreads();
  GBL T* tr = R.Qtr + R.e * 6 * 9 * N2;
  for (int it = tid; it < 6 * 9 * N2; it += BS) {
    const int ab = it % N2, fv = it / N2, v = fv % 9, f = fv / 9;
    const int d = f >> 1;
    const T* wI = sI + ((f & 1) ? N : 0) * N;
    T s = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) s += wI[i] * sQ[v * N3 + sp_line<N>(d, ab % N, ab / N, i)];
    tr[it] = s;
  }
  __syncthreads();
}

template <int N, typename T>
__global__ __launch_bounds__(block_threads<N>()) void k_traces(Launch L) {
  __shared__ __align__(16) char lds[TraceLds<N, T>::bytes];
  // one element per workgroup; no loop, so nothing per element is kept
  // live across elements
  const int64_t w = L.w0 + blockIdx.x;
  if (w >= L.n_work) return;
  traces_body<N, T>(view<T>(L, w), threadIdx.x, lds);
}

// divergence contribution of the interior flux points of family d (stored
// in sU, 9 values per point, line-major) at the SP (ia0, ia1, ia2)
template <int N, typename T>
__device__ __forceinline__ void lift_family(int d, int ia0, int ia1, int ia2, const T* sD, int ds, const T* sU,
                                            T div[9]) {
  constexpr int NP = N + 1;
  const int p = d == 0 ? ia1 : ia0, q = d == 2 ? ia1 : ia2, i = d == 0 ? ia0 : (d == 1 ? ia1 : ia2);
  const int base = (p + N * q) * (N - 1);
#pragma unroll 1
  for (int f = 1; f < N; ++f) {
    const T df = sD[(i * NP + f) * ds];
#pragma unroll
    for (int v = 0; v < 9; ++v) div[v] += df * sU[(base + f - 1) * 9 + v];
  }
}

// E. of k_volume: the lifting of the last family's fluxes, the sources (Eq.
// "M") and -div/|J| + M at this thread's SP.  Written as the partial residual
// Rp (residual mode), or, in a stage (FUSED, K input registers), as the stage
// output sum_k alpha_k u_k + beta dt (-div/|J| + M) in `out`, in FP64: the
// input registers are requested before the lifting, so that they arrive
// meanwhile, except, in FP64, the state itself, which is the SP's own point
// row (in FP32-mixed the row holds it in FP32).  k_finish then subtracts
// beta dt times the neighbour half of the viscous flux.
template <int N, typename T, bool FUSED, int K>
__device__ __forceinline__ void volume_epilogue(const Run<T>& R, const Phys<T>& P, const T* sR, const T* sD, int ds,
                                                const T* sU, int tid, int ia0, int ia1, int ia2, T div[9],
                                                const T xs[3], T ji) {
  constexpr int N3 = N * N * N;
  constexpr int RS = row_stride<T>();
  const int64_t e = R.e;
  double a[K > 0 ? K : 1][9];
  if constexpr (FUSED) {
    if (tid < N3) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (sizeof(T) != 8 || R.in[k] != R.Q) {
          const GBL double* src = R.in[k] + e * 9 * N3 + tid;
#pragma unroll
          for (int v = 0; v < 9; ++v) a[k][v] = src[v * N3];
        }
      }
    }
  }
  if (tid < N3) lift_family<N>(2, ia0, ia1, ia2, sD, ds, sU, div);
  if (tid < N3) {
    const int sp = tid;
    T q[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = sR[sp * RS + v];
    T gv[3] = {T(0), T(0), T(0)};
    if (P.GM != T(0)) {
      const T r2 = xs[0] * xs[0] + xs[1] * xs[1] + xs[2] * xs[2];
      const T sc = -P.GM * recip(r2 * sqrt_fast(r2));
      gv[0] = sc * xs[0]; gv[1] = sc * xs[1]; gv[2] = sc * xs[2];
    }
    const T ir = recip(q[0]);
    const T* row = sR + sp * RS;
    const T db = P.powell ? row[24] + row[28] + row[32] : T(0);
    const T uB = (q[1] * q[5] + q[2] * q[6] + q[3] * q[7]) * ir;
    T M[9];
    M[0] = T(0);
    M[1] = q[0] * gv[0] + T(2) * P.Omega * q[2] - db * q[5];
    M[2] = q[0] * gv[1] - T(2) * P.Omega * q[1] - db * q[6];
    M[3] = q[0] * gv[2] - db * q[7];
    M[4] = q[1] * gv[0] + q[2] * gv[1] + q[3] * gv[2] - db * uB;
    M[5] = -db * q[1] * ir;
    M[6] = -db * q[2] * ir;
    M[7] = -db * q[3] * ir;
    M[8] = -P.glm_a * q[8];
    if constexpr (FUSED) {
      // the state itself: this SP's point row (FP64 here)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (sizeof(T) == 8 && R.in[k] == R.Q) {
#pragma unroll
          for (int v = 0; v < 9; ++v) a[k][v] = (double)q[v];
        }
      }
      GBL double* out = R.out + e * 9 * N3 + sp;
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) x += R.alpha[k] * a[k][v];
        out[v * N3] = x + R.beta_dt * (double)(M[v] - div[v] * ji);
      }
    } else {
      GBL T* rp = R.Rp + e * 9 * N3 + sp;
#pragma unroll
      for (int v = 0; v < 9; ++v) rp[v * N3] = M[v] - div[v] * ji;
    }
  }
}

// ---------------------------------------------------------------------------
// k_volume
// ---------------------------------------------------------------------------
// waves per SIMD the volume pass is compiled for (its register budget is
// 512 / waves): FP64 two (LDS also admits two workgroups per CU), FP32 four,
// except N = 4, 5 and 7, whose FP32 passes need more than 128 registers
// (N = 7: and LDS admits fewer workgroups) and get three
#ifndef SDM_VOLUME_WAVES_F64
#define SDM_VOLUME_WAVES_F64 2
#endif
#ifndef SDM_VOLUME_WAVES_F32
#define SDM_VOLUME_WAVES_F32 4
#endif
template <int N, typename T>
constexpr int volume_waves() {
  return sizeof(T) == 8 ? SDM_VOLUME_WAVES_F64
                        : ((N == 4 || N == 5 || N == 7) && SDM_VOLUME_WAVES_F32 > 3 ? 3 : SDM_VOLUME_WAVES_F32);
}

// Interior flux points of one family on FP64 MFMA (v_mfma_f64_4x4x4f64, four
// 4x4 blocks per instruction; lane L supplies A[(L/4)%4][L%4][L/16] and
// B[(L/4)%4][L/16][L%4] and receives D[(L/4)%4][L/16][L%4]).  With the
// interpolation weights I[1 + m][i] as A and the point-row values of 16 lines
// as B, lane o of wave w < 2 receives flux point f = 1 + o/16 of line
// 16 w + o%16, all 36 fields in its accumulators (128 points); wave 2 takes
// the other 52 (f = 1..4 of lines 32..35, f = 5 of every line) on the VALU.
// Degree 5, FP64 only.  Measured no faster than the VALU interpolation
// (same time within 2 %), so it is off unless built with SDM_MFMA_INTERP=1.
#ifndef SDM_MFMA_INTERP
#define SDM_MFMA_INTERP 0
#endif
template <int N, typename T>
constexpr bool mfma_interior() {
  return SDM_MFMA_INTERP && N == 6 && sizeof(T) == 8;
}
// the interior flux point (line, f) of thread tid in that arrangement
__device__ __forceinline__ bool int_fp_mfma6(int tid, int& line, int& f) {
  const int w = tid >> 6, o = tid & 63;
  if (w < 2) {
    f = 1 + (o >> 4);
    line = 16 * w + (o & 15);
    return true;
  }
  if (w == 2 && o < 52) {
    f = o < 16 ? 1 + (o >> 2) : 5;
    line = o < 16 ? 32 + (o & 3) : o - 16;
    return true;
  }
  return false;
}

template <int N, typename T>
struct VolLds {
  static constexpr int N2 = N * N, N3 = N2 * N, NI = N2 * (N - 1), BS = block_threads<N>();
  static constexpr int UN = (9 * NI > 9 * 6 * N2) ? 9 * NI : 9 * 6 * N2;
  static constexpr int RS = row_stride<T>();
  // FP64 rows have two spare slots, where the basis tables live (I in slot
  // 36, D in slot 37, DI after I where the rows leave room)
  static constexpr bool PADTAB = RS >= 38;
  static constexpr bool DIPAD = PADTAB && (N + 1) * N + N * N <= N3;
  static constexpr size_t oR = 0;
  static constexpr size_t oU = al16(oR + sizeof(T) * N3 * RS);
  static constexpr size_t oRed = al16(oU + sizeof(T) * UN);
  static constexpr size_t oI = al16(oRed + sizeof(double) * (BS / 64) * 10);
  static constexpr size_t oD = al16(oI + (PADTAB ? 0 : sizeof(T) * (N + 1) * N));
  static constexpr size_t oDI = al16(oD + (PADTAB ? 0 : sizeof(T) * N * (N + 1)));
  static constexpr size_t oP = al16(oDI + (DIPAD ? 0 : sizeof(T) * N * N));
  static constexpr size_t bytes = al16(oP + sizeof(Phys<T>));
};

template <int N, typename T, bool DIAG>
__device__ __forceinline__ void volume_body(const Run<T>& R, int tid, char* lds) {
  constexpr int N2 = N * N, N3 = N2 * N, NP = N + 1, NF = NP * N2, BS = block_threads<N>();
  constexpr int NI = N2 * (N - 1);  // interior flux points of one family
  // a thread keeps its own face point / interior flux points across phases
  // when one pass covers them all
  constexpr int FL = face_lanes<N>();
  constexpr bool FACE_REG = FL <= BS;
  constexpr bool INT_REG = NI <= BS;
  using Ly = VolLds<N, T>;
  constexpr int RS = Ly::RS;
  constexpr bool PADTAB = Ly::PADTAB, DIPAD = Ly::DIPAD;
  static_assert(!PADTAB || (N + 1) * N <= N3, "tables fit the spare slots");
  // the element's point rows (Q, then grad_x Q)
  T* const sR = reinterpret_cast<T*>(lds + Ly::oR);
  T* const sU = reinterpret_cast<T*>(lds + Ly::oU);  // face jumps (common value - own trace), then fluxes: 9 per point
  double(*const sRed)[10] = reinterpret_cast<double(*)[10]>(lds + Ly::oRed);
  T* const sI = PADTAB ? sR + 36 : reinterpret_cast<T*>(lds + Ly::oI);
  T* const sD = PADTAB ? sR + 37 : reinterpret_cast<T*>(lds + Ly::oD);
  T* const sDI = DIPAD ? sR + 36 + (N + 1) * N * RS : reinterpret_cast<T*>(lds + Ly::oDI);
  constexpr int is = PADTAB ? RS : 1, ds = PADTAB ? RS : 1, dis = DIPAD ? RS : 1;
  // the physical parameters, read from LDS where they are used: held in
  // scalar registers for the whole element they overflow them
  Phys<T>& sP = *reinterpret_cast<Phys<T>*>(lds + Ly::oP);
  static_assert(BS >= N3, "one solution point per thread");
  const DevTab<T>& tb = tab<T>(N);
  const int ia0 = tid % N, ia1 = (tid / N) % N, ia2 = tid / N2;  // this thread's SP (tid < N3)

  {
    const int64_t e = R.e;
    copy_phys<T>(R.P, &sP, tid);
    const Phys<T>& P = sP;  // valid after the barrier that ends phase A
    const GBL double* Qe = R.Q + e * 9 * N3;
    const GBL T* Se = R.S_fp + e * 9 * NF;
    const GBL int32_t* nb6 = R.nbr + e * 6;
    const bool use_kr = R.kr_on;

    // A. every global read of this element is issued before any of them is
    //    used (one round trip, plus one for the neighbour gather that needs
    //    the face's neighbour code): the state and the chain-rule factors and
    //    position of this thread's SP (its state goes to its point row), the normal and outside state of this
    //    thread's face point, the metric at this thread's interior flux points
    //    of the three families, and the basis tables; then the LDS writes.
    // the six neighbour codes are uniform across the workgroup: read through
    // the scalar cache, so that the neighbour gather waits only for them and
    // not (through the in-order vector-load counter) for the element's bulk
    // loads
    int32_t nbc[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) nbc[f] = nb6[f];
    int32_t fcode = 0;
    int lf = 0, lab = 0;  // this lane's face point (face passes)
    const bool has_face = FACE_REG && face_lane<N>(tid, lf, lab);
    T qv[9];
    if (tid < N3) {
#pragma unroll
      for (int v = 0; v < 9; ++v) qv[v] = (T)Qe[v * N3 + tid];
    }
    T ji = T(0), Sj[3][3], xs[3] = {T(0), T(0), T(0)};
    if (tid < N3) {
      ji = (T)R.detJ[e * N3 + tid];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c) Sj[d][c] = (T)R.Sj_sp[(e * 9 + d * 3 + c) * N3 + tid];
#pragma unroll
      for (int c = 0; c < 3; ++c) xs[c] = (T)R.x_sp[(e * 3 + c) * N3 + tid];
    }
    T fq[9], fn[3];  // face point: outside state (neighbour trace or ghost), normal
    if (has_face) load_normal<N>(R, lf, lab, fn);
    T Sint[3][3];  // metric at this thread's interior flux point of each family
    int int_line = tid / (N - 1), int_f = 1 + tid % (N - 1);
    bool int_on = INT_REG && tid < NI;
    if constexpr (mfma_interior<N, T>()) int_on = int_fp_mfma6(tid, int_line, int_f);
    if (!DIAG && int_on) {
      const int line = int_line, f = int_f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int fi = fp_fam<N>(d, f, line % N, line / N);
#pragma unroll
        for (int c = 0; c < 3; ++c) Sint[d][c] = (T)Se[(d * 3 + c) * NF + fi];
      }
    }
    T tI = T(0), tD = T(0), tDI = T(0);
    if (tid < (N + 1) * N) {
      tI = tb.I[tid / N][tid % N];
      tD = tb.D[tid / (N + 1)][tid % (N + 1)];
    }
    if (tid < N * N) tDI = tb.DI[tid / N][tid % N];
    if (has_face) {
      fcode = nbc[0];
#pragma unroll
      for (int f = 1; f < 6; ++f) fcode = lf == f ? nbc[f] : fcode;
      load_outside_state<N>(R, lab, fcode, fq);
    }
    if (tid < N3) {
#pragma unroll
      for (int v = 0; v < 9; ++v) sR[tid * RS + v] = qv[v];
    }
    if (tid < (N + 1) * N) {
      sI[tid * is] = tI;
      sD[tid * ds] = tD;
    }
    if (tid < N * N) sDI[tid * dis] = tDI;
    if (tid < N3) ji = recip(ji);
    __syncthreads();

    // B. BR1 common solution at the 6 N^2 face points (one per thread): the
    //    own trace, and the common value from the outside (neighbour, wall or
    //    ghost) state, stored as the jump (common value - own trace) that
    //    the gradient correction uses.
    for (int it = tid; it < FL; it += BS) {
      int f, ab;
      if (!face_lane<N>(it, f, ab)) continue;
      T q_out[9], n[3];
      int32_t code;
      if (FACE_REG) {
        code = fcode;
#pragma unroll
        for (int v = 0; v < 9; ++v) q_out[v] = fq[v];
        n[0] = fn[0]; n[1] = fn[1]; n[2] = fn[2];
      } else {
        code = nb6[f];
        load_outside<N>(R, f, ab, code, q_out, n);
      }
      // the own trace: Q interpolated along the line to the face
      const int d = f >> 1;
      const int st = d == 0 ? 1 : (d == 1 ? N : N2);
      const int s0 = sp_line<N>(d, ab % N, ab / N, 0);
      const T* wI = sI + ((f & 1) ? N : 0) * N * is;
      // the rows are read two ahead of their use (as in phase C)
      T own[9], wv[N], rv[3][9];
#pragma unroll
      for (int i = 0; i < N; ++i) wv[i] = wI[i * is];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 9; ++v) rv[i][v] = sR[(s0 + i * st) * RS + v];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i + 2 < N) {
#pragma unroll
          for (int v = 0; v < 9; ++v) rv[(i + 2) % 3][v] = sR[(s0 + (i + 2) * st) * RS + v];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < 9; ++v) own[v] = i == 0 ? wv[0] * rv[0][v] : own[v] + wv[i] * rv[i % 3][v];
        __builtin_amdgcn_sched_barrier(0);
      }
      T* dst = sU + (f * N2 + ab) * 9;
      const int g = code >= 0 ? -1 : ((-code - 1) & 3);
      if (code >= 0 || g >= 2 || wsel(g, P.wall_kind) == 1) {
#pragma unroll
        for (int v = 0; v < 9; ++v) dst[v] = T(0.5) * (q_out[v] - own[v]);
      } else {
        T qo[9], qc[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) qo[v] = own[v];
        const T inn = recip(sqrt_fast(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
        const T nh[3] = {n[0] * inn, n[1] * inn, n[2] * inn};
        wall_common(qo, nh, g, P, qc);
#pragma unroll
        for (int v = 0; v < 9; ++v) dst[v] = qc[v] - qo[v];
      }
    }
    __syncthreads();

    // C. gradient at the solution points, one SP per thread: along each
    //    direction d the derivative of the solution polynomial through the
    //    line's N points plus the lifting of the line's two end jumps,
    //    dQ/dxi_d = D_i0 J_0 + D_iN J_N + sum_j DI_ij Q_j, then the chain
    //    rule grad_x Q = sum_d (S^d/|J|) dQ/dxi_d, summed in registers and
    //    written to the gradient slots of the thread's own point row (the
    //    Q slots other threads read are not written).  Each line row is
    //    read as whole 16-byte units.
    if (tid < N3) {
      T g[27];
#pragma unroll
      for (int k = 0; k < 27; ++k) g[k] = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int i = d == 0 ? ia0 : (d == 1 ? ia1 : ia2);
        const int st = d == 0 ? 1 : (d == 1 ? N : N2);
        const int pq = d == 0 ? ia1 + N * ia2 : (d == 1 ? ia0 + N * ia2 : ia0 + N * ia1);
        const T* row0 = sR + (tid - i * st) * RS;
        const T* j0 = sU + ((2 * d) * N2 + pq) * 9;
        const T* jN = sU + ((2 * d + 1) * N2 + pq) * 9;
        // the LDS reads run two rows ahead of their use (scheduling
        // barriers keep the compiler from regrouping them, which would leave
        // only a few reads in flight and a wait for each group in turn)
        const T c0 = sD[(i * NP) * ds], cN = sD[(i * NP + N) * ds];
        T a0[9], aN[9], w[N], rv[3][9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
          a0[v] = j0[v];
          aN[v] = jN[v];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) w[j] = sDI[(i * N + j) * dis];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 9; ++v) rv[j][v] = row0[j * st * RS + v];
        __builtin_amdgcn_sched_barrier(0);
        T dq[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) dq[v] = c0 * a0[v] + cN * aN[v];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          if (j + 2 < N) {
#pragma unroll
            for (int v = 0; v < 9; ++v) rv[(j + 2) % 3][v] = row0[(j + 2) * st * RS + v];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int v = 0; v < 9; ++v) dq[v] += w[j] * rv[j % 3][v];
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int v = 0; v < 9; ++v)
#pragma unroll
          for (int c = 0; c < 3; ++c) g[v * 3 + c] += Sj[d][c] * dq[v];
      }
      T* out = sR + tid * RS + 9;
#pragma unroll
      for (int k = 0; k < 27; ++k) out[k] = g[k];
    }
    __syncthreads();
    if (DIAG) {
      // per-element diagnostics: W^3 |J|-weighted sums, maxima, NaN flag
      double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      if (tid < N3) {
        const int sp = tid;
        // FP64 quadrature weights in either arithmetic
        const DevTab<double>& td = tab<double>(N);
        const double wq = td.W[ia0] * td.W[ia1] * td.W[ia2] * R.detJ64[e * N3 + sp];
        const GBL double* q = Qe + sp;
        const double rho = q[0];
        const double m2 = q[N3] * q[N3] + q[2 * N3] * q[2 * N3] + q[3 * N3] * q[3 * N3];
        const double b2 = q[5 * N3] * q[5 * N3] + q[6 * N3] * q[6 * N3] + q[7 * N3] * q[7 * N3];
        const T* row = sR + sp * RS;
        const double db = (double)row[24] + (double)row[28] + (double)row[32];
        acc[0] = wq;
        acc[1] = wq * rho;
        acc[2] = wq * q[4 * N3];
        acc[3] = wq * 0.5 * m2 / rho;
        acc[4] = wq * 0.5 * b2;
        acc[5] = fabs(db);
        acc[6] = wq * db * db;
        acc[7] = fabs(q[8 * N3]);
        bool bad = false;
        for (int v = 0; v < 9; ++v) bad = bad || !isfinite(q[v * N3]);
        acc[8] = bad ? 1.0 : 0.0;
      }
      // wave reduction in a fixed order, then across waves
      for (int k = 0; k < 9; ++k) {
        double x = acc[k];
        for (int off = 32; off > 0; off >>= 1) {
          const double y = __shfl_down(x, off, 64);
          x = (k == 5 || k == 7 || k == 8) ? fmax(x, y) : x + y;
        }
        if ((tid & 63) == 0 && tid < BS) sRed[tid >> 6][k] = x;
      }
      __syncthreads();
      if (tid == 0) {
        double out[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int wv = 0; wv < BS / 64; ++wv)
          for (int k = 0; k < 9; ++k)
            out[k] = (k == 5 || k == 7 || k == 8) ? fmax(out[k], sRed[wv][k]) : out[k] + sRed[wv][k];
        GBL double* dst = (GBL double*)R.Rp + e * 10;
        for (int k = 0; k < 10; ++k) dst[k] = out[k];
      }
      __syncthreads();
      return;
    }

    // D. fluxes and their divergence.
    //    D1: the 6 N^2 face points (common fluxes) into sU; then per family
    //    d the interior flux points (one per thread, held in registers) while
    //    the SP threads lift the previous pass's fluxes (the faces' before
    //    family 0) into the divergence; then the family's fluxes replace
    //    them in sU.  The last family is lifted after the loop.
    T div[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) div[v] = T(0);
#pragma unroll 1
    for (int it = tid; it < FL; it += BS) {
      int face, ab;
      if (!face_lane<N>(it, face, ab)) continue;
      const int p = ab % N, q = ab / N;
      const int d = face >> 1, fe = (face & 1) ? N : 0;
      const int st = d == 0 ? 1 : (d == 1 ? N : N2);
      const int s0 = sp_line<N>(d, p, q, 0);
      T qf[9], gf[27];
      T kf = interp_rows<N>(sR, sI + fe * N * is, is, s0, st, qf, gf, use_kr, R, P);
      T qx[9], n[3];
      int32_t code;
      if (FACE_REG) {
        code = fcode;
#pragma unroll
        for (int v = 0; v < 9; ++v) qx[v] = fq[v];
        n[0] = fn[0]; n[1] = fn[1]; n[2] = fn[2];
      } else {
        code = nb6[face];
        load_outside<N>(R, face, ab, code, qx, n);
      }
      T F[9];
      ViscLocal<T> vl;
      const int g = code >= 0 ? -1 : ((-code - 1) & 3);
      if (code >= 0 || g == 3) {
        // interior (or import) face: Rusanov on the symmetric normal, own half
        // of the BR1 viscous flux
        PointState<T> ps;
        point_state(qf, P, ps);
        T Fv[7];
        flux_viscous_n(qf, gf, kf, ps, n, P, Fv);
        GBL T* vt = R.Vtr + (e * 6 + face) * 7 * N2 + ab;
#pragma unroll
        for (int c = 0; c < 7; ++c) vt[c * N2] = Fv[c];
        rusanov(qf, qx, n, P, F);
#pragma unroll
        for (int c = 0; c < 7; ++c) F[1 + c] -= T(0.5) * Fv[c];
      } else if (g == 2 || wsel(g, P.wall_kind) == 1) {
        // Dirichlet: Rusanov with the ghost state, BR1 average of the viscous
        // fluxes of both states with the interior gradient
        rusanov(qf, qx, n, P, F);
        T Fv[7];
        PointState<T> ps;
        point_state(qf, P, ps);
        flux_viscous_n(qf, gf, kf, ps, n, P, Fv);
#pragma unroll
        for (int c = 0; c < 7; ++c) F[1 + c] -= T(0.5) * Fv[c];
        point_state(qx, P, ps);
        flux_viscous_n(qx, gf, kf, ps, n, P, Fv);
#pragma unroll
        for (int c = 0; c < 7; ++c) F[1 + c] -= T(0.5) * Fv[c];
      } else {
        // physical wall
        const T nn = sqrt_fast(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const T inn = recip(nn);
        const T nh[3] = {n[0] * inn, n[1] * inn, n[2] * inn};
        wall_mirror(qf, nh, g, P, qx);
        rusanov(qf, qx, n, P, F);
        wall_common(qf, nh, g, P, qx);
        viscous_local(qx, gf, kf, P, vl);
        wall_viscous_sub(vl, n, nh, nn, g, P, F);
      }
      // the flux polynomial of family d takes -F at its coordinate 0, +F at 1
      const T sg = (face & 1) ? T(1) : T(-1);
#pragma unroll
      for (int v = 0; v < 9; ++v) sU[(face * N2 + ab) * 9 + v] = sg * F[v];
    }
    __syncthreads();
    static_assert(INT_REG, "one interior flux point per thread");
    // per family d: the interior fluxes into registers while the SP threads
    // lift the fluxes of the previous pass (the faces before family 0), then
    // the fluxes go to sU once every thread has read the previous ones
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T F[9];
      T qf[9], gf[27], kf = T(0);
      const int st = d == 0 ? 1 : (d == 1 ? N : N2);
      if (mfma_interior<N, T>() && __builtin_amdgcn_readfirstlane(tid >> 6) < 2) {
        // waves 0, 1: 72 MFMAs (36 fields x two K chunks of 4 SPs, the
        // chunk past the line's 6 SPs weighted 0), every lane active
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6), o = tid & 63;
        const int m = o & 3, k = o >> 4;
        const T a0 = sI[((1 + m) * N + k) * is];
        const T a1 = (4 + k < N) ? sI[((1 + m) * N + 4 + k) * is] : T(0);
        const int lineB = 16 * w + (o & 15);
        const int s0B = sp_line<N>(d, lineB % N, lineB / N, 0);
        const T* rb0 = sR + (s0B + k * st) * RS;
        const bool ok1 = 4 + k < N;
        const T* rb1 = sR + (s0B + (ok1 ? 4 + k : 0) * st) * RS;
#pragma unroll
        for (int v = 0; v < 36; ++v) {
          const T b1 = ok1 ? rb1[v] : T(0);
          T x = __builtin_amdgcn_mfma_f64_4x4x4f64(a0, rb0[v], T(0), 0, 0, 0);
          x = __builtin_amdgcn_mfma_f64_4x4x4f64(a1, b1, x, 0, 0, 0);
          if (v < 9) qf[v] = x; else gf[v - 9] = x;
        }
        if (use_kr) {
          const int s0 = sp_line<N>(d, int_line % N, int_line / N, 0);
#pragma unroll 1
          for (int i = 0; i < N; ++i) {
            const int sidx = s0 + i * st;
            const T x[3] = {(T)R.x_sp[(R.e * 3 + 0) * N3 + sidx], (T)R.x_sp[(R.e * 3 + 1) * N3 + sidx],
                            (T)R.x_sp[(R.e * 3 + 2) * N3 + sidx]};
            kf += sI[(int_f * N + i) * is] * kappa_r(x, P);
          }
        }
      } else if (int_on) {
        const int s0 = sp_line<N>(d, int_line % N, int_line / N, 0);
        kf = interp_rows<N>(sR, sI + int_f * N * is, is, s0, st, qf, gf, use_kr, R, P);
      }
      if (int_on) {
        const T Sd[3] = {Sint[d][0], Sint[d][1], Sint[d][2]};
        PointState<T> ps;
        point_state(qf, P, ps);
        T Fv[7];
        flux_viscous_n(qf, gf, kf, ps, Sd, P, Fv);
        flux_inviscid_s(qf, ps, Sd, P, F);
#pragma unroll
        for (int c = 0; c < 7; ++c) F[1 + c] -= Fv[c];
      }
      if (tid < N3) {
        if (d == 0) {
#pragma unroll
          for (int e2 = 0; e2 < 3; ++e2) {
            const int p = e2 == 0 ? ia1 : ia0, q = e2 == 2 ? ia1 : ia2, i = e2 == 0 ? ia0 : (e2 == 1 ? ia1 : ia2);
            const int pq = p + N * q;
            const T d0 = sD[(i * NP) * ds], dN = sD[(i * NP + N) * ds];
#pragma unroll
            for (int v = 0; v < 9; ++v)
              div[v] += d0 * sU[((2 * e2) * N2 + pq) * 9 + v] + dN * sU[((2 * e2 + 1) * N2 + pq) * 9 + v];
          }
        } else {
          lift_family<N>(d - 1, ia0, ia1, ia2, sD, ds, sU, div);
        }
      }
      __syncthreads();
      if (int_on) {
        const int slot = int_line * (N - 1) + int_f - 1;
#pragma unroll
        for (int v = 0; v < 9; ++v) sU[slot * 9 + v] = F[v];
      }
      __syncthreads();
    }
    // E. the last family's lifting, then the sources and the partial
    //    residual; a stage forms its output here (volume_epilogue)
    if constexpr (!DIAG) {
      if (R.fuse) {
        switch (R.n_in) {
          case 1: volume_epilogue<N, T, true, 1>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji); break;
          case 2: volume_epilogue<N, T, true, 2>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji); break;
          case 3: volume_epilogue<N, T, true, 3>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji); break;
          case 4: volume_epilogue<N, T, true, 4>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji); break;
          default: volume_epilogue<N, T, true, 0>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji); break;
        }
      } else {
        volume_epilogue<N, T, false, 0>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji);
      }
    } else {
      volume_epilogue<N, T, false, 0>(R, P, sR, sD, ds, sU, tid, ia0, ia1, ia2, div, xs, ji);
    }
    __syncthreads();
  }
}

template <int N, typename T, bool DIAG>
__global__ __launch_bounds__(block_threads<N>()) __attribute__((amdgpu_waves_per_eu(volume_waves<N, T>())))
void k_volume(Launch L) {
  __shared__ __align__(16) char lds[VolLds<N, T>::bytes];
  // one element per workgroup; no loop, so nothing per element is kept
  // live across elements
  const int64_t w = L.w0 + blockIdx.x;
  if (w >= L.n_work) return;
  volume_body<N, T, DIAG>(view<T>(L, w), threadIdx.x, lds);
}

// the neighbour's viscous normal flux at face point `it` (face it / N^2) of
// element e: its stored flux (orientation-mapped) or, on an import face, the
// caller's; zero on walls and Dirichlet faces (completed in k_volume)
template <int N, typename T>
__device__ __forceinline__ void gather_vflux(const Run<T>& R, const GBL int32_t* nb6, int it, T fv[7]) {
  constexpr int N2 = N * N;
  const int f = it / N2, ab = it % N2;
  // per-lane code load: selecting among six uniform codes by the lane's face
  // is folded by the compiler into a private array in scratch memory
  const int32_t code = nb6[f];
  const GBL T* src = nullptr;
  if (code >= 0) {
    const int64_t en = code >> 6;
    const int fn = (code >> 3) & 7, o = code & 7;
    int a2, b2;
    omap<N>(o, ab % N, ab / N, a2, b2);
    src = R.Vtr + (en * 6 + fn) * 7 * N2 + a2 + N * b2;
  } else if (((-code - 1) & 3) == 3) {
    src = R.imp_v + (int64_t)((-code - 1) >> 2) * 7 * N2 + ab;
  }
  if (src) {
#pragma unroll
    for (int c = 0; c < 7; ++c) fv[c] = src[c * N2];
  } else {
#pragma unroll
    for (int c = 0; c < 7; ++c) fv[c] = T(0);
  }
}

// ---------------------------------------------------------------------------
// k_finish: neighbour half of the viscous common flux, then R or the stage
// ---------------------------------------------------------------------------
template <int N, typename T, bool STAGE>
struct FinLds {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr size_t oV = 0, oOut = al16(oV + sizeof(T) * 6 * 7 * N2);
  static constexpr size_t oI = al16(oOut + sizeof(double) * (STAGE ? 9 * N3 : 1));
  static constexpr size_t oD = al16(oI + sizeof(T) * (N + 1) * N);
  static constexpr size_t bytes = al16(oD + sizeof(T) * N * (N + 1));
};

template <int N, typename T, bool STAGE>
__device__ __forceinline__ void finish_body(const Run<T>& R, int tid, char* lds) {
  constexpr int N2 = N * N, N3 = N2 * N, NP = N + 1, BS = finish_threads<N>();
  static_assert(BS >= N3, "one solution point per thread");
  using Ly = FinLds<N, T, STAGE>;
  T* const sV = reinterpret_cast<T*>(lds + Ly::oV);
  double* const sOut = reinterpret_cast<double*>(lds + Ly::oOut);
  T* const sI = reinterpret_cast<T*>(lds + Ly::oI);
  T* const sD = reinterpret_cast<T*>(lds + Ly::oD);
  {
    const int64_t e = R.e;
    const GBL int32_t* nb6 = R.nbr + e * 6;
    // the neighbours' viscous normal fluxes on the six faces: with one face
    // point per thread they are requested first, into registers, so that
    // they travel with the own-element loads below (one memory round trip)
    constexpr bool GREG = 6 * N2 <= BS;
    T fv[7];
    if constexpr (GREG) {
      if (tid < 6 * N2) gather_vflux<N>(R, nb6, tid, fv);
    }
    // this thread's SP: 1/|J|, and either (stage) the stage output k_volume
    // formed without the neighbour half, or (residual) the partial residual
    const int sp = tid;
    T ji = T(0), rpv[9];  // |J| here; its reciprocal once the loads are issued
    double u[9];
    if (sp < N3) {
      ji = (T)R.detJ[e * N3 + sp];
      if constexpr (STAGE) {
        const GBL double* o = R.out + e * 9 * N3 + sp;
#pragma unroll
        for (int v = 0; v < 9; ++v) u[v] = o[v * N3];
      } else {
        const GBL T* rp = R.Rp + e * 9 * N3 + sp;
#pragma unroll
        for (int v = 0; v < 9; ++v) rpv[v] = rp[v * N3];
      }
    }
    if constexpr (GREG) {
      if (tid < 6 * N2) {
#pragma unroll
        for (int c = 0; c < 7; ++c) sV[((tid / N2) * 7 + c) * N2 + tid % N2] = fv[c];
      }
    } else {
      for (int it = tid; it < 6 * N2; it += BS) {
        gather_vflux<N>(R, nb6, it, fv);
#pragma unroll
        for (int c = 0; c < 7; ++c) sV[((it / N2) * 7 + c) * N2 + it % N2] = fv[c];
      }
    }
    stage_tables<N>(sI, sD, tid, BS);
    __syncthreads();
    if (sp < N3) {
      ji = recip(ji);
      const int ia[3] = {sp % N, (sp / N) % N, sp / N2};
      T corr[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int p = d == 0 ? ia[1] : ia[0], q = d == 2 ? ia[1] : ia[2], i = ia[d];
        const int pq = p + N * q;
        const T w0 = T(-0.5) * sD[i * NP], wN = T(0.5) * sD[i * NP + N];
#pragma unroll
        for (int c = 0; c < 7; ++c)
          corr[c] += w0 * sV[((2 * d) * 7 + c) * N2 + pq] + wN * sV[((2 * d + 1) * 7 + c) * N2 + pq];
      }
      if constexpr (STAGE) {
        // the stage output less beta dt times the neighbour half; rho and psi
        // (no viscous flux) are final as k_volume wrote them
        GBL double* out = R.out + e * 9 * N3 + sp;
#pragma unroll
        for (int v = 0; v < 9; ++v) {
          const double x = (v >= 1 && v <= 7) ? u[v] - R.beta_dt * (double)(corr[v - 1] * ji) : u[v];
          if (v >= 1 && v <= 7) out[v * N3] = x;
          sOut[v * N3 + sp] = x;
        }
      } else {
        GBL double* Ro = R.R + e * 9 * N3 + sp;
#pragma unroll
        for (int v = 0; v < 9; ++v) {
          const T c = (v >= 1 && v <= 7) ? corr[v - 1] : T(0);
          Ro[v * N3] = (double)(rpv[v] - c * ji);
        }
      }
    }
    if (STAGE && R.write_traces) {
      // the new state's face traces for the next stage
      __syncthreads();
      GBL T* tr = R.Qtr + e * 6 * 9 * N2;
      for (int it = tid; it < 6 * 9 * N2; it += BS) {
        const int ab = it % N2, fv = it / N2, v = fv % 9, f = fv / 9;
        const int d = f >> 1;
        const T* wI = sI + ((f & 1) ? N : 0) * N;
        T s = T(0);
#pragma unroll
        for (int i = 0; i < N; ++i) s += wI[i] * (T)sOut[v * N3 + sp_line<N>(d, ab % N, ab / N, i)];
        tr[it] = s;
      }
    }
  }
}

template <int N, typename T, bool STAGE>
__global__ __launch_bounds__(finish_threads<N>()) void k_finish(Launch L) {
  __shared__ __align__(16) char lds[FinLds<N, T, STAGE>::bytes];
  // one element per workgroup; no loop, so nothing per element is kept
  // live across elements
  const int64_t w = L.w0 + blockIdx.x;
  if (w >= L.n_work) return;
  finish_body<N, T, STAGE>(view<T>(L, w), threadIdx.x, lds);
}

// ---------------------------------------------------------------------------
// k_sph_profile: spherical-component sums of one (r, theta) bin per
// workgroup (Sec. "Results": V_phi and V_mer = sqrt(V_r^2 + V_theta^2) for
// the longitude averages, (B_r^2 + B_theta^2)/2 and B_phi^2/2 for the
// poloidal and toroidal energies), weights W_a W_b W_c |J|.  Each thread
// sums its strided share of the bin's SP list in list order, then a fixed
// reduction tree: results are bitwise reproducible.  On the polar axis
// phi_hat = (0, 1, 0) and theta_hat = (sign z, 0, 0).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_sph_profile(const double* Q, const double* x_sp, const double* detJ,
                                                     const int32_t* order, const int64_t* offsets, double* out) {
  constexpr int N3 = N * N * N;
  const DevTab<double>& tb = tab<double>(N);
  const int64_t o0 = offsets[blockIdx.x], o1 = offsets[blockIdx.x + 1];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t j = o0 + threadIdx.x; j < o1; j += 256) {
    const int64_t g = order[j], e = g / N3;
    const int q = (int)(g % N3);
    const double w = tb.W[q % N] * tb.W[(q / N) % N] * tb.W[q / (N * N)] * detJ[e * N3 + q];
    const double x = x_sp[(e * 3 + 0) * N3 + q], y = x_sp[(e * 3 + 1) * N3 + q], z = x_sp[(e * 3 + 2) * N3 + q];
    const double rc = sqrt(x * x + y * y), r = sqrt(x * x + y * y + z * z);
    const double rh[3] = {x / r, y / r, z / r};
    double ph[3], th[3];
    if (rc > 0.0) {
      ph[0] = -y / rc; ph[1] = x / rc; ph[2] = 0.0;
      th[0] = ph[1] * rh[2] - ph[2] * rh[1];
      th[1] = ph[2] * rh[0] - ph[0] * rh[2];
      th[2] = ph[0] * rh[1] - ph[1] * rh[0];
    } else {
      ph[0] = 0.0; ph[1] = 1.0; ph[2] = 0.0;
      th[0] = z >= 0.0 ? 1.0 : -1.0; th[1] = 0.0; th[2] = 0.0;
    }
    const double* s = Q + e * 9 * N3 + q;
    const double u[3] = {s[N3] / s[0], s[2 * N3] / s[0], s[3 * N3] / s[0]};
    const double B[3] = {s[5 * N3], s[6 * N3], s[7 * N3]};
    double ur = 0, ut = 0, up = 0, br = 0, bt = 0, bp = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ur += u[k] * rh[k]; ut += u[k] * th[k]; up += u[k] * ph[k];
      br += B[k] * rh[k]; bt += B[k] * th[k]; bp += B[k] * ph[k];
    }
    acc[0] += w;
    acc[1] += w * up;
    acc[2] += w * sqrt(ur * ur + ut * ut);
    acc[3] += w * 0.5 * (br * br + bt * bt);
    acc[4] += w * 0.5 * bp * bp;
  }
  __shared__ double red[4][5];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int k = threadIdx.x;
    out[blockIdx.x * 5 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// FP64 -> FP32 (round to nearest) copy of n values, grid-stride
__global__ __launch_bounds__(256) void k_to_f32(const double* src, float* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = (float)src[i];
}

// ---------------------------------------------------------------------------
// diagnostics reduction (one block, fixed order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag_reduce(const double* part, int64_t E, double* out) {
  __shared__ double s[256][9];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t e = threadIdx.x; e < E; e += 256)
    for (int k = 0; k < 9; ++k) {
      const double x = part[e * 10 + k];
      acc[k] = (k == 5 || k == 7 || k == 8) ? fmax(acc[k], x) : acc[k] + x;
    }
  for (int k = 0; k < 9; ++k) s[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < 256; ++t)
      for (int k = 0; k < 9; ++k) r[k] = (k == 5 || k == 7 || k == 8) ? fmax(r[k], s[t][k]) : r[k] + s[t][k];
    const double V = r[0];
    out[0] = V;
    out[1] = r[1];
    out[2] = r[2];
    out[3] = r[3] / V;
    out[4] = r[4] / V;
    out[5] = r[5];
    out[6] = sqrt(r[6] / V);
    out[7] = r[7];
    out[8] = r[8];
    for (int k = 9; k < 16; ++k) out[k] = 0.0;
  }
}

}  // namespace sdm

// ===========================================================================
// host side: contexts, launches, C ABI
// ===========================================================================
using namespace sdm;

namespace {

thread_local std::string g_err;

sdm_status fail(sdm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(SDM_EHIP, std::string(#expr ": ") + hipGetErrorString(_e));          \
  } while (0)

std::mutex g_tab_mu;
bool g_tab_ready[64] = {false};

sdm_status upload_tables(int device) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  if (device < 0 || device >= 64) return fail(SDM_EINVAL, "device index out of range");
  if (g_tab_ready[device]) return SDM_OK;
  std::vector<DevTab<double>> td(kNMax + 1);
  std::vector<DevTab<float>> tf(kNMax + 1);
  std::memset(td.data(), 0, sizeof(DevTab<double>) * td.size());
  std::memset(tf.data(), 0, sizeof(DevTab<float>) * tf.size());
  for (int N = 2; N <= kNMax; ++N) {
    Tables1D t = make_tables(N);
    for (int f = 0; f <= N; ++f)
      for (int i = 0; i < N; ++i) td[N].I[f][i] = t.I[f * N + i];
    for (int i = 0; i < N; ++i)
      for (int f = 0; f <= N; ++f) td[N].D[i][f] = t.D[i * (N + 1) + f];
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) td[N].DI[i][j] = t.DI[i * N + j];
    for (int i = 0; i < N; ++i) td[N].W[i] = t.W[i];
    const double* s = (const double*)&td[N];
    float* d = (float*)&tf[N];
    for (size_t k = 0; k < sizeof(DevTab<double>) / sizeof(double); ++k) d[k] = (float)s[k];
  }
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_d), td.data(), sizeof(DevTab<double>) * td.size()));
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_f), tf.data(), sizeof(DevTab<float>) * tf.size()));
  g_tab_ready[device] = true;
  return SDM_OK;
}

std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {nullptr};

// Device address of `scratch` on `device` (which must be current): looked up
// once per device; each device holds its own copy at its own address.
sdm_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= 64) return fail(SDM_EINVAL, "device index out of range");
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SDM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return SDM_OK;
}

Phys<double> to_phys(const sdm_params* p) {
  Phys<double> o;
  o.gamma = p->gamma;
  o.gm1 = p->gamma - 1.0;
  o.Rgas = p->Rgas;
  o.cp = p->gamma * p->Rgas / (p->gamma - 1.0);
  o.inv_R = 1.0 / p->Rgas;
  o.inv_gamma = 1.0 / p->gamma;
  o.inv_gm1 = 1.0 / (p->gamma - 1.0);
  o.GM = p->GM; o.Omega = p->Omega; o.nu = p->nu; o.kappa = p->kappa; o.eta = p->eta;
  o.kr_scale = p->kr_scale; o.kr_c0 = p->kr_c0; o.kr_c1 = p->kr_c1; o.kr_c2 = p->kr_c2;
  o.kr_w = p->kr_omega_per_r;
  o.c_h = p->c_h; o.glm_a = p->glm_a;
  o.q_wall[0] = p->q_wall[0]; o.q_wall[1] = p->q_wall[1];
  o.T_wall[0] = p->T_wall[0]; o.T_wall[1] = p->T_wall[1];
  o.powell = p->powell;
  for (int g = 0; g < 2; ++g) {
    o.wall_kind[g] = p->wall_kind[g];
    o.wall_mag[g] = p->wall_mag[g];
    o.wall_th[g] = p->wall_th[g];
  }
  return o;
}

}  // namespace

struct sdm_ctx {
  int device = 0;
  void* scratch = nullptr;  // device address of this device's `scratch`
  int p = 5;
  int N = 6;
  int arith = 0;
  bool bound = false;
  sdm_mesh mesh{};
  // mixed arithmetic: FP32 copies of x_sp, detJ, S_fp, Sj_sp, n_face (one
  // device allocation, made by sdm_mesh_bind, released by sdm_destroy)
  float* geo32 = nullptr;
  size_t geo32_off[5] = {0, 0, 0, 0, 0};
  int64_t n_group[4] = {0, 0, 0, 0};  // boundary faces per group
  // optional per-kernel timing: events recorded around every launch
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (kernel id, start event index)
};

namespace {

size_t real_size(const sdm_ctx* c) { return c->arith ? sizeof(float) : sizeof(double); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// workspace pieces: Qtr | Vtr | Rp (Rp also holds diagnostics partials)
void ws_layout(const sdm_ctx* c, size_t off[4]) {
  const int64_t E = c->mesh.n_elem;
  const int N = c->N;
  const size_t rs = real_size(c);
  const size_t qtr = align256((size_t)E * 6 * 9 * N * N * rs);
  const size_t vtr = align256((size_t)E * 6 * 7 * N * N * rs);
  const size_t rp = align256(std::max((size_t)E * 9 * N * N * N * rs, (size_t)E * 10 * sizeof(double)));
  off[0] = 0;
  off[1] = qtr;
  off[2] = qtr + vtr;
  off[3] = qtr + vtr + rp;
}

sdm_status check_params(const sdm_ctx* c, const sdm_params* p) {
  if (!p) return fail(SDM_EINVAL, "params is NULL");
  if (!(p->gamma > 1.0) || !(p->Rgas > 0.0)) return fail(SDM_EINVAL, "gamma must exceed 1 and Rgas be positive");
  for (int g = 0; g < 2; ++g) {
    if (p->wall_kind[g] < 0 || p->wall_kind[g] > 1 || p->wall_mag[g] < 0 || p->wall_mag[g] > 1 ||
        p->wall_th[g] < 0 || p->wall_th[g] > 1)
      return fail(SDM_EINVAL, "wall selector out of range");
  }
  const bool need_ghost = c->n_group[2] > 0 || (c->n_group[0] > 0 && p->wall_kind[0] == 1) ||
                          (c->n_group[1] > 0 && p->wall_kind[1] == 1);
  if (need_ghost && !p->ghost) return fail(SDM_EINVAL, "Dirichlet faces present but ghost is NULL");
  if (c->n_group[3] > 0 && (!p->import_q || !p->import_v))
    return fail(SDM_EINVAL, "import faces present but import_q or import_v is NULL");
  return SDM_OK;
}

RunDesc make_desc(const sdm_ctx* c, const sdm_params* p, const double* Q, void* ws) {
  RunDesc r;
  std::memset(&r, 0, sizeof r);
  size_t off[4];
  ws_layout(c, off);
  r.N = c->N;
  r.E = c->mesh.n_elem;
  r.n_bfaces = c->mesh.n_bfaces;
  r.x_sp = c->mesh.x_sp;
  r.detJ = c->mesh.detJ;
  r.S_fp = c->mesh.S_fp;
  r.Sj_sp = c->mesh.Sj_sp;
  r.nbr = c->mesh.nbr;
  r.n_face = c->mesh.n_face;
  if (c->geo32) {
    r.x_sp_f = c->geo32 + c->geo32_off[0];
    r.detJ_f = c->geo32 + c->geo32_off[1];
    r.S_fp_f = c->geo32 + c->geo32_off[2];
    r.Sj_sp_f = c->geo32 + c->geo32_off[3];
    r.n_face_f = c->geo32 + c->geo32_off[4];
  }
  r.ghost = p ? p->ghost : nullptr;
  r.imp_q = p ? p->import_q : nullptr;
  r.imp_v = p ? p->import_v : nullptr;
  r.Q = Q;
  r.Qtr = (char*)ws + off[0];
  r.Vtr = (char*)ws + off[1];
  r.Rp = (char*)ws + off[2];
  if (p) r.P = to_phys(p);
  return r;
}

template <int N, typename T>
hipError_t launch_all(int which, const Launch& L, hipStream_t s, int64_t cap) {
  constexpr int BS = block_threads<N>();
  // at most `cap` workgroups per launch: consecutive launches cover the work
  const int64_t step = std::min<int64_t>(cap, (int64_t)1 << 30);
  for (int64_t w0 = L.w0; w0 < L.n_work; w0 += step) {
    Launch Lc = L;
    Lc.w0 = w0;
    const unsigned grid = (unsigned)std::min<int64_t>(L.n_work - w0, step);
    switch (which) {
      case 0: hipLaunchKernelGGL((k_traces<N, T>), dim3(grid), dim3(BS), 0, s, Lc); break;
      case 1: hipLaunchKernelGGL((k_volume<N, T, false>), dim3(grid), dim3(BS), 0, s, Lc); break;
      case 2: hipLaunchKernelGGL((k_volume<N, T, true>), dim3(grid), dim3(BS), 0, s, Lc); break;
      case 3: hipLaunchKernelGGL((k_finish<N, T, false>), dim3(grid), dim3(finish_threads<N>()), 0, s, Lc); break;
      case 4: hipLaunchKernelGGL((k_finish<N, T, true>), dim3(grid), dim3(finish_threads<N>()), 0, s, Lc); break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t dispatch_N(int N, int which, const Launch& L, hipStream_t s, int64_t cap);
template <typename T>
hipError_t dispatch_N(int N, int which, const Launch& L, hipStream_t s) {
  return dispatch_N<T>(N, which, L, s, (int64_t)1 << 30);
}
template <typename T>
hipError_t dispatch_N(int N, int which, const Launch& L, hipStream_t s, int64_t cap) {
  switch (N) {
    case 2: return launch_all<2, T>(which, L, s, cap);
    case 3: return launch_all<3, T>(which, L, s, cap);
    case 4: return launch_all<4, T>(which, L, s, cap);
    case 5: return launch_all<5, T>(which, L, s, cap);
    case 6: return launch_all<6, T>(which, L, s, cap);
    case 7: return launch_all<7, T>(which, L, s, cap);
    default: return hipErrorInvalidValue;
  }
}

sdm_status run_capped(sdm_ctx* c, int which, const Launch& L, hipStream_t s, int64_t cap);
sdm_status run(sdm_ctx* c, int which, const Launch& L, hipStream_t s) { return run_capped(c, which, L, s, (int64_t)1 << 30); }
sdm_status run_capped(sdm_ctx* c, int which, const Launch& L, hipStream_t s, int64_t cap) {
  size_t e0 = 0;
  if (c->prof) {
    while (c->ev.size() < c->ev_used + 2) {
      hipEvent_t h;
      HIP_TRY(hipEventCreate(&h));
      c->ev.push_back(h);
    }
    e0 = c->ev_used;
    c->ev_used += 2;
    HIP_TRY(hipEventRecord(c->ev[e0], s));
  }
  hipError_t e = c->arith ? dispatch_N<float>(c->N, which, L, s, cap) : dispatch_N<double>(c->N, which, L, s, cap);
  if (e != hipSuccess) return fail(SDM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  if (c->prof) {
    HIP_TRY(hipEventRecord(c->ev[e0 + 1], s));
    c->marks.emplace_back(which, e0);
  }
  return SDM_OK;
}

Launch single(const RunDesc& r) {
  Launch L;
  std::memset(&L, 0, sizeof L);
  L.one = r;
  L.many = nullptr;
  L.prefix = nullptr;
  L.n_run = 1;
  L.n_work = r.E;
  return L;
}

}  // namespace

namespace {

// Pinned host staging for batch descriptor tables: a small ring of buffers,
// each reused only after the copy that last read it has completed.
struct Staging {
  std::mutex mu;
  struct Slot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
  };
  Slot slot[8];
  int next = 0;
};
Staging g_stage;

sdm_status stage_copy(const void* src, size_t bytes, void* dst_dev, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_stage.mu);
  Staging::Slot& sl = g_stage.slot[g_stage.next];
  g_stage.next = (g_stage.next + 1) % 8;
  if (sl.pending) {
    HIP_TRY(hipEventSynchronize(sl.done));
    sl.pending = false;
  }
  if (sl.cap < bytes) {
    if (sl.host) HIP_TRY(hipHostFree(sl.host));
    sl.host = nullptr;
    sl.cap = 0;
    HIP_TRY(hipHostMalloc(&sl.host, bytes, hipHostMallocDefault));
    sl.cap = bytes;
  }
  if (!sl.done) HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  std::memcpy(sl.host, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst_dev, sl.host, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(sl.done, s));
  sl.pending = true;
  return SDM_OK;
}

// Batch workspace: the work lists of the batch, one per pass kind, each
// with the runs of every degree group stored contiguously (descriptors, then
// element offsets with one extra entry per group): [runs | offsets] for the
// volume and finish passes, then the same for the runs whose traces must be
// computed first.  At most kBatchGroups degrees (N = 2 .. 7).
constexpr int kBatchGroups = 6;
size_t batch_list_bytes(int n) {
  return align256(sizeof(RunDesc) * (size_t)n) + align256(sizeof(int64_t) * (size_t)(n + kBatchGroups));
}
size_t batch_ws_bytes(int n) { return 2 * batch_list_bytes(n); }

// Library-owned streams and events of one device for the degree groups of a
// batch after the first (default priority; created once, kept until exit).
struct BatchStreams {
  hipStream_t side[kBatchGroups] = {};
  hipEvent_t fork = nullptr, join[kBatchGroups] = {};
};
std::mutex g_bs_mu;
BatchStreams g_bs[64];
// held while one call enqueues on a device's library streams and records
// their fork and join events, so that calls from several host threads do
// not interleave their records and waits
std::mutex g_bs_enqueue[64];

sdm_status batch_streams(int device, int n_side, BatchStreams** out) {
  std::lock_guard<std::mutex> lk(g_bs_mu);
  BatchStreams& b = g_bs[device];
  if (!b.fork) HIP_TRY(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
  for (int k = 0; k < n_side; ++k) {
    if (!b.side[k]) HIP_TRY(hipStreamCreateWithFlags(&b.side[k], hipStreamNonBlocking));
    if (!b.join[k]) HIP_TRY(hipEventCreateWithFlags(&b.join[k], hipEventDisableTiming));
  }
  *out = &b;
  return SDM_OK;
}
}  // namespace

extern "C" {

const char* sdm_last_error(void) { return g_err.c_str(); }

const char* sdm_version(void) { return "sdmhd-gfx950 0.1"; }

sdm_status sdm_shell_sizes(int Nz, int Nr, int64_t* n_elem, int64_t* n_bfaces) {
  if (Nz < 1 || Nr < 1 || !n_elem) return fail(SDM_EINVAL, "shell sizes: Nz, Nr >= 1 and n_elem required");
  *n_elem = 6LL * Nz * Nz * Nr;
  if (n_bfaces) *n_bfaces = 12LL * Nz * Nz;
  return SDM_OK;
}

sdm_status sdm_shell_build(int Nz, int Nr, int p, double rb, double rt, double* x_sp, double* detJ,
                           double* S_fp, double* Sj_sp, int32_t* nbr, double* n_face) {
  if (Nz < 1 || Nr < 1 || p < 1 || p > kNMax - 1 || !(rb > 0) || !(rt > rb))
    return fail(SDM_EINVAL, "shell build: need Nz, Nr >= 1, 1 <= p <= 7, 0 < rb < rt");
  if (!x_sp || !detJ || !S_fp || !Sj_sp || !nbr || !n_face) return fail(SDM_EINVAL, "shell build: NULL output");
  if (shell_build(Nz, Nr, p, rb, rt, x_sp, detJ, S_fp, Sj_sp, nbr, n_face))
    return fail(SDM_EINVAL, "shell connectivity failed");
  return SDM_OK;
}

sdm_status sdm_box_sizes(int nx, int ny, int nz, int periodic, int64_t* n_elem, int64_t* n_bfaces) {
  const int n[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || (((periodic >> d) & 1) && n[d] < 3))
      return fail(SDM_EINVAL, "box: >= 1 element per direction, >= 3 in periodic ones");
  if (!n_elem) return fail(SDM_EINVAL, "box sizes: n_elem is NULL");
  *n_elem = (int64_t)nx * ny * nz;
  if (n_bfaces) {
    int64_t nb = 0;
    if (!(periodic & 1)) nb += 2LL * ny * nz;
    if (!(periodic & 2)) nb += 2LL * nx * nz;
    if (!(periodic & 4)) nb += 2LL * nx * ny;
    *n_bfaces = nb;
  }
  return SDM_OK;
}

sdm_status sdm_box_build(int nx, int ny, int nz, double Lx, double Ly, double Lz, int periodic, double warp,
                         int p, double* x_sp, double* detJ, double* S_fp, double* Sj_sp, int32_t* nbr,
                         double* n_face) {
  int64_t E;
  sdm_status st = sdm_box_sizes(nx, ny, nz, periodic, &E, nullptr);
  if (st != SDM_OK) return st;
  if (p < 1 || p > kNMax - 1 || !(Lx > 0) || !(Ly > 0) || !(Lz > 0))
    return fail(SDM_EINVAL, "box build: need 1 <= p <= 7 and positive lengths");
  if (!x_sp || !detJ || !S_fp || !Sj_sp || !nbr || !n_face) return fail(SDM_EINVAL, "box build: NULL output");
  if (box_build(nx, ny, nz, Lx, Ly, Lz, periodic, warp, p, x_sp, detJ, S_fp, Sj_sp, nbr, n_face))
    return fail(SDM_EINVAL, "box connectivity failed");
  return SDM_OK;
}

sdm_status sdm_tables(int p, double* xs, double* xf, double* I, double* D, double* W) {
  if (p < 1 || p > kNMax - 1) return fail(SDM_EINVAL, "tables: 1 <= p <= 7");
  if (!xs || !xf || !I || !D || !W) return fail(SDM_EINVAL, "tables: NULL output");
  Tables1D t = make_tables(p + 1);
  std::copy(t.xs.begin(), t.xs.end(), xs);
  std::copy(t.xf.begin(), t.xf.end(), xf);
  std::copy(t.I.begin(), t.I.end(), I);
  std::copy(t.D.begin(), t.D.end(), D);
  std::copy(t.W.begin(), t.W.end(), W);
  return SDM_OK;
}

sdm_status sdm_create(int device, int p, int arith, sdm_ctx** out) {
  if (!out) return fail(SDM_EINVAL, "create: out is NULL");
  if (p < 1 || p > 6) return fail(SDM_EUNSUPPORTED, "create: the device kernels support 1 <= p <= 6");
  if (arith != 0 && arith != 1) return fail(SDM_EINVAL, "create: arith must be 0 (FP64) or 1 (mixed)");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SDM_EINVAL, "create: no such device");
  HIP_TRY(hipSetDevice(device));
  sdm_status st = upload_tables(device);
  if (st != SDM_OK) return st;
  void* scr = nullptr;
  if ((st = scratch_address(device, &scr)) != SDM_OK) return st;
  sdm_ctx* c = new sdm_ctx;
  c->device = device;
  c->scratch = scr;
  c->p = p;
  c->N = p + 1;
  c->arith = arith;
  *out = c;
  return SDM_OK;
}

sdm_status sdm_destroy(sdm_ctx* c) {
  if (c) {
    (void)hipSetDevice(c->device);
    for (hipEvent_t h : c->ev) (void)hipEventDestroy(h);
    if (c->geo32) (void)hipFree(c->geo32);
  }
  delete c;
  return SDM_OK;
}

sdm_status sdm_profile_enable(sdm_ctx* c, int enable) {
  if (!c) return fail(SDM_EINVAL, "profile_enable: NULL context");
  c->prof = enable != 0;
  c->ev_used = 0;
  c->marks.clear();
  return SDM_OK;
}

sdm_status sdm_profile_read(sdm_ctx* c, double* ms, int64_t* count) {
  if (!c || !ms || !count) return fail(SDM_EINVAL, "profile_read: NULL argument");
  for (int k = 0; k < 8; ++k) { ms[k] = 0.0; count[k] = 0; }
  HIP_TRY(hipSetDevice(c->device));
  for (const auto& m : c->marks) {
    HIP_TRY(hipEventSynchronize(c->ev[m.second + 1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, c->ev[m.second], c->ev[m.second + 1]));
    ms[m.first] += t;
    count[m.first] += 1;
  }
  c->ev_used = 0;
  c->marks.clear();
  return SDM_OK;
}

sdm_status sdm_mesh_bind(sdm_ctx* c, const sdm_mesh* m) {
  if (!c || !m) return fail(SDM_EINVAL, "mesh_bind: NULL argument");
  if (m->n_elem < 1 || m->n_bfaces < 0 || m->n_elem >= ((int64_t)1 << 25))
    return fail(SDM_EINVAL, "mesh_bind: 1 <= n_elem < 2^25 required");
  if (!m->x_sp || !m->detJ || !m->S_fp || !m->Sj_sp || !m->nbr || !m->n_face)
    return fail(SDM_EINVAL, "mesh_bind: NULL array");
  // validate the neighbour table on the host: every code must decode into range
  std::vector<int32_t> nb((size_t)m->n_elem * 6);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpy(nb.data(), m->nbr, sizeof(int32_t) * nb.size(), hipMemcpyDeviceToHost));
  int64_t ng[4] = {0, 0, 0, 0};
  for (int64_t i = 0; i < (int64_t)nb.size(); ++i) {
    const int32_t code = nb[i];
    if (code >= 0) {
      const int64_t en = code >> 6;
      const int fn = (code >> 3) & 7;
      if (en >= m->n_elem || fn > 5) return fail(SDM_EINVAL, "mesh_bind: neighbour code out of range");
    } else {
      const int64_t c2 = -(int64_t)code - 1;
      const int g = (int)(c2 & 3);
      const int64_t bf = c2 >> 2;
      if (bf >= m->n_bfaces) return fail(SDM_EINVAL, "mesh_bind: boundary code out of range");
      ++ng[g];
    }
  }
  if (c->geo32) {
    HIP_TRY(hipFree(c->geo32));
    c->geo32 = nullptr;
  }
  c->bound = false;
  if (c->arith == 1) {
    // the FP32 kernels convert every geometry value to FP32 on use; they read
    // these copies instead (the same values, half the bytes)
    const int64_t E = m->n_elem, N = c->N, N2 = N * N, N3 = N2 * N, NF = (N + 1) * N2;
    const int64_t cnt[5] = {E * 3 * N3, E * N3, E * 9 * NF, E * 9 * N3, E * 6 * 3 * N2};
    const double* src[5] = {m->x_sp, m->detJ, m->S_fp, m->Sj_sp, m->n_face};
    size_t total = 0;
    for (int k = 0; k < 5; ++k) {
      c->geo32_off[k] = total;
      total += (size_t)((cnt[k] + 63) & ~int64_t(63));  // 256-byte aligned pieces
    }
    HIP_TRY(hipMalloc((void**)&c->geo32, total * sizeof(float)));
    for (int k = 0; k < 5; ++k) {
      const int64_t blocks = std::min<int64_t>((cnt[k] + 255) / 256, 65536);
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, nullptr, src[k], c->geo32 + c->geo32_off[k],
                         cnt[k]);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(nullptr));
  }
  c->mesh = *m;
  for (int g = 0; g < 4; ++g) c->n_group[g] = ng[g];
  c->bound = true;
  return SDM_OK;
}

sdm_status sdm_background_profile(const sdm_background* bg, int64_t n, const double* r, double* rho, double* p,
                                  double* T) {
  if (!bg || n < 0 || (n > 0 && (!r || !rho || !p || !T))) return fail(SDM_EINVAL, "background_profile: NULL argument");
  Background b;
  b.GM = bg->GM; b.Rgas = bg->Rgas; b.gamma = bg->gamma; b.rb = bg->rb; b.rt = bg->rt;
  b.rho_b = bg->rho_b; b.N_rho = bg->N_rho; b.L = bg->L; b.kappa = bg->kappa;
  b.kr_scale = bg->kr_scale; b.kr_c0 = bg->kr_c0; b.kr_c1 = bg->kr_c1; b.kr_c2 = bg->kr_c2;
  b.kr_w = bg->kr_omega_per_r; b.flux_balanced = bg->flux_balanced;
  switch (background_profile(b, n, r, rho, p, T)) {
    case 0: return SDM_OK;
    case 2: return fail(SDM_EINVAL, "background_profile: radius outside [rb, rt]");
    case 3: return fail(SDM_EINVAL, "background_profile: the flux-balanced density reaches zero (no hydrostatic profile)");
    default: return fail(SDM_EINVAL, "background_profile: need gamma > 1, Rgas, GM, rho_b, N_rho > 0, 0 < rb < rt "
                                     "and kappa > 0 for the flux-balanced profile");
  }
}

sdm_status sdm_workspace_size(const sdm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(SDM_EINVAL, "workspace_size: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "workspace_size: no mesh bound");
  size_t off[4];
  ws_layout(c, off);
  *bytes = off[3];
  return SDM_OK;
}

sdm_status sdm_workspace_traces(const sdm_ctx* c, void* ws, void** q_traces, void** v_traces) {
  if (!c || !ws || !q_traces || !v_traces) return fail(SDM_EINVAL, "workspace_traces: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "workspace_traces: no mesh bound");
  size_t off[4];
  ws_layout(c, off);
  *q_traces = (char*)ws + off[0];
  *v_traces = (char*)ws + off[1];
  return SDM_OK;
}

sdm_status sdm_residual(sdm_ctx* c, const sdm_params* p, const double* Q, double* R, void* ws, void* stream) {
  if (!c || !Q || !R || !ws) return fail(SDM_EINVAL, "residual: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "residual: no mesh bound");
  sdm_status st = check_params(c, p);
  if (st != SDM_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  RunDesc r = make_desc(c, p, Q, ws);
  r.R = R;
  Launch L = single(r);
  if ((st = run(c, 0, L, s)) != SDM_OK) return st;
  if ((st = run(c, 1, L, s)) != SDM_OK) return st;
  return run(c, 3, L, s);
}

namespace {
// the launches of one stage: `parts` bit 0 = traces (unless valid) and
// volume, bit 1 = finish (neighbour viscous half + Shu-Osher update)
sdm_status stage_parts(sdm_ctx* c, const sdm_params* p, double* const* regs, int n_regs, const sdm_stage* stg,
                       double dt, void* ws, void* stream, int parts, const char* who) {
  if (!c || !regs || !stg || !ws) return fail(SDM_EINVAL, std::string(who) + ": NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, std::string(who) + ": no mesh bound");
  if (n_regs < 1 || n_regs > 16) return fail(SDM_EINVAL, std::string(who) + ": 1 <= n_regs <= 16");
  if (stg->n_in < 0 || stg->n_in > 4) return fail(SDM_EINVAL, std::string(who) + ": 0 <= n_in <= 4");
  auto okreg = [&](int i) { return i >= 0 && i < n_regs && regs[i] != nullptr; };
  if (!okreg(stg->cur) || !okreg(stg->out))
    return fail(SDM_EINVAL, std::string(who) + ": register index out of range");
  for (int k = 0; k < stg->n_in; ++k)
    if (!okreg(stg->in_idx[k])) return fail(SDM_EINVAL, std::string(who) + ": input register out of range");
  sdm_status st = check_params(c, p);
  if (st != SDM_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  RunDesc r = make_desc(c, p, regs[stg->cur], ws);
  for (int k = 0; k < stg->n_in; ++k) {
    r.in[k] = regs[stg->in_idx[k]];
    r.alpha[k] = stg->alpha[k];
  }
  r.n_in = stg->n_in;
  r.out = regs[stg->out];
  r.beta_dt = stg->beta * dt;
  r.write_traces = 1;
  r.fuse = 1;  // k_volume forms the stage output
  r.Rp = nullptr;  // a stage never uses the partial-residual region
  Launch L = single(r);
  if (parts & 1) {
    if (!stg->traces_valid && (st = run(c, 0, L, s)) != SDM_OK) return st;
    if ((st = run(c, 1, L, s)) != SDM_OK) return st;
  }
  if (parts & 2) return run(c, 4, L, s);
  return SDM_OK;
}
}  // namespace

sdm_status sdm_rk_stage(sdm_ctx* c, const sdm_params* p, double* const* regs, int n_regs,
                        const sdm_stage* stg, double dt, void* ws, void* stream) {
  return stage_parts(c, p, regs, n_regs, stg, dt, ws, stream, 3, "rk_stage");
}

sdm_status sdm_rk_stage_volume(sdm_ctx* c, const sdm_params* p, double* const* regs, int n_regs,
                               const sdm_stage* stg, double dt, void* ws, void* stream) {
  return stage_parts(c, p, regs, n_regs, stg, dt, ws, stream, 1, "rk_stage_volume");
}

sdm_status sdm_rk_stage_finish(sdm_ctx* c, const sdm_params* p, double* const* regs, int n_regs,
                               const sdm_stage* stg, double dt, void* ws, void* stream) {
  return stage_parts(c, p, regs, n_regs, stg, dt, ws, stream, 2, "rk_stage_finish");
}

sdm_status sdm_ssprk53_stages(sdm_stage* out, double* c) {
  if (!out) return fail(SDM_EINVAL, "ssprk53_stages: out is NULL");
  ShuOsherStage st[5];
  double cc[5];
  ssprk53_stages(st, cc);
  for (int i = 0; i < 5; ++i) {
    sdm_stage& o = out[i];
    std::memset(&o, 0, sizeof o);
    o.n_in = st[i].n_in;
    for (int k = 0; k < 4; ++k) {
      o.in_idx[k] = st[i].in_idx[k];
      o.alpha[k] = st[i].alpha[k];
    }
    o.cur = st[i].cur;
    o.out = st[i].out;
    o.beta = st[i].beta;
    o.traces_valid = 1;  // each stage's input is the previous stage's output
  }
  out[0].traces_valid = 0;
  if (c) std::copy(cc, cc + 5, c);
  return SDM_OK;
}

sdm_status sdm_ssprk53_step(sdm_ctx* c, const sdm_params* p, double* const* regs, double dt, int traces_valid,
                            void* ws, void* stream) {
  if (!regs) return fail(SDM_EINVAL, "ssprk53_step: NULL argument");
  sdm_stage st[5];
  sdm_status s = sdm_ssprk53_stages(st, nullptr);
  if (s != SDM_OK) return s;
  st[0].traces_valid = traces_valid ? 1 : 0;
  for (int i = 0; i < 5; ++i)
    if ((s = stage_parts(c, p, regs, 4, &st[i], dt, ws, stream, 3, "ssprk53_step")) != SDM_OK) return s;
  return SDM_OK;
}

sdm_status sdm_ssprk53_step_noalloc(sdm_ctx* c, const sdm_params* p, double* const* regs, double dt,
                                    void* stream) {
  if (!c || !regs) return fail(SDM_EINVAL, "ssprk53_step_noalloc: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "ssprk53_step_noalloc: no mesh bound");
  if (!c->scratch) return fail(SDM_ESTATE, "ssprk53_step_noalloc: no scratch address for this device");
  size_t off[4];
  ws_layout(c, off);
  const size_t need = off[2];  // the two trace regions; a stage leaves the rest unused
  if (need > kScratchBytes) {
    const size_t per = need / (size_t)c->mesh.n_elem;
    return fail(SDM_EINVAL, "ssprk53_step_noalloc: the mesh needs " + std::to_string(need) +
                                " bytes of face-trace scratch, the maximum is " + std::to_string(kScratchBytes) +
                                " (" + std::to_string(kScratchBytes / per) + " elements at this degree and arithmetic)");
  }
  sdm_stage st[5];
  sdm_status s = sdm_ssprk53_stages(st, nullptr);
  if (s != SDM_OK) return s;
  // the scratch holds whatever the last call on this device left: the first
  // stage always computes the traces of regs[0]
  st[0].traces_valid = 0;
  for (int i = 0; i < 5; ++i)
    if ((s = stage_parts(c, p, regs, 4, &st[i], dt, c->scratch, stream, 3, "ssprk53_step_noalloc")) != SDM_OK)
      return s;
  return SDM_OK;
}

sdm_status sdm_diagnostics(sdm_ctx* c, const sdm_params* p, const double* Q, double* out, void* ws,
                           void* stream) {
  if (!c || !Q || !out || !ws) return fail(SDM_EINVAL, "diagnostics: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "diagnostics: no mesh bound");
  sdm_status st = check_params(c, p);
  if (st != SDM_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  RunDesc r = make_desc(c, p, Q, ws);
  Launch L = single(r);
  if ((st = run(c, 0, L, s)) != SDM_OK) return st;
  if ((st = run(c, 2, L, s)) != SDM_OK) return st;
  hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(256), 0, s, (const double*)r.Rp, r.E, out);
  HIP_TRY(hipGetLastError());
  return SDM_OK;
}


sdm_status sdm_sph_bins(int64_t n_elem, int p, const double* x_sp, double rb, double rt, int n_r, int n_th,
                        int32_t* order, int64_t* offsets) {
  if (n_elem < 1 || p < 1 || p > kNMax - 1 || !x_sp || !order || !offsets)
    return fail(SDM_EINVAL, "sph_bins: need n_elem >= 1, 1 <= p <= 7 and non-NULL buffers");
  if (n_r < 1 || n_th < 1 || !(rt > rb)) return fail(SDM_EINVAL, "sph_bins: need n_r, n_th >= 1 and rt > rb");
  const int64_t N = p + 1;
  if (n_elem * N * N * N > INT32_MAX) return fail(SDM_EINVAL, "sph_bins: more than 2^31 solution points");
  sph_bins(n_elem, (int)N, x_sp, rb, rt, n_r, n_th, order, offsets);
  return SDM_OK;
}

sdm_status sdm_sph_profiles(sdm_ctx* c, const double* Q, const int32_t* order, const int64_t* offsets, int n_bins,
                            double* out, void* stream) {
  if (!c || !Q || !order || !offsets || !out) return fail(SDM_EINVAL, "sph_profiles: NULL argument");
  if (!c->bound) return fail(SDM_ESTATE, "sph_profiles: no mesh bound");
  if (n_bins < 1) return fail(SDM_EINVAL, "sph_profiles: n_bins >= 1 required");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const double* x = c->mesh.x_sp;
  const double* dj = c->mesh.detJ;
  switch (c->N) {
    case 2: hipLaunchKernelGGL(k_sph_profile<2>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    case 3: hipLaunchKernelGGL(k_sph_profile<3>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    case 4: hipLaunchKernelGGL(k_sph_profile<4>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    case 5: hipLaunchKernelGGL(k_sph_profile<5>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    case 6: hipLaunchKernelGGL(k_sph_profile<6>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    case 7: hipLaunchKernelGGL(k_sph_profile<7>, dim3(n_bins), dim3(256), 0, s, Q, x, dj, order, offsets, out); break;
    default: return fail(SDM_EUNSUPPORTED, "sph_profiles: unsupported p");
  }
  HIP_TRY(hipGetLastError());
  return SDM_OK;
}

sdm_status sdm_batch_workspace_size(int n_items, size_t* bytes) {
  if (n_items < 1 || !bytes) return fail(SDM_EINVAL, "batch_workspace_size: n_items >= 1 and bytes required");
  *bytes = batch_ws_bytes(n_items);
  return SDM_OK;
}

sdm_status sdm_batch_stage(const sdm_batch_item* items, int n_items, void* batch_ws, size_t ws_bytes,
                           int max_blocks, void* stream) {
  if (!items || n_items < 1 || !batch_ws) return fail(SDM_EINVAL, "batch_stage: NULL argument or no items");
  if (ws_bytes < batch_ws_bytes(n_items)) return fail(SDM_EINVAL, "batch_stage: batch workspace too small");
  if ((uintptr_t)batch_ws % 256 != 0) return fail(SDM_EINVAL, "batch_stage: batch workspace not 256-byte aligned");
  sdm_ctx* c0 = items[0].ctx;
  if (!c0) return fail(SDM_EINVAL, "batch_stage: NULL context");
  // the stage descriptor of every item, grouped by degree (groups in order
  // of first appearance, items in their given order within a group)
  std::vector<int> degrees;
  std::vector<std::vector<RunDesc>> all(kBatchGroups), tr(kBatchGroups);
  for (int k = 0; k < n_items; ++k) {
    const sdm_batch_item& it = items[k];
    sdm_ctx* c = it.ctx;
    if (!c || !c->bound) return fail(SDM_ESTATE, "batch_stage: item without a bound mesh");
    if (c->arith != c0->arith || c->device != c0->device)
      return fail(SDM_EINVAL, "batch_stage: items must share the arithmetic and the device");
    if (!it.regs || !it.ws || it.n_regs < 1 || it.n_regs > 16) return fail(SDM_EINVAL, "batch_stage: bad registers");
    const sdm_stage& st = it.stage;
    if (st.n_in < 0 || st.n_in > 4) return fail(SDM_EINVAL, "batch_stage: 0 <= n_in <= 4");
    auto okreg = [&](int i) { return i >= 0 && i < it.n_regs && it.regs[i] != nullptr; };
    if (!okreg(st.cur) || !okreg(st.out)) return fail(SDM_EINVAL, "batch_stage: register index out of range");
    for (int q = 0; q < st.n_in; ++q)
      if (!okreg(st.in_idx[q])) return fail(SDM_EINVAL, "batch_stage: input register out of range");
    sdm_status ps = check_params(c, it.prm);
    if (ps != SDM_OK) return ps;
    RunDesc r = make_desc(c, it.prm, it.regs[st.cur], it.ws);
    for (int q = 0; q < st.n_in; ++q) {
      r.in[q] = it.regs[st.in_idx[q]];
      r.alpha[q] = st.alpha[q];
    }
    r.n_in = st.n_in;
    r.out = it.regs[st.out];
    r.beta_dt = st.beta * it.dt;
    r.write_traces = 1;
    r.fuse = 1;
    r.Rp = nullptr;  // a stage never uses the partial-residual region
    size_t g = std::find(degrees.begin(), degrees.end(), c->N) - degrees.begin();
    if (g == degrees.size()) degrees.push_back(c->N);
    all[g].push_back(r);
    if (!st.traces_valid) tr[g].push_back(r);
  }
  const int G = (int)degrees.size();
  HIP_TRY(hipSetDevice(c0->device));
  hipStream_t s = (hipStream_t)stream;
  // one host image of both work lists, one copy
  const size_t lb = batch_list_bytes(n_items);
  const size_t pre_off = align256(sizeof(RunDesc) * (size_t)n_items);
  std::vector<char> host(batch_ws_bytes(n_items), 0);
  struct Span { size_t run0, pre0; int n; int64_t E; };
  std::vector<Span> sp_all(G), sp_tr(G);
  auto pack = [&](size_t off, const std::vector<std::vector<RunDesc>>& lists, std::vector<Span>& spans) {
    size_t run0 = 0;
    for (int g = 0; g < G; ++g) {
      const std::vector<RunDesc>& d = lists[g];
      std::vector<int64_t> pre{0};
      for (const RunDesc& r : d) pre.push_back(pre.back() + r.E);
      std::memcpy(host.data() + off + sizeof(RunDesc) * run0, d.data(), sizeof(RunDesc) * d.size());
      std::memcpy(host.data() + off + pre_off + sizeof(int64_t) * (run0 + g), pre.data(), sizeof(int64_t) * pre.size());
      spans[g] = Span{run0, run0 + g, (int)d.size(), pre.back()};
      run0 += d.size();
    }
  };
  pack(0, all, sp_all);
  pack(lb, tr, sp_tr);
  sdm_status st = stage_copy(host.data(), host.size(), batch_ws, s);
  if (st != SDM_OK) return st;
  // the first degree group runs on the caller's stream, the others on
  // library streams that wait for the table copy; the caller's stream then
  // waits for them, so work of different degrees overlaps on the device
  BatchStreams* bs = nullptr;
  std::unique_lock<std::mutex> enqueue;
  if (G > 1) {
    if ((st = batch_streams(c0->device, G - 1, &bs)) != SDM_OK) return st;
    enqueue = std::unique_lock<std::mutex>(g_bs_enqueue[c0->device]);
    HIP_TRY(hipEventRecord(bs->fork, s));
  }
  char* base = (char*)batch_ws;
  const int64_t cap = max_blocks > 0 ? max_blocks : ((int64_t)1 << 30);
  for (int g = 0; g < G; ++g) {
    hipStream_t sg = g == 0 ? s : bs->side[g - 1];
    if (g > 0) HIP_TRY(hipStreamWaitEvent(sg, bs->fork, 0));
    auto launch_of = [&](size_t off, const Span& sp) {
      Launch L;
      std::memset(&L, 0, sizeof L);
      L.one.N = degrees[g];
      L.many = (const RunDesc*)(base + off + sizeof(RunDesc) * sp.run0);
      L.prefix = (const int64_t*)(base + off + pre_off + sizeof(int64_t) * sp.pre0);
      L.n_run = sp.n;
      L.n_work = sp.E;
      return L;
    };
    auto go = [&](int which, const Launch& L) -> sdm_status {
      const hipError_t e = c0->arith ? dispatch_N<float>(degrees[g], which, L, sg, cap)
                                     : dispatch_N<double>(degrees[g], which, L, sg, cap);
      return e == hipSuccess ? SDM_OK : fail(SDM_EHIP, std::string("batch kernel launch: ") + hipGetErrorString(e));
    };
    if (sp_tr[g].n > 0 && (st = go(0, launch_of(lb, sp_tr[g]))) != SDM_OK) return st;
    const Launch La = launch_of(0, sp_all[g]);
    if ((st = go(1, La)) != SDM_OK) return st;
    if ((st = go(4, La)) != SDM_OK) return st;
    if (g > 0) {
      HIP_TRY(hipEventRecord(bs->join[g - 1], sg));
      HIP_TRY(hipStreamWaitEvent(s, bs->join[g - 1], 0));
    }
  }
  return SDM_OK;
}

}  // extern "C"
