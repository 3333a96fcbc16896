/* abi_step.c -- a plain C caller of the library's C ABI (include/sdmhd.h),
 * used by tests/test_gpu_abi_c.py.  It builds the cubed-sphere shell with the
 * library's host builder, uploads it with the HIP runtime, and advances the
 * state by SSPRK(5,3) steps with sdm_ssprk53_step only.
 *
 * usage: abi_step IN OUT
 *   IN   Nz, Nr, p, steps (int32 each), the sdm_params struct as raw bytes
 *        (no ghost or import buffers), dt (double), Q ([E][9][(p+1)^3]
 *        doubles)
 *   OUT  Q after the steps, same layout
 * Exit status 0 on success; a message on stderr otherwise. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/sdmhd.h"

#define CHECK_SDM(x)                                                     \
  do {                                                                   \
    sdm_status s_ = (x);                                                 \
    if (s_ != SDM_OK) {                                                  \
      fprintf(stderr, "%s: %d %s\n", #x, (int)s_, sdm_last_error());     \
      return 1;                                                          \
    }                                                                    \
  } while (0)
#define CHECK_HIP(x)                                                     \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      return 1;                                                          \
    }                                                                    \
  } while (0)

static int upload(void** dev, const void* host, size_t bytes) {
  if (hipMalloc(dev, bytes) != hipSuccess) return 1;
  return hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice) != hipSuccess;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: abi_step IN OUT\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) {
    perror(argv[1]);
    return 1;
  }
  int32_t hdr[4];
  sdm_params prm;
  double dt;
  if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&prm, sizeof prm, 1, f) != 1 || fread(&dt, sizeof dt, 1, f) != 1) {
    fprintf(stderr, "short input header\n");
    return 1;
  }
  const int Nz = hdr[0], Nr = hdr[1], p = hdr[2], steps = hdr[3], N = p + 1;
  prm.ghost = NULL;
  prm.import_q = NULL;
  prm.import_v = NULL;
  int64_t E = 0, NB = 0;
  CHECK_SDM(sdm_shell_sizes(Nz, Nr, &E, &NB));
  const size_t N3 = (size_t)N * N * N, NF = (size_t)(N + 1) * N * N, N2 = (size_t)N * N;
  const size_t nq = (size_t)E * 9 * N3;
  double* Q = (double*)malloc(sizeof(double) * nq);
  if (fread(Q, sizeof(double), nq, f) != nq) {
    fprintf(stderr, "short state\n");
    return 1;
  }
  fclose(f);

  double* x_sp = (double*)malloc(sizeof(double) * E * 3 * N3);
  double* detJ = (double*)malloc(sizeof(double) * E * N3);
  double* S_fp = (double*)malloc(sizeof(double) * E * 9 * NF);
  double* Sj_sp = (double*)malloc(sizeof(double) * E * 9 * N3);
  int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * E * 6);
  double* n_face = (double*)malloc(sizeof(double) * E * 18 * N2);
  CHECK_SDM(sdm_shell_build(Nz, Nr, p, 0.70, 0.98, x_sp, detJ, S_fp, Sj_sp, nbr, n_face));

  sdm_mesh m;
  memset(&m, 0, sizeof m);
  m.n_elem = E;
  m.n_bfaces = NB;
  void *d_x, *d_J, *d_S, *d_Sj, *d_nb, *d_n;
  if (upload(&d_x, x_sp, sizeof(double) * E * 3 * N3) || upload(&d_J, detJ, sizeof(double) * E * N3) ||
      upload(&d_S, S_fp, sizeof(double) * E * 9 * NF) || upload(&d_Sj, Sj_sp, sizeof(double) * E * 9 * N3) ||
      upload(&d_nb, nbr, sizeof(int32_t) * E * 6) || upload(&d_n, n_face, sizeof(double) * E * 18 * N2)) {
    fprintf(stderr, "mesh upload failed\n");
    return 1;
  }
  m.x_sp = (const double*)d_x;
  m.detJ = (const double*)d_J;
  m.S_fp = (const double*)d_S;
  m.Sj_sp = (const double*)d_Sj;
  m.nbr = (const int32_t*)d_nb;
  m.n_face = (const double*)d_n;

  sdm_ctx* ctx = NULL;
  CHECK_SDM(sdm_create(0, p, 0, &ctx));
  CHECK_SDM(sdm_mesh_bind(ctx, &m));
  size_t ws_bytes = 0;
  CHECK_SDM(sdm_workspace_size(ctx, &ws_bytes));
  void* ws = NULL;
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  double* regs[4];
  for (int k = 0; k < 4; ++k) CHECK_HIP(hipMalloc((void**)&regs[k], sizeof(double) * nq));
  CHECK_HIP(hipMemcpy(regs[0], Q, sizeof(double) * nq, hipMemcpyHostToDevice));
  for (int s = 0; s < steps; ++s) CHECK_SDM(sdm_ssprk53_step(ctx, &prm, regs, dt, s > 0, ws, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(Q, regs[0], sizeof(double) * nq, hipMemcpyDeviceToHost));

  FILE* g = fopen(argv[2], "wb");
  if (!g || fwrite(Q, sizeof(double), nq, g) != nq) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    return 1;
  }
  fclose(g);
  CHECK_SDM(sdm_destroy(ctx));
  for (int k = 0; k < 4; ++k) (void)hipFree(regs[k]);
  (void)hipFree(ws);
  (void)hipFree(d_x); (void)hipFree(d_J); (void)hipFree(d_S); (void)hipFree(d_Sj); (void)hipFree(d_nb);
  (void)hipFree(d_n);
  free(Q); free(x_sp); free(detJ); free(S_fp); free(Sj_sp); free(nbr); free(n_face);
  printf("abi_step: %lld elements, p = %d, %d steps\n", (long long)E, p, steps);
  return 0;
}
