/*
 * Drives liblbm.so through include/lbm.h alone: plain C, no Python, no torch,
 * the library's own device memory and the null stream.
 *
 *   lid_cavity OUT.bin      (needs a GPU)
 *   lid_cavity --check-only (validation only: no device call)
 *
 * A 12 x 10 x 8 iD3Q14 FP64 lattice (AA pattern): walls on every face, the
 * +z lid moving along x, a body force, initial state f_eq(p0, u0); 25 steps
 * with the monitor every 5.  Writes p[N] then u[3][N] (doubles) to OUT.bin
 * and prints the mass and residual.  Also checks that an invalid spec is
 * refused with a message.  Then a batch on the null stream: a D3Q18 FP32
 * duct with a pressure inlet and outlet and a D3Q14 FP32 lid cavity, each
 * also run alone with lbm_step; the batch (step budget 12 for the cavity)
 * advances them by 10 and 7 steps, and their populations must equal the
 * single runs byte for byte.  Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/lbm.h"

#define CHECK(call)                                                              \
  do {                                                                           \
    int rc_ = (call);                                                            \
    if (rc_ != LBM_OK) {                                                         \
      fprintf(stderr, "%s failed: %s (%s)\n", #call, lbm_status_string(rc_),     \
              lbm_last_error(ctx));                                              \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

/* Two lattices, each created twice: [k][0] runs alone, [k][1] in the batch. */
static int run_batch(void) {
  const double s18[18] = {1.0, 1.19, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, 1.5,
                          1.4, 1.5, 1.4, 1.5, 1.5, 1.5, 0.98, 0.98, 0.98};
  const double s14[14] = {1.0, 1.19, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2,
                          1.3, 1.3, 1.3, 1.3, 1.3, 0.98};
  const int dims[2][3] = {{20, 9, 7}, {11, 10, 9}};
  lbm_ctx* ctx = NULL;
  lbm_ctx* lat[2][2] = {{NULL, NULL}, {NULL, NULL}};
  lbm_batch* b = NULL;
  lbm_spec sp;
  int k, j;
  for (k = 0; k < 2; ++k) {
    lbm_spec_default(&sp);
    sp.storage = LBM_F32;
    sp.pattern = LBM_AA;
    if (k == 0) { /* duct: pressure faces on x, walls elsewhere */
      sp.face[0] = LBM_PRESSURE;
      sp.face[1] = LBM_PRESSURE;
      sp.face_p[0] = 0.003;
      sp.face_p[1] = -0.002;
    } else { /* cavity with a lid along +x and a weak body force */
      sp.wall_u[5][0] = 0.08;
      sp.F0[1] = 2e-5;
    }
    for (j = 0; j < 2; ++j)
      CHECK(lbm_create(&lat[k][j], k == 0 ? 18 : 14, dims[k][0], dims[k][1], dims[k][2],
                       k == 0 ? s18 : s14, &sp));
  }
  if (lbm_batch_create(&b, NULL) != LBM_OK) {
    fprintf(stderr, "lbm_batch_create failed\n");
    return 1;
  }
  if (lbm_batch_add(b, lat[0][1], 1000) != LBM_OK || lbm_batch_add(b, lat[1][1], 12) != LBM_OK ||
      lbm_batch_step(b, 10) != LBM_OK || lbm_batch_step(b, 7) != LBM_OK) {
    fprintf(stderr, "batch failed: %s\n", lbm_batch_last_error(b));
    return 1;
  }
  if (lbm_batch_remaining(b, lat[1][1]) != 0 || lbm_batch_remaining(b, lat[0][1]) != 983) {
    fprintf(stderr, "step budgets not kept\n");
    return 1;
  }
  ctx = lat[0][0];
  CHECK(lbm_step(lat[0][0], 17));
  ctx = lat[1][0];
  CHECK(lbm_step(lat[1][0], 12));
  for (k = 0; k < 2; ++k) {
    const int q = k == 0 ? 18 : 14;
    const size_t n = (size_t)q * dims[k][0] * dims[k][1] * dims[k][2];
    double* fa = (double*)malloc(sizeof(double) * n);
    double* fb = (double*)malloc(sizeof(double) * n);
    if (!fa || !fb) return 1;
    ctx = lat[k][0];
    CHECK(lbm_get_f(lat[k][0], fa));
    ctx = lat[k][1];
    CHECK(lbm_get_f(lat[k][1], fb));
    if (lbm_time(lat[k][0]) != lbm_time(lat[k][1]) || memcmp(fa, fb, sizeof(double) * n) != 0) {
      fprintf(stderr, "batched lattice %d differs from its single run\n", k);
      return 1;
    }
    free(fa);
    free(fb);
  }
  printf("batch: duct t=%lld, cavity t=%lld, bit-identical to single runs\n",
         lbm_time(lat[0][1]), lbm_time(lat[1][1]));
  if (lbm_batch_destroy(b) != LBM_OK) return 1;
  for (k = 0; k < 2; ++k)
    for (j = 0; j < 2; ++j)
      if (lbm_destroy(lat[k][j]) != LBM_OK) return 1;
  return 0;
}

int main(int argc, char** argv) {
  const int nx = 12, ny = 10, nz = 8, N = nx * ny * nz;
  const double s14[14] = {1.0, 1.19, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2,
                          1.6, 1.6, 1.6, 1.6, 1.6, 0.98};
  lbm_ctx* ctx = NULL;
  lbm_spec sp;
  double *p, *u, mass = 0.0, res = 0.0;
  FILE* fh;
  if (argc != 2) {
    fprintf(stderr, "usage: %s OUT.bin | --check-only\n", argv[0]);
    return 2;
  }
  /* an invalid spec (unpaired periodic face) is refused before any device call */
  lbm_spec_default(&sp);
  sp.face[0] = LBM_PERIODIC;
  if (lbm_create(&ctx, 14, nx, ny, nz, s14, &sp) != LBM_EINVAL || ctx != NULL ||
      strlen(lbm_last_error(NULL)) == 0) {
    fprintf(stderr, "invalid spec was not refused\n");
    return 1;
  }
  if (lbm_footprint_bytes(14, nx, ny, nz, &sp) != 0) {
    fprintf(stderr, "footprint of an invalid spec is not 0\n");
    return 1;
  }
  if (strcmp(argv[1], "--check-only") == 0) {
    printf("lid_cavity: validation ok (%s)\n", lbm_last_error(NULL));
    return 0;
  }
  lbm_spec_default(&sp);
  sp.storage = LBM_F64;
  sp.pattern = LBM_AA;
  sp.wall_u[5][0] = 0.06;
  sp.F0[0] = 1e-5;
  sp.F0[2] = -2e-5;
  sp.p0 = 0.002;
  sp.u0[0] = 0.01;
  sp.u0[1] = -0.005;
  sp.monitor_every = 5;
  CHECK(lbm_create(&ctx, 14, nx, ny, nz, s14, &sp));
  CHECK(lbm_step(ctx, 25));
  p = (double*)malloc(sizeof(double) * N);
  u = (double*)malloc(sizeof(double) * 3 * N);
  if (!p || !u) return 1;
  CHECK(lbm_macros(ctx, p, u));
  CHECK(lbm_mass(ctx, &mass));
  CHECK(lbm_residual(ctx, &res));
  if (lbm_time(ctx) != 25) {
    fprintf(stderr, "time level %lld, expected 25\n", lbm_time(ctx));
    return 1;
  }
  fh = fopen(argv[1], "wb");
  if (!fh || fwrite(p, sizeof(double), N, fh) != (size_t)N ||
      fwrite(u, sizeof(double), 3 * (size_t)N, fh) != 3 * (size_t)N || fclose(fh) != 0) {
    fprintf(stderr, "cannot write %s\n", argv[1]);
    return 1;
  }
  printf("lid_cavity: t=%lld mass=%.17g residual=%.6e\n", lbm_time(ctx), mass, res);
  free(p);
  free(u);
  if (lbm_destroy(ctx) != LBM_OK) {
    fprintf(stderr, "lbm_destroy failed\n");
    return 1;
  }
  return run_batch();
}
