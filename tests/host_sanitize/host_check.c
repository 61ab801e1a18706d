/* Host-side checks of libshgb built with AddressSanitizer and UBSan on its
 * host code (the argument validation, the workspace and checkpoint sizes,
 * the batch table writer and the zero-work early returns): every call here
 * returns before any device work, so the program runs without a GPU.  It
 * exits non-zero on the first wrong return code; the sanitizers abort on a
 * memory or undefined-behaviour error in the library's host code. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "shgb.h"

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "host_check: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static shgb_model qcle(int d) {
  shgb_model m;
  memset(&m, 0, sizeof m);
  m.kind = SHGB_MODEL_QCLE;
  m.d = d;
  m.mass = 2000.0;
  m.eps = d == 1 ? 0.01 : 0.02;
  m.A = 0.01;
  m.B = 1.6;
  m.C = 0.005;
  m.D = 1.0;
  m.lam = d == 1 ? 0.0 : 1e-3;
  for (int k = 0; k + 1 < d; ++k) m.bath_omega[k] = 0.002 + 0.001 * k;
  return m;
}

static shgb_state desc(int64_t n, int32_t m, int64_t ld, uintptr_t fake) {
  shgb_state s;
  memset(&s, 0, sizeof s);
  s.f64 = (double *)fake;
  s.comp = (int32_t *)fake;
  s.nhop = (uint32_t *)fake;
  s.n_beams = n;
  s.ld = ld;
  s.m = m;
  s.precision = SHGB_FP64;
  return s;
}

int main(void) {
  const uintptr_t F = 0x1000;
  void *nul = NULL;
  shgb_model m1 = qcle(1), m12 = qcle(12);
  shgb_state st = desc(16, 2, 16, F), st24 = desc(16, 24, 16, F);
  shgb_init_spec spec = {-5.0, 0.5, SHGB_DIST_NORMAL, 20.0, 1.0, 1, 0.0};

  /* null pointers, inconsistent shapes, bad parameters */
  CHECK(shgb_init_beams(NULL, &spec, &st, 1, nul) == SHGB_EINVAL);
  CHECK(shgb_init_beams(&m1, NULL, &st, 1, nul) == SHGB_EINVAL);
  CHECK(shgb_step_ensemble(&m1, NULL, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  shgb_state bad = desc(16, 4, 16, F);
  CHECK(shgb_step_ensemble(&m1, &bad, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  bad = desc(16, 2, 3, F);
  CHECK(shgb_step_ensemble(&m1, &bad, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  bad = desc(16, 2, 16, 0);
  CHECK(shgb_step_ensemble(&m1, &bad, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  bad = desc(16, 2, 16, F);
  bad.precision = 7;
  CHECK(shgb_step_ensemble(&m1, &bad, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  bad.precision = SHGB_MIXED;   /* no FP32 block */
  CHECK(shgb_step_ensemble(&m1, &bad, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  CHECK(shgb_step_ensemble(&m1, &st, -1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  CHECK(shgb_step_ensemble(&m1, &st, 1, 0.0, 1, NULL, nul) == SHGB_EINVAL);
  CHECK(shgb_step_ensemble(&m1, &st, 1, NAN, 1, NULL, nul) == SHGB_EINVAL);
  CHECK(shgb_step_ensemble_scheme(&m1, &st, 1, 0.5, 1, 2, NULL, nul) == SHGB_EINVAL);
  shgb_model mb = qcle(1);
  mb.mass = 0.0;
  CHECK(shgb_step_ensemble(&mb, &st, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  mb = qcle(1);
  mb.A = INFINITY;
  CHECK(shgb_step_ensemble(&mb, &st, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  mb = qcle(3);
  mb.bath_omega[1] = 0.0;
  shgb_state st6 = desc(16, 6, 16, F);
  CHECK(shgb_step_ensemble(&mb, &st6, 1, 0.5, 1, NULL, nul) == SHGB_EINVAL);
  shgb_init_spec sb = spec;
  sb.q_std = -0.5;
  CHECK(shgb_init_beams(&m1, &sb, &st, 1, nul) == SHGB_EINVAL);
  sb = spec;
  sb.comp0 = 4;
  CHECK(shgb_init_beams(&m1, &sb, &st, 1, nul) == SHGB_EINVAL);
  CHECK(shgb_hop(&m1, &st, NULL, 3, 1, NULL, nul) == SHGB_EINVAL);
  CHECK(shgb_hop(&m1, &st, (const int32_t *)F, -1, 1, NULL, nul) == SHGB_EINVAL);

  /* workspace and checkpoint sizes, and the calls that check them */
  const int64_t wp = shgb_populations_workspace(16, 2);
  CHECK(wp > 0);
  CHECK(shgb_populations_workspace(-1, 2) == -1 && shgb_populations_workspace(4, 3) == -1);
  CHECK(shgb_populations(&m1, &st, (double *)F, (void *)F, wp - 1, nul, nul) == SHGB_EWORKSPACE);
  const int64_t wr = shgb_reconstruct_workspace(16, 2, 100);
  CHECK(wr > 0);
  CHECK(shgb_reconstruct(&m1, &st, (const double *)F, 100, (double *)F, (void *)F, wr - 1, nul) ==
        SHGB_EWORKSPACE);
  CHECK(shgb_reconstruct(&m1, &st, NULL, 100, (double *)F, (void *)F, wr, nul) == SHGB_EINVAL);
  CHECK(shgb_reconstruct_workspace_mode(16, 24, 100, SHGB_FIELD_FP32_MATRIX) > 0);
  CHECK(shgb_reconstruct_mode(&m1, &st, (const double *)F, 100, (double *)F, (void *)F, wr, SHGB_FIELD_FP32_MATRIX,
                              nul) == SHGB_EUNSUPPORTED);
  CHECK(shgb_reconstruct_mode(&m12, &st24, (const double *)F, 100, (double *)F, (void *)F, 1 << 30, 9, nul) ==
        SHGB_EINVAL);
  CHECK(shgb_population_tangent_workspace(16) > 0);
  for (int d = 1; d <= 12; ++d) {
    const int64_t cb = shgb_checkpoint_bytes(1000, 2 * d, 1000, 100);
    const int64_t aw = shgb_population_adjoint_workspace(1000, 2 * d, 100);
    CHECK(cb > 0);
    if (d == 1 || d == 2 || d == 3 || d == 4 || d == 12) CHECK(aw > 0);
    else CHECK(aw == -1);
  }
  CHECK(shgb_checkpoint_bytes(16, 2, 10, 0) == -1);
  CHECK(shgb_step_checkpointed(&m1, &st, 10, 0.5, 1, 0, (void *)F, 1 << 20, nul, nul) == SHGB_EINVAL);
  const int64_t cb = shgb_checkpoint_bytes(16, 2, 10, 4);
  CHECK(shgb_step_checkpointed(&m1, &st, 10, 0.5, 1, 4, (void *)F, cb - 1, nul, nul) == SHGB_EWORKSPACE);
  CHECK(shgb_philox(1, NULL, NULL, 5, nul) == SHGB_EINVAL);

  /* the batch table writer: sizes, configurations, mixed instances */
  enum { NI = 5 };
  shgb_model models[NI];
  shgb_state states[NI];
  uint64_t seeds[NI];
  const int64_t sizes[NI] = {0, 9, 17, 1, 130};
  for (int i = 0; i < NI; ++i) {
    models[i] = qcle(12);
    states[i] = desc(sizes[i], 24, sizes[i] > 0 ? sizes[i] : 1, F);
    seeds[i] = 100 + i;
  }
  const int64_t tb = shgb_batch_table_bytes(NI);
  CHECK(tb > 0 && shgb_batch_table_bytes(0) == -1);
  unsigned char *host = (unsigned char *)malloc((size_t)tb);
  shgb_batch batch;
  shgb_batch_config cfg = {4, 2, 1};
  CHECK(shgb_batch_prepare(models, states, seeds, NI, &cfg, host, tb, &batch) == SHGB_OK);
  int64_t tiles = 0;
  for (int i = 0; i < NI; ++i) tiles += (sizes[i] + 7) / 8;
  CHECK(batch.total_tiles == tiles && batch.d == 12 && batch.n_inst == NI);
  CHECK(shgb_batch_prepare(models, states, seeds, NI, &cfg, host, tb - 1, &batch) == SHGB_EINVAL);
  const shgb_batch_config bad_cfg[4] = {{3, 2, 1}, {4, 0, 1}, {4, 17, 1}, {4, 2, 0}};
  for (int k = 0; k < 4; ++k)
    CHECK(shgb_batch_prepare(models, states, seeds, NI, &bad_cfg[k], host, tb, &batch) == SHGB_EINVAL);
  states[2].precision = SHGB_MIXED;
  states[2].f32 = (float *)F;
  CHECK(shgb_batch_prepare(models, states, seeds, NI, &cfg, host, tb, &batch) == SHGB_EINVAL);
  states[2].precision = SHGB_FP64;
  CHECK(shgb_batch_prepare(models, states, seeds, NI, &cfg, host, tb, &batch) == SHGB_OK);
  CHECK(shgb_step_batched(&batch, 0, 0.5, (void *)F, SHGB_BATCH_WORK_BYTES, nul, nul) == SHGB_OK);
  CHECK(shgb_step_batched(&batch, 5, 0.5, (void *)F, SHGB_BATCH_WORK_BYTES - 1, nul, nul) == SHGB_EINVAL);
  free(host);

  /* zero work returns without touching a device */
  shgb_state empty = desc(0, 2, 0, 0);
  CHECK(shgb_init_beams(&m1, &spec, &empty, 1, nul) == SHGB_OK);
  CHECK(shgb_step_ensemble(&m1, &empty, 10, 0.5, 1, NULL, nul) == SHGB_OK);
  CHECK(shgb_step_ensemble(&m1, &st, 0, 0.5, 1, NULL, nul) == SHGB_OK);
  CHECK(shgb_hop(&m1, &st, NULL, 0, 1, NULL, nul) == SHGB_OK);
  CHECK(shgb_philox(1, NULL, NULL, 0, nul) == SHGB_OK);

  /* sizes, version and every error string */
  int64_t sz[16];
  memset(sz, 0, sizeof sz);
  shgb_abi_sizes(sz);
  CHECK(sz[0] == (int64_t)sizeof(shgb_model) && sz[1] == (int64_t)sizeof(shgb_state));
  CHECK(shgb_version() > 0);
  for (int code = 0; code >= -8; --code) CHECK(shgb_strerror(code) != NULL && strlen(shgb_strerror(code)) > 0);

  if (failures) {
    fprintf(stderr, "host_check: %d failures\n", failures);
    return 1;
  }
  printf("host_check: all checks passed\n");
  return 0;
}
