/* Drives the host side of libacs's C ABI without a GPU, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer on the host code
 * (tests/test_oracle_sanitized.py): defaults, workspace sizes over many
 * shapes, every argument check, the no-device error path of the create
 * calls, calls on NULL handles and the thread-local error text from several
 * threads.  Exits 0 when each call returns what the header states. */
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/acs.h"

static int fails = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, \
              acs_last_error());                                      \
      fails++;                                                        \
    }                                                                 \
  } while (0)

static void *thread_body(void *arg) {
  acs_params p;
  acs_default_params(&p);
  p.q0 = 2.0 + (double)(size_t)arg;
  size_t ws = 0;
  int *ok = malloc(sizeof(int));
  *ok = acs_workspace_bytes(100, &p, &ws) == ACS_E_INVALID && strstr(acs_last_error(), "q0");
  return ok;
}

int main(void) {
  acs_params p;
  CHECK(acs_default_params(&p) == ACS_OK);
  CHECK(p.struct_size == sizeof(acs_params) && p.cl == 32 && p.local_update_period == 1);
  CHECK(acs_default_params(NULL) != ACS_OK);
  size_t ws = 0, prev = 0;
  /* workspace sizes over memory kinds, modes and sizes */
  for (uint32_t mem = 0; mem < 2; ++mem)
    for (uint32_t mode = 0; mode < 4; ++mode)
      for (int n = 3; n < 30000; n = n * 3 + 1) {
        acs_default_params(&p);
        p.memory = mem;
        p.mode = mode;
        p.m = mode == 3 ? 64 : 0;
        const int rc = acs_workspace_bytes(n, &p, &ws);
        CHECK(rc == ACS_OK || rc == ACS_E_UNSUPPORTED);
        (void)prev;
      }
  /* argument checks */
  struct { int n; int field; double v; int want; } bad[] = {
      {2, 0, 0, ACS_E_INVALID},   {100, 1, -0.5, ACS_E_INVALID}, {100, 1, 1.5, ACS_E_INVALID},
      {100, 2, 0.0, ACS_E_INVALID}, {100, 2, 1.0, ACS_E_INVALID}, {100, 3, 0.0, ACS_E_INVALID},
      {100, 4, 0, ACS_E_INVALID},  {100, 5, 9, ACS_E_INVALID},    {100, 6, 7, ACS_E_INVALID},
      {100, 7, 5, ACS_E_INVALID},  {100, 8, 65, ACS_E_INVALID}};
  for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
    acs_default_params(&p);
    switch (bad[i].field) {
      case 1: p.q0 = bad[i].v; break;
      case 2: p.phi = bad[i].v; break;
      case 3: p.rho = bad[i].v; break;
      case 4: p.memory = 1; p.spm_s = 0; break;
      case 5: p.mode = (uint32_t)bad[i].v; break;
      case 6: p.local_search = (uint32_t)bad[i].v; break;
      case 7: p.update_path = (uint32_t)bad[i].v; break;
      case 8: p.cl = (uint32_t)bad[i].v; break;
      default: break;
    }
    const int rc = acs_workspace_bytes(bad[i].n, &p, &ws);
    CHECK(rc != ACS_OK);
    CHECK(strlen(acs_last_error()) > 0);
  }
  /* create without a device, and with invalid coordinates */
  const int n = 200;
  double *xy = malloc(sizeof(double) * 2 * n);
  for (int i = 0; i < 2 * n; ++i) xy[i] = (double)((i * 7919) % 1000);
  struct acs_t *h = (struct acs_t *)0x1;
  acs_default_params(&p);
  CHECK(acs_create(xy, n, &p, &h) == ACS_E_DEVICE && h == NULL);
  xy[5] = 0.0 / 0.0;
  CHECK(acs_create(xy, n, &p, &h) == ACS_E_INVALID);
  xy[5] = 1.0;
  CHECK(acs_create(NULL, n, &p, &h) == ACS_E_INVALID);
  CHECK(acs_create(xy, n, NULL, &h) == ACS_E_INVALID);
  /* calls on a NULL handle */
  int32_t tour[4];
  int64_t len = 0;
  acs_stats_t st;
  CHECK(acs_iterate(NULL, 1) == ACS_E_STATE);
  CHECK(acs_best_tour(NULL, tour, &len) == ACS_E_STATE);
  CHECK(acs_stats(NULL, &st) == ACS_E_STATE);
  CHECK(acs_tours(NULL, tour, 4) == ACS_E_STATE);
  CHECK(acs_set_candidate_scores(NULL, NULL) == ACS_E_STATE);
  acs_destroy(NULL);
  /* the static entry point checks its arguments before any device work */
  acs_default_params(&p);
  p.workspace = (void *)0x1000;
  p.workspace_bytes = 16;
  CHECK(acs_solve_static(xy, n, &p, 1, NULL, &len) != ACS_OK);
  /* batches */
  const double *coords[2] = {xy, xy};
  const int32_t ns[2] = {n, 2};
  acs_batch_t *b = NULL;
  acs_default_params(&p);
  p.mode = 1;
  CHECK(acs_batch_workspace_bytes(ns, 2, &p, &ws) == ACS_E_INVALID);
  CHECK(acs_batch_create(coords, ns, 2, &p, &b) == ACS_E_INVALID && b == NULL);
  CHECK(acs_batch_iterate(NULL, 1) == ACS_E_STATE);
  acs_batch_destroy(NULL);
  /* the error text is per thread */
  pthread_t th[4];
  for (size_t i = 0; i < 4; ++i) pthread_create(&th[i], NULL, thread_body, (void *)i);
  for (int i = 0; i < 4; ++i) {
    void *r = NULL;
    pthread_join(th[i], &r);
    CHECK(r && *(int *)r);
    free(r);
  }
  free(xy);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
