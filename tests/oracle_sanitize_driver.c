/* Drives every entry point of the CPU oracle once on small instances, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py).  Exits 0 when every call behaves as its
 * header states; a sanitizer report ends the process with an error. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/acs_oracle.h"

static int fails = 0;
#define CHECK(c)                                                \
  do {                                                          \
    if (!(c)) {                                                 \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      fails++;                                                  \
    }                                                           \
  } while (0)

static uint64_t lcg = 12345;
static double rnd(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) / 9007199254740992.0;
}

static void run(int n, int m, int cl, int memory, int s, int mode, int period, int ls) {
  double *xy = malloc(sizeof(double) * 2 * (size_t)n);
  for (int i = 0; i < 2 * n; ++i) xy[i] = (double)(int)(rnd() * 1000.0);
  orc *o = orc_create(xy, n, m, cl, 2.0, 0.9, 0.1, 0.1, 0.0, memory, s, mode, 7, 0);
  CHECK(o != NULL);
  if (!o) {
    free(xy);
    return;
  }
  CHECK(orc_set_local_period(o, period) == 0);
  if (memory == ORC_DENSE) CHECK(orc_set_local_search(o, ls) == 0);
  const int32_t cle = orc_cl(o);
  float *w = malloc(sizeof(float) * (size_t)n * (size_t)cle);
  for (int i = 0; i < n * cle; ++i) w[i] = 0.01f + (float)rnd();
  CHECK(orc_set_candidate_weights(o, w) == 0);
  orc_iterate(o, 2);
  CHECK(orc_set_candidate_weights(o, NULL) == 0);
  orc_construct(o);
  orc_local_search(o);
  orc_select_best(o);
  orc_global_update(o);
  CHECK(orc_iteration(o) >= 2);
  int32_t *tours = malloc(sizeof(int32_t) * (size_t)m * (size_t)n);
  int64_t *lens = malloc(sizeof(int64_t) * (size_t)m);
  orc_get_tours(o, tours);
  orc_get_lengths(o, lens);
  for (int a = 0; a < m; ++a) {
    char *seen = calloc((size_t)n, 1);
    for (int p = 0; p < n; ++p) seen[tours[(size_t)a * n + p]]++;
    for (int c = 0; c < n; ++c) CHECK(seen[c] == 1);
    free(seen);
    CHECK(lens[a] > 0);
  }
  int32_t *best = malloc(sizeof(int32_t) * (size_t)n);
  CHECK(orc_get_best(o, best) > 0);
  CHECK(orc_set_best(o, best, orc_get_best(o, best)) == 0);
  int32_t ant = -1;
  CHECK(orc_get_iter_best(o, &ant) > 0 && ant >= 0 && ant < m);
  int32_t *dist = malloc(sizeof(int32_t) * (size_t)n * (size_t)n);
  int32_t *cand = malloc(sizeof(int32_t) * (size_t)n * (size_t)cle);
  orc_get_dist(o, dist);
  orc_get_cand(o, cand);
  float eta[64];
  orc_get_eta(o, eta, 64);
  int64_t lnn = 0, cnt[6];
  float t0, al, bl, ag;
  uint32_t q24;
  orc_constants(o, &lnn, &t0, &al, &bl, &ag, &q24);
  CHECK(lnn > 0 && t0 > 0.f);
  orc_get_counts(o, cnt);
  if (memory == ORC_DENSE) {
    float *tau = malloc(sizeof(float) * (size_t)n * (size_t)n);
    orc_get_tau(o, tau);
    CHECK(orc_set_tau(o, tau) == 0);
    free(tau);
    int64_t moves = 0, kinds[6];
    for (int p = 0; p < n; ++p) best[p] = (p * 7) % n;  /* n is not a multiple of 7 */
    int64_t L = 0;
    for (int p = 0; p < n; ++p) L += dist[(size_t)best[p] * n + best[(p + 1) % n]];
    const int64_t L2 = orc_local_search_tour(o, best, L, &moves, kinds);
    CHECK(L2 > 0 && L2 <= L);
    CHECK(orc_set_local_search_cap(o, 1) == 0);
    CHECK(orc_set_local_search_cap(o, -1) == -1);
  } else {
    int32_t *nodes = malloc(sizeof(int32_t) * (size_t)n * (size_t)s);
    float *vals = malloc(sizeof(float) * (size_t)n * (size_t)s);
    int32_t *tail = malloc(sizeof(int32_t) * (size_t)n);
    orc_get_spm(o, nodes, vals, tail);
    CHECK(orc_spm_update(o, 0, 1, al, bl) == 0);
    free(nodes);
    free(vals);
    free(tail);
  }
  CHECK(orc_set_local_period(o, 0) == -1);
  CHECK(orc_set_local_search(o, 3) == -1);
  CHECK(orc_local_map_k(o, t0, 3) > 0.f);
  free(w);
  free(tours);
  free(lens);
  free(best);
  free(dist);
  free(cand);
  orc_destroy(o);
  free(xy);
}

int main(void) {
  orc_set_threads(2);
  run(61, 12, 8, ORC_DENSE, 8, ORC_SYNC, 1, 2);
  run(61, 12, 8, ORC_DENSE, 8, ORC_SEQUENTIAL, 3, 1);
  run(53, 9, 6, ORC_SPM, 3, ORC_SYNC, 1, 0);
  run(53, 9, 6, ORC_SPM, 1, ORC_SEQUENTIAL, 2, 0);
  run(5, 3, 4, ORC_DENSE, 8, ORC_SYNC, 1, 2);
  /* colonies and their exchange */
  double xy[2 * 40];
  for (int i = 0; i < 80; ++i) xy[i] = (double)(int)(rnd() * 500.0);
  orc *cols[3];
  for (int c = 0; c < 3; ++c) {
    cols[c] = orc_create(xy, 40, 6, 8, 2.0, 0.9, 0.1, 0.1, 0.0, ORC_DENSE, 8, ORC_SYNC,
                         (uint64_t)c, (uint32_t)c);
    CHECK(cols[c] != NULL);
    orc_iterate(cols[c], 2);
  }
  CHECK(orc_exchange_best(cols, 3, 0) == 0);
  CHECK(orc_exchange_best(cols, 3, 1) == 0);
  for (int c = 0; c < 3; ++c) orc_destroy(cols[c]);
  /* invalid arguments */
  CHECK(orc_create(xy, 2, 1, 1, 2.0, 0.9, 0.1, 0.1, 0.0, ORC_DENSE, 8, ORC_SYNC, 0, 0) == NULL);
  CHECK(orc_create(xy, 40, 4, 8, 2.0, 1.5, 0.1, 0.1, 0.0, ORC_DENSE, 8, ORC_SYNC, 0, 0) == NULL);
  /* stand-alone helpers */
  const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
  uint32_t out[4];
  orc_philox(ctr, key, out);
  CHECK(orc_exact_dist(0.0, 0.0, 3.0, 4.0) == 5);
  const float wt[4] = {1.f, 2.f, 0.f, 4.f};
  const uint8_t un[4] = {1, 1, 1, 0};
  const int32_t k = orc_roulette_pick(wt, un, 4, 1u << 23);
  CHECK(k >= 0 && k < 3);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
