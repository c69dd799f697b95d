/*
 * CPU oracle for the Ant Colony System hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, no blocking, no fusion, no reordering beyond what the definitions
 * state.  Compiled with -ffp-contract=off so that every float expression is
 * the sequence of IEEE-754 single operations written here; the only fused
 * operation is the explicit fmaf() of the pheromone maps.
 *
 * Paper: R. Skinderowicz, "The GPU-based Parallel Ant Colony System",
 * JPDC 2016 (arXiv:1605.02669).
 *   Sec. 3, Eq. 1 and Eq. 2: pseudo-random-proportional transition rule.
 *   Sec. 3, Eq. 3: local pheromone update, applied after each crossing.
 *   Sec. 3, Eq. 4: global pheromone update on the best-so-far tour.
 *   Alg. 1: one iteration (first nodes, n-1 steps with local updates, the
 *           closing edges, iteration best, best-so-far, global update).
 *   Alg. 2: next-node selection over the candidate set, greedy fallback over
 *           all unvisited nodes when the candidate set is empty.
 *   Sec. 3.2, Alg. 3: selective pheromone memory (SPM) update.
 */
#include "acs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc {
  int32_t n, m, cl;
  double beta, q0, phi, rho;
  int32_t memory, spm_s, mode;
  uint64_t seed;
  uint32_t instance;
  uint32_t iter;
  int32_t lperiod; /* local update after every lperiod-th selected edge */

  double *xy;
  int32_t *dist;  /* n*n exact integer distances */
  int32_t *cand;  /* n*cl nearest neighbours sorted by (d, j) */
  float *eta;     /* eta^beta indexed by integer distance, 0..dmax */
  float *cw;      /* NULL, or n*cl weights that replace eta^beta of the
                     candidates in Eq. 1 and Eq. 2 (learned scores) */
  int32_t dmax;
  int64_t lnn;
  float tau0, a_loc, b_loc, a_glob;
  uint32_t q0_24;

  float *tau;        /* dense: n*n */
  int32_t *spm_node; /* SPM: n*s, -1 = empty slot */
  float *spm_val;    /* SPM: n*s */
  int32_t *spm_tail; /* SPM: n, index of the most recently added slot */

  int32_t *tour;   /* m*n */
  int64_t *len;    /* m */
  uint8_t *vis;    /* m*n visited flags */
  int32_t *choice; /* m, selection of the current step */
  uint8_t *kind;   /* m, 0 greedy, 1 roulette, 2 fallback */

  int32_t *best;
  int64_t lgb; /* -1 = no best yet (+infinity) */
  int64_t lib;
  int32_t ib;

  int64_t cnt_steps, cnt_greedy, cnt_roul, cnt_fb, cnt_hit, cnt_miss;
  int32_t ls;       /* local search after construction: 0 none, 1 2-opt + Or-opt,
                       2 the same and the four pure 3-opt reconnections */
  int64_t cnt_ls;   /* improving local-search moves applied */
  int64_t ls_cap;   /* moves per descent, 0: 50 n (a smaller cap is for tests) */
};

static int g_threads = 1;
void orc_set_threads(int32_t threads) { g_threads = threads > 0 ? threads : 1; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC 2011): ten rounds of the 4x32 Philox S-box; the key  */
/* is bumped by the Weyl constants between rounds.                           */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw for (iteration, ant, step): counter = (step, ant, iteration,
 * instance), key = the 64-bit seed.  Word 0 is q, word 1 the roulette draw,
 * word 2 the start city (step 0). */
static void draw(const orc *o, uint32_t step, uint32_t ant, uint32_t w[4]) {
  uint32_t ctr[4] = {step, ant, o->iter, o->instance};
  uint32_t key[2] = {(uint32_t)o->seed, (uint32_t)(o->seed >> 32)};
  orc_philox(ctr, key, w);
}

/* ------------------------------------------------------------------------ */
/* Costs d_ij of Sec. 3: TSPLIB EUC_2D (nearest integer of the Euclidean    */
/* distance), made exact: with s = dx*dx + dy*dy evaluated in double, d is   */
/* the unique integer with (d - 1/2)^2 <= s < (d + 1/2)^2 (d = 0 iff         */
/* s < 1/4).                                                                  */
/* ------------------------------------------------------------------------ */
int32_t orc_exact_dist(double xi, double yi, double xj, double yj) {
  double dx = xi - xj;
  double dy = yi - yj;
  double sx = dx * dx;
  double sy = dy * dy;
  double s = sx + sy;
  if (s < 0.25) return 0;
  int32_t d = (int32_t)sqrt(s);
  while ((d + 0.5) * (d + 0.5) <= s) d++;
  while (d > 0 && (d - 0.5) * (d - 0.5) > s) d--;
  return d;
}

static inline int32_t D(const orc *o, int32_t i, int32_t j) {
  return o->dist[(size_t)i * o->n + j];
}

/* eta = 1/d (Eq. 1); eta^beta tabulated in double and rounded once to float.
 * A zero distance (coincident points) is treated as d = 1/2. */
static float eta_beta(double beta, int32_t d) {
  if (d == 0) return (float)pow(2.0, beta);
  return (float)(1.0 / pow((double)d, beta));
}

/* ------------------------------------------------------------------------ */
/* Pheromone memory.                                                          */
/* ------------------------------------------------------------------------ */
static inline float local_map(const orc *o, float x) {  /* Eq. 3 */
  return fmaf(o->a_loc, x, o->b_loc);
}

/* Pheromone on the directed entry (i, j) as read by an ant at i. */
static float tau_read(const orc *o, int32_t i, int32_t j) {
  if (o->memory == ORC_DENSE) return o->tau[(size_t)i * o->n + j];
  const int32_t s = o->spm_s;
  for (int32_t k = 0; k < s; ++k)
    if (o->spm_node[(size_t)i * s + k] == j) return o->spm_val[(size_t)i * s + k];
  return o->tau0; /* every edge not in the record holds the minimum, tau0 */
}

/* Alg. 3 on the record of u for neighbour v.  An existing trail gets the map
 * applied; otherwise the map is applied to tau0 and the result overwrites the
 * least recently added slot of the circular buffer. */
static void spm_update(orc *o, int32_t u, int32_t v, float a, float b) {
  const int32_t s = o->spm_s;
  int32_t *node = o->spm_node + (size_t)u * s;
  float *val = o->spm_val + (size_t)u * s;
  for (int32_t k = 0; k < s; ++k) {
    if (node[k] == v) {
      val[k] = fmaf(a, val[k], b);
      o->cnt_hit++;
      return;
    }
  }
  o->spm_tail[u] = (o->spm_tail[u] + 1) % s;
  node[o->spm_tail[u]] = v;
  val[o->spm_tail[u]] = fmaf(a, o->tau0, b);
  o->cnt_miss++;
}

/* Local update (Eq. 3) of the undirected edge {u, v}. */
static void local_update(orc *o, int32_t u, int32_t v) {
  if (o->memory == ORC_DENSE) {
    float *t = o->tau;
    t[(size_t)u * o->n + v] = local_map(o, t[(size_t)u * o->n + v]);
    t[(size_t)v * o->n + u] = local_map(o, t[(size_t)v * o->n + u]);
  } else {
    spm_update(o, u, v, o->a_loc, o->b_loc);
    spm_update(o, v, u, o->a_loc, o->b_loc);
  }
}

/* ------------------------------------------------------------------------ */
/* Instance preparation.                                                      */
/* ------------------------------------------------------------------------ */
static int build_candidates(orc *o) {
  const int32_t n = o->n, cl = o->cl;
  /* Insertion of every j != i into a list kept sorted by (d, j); only the
   * first cl entries are kept. */
  int32_t *bd = (int32_t *)malloc(sizeof(int32_t) * (size_t)cl);
  int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)cl);
  if (!bd || !bj) { free(bd); free(bj); return -1; }
  for (int32_t i = 0; i < n; ++i) {
    int32_t cnt = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      int32_t d = D(o, i, j);
      if (cnt == cl && (d > bd[cl - 1] || (d == bd[cl - 1] && j > bj[cl - 1])))
        continue;
      int32_t p = cnt < cl ? cnt : cl - 1;
      while (p > 0 && (bd[p - 1] > d || (bd[p - 1] == d && bj[p - 1] > j))) {
        bd[p] = bd[p - 1];
        bj[p] = bj[p - 1];
        --p;
      }
      bd[p] = d;
      bj[p] = j;
      if (cnt < cl) ++cnt;
    }
    memcpy(o->cand + (size_t)i * cl, bj, sizeof(int32_t) * (size_t)cl);
  }
  free(bd);
  free(bj);
  return 0;
}

/* Length of the nearest-neighbour tour from city 0 (ties: lowest index). */
static int64_t nn_tour_length(const orc *o) {
  const int32_t n = o->n;
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  int32_t cur = 0;
  int64_t L = 0;
  seen[0] = 1;
  for (int32_t step = 1; step < n; ++step) {
    int32_t bj = -1, bdist = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (seen[j]) continue;
      if (bj < 0 || D(o, cur, j) < bdist) { bj = j; bdist = D(o, cur, j); }
    }
    L += bdist;
    seen[bj] = 1;
    cur = bj;
  }
  L += D(o, cur, 0);
  free(seen);
  return L;
}

orc *orc_create(const double *xy, int32_t n, int32_t m, int32_t cl,
                double beta, double q0, double phi, double rho, double tau0,
                int32_t memory, int32_t spm_s, int32_t mode, uint64_t seed,
                uint32_t instance) {
  if (n < 3 || m < 1 || cl < 1 || cl > 256 || !(q0 >= 0.0 && q0 <= 1.0) ||
      !(phi > 0.0 && phi < 1.0) || !(rho > 0.0 && rho < 1.0) ||
      !(beta >= 0.0) || (memory != ORC_DENSE && memory != ORC_SPM) ||
      (memory == ORC_SPM && spm_s < 1) ||
      (mode != ORC_SYNC && mode != ORC_SEQUENTIAL))
    return NULL;
  for (int32_t i = 0; i < 2 * n; ++i)
    if (!isfinite(xy[i])) return NULL;
  orc *o = (orc *)calloc(1, sizeof(orc));
  if (!o) return NULL;
  o->n = n;
  o->m = m;
  o->cl = cl < n - 1 ? cl : n - 1;
  o->beta = beta; o->q0 = q0; o->phi = phi; o->rho = rho;
  o->memory = memory;
  o->spm_s = spm_s;
  o->mode = mode;
  o->seed = seed;
  o->instance = instance;
  o->lgb = -1;
  o->lperiod = 1;
  o->ib = -1;
  o->lib = -1;

  size_t nn = (size_t)n * n;
  o->xy = (double *)malloc(sizeof(double) * 2 * (size_t)n);
  o->dist = (int32_t *)malloc(sizeof(int32_t) * nn);
  o->cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * o->cl);
  o->tour = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * n);
  o->len = (int64_t *)calloc((size_t)m, sizeof(int64_t));
  o->vis = (uint8_t *)malloc((size_t)m * n);
  o->choice = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  o->kind = (uint8_t *)malloc((size_t)m);
  o->best = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!o->xy || !o->dist || !o->cand || !o->tour || !o->len || !o->vis ||
      !o->choice || !o->kind || !o->best) {
    orc_destroy(o);
    return NULL;
  }
  memcpy(o->xy, xy, sizeof(double) * 2 * (size_t)n);

  o->dmax = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = 0; j < n; ++j) {
      int32_t d = i == j ? 0 : orc_exact_dist(xy[2 * i], xy[2 * i + 1], xy[2 * j], xy[2 * j + 1]);
      o->dist[(size_t)i * n + j] = d;
      if (d > o->dmax) o->dmax = d;
    }
  o->eta = (float *)malloc(sizeof(float) * ((size_t)o->dmax + 1));
  if (!o->eta || build_candidates(o) != 0) { orc_destroy(o); return NULL; }
  for (int32_t d = 0; d <= o->dmax; ++d) o->eta[d] = eta_beta(beta, d);

  o->lnn = nn_tour_length(o);
  o->tau0 = tau0 > 0.0 ? (float)tau0 : (float)(1.0 / ((double)n * (double)o->lnn));
  o->a_loc = (float)(1.0 - phi);
  o->b_loc = (float)(phi * (double)o->tau0);
  o->a_glob = (float)(1.0 - rho);
  o->q0_24 = (uint32_t)ceil(q0 * 16777216.0);

  if (memory == ORC_DENSE) {
    o->tau = (float *)malloc(sizeof(float) * nn);
    if (!o->tau) { orc_destroy(o); return NULL; }
    for (size_t e = 0; e < nn; ++e) o->tau[e] = o->tau0;
  } else {
    size_t ns = (size_t)n * spm_s;
    o->spm_node = (int32_t *)malloc(sizeof(int32_t) * ns);
    o->spm_val = (float *)malloc(sizeof(float) * ns);
    o->spm_tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!o->spm_node || !o->spm_val || !o->spm_tail) { orc_destroy(o); return NULL; }
    for (size_t e = 0; e < ns; ++e) { o->spm_node[e] = -1; o->spm_val[e] = o->tau0; }
    for (int32_t i = 0; i < n; ++i) o->spm_tail[i] = spm_s - 1;
  }
  return o;
}

void orc_destroy(orc *o) {
  if (!o) return;
  free(o->xy); free(o->dist); free(o->cand); free(o->eta); free(o->cw); free(o->tau);
  free(o->spm_node); free(o->spm_val); free(o->spm_tail); free(o->tour);
  free(o->len); free(o->vis); free(o->choice); free(o->kind); free(o->best);
  free(o);
}

/* ------------------------------------------------------------------------ */
/* Eq. 2 by roulette wheel: the inclusive prefix sums P of the weights are   */
/* formed by the Hillis-Steele scan (rounds with offsets 1, 2, 4, ... < cl,  */
/* each reading the previous round's values); r = u * P[cl-1] and the pick is*/
/* the first member of the candidate set whose prefix sum exceeds r (the     */
/* scan's rounding is not monotone, so a visited position can have a larger  */
/* sum than its predecessor and must be skipped).  If no member does, the    */
/* last member of the candidate set is taken.                                */
/* ------------------------------------------------------------------------ */
int32_t orc_roulette_pick(const float *w, const uint8_t *unvisited, int32_t cl,
                          uint32_t u24) {
  float P[256], nxt[256];
  for (int32_t k = 0; k < cl; ++k) P[k] = w[k];
  for (int32_t off = 1; off < cl; off <<= 1) {
    for (int32_t k = 0; k < cl; ++k) nxt[k] = k >= off ? P[k] + P[k - off] : P[k];
    for (int32_t k = 0; k < cl; ++k) P[k] = nxt[k];
  }
  float u = (float)u24 * 0x1p-24f;
  float r = u * P[cl - 1];
  for (int32_t k = 0; k < cl; ++k)
    if (unvisited[k] && P[k] > r) return k;
  int32_t last = -1;
  for (int32_t k = 0; k < cl; ++k)
    if (unvisited[k]) last = k;
  return last;
}

void orc_roulette_hist(const float *w, const uint8_t *unvisited, int32_t cl,
                       int64_t *counts) {
  for (int32_t k = 0; k < cl; ++k) counts[k] = 0;
  for (uint32_t u = 0; u < (1u << 24); ++u) {
    int32_t k = orc_roulette_pick(w, unvisited, cl, u);
    if (k >= 0) counts[k]++;
  }
}

/* Heuristic factor of candidate k of city i in Eq. 1 and Eq. 2: eta^beta of
 * the edge, or the weight set by orc_set_candidate_weights in its place. */
static float cand_weight(const orc *o, int32_t i, int32_t k) {
  if (o->cw) return o->cw[(size_t)i * o->cl + k];
  return o->eta[D(o, i, o->cand[(size_t)i * o->cl + k])];
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: next node of ant a standing at cur after step t's draw.            */
/* ------------------------------------------------------------------------ */
static int32_t select_next(const orc *o, int32_t a, int32_t t, int32_t cur,
                           uint8_t *kind) {
  const int32_t n = o->n, cl = o->cl;
  const uint8_t *vis = o->vis + (size_t)a * n;
  const int32_t *cn = o->cand + (size_t)cur * cl;
  float w[256];
  uint8_t unv[256];
  int32_t any = 0;
  uint32_t r4[4];
  draw(o, (uint32_t)t, (uint32_t)a, r4);

  /* candidate set = unvisited members of the cl nearest neighbours */
  for (int32_t k = 0; k < cl; ++k) {
    int32_t j = cn[k];
    unv[k] = vis[j] ? 0 : 1;
    w[k] = unv[k] ? tau_read(o, cur, j) * cand_weight(o, cur, k) : 0.0f;
    any |= unv[k];
  }
  if (any) {
    if ((r4[0] >> 8) < o->q0_24) {
      /* Eq. 1, exploitation: maximum of tau * eta^beta, ties -> lowest
       * position in the (d, j)-sorted list */
      int32_t bk = -1;
      for (int32_t k = 0; k < cl; ++k)
        if (unv[k] && (bk < 0 || w[k] > w[bk])) bk = k;
      *kind = 0;
      return cn[bk];
    }
    /* Eq. 1, exploration: Eq. 2 over the candidate set */
    *kind = 1;
    return cn[orc_roulette_pick(w, unv, cl, r4[1] >> 8)];
  }
  /* empty candidate set: greedy over every unvisited node, ties -> lowest j;
   * the heuristic factor here is always eta^beta of the edge */
  *kind = 2;
  int32_t bj = -1;
  float bv = 0.0f;
  for (int32_t j = 0; j < n; ++j) {
    if (vis[j]) continue;
    float v = tau_read(o, cur, j) * o->eta[D(o, cur, j)];
    if (bj < 0 || v > bv) { bj = j; bv = v; }
  }
  return bj;
}

static void move_ant(orc *o, int32_t a, int32_t t, int32_t next) {
  const int32_t n = o->n;
  int32_t cur = o->tour[(size_t)a * n + t - 1];
  o->tour[(size_t)a * n + t] = next;
  o->vis[(size_t)a * n + next] = 1;
  o->len[a] += D(o, cur, next);
}

static void count_kind(orc *o, uint8_t k) {
  o->cnt_steps++;
  if (k == 0) o->cnt_greedy++;
  else if (k == 1) o->cnt_roul++;
  else o->cnt_fb++;
}

/* Construction part of Alg. 1 for every ant of this iteration. */
void orc_construct(orc *o) {
  const int32_t n = o->n, m = o->m;
  memset(o->vis, 0, (size_t)m * n);
  for (int32_t a = 0; a < m; ++a) {
    uint32_t r4[4];
    draw(o, 0u, (uint32_t)a, r4);
    int32_t start = (int32_t)(((uint64_t)r4[2] * (uint64_t)n) >> 32);
    o->tour[(size_t)a * n] = start;
    o->vis[(size_t)a * n + start] = 1;
    o->len[a] = 0;
  }
  for (int32_t t = 1; t < n; ++t) {
    if (o->mode == ORC_SYNC) {
      /* every ant selects from the pheromone as it is at the start of step t
       * (no writes happen in this loop, so the ants are independent) */
#pragma omp parallel for schedule(static) num_threads(g_threads)
      for (int32_t a = 0; a < m; ++a) {
        int32_t cur = o->tour[(size_t)a * n + t - 1];
        o->choice[a] = select_next(o, a, t, cur, &o->kind[a]);
      }
      for (int32_t a = 0; a < m; ++a) {
        move_ant(o, a, t, o->choice[a]);
        count_kind(o, o->kind[a]);
      }
      if (t % o->lperiod == 0)
        for (int32_t a = 0; a < m; ++a)
          local_update(o, o->tour[(size_t)a * n + t - 1], o->tour[(size_t)a * n + t]);
    } else {
      for (int32_t a = 0; a < m; ++a) {
        int32_t cur = o->tour[(size_t)a * n + t - 1];
        uint8_t k;
        int32_t next = select_next(o, a, t, cur, &k);
        move_ant(o, a, t, next);
        count_kind(o, k);
        if (t % o->lperiod == 0) local_update(o, cur, next);
      }
    }
  }
  /* closing edges: length and local update (the last step of the schedule;
   * updated whatever the period) */
  for (int32_t a = 0; a < m; ++a) {
    int32_t last = o->tour[(size_t)a * n + n - 1], first = o->tour[(size_t)a * n];
    o->len[a] += D(o, last, first);
  }
  for (int32_t a = 0; a < m; ++a)
    local_update(o, o->tour[(size_t)a * n + n - 1], o->tour[(size_t)a * n]);
}

/* ------------------------------------------------------------------------ */
/* Local search (Sec. 5.1 leaves "a local search heuristic, e.g. 3-Opt" as   */
/* further research).  Reading: first-improvement descent over 2-opt moves   */
/* and Or-opt moves (a segment of 1..3 cities moved elsewhere, a subset of   */
/* the 3-opt exchanges), every move creating an edge from the examined city  */
/* a to one of its candidates (the cl nearest), with a FIFO queue of cities  */
/* to examine (don't-look bits).  Distances are integers, so a move is taken */
/* only if it shortens the tour by at least 1 and the descent ends.          */
/*                                                                            */
/* For a popped city a the moves are tried in this order, the first that     */
/* shortens the tour is applied:                                              */
/*  1. 2-opt on a's successor b: for each candidate c (k ascending) while    */
/*     d(a,c) < d(a,b), e = succ(c): edges (a,b), (c,e) -> (a,c), (b,e).      */
/*  2. 2-opt on a's predecessor b: for each c while d(a,c) < d(b,a),          */
/*     e = pred(c): edges (b,a), (e,c) -> (a,c), (b,e).                        */
/*  3. Or-opt, L = 1, 2, 3: the segment S = a and the L - 1 cities after it,  */
/*     p = pred(a), x the city after S; for each candidate c (k ascending):   */
/*     (A) S between c and e = succ(c), a next to c;                          */
/*     (B) S reversed between f = pred(c) and c, a next to c.                 */
/*  4. (kind 2 only) 3-opt: with b = succ(a), the tour a [B = b..c]           */
/*     [C = d..e] f becomes a X Y f, one of the four reconnections that      */
/*     replace all three removed edges (a,b), (c,d), (e,f), tried in this    */
/*     order, the first created edge joining a to a candidate x with         */
/*     d(a,x) < d(a,b) (x's candidate index k ascending), the second one     */
/*     joining the named city to one of its candidates y (ascending) while   */
/*     the partial gain stays positive:                                       */
/*     (i)   C B:   x = d, y = e from b's candidates: (a,d), (e,b), (c,f);    */
/*     (ii)  C B':  x = d, y = e from c's candidates: (a,d), (c,e), (b,f);    */
/*     (iii) C' B:  x = e, y = d from b's candidates: (a,e), (b,d), (c,f);    */
/*     (iv)  B' C': x = c, y = e from b's candidates: (a,c), (b,e), (d,f).    */
/*     The positions after a are rewritten in place by reversals of B, C or  */
/*     both together; a, b, c, d, e, f are queued.                            */
/* Then the cities at the ends of the changed edges are queued, in the order  */
/* listed at each move, if not queued already.  The queue starts with the    */
/* tour in order.  At most 50 n moves are applied.                           */
/*                                                                            */
/* The array holds the cycle; how a move rewrites it is fixed as well: a     */
/* 2-opt move reverses the forward path between the two cities when it holds */
/* at most half of them, else the rest of the tour (the same cycle); an      */
/* Or-opt move shifts the shorter of the two blocks between the segment's    */
/* old and new places by L positions and writes the segment into the gap.    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n;
  int32_t *t, *pos, *q;
  uint8_t *inq;
  int32_t qh, qn;
} ls_state;

static int32_t ls_at(const ls_state *w, int32_t i) { return w->t[((i % w->n) + w->n) % w->n]; }
static int32_t ls_succ(const ls_state *w, int32_t c) { return ls_at(w, w->pos[c] + 1); }
static int32_t ls_pred(const ls_state *w, int32_t c) { return ls_at(w, w->pos[c] - 1); }

static void ls_put(ls_state *w, int32_t i, int32_t c) {
  i = ((i % w->n) + w->n) % w->n;
  w->t[i] = c;
  w->pos[c] = i;
}

static void ls_push(ls_state *w, int32_t c) {
  if (w->inq[c]) return;
  w->inq[c] = 1;
  w->q[(w->qh + w->qn) % w->n] = c;
  w->qn++;
}

/* the forward path from city u to city v, reversed (or the rest of the tour) */
static void ls_reverse(ls_state *w, int32_t u, int32_t v) {
  const int32_t n = w->n;
  int32_t i = w->pos[u], j = w->pos[v];
  int32_t len = (j - i + n) % n + 1;
  if (2 * len > n) {
    const int32_t i2 = (j + 1) % n, j2 = (i - 1 + n) % n;
    i = i2;
    j = j2;
    len = n - len;
  }
  for (int32_t s = 0; s < len / 2; ++s) {
    const int32_t a = ls_at(w, i + s), b = ls_at(w, j - s);
    ls_put(w, i + s, b);
    ls_put(w, j - s, a);
  }
}

/* Or-opt: the segment of L cities at positions i .. i + L - 1 goes between
 * cities c and e = succ(c) in its own orientation (side 0), or reversed
 * between f = pred(c) and c (side 1). */
static void ls_oropt(ls_state *w, int32_t i, int32_t L, int32_t c, int32_t side) {
  const int32_t n = w->n;
  int32_t seg[3];
  for (int32_t q = 0; q < L; ++q) seg[q] = ls_at(w, i + q);
  if (side == 0) {
    /* cycle p S [x .. c] e ... : blocks B = x..c, C = e..p */
    const int32_t nb = (w->pos[c] - (i + L) % n + n) % n + 1, nc = n - L - nb;
    if (nb <= nc) {
      for (int32_t r = 0; r < nb; ++r) ls_put(w, i + r, ls_at(w, i + L + r));
      for (int32_t q = 0; q < L; ++q) ls_put(w, i + nb + q, seg[q]);
    } else {
      const int32_t e0 = (w->pos[c] + 1) % n;
      for (int32_t r = nc - 1; r >= 0; --r) ls_put(w, e0 + r + L, ls_at(w, e0 + r));
      for (int32_t q = 0; q < L; ++q) ls_put(w, e0 + q, seg[q]);
    }
  } else {
    /* cycle f [c .. p] S x ... : blocks C = c..p, B = x..f */
    const int32_t c0 = w->pos[c];
    const int32_t nc = (i - 1 - c0 + 2 * n) % n + 1, nb = n - L - nc;
    if (nc <= nb) {
      for (int32_t r = nc - 1; r >= 0; --r) ls_put(w, c0 + r + L, ls_at(w, c0 + r));
      for (int32_t q = 0; q < L; ++q) ls_put(w, c0 + q, seg[L - 1 - q]);
    } else {
      for (int32_t r = 0; r < nb; ++r) ls_put(w, i + r, ls_at(w, i + L + r));
      for (int32_t q = 0; q < L; ++q) ls_put(w, i + nb + q, seg[L - 1 - q]);
    }
  }
}

/* the cities at positions i .. j (forward, j reached from i) in reverse order */
static void ls_reverse_at(ls_state *w, int32_t i, int32_t j) {
  const int32_t n = w->n;
  const int32_t len = (j - i + n) % n + 1;
  for (int32_t s = 0; s < len / 2; ++s) {
    const int32_t a = ls_at(w, i + s), b = ls_at(w, j - s);
    ls_put(w, i + s, b);
    ls_put(w, j - s, a);
  }
}

/* 3-opt step of the descent (move 4 above) for the popped city a; returns
 * 1 + the reconnection's index (0 .. 3) if a move was applied, else 0. */
static int ls_three_opt(const orc *o, ls_state *w, int32_t a, int64_t *len) {
  const int32_t n = o->n, cl = o->cl;
  const int32_t *ca = o->cand + (size_t)a * cl;
  const int32_t pa = w->pos[a];
  const int32_t b = ls_at(w, pa + 1);
  const int64_t dab = D(o, a, b);
  for (int32_t type = 0; type < 4; ++type) {
    for (int32_t kx = 0; kx < cl; ++kx) {
      const int32_t x = ca[kx];
      const int64_t dax = D(o, a, x);
      if (dax >= dab) break;
      const int32_t ox = (w->pos[x] - pa + n) % n; /* offset of x after a */
      /* the city whose candidates give y, and the gain so far */
      int32_t from;
      int64_t g;
      if (type == 0 || type == 1) { /* x = d */
        if (ox < 2) continue;
        const int32_t c = ls_at(w, pa + ox - 1);
        from = type == 0 ? b : c;
        g = dab - dax + D(o, c, x);
      } else if (type == 2) { /* x = e */
        if (ox < 3) continue;
        from = b;
        g = dab - dax + D(o, x, ls_at(w, pa + ox + 1));
      } else { /* x = c */
        if (ox < 2 || ox > n - 3) continue;
        from = b;
        g = dab - dax + D(o, x, ls_at(w, pa + ox + 1));
      }
      const int32_t *cy = o->cand + (size_t)from * cl;
      for (int32_t ky = 0; ky < cl; ++ky) {
        const int32_t y = cy[ky];
        const int64_t dfy = D(o, from, y);
        if (dfy >= g) break;
        const int32_t oy = (w->pos[y] - pa + n) % n;
        int32_t c, d, e, f, oe, od;
        int64_t delta;
        if (type == 0 || type == 1) {
          od = ox;
          oe = oy;
          if (type == 0 ? oe < od : oe <= od) continue;
        } else if (type == 2) {
          od = oy;
          oe = ox;
          if (od < 2 || od >= oe) continue;
        } else {
          od = ox + 1;
          oe = oy;
          if (oe <= od) continue;
        }
        c = ls_at(w, pa + od - 1);
        d = ls_at(w, pa + od);
        e = ls_at(w, pa + oe);
        f = ls_at(w, pa + oe + 1);
        const int64_t removed = dab + D(o, c, d) + D(o, e, f);
        if (type == 0) delta = D(o, a, d) + D(o, e, b) + D(o, c, f) - removed;
        else if (type == 1) delta = D(o, a, d) + D(o, c, e) + D(o, b, f) - removed;
        else if (type == 2) delta = D(o, a, e) + D(o, b, d) + D(o, c, f) - removed;
        else delta = D(o, a, c) + D(o, b, e) + D(o, d, f) - removed;
        if (delta >= 0) continue;
        /* positions pa + 1 .. pa + oe hold B (od - 1 cities) then C */
        const int32_t p0 = pa + 1, nb = od - 1, nc = oe - od + 1;
        if (type == 0) {          /* C B */
          ls_reverse_at(w, p0 % n, (p0 + oe - 1) % n);
          ls_reverse_at(w, p0 % n, (p0 + nc - 1) % n);
          ls_reverse_at(w, (p0 + nc) % n, (p0 + oe - 1) % n);
        } else if (type == 1) {   /* C B' */
          ls_reverse_at(w, p0 % n, (p0 + oe - 1) % n);
          ls_reverse_at(w, p0 % n, (p0 + nc - 1) % n);
        } else if (type == 2) {   /* C' B */
          ls_reverse_at(w, p0 % n, (p0 + oe - 1) % n);
          ls_reverse_at(w, (p0 + nc) % n, (p0 + oe - 1) % n);
        } else {                  /* B' C' */
          ls_reverse_at(w, p0 % n, (p0 + nb - 1) % n);
          ls_reverse_at(w, (p0 + nb) % n, (p0 + oe - 1) % n);
        }
        *len += delta;
        ls_push(w, a); ls_push(w, b); ls_push(w, c);
        ls_push(w, d); ls_push(w, e); ls_push(w, f);
        return 1 + type;
      }
    }
  }
  return 0;
}

/* One descent on tour[0..n-1] (rewritten in place); returns the new length,
 * *moves the number of moves applied, kinds[0 .. 5] (if not NULL) the moves
 * by kind: 2-opt, Or-opt, 3-opt (i) .. (iv). */
static int64_t ls_descent(const orc *o, int32_t *tour, int64_t len, ls_state *w, int64_t *moves,
                          int64_t *kinds) {
  const int32_t n = o->n, cl = o->cl;
  w->t = tour;
  for (int32_t p = 0; p < n; ++p) w->pos[tour[p]] = p;
  memset(w->inq, 0, (size_t)n);
  w->qh = 0;
  w->qn = 0;
  for (int32_t p = 0; p < n; ++p) ls_push(w, tour[p]);
  const int64_t cap = o->ls_cap > 0 ? o->ls_cap : 50 * (int64_t)n;
  int64_t mv = 0;
  while (w->qn > 0 && mv < cap) {
    const int32_t a = w->q[w->qh];
    w->qh = (w->qh + 1) % n;
    w->qn--;
    w->inq[a] = 0;
    const int32_t *ca = o->cand + (size_t)a * cl;
    int done = 0;
    /* 1. 2-opt on the successor */
    {
      const int32_t b = ls_succ(w, a);
      for (int32_t k = 0; k < cl && !done; ++k) {
        const int32_t c = ca[k];
        if (D(o, a, c) >= D(o, a, b)) break;
        const int32_t e = ls_succ(w, c);
        if (c == b || e == a) continue;
        const int64_t delta = (int64_t)D(o, a, c) + D(o, b, e) - D(o, a, b) - D(o, c, e);
        if (delta < 0) {
          ls_reverse(w, b, c);
          len += delta;
          ls_push(w, a); ls_push(w, b); ls_push(w, c); ls_push(w, e);
          done = 1;
          if (kinds) kinds[0]++;
        }
      }
    }
    /* 2. 2-opt on the predecessor */
    if (!done) {
      const int32_t b = ls_pred(w, a);
      for (int32_t k = 0; k < cl && !done; ++k) {
        const int32_t c = ca[k];
        if (D(o, a, c) >= D(o, b, a)) break;
        const int32_t e = ls_pred(w, c);
        if (c == b || e == a) continue;
        const int64_t delta = (int64_t)D(o, a, c) + D(o, b, e) - D(o, b, a) - D(o, e, c);
        if (delta < 0) {
          ls_reverse(w, a, e);
          len += delta;
          ls_push(w, a); ls_push(w, b); ls_push(w, c); ls_push(w, e);
          done = 1;
          if (kinds) kinds[0]++;
        }
      }
    }
    /* 3. Or-opt */
    for (int32_t L = 1; L <= 3 && !done; ++L) {
      if (n < L + 3) break;
      const int32_t i = w->pos[a];
      const int32_t s1 = a, sL = ls_at(w, i + L - 1);
      const int32_t p = ls_at(w, i - 1), x = ls_at(w, i + L);
      const int64_t g = (int64_t)D(o, p, s1) + D(o, sL, x) - D(o, p, x);
      for (int32_t k = 0; k < cl && !done; ++k) {
        const int32_t c = ca[k];
        const int32_t off = (w->pos[c] - i + n) % n;
        if (off < L) continue; /* c inside the segment */
        /* (A) between c and its successor */
        if (c != p) {
          const int32_t e = ls_succ(w, c);
          const int64_t delta = (int64_t)D(o, c, s1) + D(o, sL, e) - D(o, c, e) - g;
          if (delta < 0) {
            ls_oropt(w, i, L, c, 0);
            len += delta;
            ls_push(w, p); ls_push(w, x); ls_push(w, s1); ls_push(w, sL);
            ls_push(w, c); ls_push(w, e);
            done = 1;
            if (kinds) kinds[1]++;
            break;
          }
        }
        /* (B) reversed, between the predecessor of c and c */
        if (c != x) {
          const int32_t f = ls_pred(w, c);
          const int64_t delta = (int64_t)D(o, f, sL) + D(o, s1, c) - D(o, f, c) - g;
          if (delta < 0) {
            ls_oropt(w, i, L, c, 1);
            len += delta;
            ls_push(w, p); ls_push(w, x); ls_push(w, s1); ls_push(w, sL);
            ls_push(w, f); ls_push(w, c);
            done = 1;
            if (kinds) kinds[1]++;
            break;
          }
        }
      }
    }
    /* 4. 3-opt */
    if (!done && o->ls >= 2 && n >= 6) {
      const int r = ls_three_opt(o, w, a, &len);
      if (r) {
        done = 1;
        if (kinds) kinds[1 + r]++;
      }
    }
    if (done) mv++;
  }
  *moves = mv;
  return len;
}

int64_t orc_local_search_tour(const orc *o, int32_t *tour, int64_t len, int64_t *moves,
                              int64_t *kinds) {
  const int32_t n = o->n;
  ls_state w;
  w.n = n;
  w.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  w.q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  w.inq = (uint8_t *)malloc((size_t)n);
  int64_t mv = 0;
  if (kinds)
    for (int k = 0; k < 6; ++k) kinds[k] = 0;
  if (w.pos && w.q && w.inq) len = ls_descent(o, tour, len, &w, &mv, kinds);
  else len = -1;
  free(w.pos);
  free(w.q);
  free(w.inq);
  if (moves) *moves = mv;
  return len;
}

int orc_set_local_search(orc *o, int32_t kind) {
  if (kind < 0 || kind > 2) return -1;
  o->ls = kind;
  return 0;
}

int orc_set_local_search_cap(orc *o, int64_t moves) {
  if (moves < 0) return -1;
  o->ls_cap = moves;
  return 0;
}

/* The local search on every ant's tour, after the construction (and its
 * local updates) and before the iteration best is chosen. */
void orc_local_search(orc *o) {
  if (!o->ls) return;
  const int32_t n = o->n, m = o->m;
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads) reduction(+ : total)
  for (int32_t a = 0; a < m; ++a) {
    int64_t mv = 0;
    o->len[a] = orc_local_search_tour(o, o->tour + (size_t)a * n, o->len[a], &mv, NULL);
    total += mv;
  }
  o->cnt_ls += total;
}

/* Alg. 1: iteration best (lowest ant index among equal lengths); it becomes
 * the best-so-far only if strictly shorter. */
void orc_select_best(orc *o) {
  int32_t ib = 0;
  for (int32_t a = 1; a < o->m; ++a)
    if (o->len[a] < o->len[ib]) ib = a;
  o->ib = ib;
  o->lib = o->len[ib];
  if (o->lgb < 0 || o->lib < o->lgb) {
    o->lgb = o->lib;
    memcpy(o->best, o->tour + (size_t)ib * o->n, sizeof(int32_t) * (size_t)o->n);
  }
}

/* Eq. 4 restricted to the edges of the best-so-far tour (deposit 1/L_gb). */
void orc_global_update(orc *o) {
  const int32_t n = o->n;
  if (o->lgb < 0) return;
  float a = o->a_glob;
  float b = (float)(o->rho / (double)o->lgb);
  for (int32_t p = 0; p < n; ++p) {
    int32_t u = o->best[p], v = o->best[(p + 1) % n];
    if (o->memory == ORC_DENSE) {
      o->tau[(size_t)u * n + v] = fmaf(a, o->tau[(size_t)u * n + v], b);
      o->tau[(size_t)v * n + u] = fmaf(a, o->tau[(size_t)v * n + u], b);
    } else {
      spm_update(o, u, v, a, b);
      spm_update(o, v, u, a, b);
    }
  }
}

/* Sec. 4, limiting the number of local updates: the update follows only
 * every k-th edge an ant selects, i.e. the edges of steps t = k, 2k, ...
 * (1-based); the closing edge keeps its update. */
int orc_set_local_period(orc *o, int32_t k) {
  if (k < 1) return -1;
  o->lperiod = k;
  return 0;
}

/* Learned candidate scores: w[i * cl + k] replaces eta^beta of candidate k
 * of city i in Eq. 1 and Eq. 2; the fallback over all unvisited cities keeps
 * eta^beta.  Every weight must be positive and finite (else -1, nothing
 * changed); NULL restores eta^beta. */
int orc_set_candidate_weights(orc *o, const float *w) {
  const size_t cnt = (size_t)o->n * o->cl;
  if (!w) {
    free(o->cw);
    o->cw = NULL;
    return 0;
  }
  for (size_t e = 0; e < cnt; ++e)
    if (!(w[e] > 0.0f) || !isfinite(w[e])) return -1;
  if (!o->cw) {
    o->cw = (float *)malloc(sizeof(float) * cnt);
    if (!o->cw) return -1;
  }
  memcpy(o->cw, w, sizeof(float) * cnt);
  return 0;
}

/* Sets the dense pheromone matrix (n*n, row-major, positive finite values),
 * for the pin tests that start from a chosen state (dense only; -1
 * otherwise). */
int orc_set_tau(orc *o, const float *tau) {
  const size_t nn = (size_t)o->n * o->n;
  if (o->memory != ORC_DENSE) return -1;
  for (size_t e = 0; e < nn; ++e)
    if (!(tau[e] > 0.0f) || !isfinite(tau[e])) return -1;
  memcpy(o->tau, tau, sizeof(float) * nn);
  return 0;
}

/* Alg. 3 on the record of u for neighbour v with the map x -> fmaf(a, x, b),
 * exposed for the pin tests (SPM only; -1 otherwise). */
int orc_spm_update(orc *o, int32_t u, int32_t v, float a, float b) {
  if (o->memory != ORC_SPM || u < 0 || u >= o->n || v < 0 || v >= o->n) return -1;
  spm_update(o, u, v, a, b);
  return 0;
}

/* Replaces the best-so-far tour and its length (the receiving side of an
 * exchange between colonies).  The tour must be a permutation of 0..n-1
 * (else -1, nothing changed). */
int orc_set_best(orc *o, const int32_t *tour, int64_t len) {
  const int32_t n = o->n;
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  if (!seen || len < 0) { free(seen); return -1; }
  for (int32_t p = 0; p < n; ++p) {
    if (tour[p] < 0 || tour[p] >= n || seen[tour[p]]) { free(seen); return -1; }
    seen[tour[p]] = 1;
  }
  free(seen);
  memcpy(o->best, tour, sizeof(int32_t) * (size_t)n);
  o->lgb = len;
  return 0;
}

/* Exchange of the best solutions between C colonies of one instance
 * (the multi-colony model of Sec. 2: periodic exchange along a
 * communication topology).  Every colony first offers its best-so-far as it
 * is before the exchange; then colony c takes the offer of its source if
 * that is strictly shorter than its own.  topology 0: the source of every
 * colony is the colony with the shortest best-so-far (lowest index among
 * equals); topology 1 (ring): the source of colony c is colony c - 1
 * (colony 0: colony C - 1).  Colonies without a best-so-far offer nothing.
 * Returns -1 for an invalid call. */
int orc_exchange_best(orc **cols, int32_t count, int32_t topology) {
  if (count < 1 || (topology != 0 && topology != 1)) return -1;
  const int32_t n = cols[0]->n;
  for (int32_t c = 1; c < count; ++c)
    if (cols[c]->n != n) return -1;
  int32_t *offer = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * count);
  int64_t *olen = (int64_t *)malloc(sizeof(int64_t) * (size_t)count);
  if (!offer || !olen) { free(offer); free(olen); return -1; }
  for (int32_t c = 0; c < count; ++c) {
    olen[c] = cols[c]->lgb;
    memcpy(offer + (size_t)c * n, cols[c]->best, sizeof(int32_t) * (size_t)n);
  }
  int32_t g = -1;
  for (int32_t c = 0; c < count; ++c)
    if (olen[c] >= 0 && (g < 0 || olen[c] < olen[g])) g = c;
  for (int32_t c = 0; c < count; ++c) {
    const int32_t src = topology == 0 ? g : (c + count - 1) % count;
    if (src < 0 || olen[src] < 0) continue;
    if (cols[c]->lgb < 0 || olen[src] < cols[c]->lgb) {
      memcpy(cols[c]->best, offer + (size_t)src * n, sizeof(int32_t) * (size_t)n);
      cols[c]->lgb = olen[src];
    }
  }
  free(offer);
  free(olen);
  return 0;
}

void orc_iterate(orc *o, int32_t k) {
  for (int32_t i = 0; i < k; ++i) {
    orc_construct(o);
    orc_local_search(o);
    orc_select_best(o);
    orc_global_update(o);
    o->iter++;
  }
}

/* ------------------------------------------------------------------------ */
/* Accessors                                                                  */
/* ------------------------------------------------------------------------ */
int32_t orc_n(const orc *o) { return o->n; }
int32_t orc_m(const orc *o) { return o->m; }
int32_t orc_cl(const orc *o) { return o->cl; }
uint32_t orc_iteration(const orc *o) { return o->iter; }

void orc_constants(const orc *o, int64_t *lnn, float *tau0, float *a_loc,
                   float *b_loc, float *a_glob, uint32_t *q0_24) {
  *lnn = o->lnn; *tau0 = o->tau0; *a_loc = o->a_loc; *b_loc = o->b_loc;
  *a_glob = o->a_glob; *q0_24 = o->q0_24;
}

void orc_get_dist(const orc *o, int32_t *out) {
  memcpy(out, o->dist, sizeof(int32_t) * (size_t)o->n * o->n);
}
void orc_get_cand(const orc *o, int32_t *out) {
  memcpy(out, o->cand, sizeof(int32_t) * (size_t)o->n * o->cl);
}
void orc_get_eta(const orc *o, float *out, int32_t count) {
  for (int32_t d = 0; d < count; ++d) out[d] = eta_beta(o->beta, d);
}
void orc_get_tau(const orc *o, float *out) {
  for (int32_t i = 0; i < o->n; ++i)
    for (int32_t j = 0; j < o->n; ++j) out[(size_t)i * o->n + j] = tau_read(o, i, j);
}
void orc_get_spm(const orc *o, int32_t *nodes, float *vals, int32_t *tail) {
  if (o->memory != ORC_SPM) return;
  size_t ns = (size_t)o->n * o->spm_s;
  memcpy(nodes, o->spm_node, sizeof(int32_t) * ns);
  memcpy(vals, o->spm_val, sizeof(float) * ns);
  memcpy(tail, o->spm_tail, sizeof(int32_t) * (size_t)o->n);
}
void orc_get_tours(const orc *o, int32_t *out) {
  memcpy(out, o->tour, sizeof(int32_t) * (size_t)o->m * o->n);
}
void orc_get_lengths(const orc *o, int64_t *out) {
  memcpy(out, o->len, sizeof(int64_t) * (size_t)o->m);
}
int64_t orc_get_best(const orc *o, int32_t *tour) {
  if (o->lgb >= 0 && tour) memcpy(tour, o->best, sizeof(int32_t) * (size_t)o->n);
  return o->lgb;
}
int64_t orc_get_iter_best(const orc *o, int32_t *ant) {
  if (ant) *ant = o->ib;
  return o->lib;
}
int64_t orc_ls_moves(const orc *o) { return o->cnt_ls; }

void orc_get_counts(const orc *o, int64_t *out6) {
  out6[0] = o->cnt_steps; out6[1] = o->cnt_greedy; out6[2] = o->cnt_roul;
  out6[3] = o->cnt_fb; out6[4] = o->cnt_hit; out6[5] = o->cnt_miss;
}

float orc_local_map_k(const orc *o, float x, int32_t k) {
  for (int32_t i = 0; i < k; ++i) x = local_map(o, x);
  return x;
}
