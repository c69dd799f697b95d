/*
 * CPU oracle for the Ant Colony System hot path (Skinderowicz, "The
 * GPU-based Parallel Ant Colony System", JPDC 2016, arXiv:1605.02669).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately unoptimised
 * C implementation used to check the HIP library.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Every value is computed from the definitions of Sec. 3 of the paper:
 * the pseudo-random-proportional rule (Eq. 1, Eq. 2, Alg. 2), the local
 * update (Eq. 3), the global update (Eq. 4), the iteration of Alg. 1 and the
 * selective pheromone memory update of Alg. 3 (Sec. 3.2).  Where the paper is
 * silent the readings are the ones listed in the design notes (exact integer
 * EUC_2D distance, eta = 1/d, Philox4x32-10 draws keyed by
 * (seed, iteration, ant, step), tie rules, synchronous-step semantics).
 */
#ifndef ACS_ORACLE_H
#define ACS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc;

enum { ORC_DENSE = 0, ORC_SPM = 1 };
/* ORC_SYNC: all ants select from the pheromone as it was at the start of the
 * step, then every crossing of the step is applied (ant index ascending).
 * ORC_SEQUENTIAL: Alg. 1 read literally, ant j sees the updates of ants < j
 * within the same step. */
enum { ORC_SYNC = 0, ORC_SEQUENTIAL = 1 };

/* Returns NULL on invalid arguments.  xy is n (x, y) pairs, copied. */
orc *orc_create(const double *xy, int32_t n, int32_t m, int32_t cl,
                double beta, double q0, double phi, double rho, double tau0,
                int32_t memory, int32_t spm_s, int32_t mode, uint64_t seed,
                uint32_t instance);
void orc_destroy(orc *o);
void orc_set_threads(int32_t threads);
/* Local update only after every k-th selected edge (k >= 1; default 1);
 * returns 0, or -1 for k < 1. */
int orc_set_local_period(orc *o, int32_t k);

/* Learned candidate scores (n*cl floats, each positive and finite) replace
 * eta^beta of the candidates in Eq. 1 and Eq. 2; the greedy fallback over
 * all unvisited cities keeps eta^beta.  NULL restores eta^beta.  Returns 0,
 * or -1 for an invalid weight (nothing changed). */
int orc_set_candidate_weights(orc *o, const float *w);
/* Replaces the best-so-far tour (a permutation of 0..n-1) and its length;
 * 0, or -1 if the tour is not a permutation. */
int orc_set_best(orc *o, const int32_t *tour, int64_t len);
/* Exchange of best-so-far solutions between `count` colonies of one
 * instance: each colony takes its source's best-so-far (as it was before the
 * exchange) if strictly shorter than its own.  topology 0: the source is the
 * colony with the shortest best-so-far (lowest index among equals); 1: ring,
 * the source of colony c is colony c - 1 mod count.  0, or -1. */
int orc_exchange_best(orc **cols, int32_t count, int32_t topology);

/* Local search after the construction (kind 1: 2-opt and Or-opt descent over
 * the candidate lists on every ant's tour; kind 2: the same with the four
 * pure 3-opt reconnections as a fourth move; 0: none, the default).  0, or
 * -1. */
int orc_set_local_search(orc *o, int32_t kind);
/* At most `moves` moves per descent (0: the default 50 n); lets a test look
 * at the tour after the first move.  0, or -1. */
int orc_set_local_search_cap(orc *o, int64_t moves);
/* The descent on one tour (n cities, rewritten in place) of length len:
 * returns the new length; *moves (may be NULL) the moves applied; kinds
 * (may be NULL, 6 entries) the moves by kind: 2-opt, Or-opt, 3-opt
 * reconnections (i) .. (iv). */
int64_t orc_local_search_tour(const orc *o, int32_t *tour, int64_t len, int64_t *moves,
                              int64_t *kinds);

/* One full iteration of Alg. 1 = construct (+ local search, if set) +
 * select_best + global_update. */
void orc_iterate(orc *o, int32_t k);
/* The three parts of one iteration, for tests of each part. */
void orc_construct(orc *o);
void orc_select_best(orc *o);
void orc_global_update(orc *o);
void orc_local_search(orc *o);

/* Accessors (caller-owned outputs). */
int32_t orc_n(const orc *o);
int32_t orc_m(const orc *o);
int32_t orc_cl(const orc *o);
uint32_t orc_iteration(const orc *o);
void orc_constants(const orc *o, int64_t *lnn, float *tau0, float *a_loc,
                   float *b_loc, float *a_glob, uint32_t *q0_24);
void orc_get_dist(const orc *o, int32_t *out);          /* n*n */
void orc_get_cand(const orc *o, int32_t *out);          /* n*cl */
void orc_get_eta(const orc *o, float *out, int32_t count); /* eta^beta by d */
void orc_get_tau(const orc *o, float *out);              /* n*n logical tau */
void orc_get_spm(const orc *o, int32_t *nodes, float *vals, int32_t *tail);
void orc_get_tours(const orc *o, int32_t *out);          /* m*n */
void orc_get_lengths(const orc *o, int64_t *out);        /* m */
int64_t orc_get_best(const orc *o, int32_t *tour);      /* n; -1 if none */
int64_t orc_get_iter_best(const orc *o, int32_t *ant);
/* counters since create: [steps, greedy, roulette, fallback, spm_hits,
 * spm_misses] */
void orc_get_counts(const orc *o, int64_t *out6);
/* Local-search moves applied since create. */
int64_t orc_ls_moves(const orc *o);

/* Pieces exposed for the pin tests. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int32_t orc_exact_dist(double xi, double yi, double xj, double yj);
/* Roulette selection over cl candidate weights; unvisited[k] != 0 marks the
 * members of the candidate set, u24 is the 24-bit draw. */
int32_t orc_roulette_pick(const float *w, const uint8_t *unvisited,
                          int32_t cl, uint32_t u24);
/* Histogram of orc_roulette_pick over every u24 in [0, 2^24). */
void orc_roulette_hist(const float *w, const uint8_t *unvisited, int32_t cl,
                       int64_t *counts);
/* Sets the dense pheromone matrix (n*n positive finite floats), for pins
 * that start from a chosen state (dense handles only; 0, or -1). */
int orc_set_tau(orc *o, const float *tau);
/* Alg. 3 on the record of u for neighbour v with the map x -> fmaf(a, x, b)
 * (SPM handles only; 0, or -1). */
int orc_spm_update(orc *o, int32_t u, int32_t v, float a, float b);
/* The local map of Eq. 3 with this instance's constants, applied k times. */
float orc_local_map_k(const orc *o, float x, int32_t k);

#ifdef __cplusplus
}
#endif
#endif
