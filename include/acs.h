/*
 * libacs -- Ant Colony System hot path for AMD Instinct MI355X (gfx950).
 *
 * Method: R. Skinderowicz, "The GPU-based Parallel Ant Colony System",
 * J. Parallel Distrib. Comput. 2016 (arXiv:1605.02669), Sec. 3.
 *
 * One handle holds one colony on one symmetric Euclidean TSP instance
 * (the complete graph of Sec. 3).  Each call of acs_iterate runs whole
 * iterations of Alg. 1: every ant picks a start city, extends its tour with
 * the pseudo-random-proportional rule (Eq. 1, Eq. 2) over its candidate set
 * of nearest neighbours and falls back to the greedy choice over all
 * unvisited cities when that set is empty (Alg. 2); every crossing is
 * followed by the local update (Eq. 3); the iteration ends with the global
 * update (Eq. 4) on the best-so-far tour.  The pheromone lives either in a
 * dense n x n matrix or in the selective pheromone memory of Sec. 3.2
 * (Alg. 3), which keeps at most s trails per city and reads every other
 * trail as tau0.
 *
 * Conventions for every entry point:
 *   - Return 0 (ACS_OK) on success, a negative ACS_E_* code otherwise; the
 *     message of the last failure on the calling thread is acs_last_error().
 *   - Host pointers are plain host memory owned by the caller; inputs are
 *     copied, outputs are written to caller-owned buffers of the stated size.
 *     Device pointers appear only as the optional stream and workspace.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Nothing here falls back to the CPU: the iteration runs in the
 *     library's HIP kernels, and a missing or unusable GPU is an error.
 */
#ifndef ACS_H
#define ACS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACS_OK 0
#define ACS_E_INVALID (-1)     /* argument out of range */
#define ACS_E_NOMEM (-2)       /* device or host allocation failed */
#define ACS_E_DEVICE (-3)      /* a HIP call or kernel failed */
#define ACS_E_BUFSIZE (-4)     /* caller buffer or workspace too small */
#define ACS_E_STATE (-5)       /* NULL or destroyed handle */
#define ACS_E_UNSUPPORTED (-6) /* valid request this handle cannot serve */

typedef struct acs_t acs_t; /* opaque handle, owned by the library */

enum acs_memory { ACS_DENSE = 0, ACS_SPM = 1 };

/* ACS_SYNC: within a step every ant selects from the pheromone as it was at
 * the start of the step; then every crossing of that step is applied (an
 * edge crossed k times gets the map k times).  Tours and pheromone are a
 * deterministic function of (instance, parameters, seed).
 * ACS_ASYNC_ATOMIC: every ant runs its whole tour without waiting for the
 * others and applies the local update of Eq. 3 right after each move with an
 * atomic compare-and-swap; reads see whatever the other ants have written
 * so far (the unsynchronised single-kernel construction of Sec. 3.1.2).
 * ACS_ASYNC_RACY: as ACS_ASYNC_ATOMIC, but each update writes the map of the
 * value the ant read with a plain store, so updates that race are lost: the
 * paper's ACS-GPU-Alt (Sec. 3.1.2, the variant without atomic operations).
 * ACS_SEQUENTIAL: Alg. 1 read literally, step by step and within a step ant
 * by ant: ant a selects from the pheromone after the local updates of ants
 * 0..a-1 of the same step (in-step Gauss-Seidel).  Deterministic like
 * ACS_SYNC; dense memory only (ACS_E_UNSUPPORTED otherwise).  One block runs
 * it: ants whose current city no earlier ant of the step touches select in
 * parallel, so its speed depends on how often ants meet. */
enum acs_mode { ACS_SYNC = 0, ACS_ASYNC_ATOMIC = 1, ACS_ASYNC_RACY = 2, ACS_SEQUENTIAL = 3 };

typedef struct acs_params {
  uint32_t struct_size;  /* = sizeof(acs_params) */
  uint32_t m;            /* ants; 0 -> n */
  uint32_t cl;           /* candidate-list length; clamped to n-1; <= 64 */
  uint32_t memory;       /* enum acs_memory */
  uint32_t spm_s;        /* SPM trails per city (Sec. 3.2), >= 1 */
  uint32_t mode;         /* enum acs_mode */
  uint32_t local_update_period; /* k >= 1: the local update of Eq. 3 follows only
                                   the edges selected at steps k, 2k, ... (and
                                   the closing edge); Sec. 4, limiting the
                                   number of local pheromone updates */
  uint32_t instance;     /* fourth word of every random-number counter */
  double beta;           /* exponent of eta = 1/d in Eq. 1-2, >= 0 */
  double q0;             /* exploitation probability of Eq. 1, in [0, 1] */
  double phi;            /* local evaporation of Eq. 3, in (0, 1) */
  double rho;            /* global evaporation of Eq. 4, in (0, 1) */
  double tau0;           /* > 0: initial pheromone; <= 0: 1/(n * L_nn) */
  uint64_t seed;         /* key of the Philox4x32-10 draws */
  void *stream;          /* hipStream_t to run on; NULL: the library's own */
  void *workspace;       /* optional device buffer (e.g. a torch tensor) */
  size_t workspace_bytes;
  uint32_t lanes_per_ant; /* asynchronous dense kernels: lanes of a wavefront
                             that carry one ant, 64, 32 or 16 (at least cl);
                             0: 64 for one instance, chosen by timing for a
                             batch.  Never changes a decision, only how many
                             ants share a wavefront. */
  uint32_t update_path;  /* asynchronous modes, 64 lanes per ant: 1 the ant
                            wave issues its local updates itself; 2 (and 0,
                            the default) the ant waves hand them to one
                            updater wavefront per workgroup through LDS, so
                            an ant never waits for an atomic */
  uint32_t wait_limit;   /* polls after which a bounded device wait (grid
                            barrier, update ring) gives up; 0: the library's
                            own limits.  A wait that gives up makes the
                            iterate call return ACS_E_DEVICE (its results are
                            then not to be trusted); every kernel still runs
                            to its end.  Small values force that path, for
                            tests of the error handling. */
  uint32_t local_search; /* 1: after the construction every ant's tour is
                            improved by a first-improvement descent over
                            2-opt and Or-opt moves (segments of 1 to 3
                            cities) along the candidate lists, before the
                            iteration best and the global update (the local
                            search the paper's Sec. 5.1 proposes to study);
                            2: the same with 3-opt moves as well (the four
                            reconnections that replace three edges by three
                            new ones); dense memory, n <= 8192, one
                            instance.  0: none */
} acs_params;

typedef struct acs_stats {
  uint32_t struct_size;      /* = sizeof(acs_stats_t) */
  uint32_t iteration;        /* iterations completed */
  int64_t best_length;       /* best-so-far L_gb, -1 before the first */
  int64_t iter_best_length;  /* best of the last iteration */
  int32_t iter_best_ant;
  int32_t n, m, cl;
  int64_t nn_length;         /* L_nn of the nearest-neighbour tour from 0 */
  float tau0;
  float pad0;
  int64_t steps;             /* construction steps since create */
  int64_t greedy;            /* ... decided by the argmax of Eq. 1 */
  int64_t roulette;          /* ... decided by Eq. 2 */
  int64_t fallback;          /* ... with an empty candidate set */
  int64_t spm_hits;          /* SPM updates that found the trail */
  int64_t spm_misses;        /* SPM updates that inserted it */
  int64_t fallback_unvisited;/* sum over fallback steps of the unvisited
                                cities the greedy scan had to consider */
  int64_t cas_retries;       /* local-update compare-and-swaps that found
                                the entry changed and were repeated */
  double construct_ms;       /* device time of the construction kernel
                                launches of the last acs_iterate call: HIP
                                events recorded right around each one, so
                                the small bound and copy kernels beside it
                                are not counted (iterate_ms has them) */
  int32_t construct_launches;/* construction launches of that call */
  int32_t pad1;
  double iterate_ms;         /* device time of the whole last acs_iterate */
  int64_t ls_moves;          /* local-search moves applied since create */
} acs_stats_t;

/* Fills *p with the defaults: m = n, cl = 32, dense, s = 8, sync,
 * beta = 2, q0 = 0.9, phi = rho = 0.1, tau0 = 1/(n L_nn), seed 0. */
int acs_default_params(acs_params *p);

/* Device bytes the library needs for an instance of n cities with these
 * parameters; a workspace of at least this size makes acs_create allocate
 * nothing on the device. */
int acs_workspace_bytes(int32_t n, const acs_params *p, size_t *out);

/* Builds the instance on the device: exact integer EUC_2D costs (the
 * d_ij of Sec. 3), the cl nearest neighbours of each city sorted by
 * (d, index) (the candidate set of Sec. 3), eta^beta, the nearest-neighbour
 * tour from city 0 and tau0, and the initial pheromone (dense: tau0
 * everywhere; SPM: empty records).  Dense memory with n - 1 > cl + 128 also
 * gets the 128 cities after each city's candidates, which let the greedy
 * fallback of Alg. 2 stop early when that is exact.
 * coords_xy: n (x, y) pairs of finite doubles, copied.  n >= 3.
 * Errors: ACS_E_INVALID (bad n, coordinates or parameters), ACS_E_NOMEM,
 * ACS_E_DEVICE, ACS_E_UNSUPPORTED (cl > 64, n > 65535, distances > 65535,
 * or m beyond what one synchronous launch can hold). */
int acs_create(const double *coords_xy, int32_t n, const acs_params *p,
               struct acs_t **out);

/* Runs k >= 0 iterations of Alg. 1 on the handle's stream and returns once
 * they have finished.  The iteration counter persists across calls, so
 * acs_iterate(h, 2) equals acs_iterate(h, 1) twice.  ACS_E_DEVICE if a
 * kernel failed or a bounded device wait gave up during the call. */
int acs_iterate(struct acs_t *h, int32_t k);

/* Best-so-far tour (n cities, starting at its ant's start city) and its
 * length.  Before the first iteration: ACS_E_STATE. */
int acs_best_tour(struct acs_t *h, int32_t *tour_out, int64_t *len_out);

/* Logical pheromone tau(i, j) as the ants read it, row-major n x n floats
 * (count must be >= n*n).  Dense handles only (SPM: ACS_E_UNSUPPORTED). */
int acs_pheromone_snapshot(struct acs_t *h, float *out, size_t count);

/* SPM records of Alg. 3: nodes[n*s] (-1 = empty slot), vals[n*s],
 * tail[n] (index of the most recently added slot).  SPM handles only. */
int acs_spm_snapshot(struct acs_t *h, int32_t *nodes, float *vals,
                     int32_t *tail);

/* Tours (m x n) and lengths (m) of the last iteration. */
int acs_tours(struct acs_t *h, int32_t *out, size_t count);
int acs_lengths(struct acs_t *h, int64_t *out, size_t count);

/* Candidate lists (n x cl, the nearest neighbours of Sec. 3) as built. */
int acs_candidates(struct acs_t *h, int32_t *out, size_t count);

int acs_stats(struct acs_t *h, acs_stats_t *out);

/* Releases every resource of the handle; NULL is a no-op. */
void acs_destroy(struct acs_t *h);

/* For callers that cannot allocate device memory (work recorded for a HIP
 * graph, tight serving loops, harnesses that forbid allocation): the same
 * result as acs_create, acs_iterate(iterations) and acs_best_tour on a
 * handle, with the device workspace in one static array of the library
 * (ACS_STATIC_WORKSPACE_BYTES per GPU, held from the library's first use on
 * that GPU until the process ends) instead of an allocation.  The call
 * creates no stream, event or device buffer: it runs on params.stream (NULL:
 * the null stream) and returns when the best tour is copied out.
 * coords_xy: n (x, y) pairs as for acs_create; iterations >= 1;
 * tour_out: n ints, len_out: one int64, both caller-owned host memory.
 * params.workspace must be NULL.  Every call on one GPU uses that GPU's one
 * array and leaves its last contents there; calls within the process are
 * serialised by a lock (calls that overlapped on one GPU would race).
 * Errors: as acs_create and acs_iterate; ACS_E_BUFSIZE when the instance
 * needs more device memory than the array holds (acs_workspace_bytes tells
 * the need: about n^2 * 14 bytes for dense memory with m = n, plus another
 * 4 n^2 in ACS_SYNC). */
#define ACS_STATIC_WORKSPACE_BYTES (128u << 20)
int acs_solve_static(const double *coords_xy, int32_t n, const acs_params *p,
                     int32_t iterations, int32_t *tour_out, int64_t *len_out);

/* Message of the last failing call on this thread ("" if none). */
const char *acs_last_error(void);

/* ------------------------------------------------------------------------
 * Batches: many independent instances solved together, each by its own
 * colony (the independent-colony setting the paper names as future work,
 * Sec. 5), one launch per iteration over every ant of every instance.
 * The iteration (construction, iteration best, global update of Alg. 1)
 * is captured once as a HIP graph and replayed.  Batches run in the
 * asynchronous atomic mode on the dense memory (other combinations:
 * ACS_E_UNSUPPORTED).  Instance i uses the random-number counter word
 * params->instance + i and otherwise the same parameters, so it reproduces
 * a single-instance handle created with that instance value.
 * ------------------------------------------------------------------------ */
typedef struct acs_batch_t acs_batch_t;

/* Device bytes for a batch of `count` instances of sizes n[0..count). */
int acs_batch_workspace_bytes(const int32_t *n, int32_t count, const acs_params *p,
                              size_t *out);

/* coords[i]: n[i] (x, y) pairs of instance i, copied.  params as for
 * acs_create (mode ACS_ASYNC_ATOMIC or ACS_ASYNC_RACY, memory ACS_DENSE); a given
 * workspace must hold acs_batch_workspace_bytes. */
int acs_batch_create(const double *const *coords, const int32_t *n, int32_t count,
                     const acs_params *p, acs_batch_t **out);

/* k iterations of every instance; returns once they have finished
 * (ACS_E_DEVICE if a bounded device wait gave up in any instance).  The
 * first iterations also choose the launch shape: one untimed iteration,
 * then one timed iteration with each candidate, later iterations with the
 * fastest.  The candidates are 64 lanes per ant with the ant issuing its
 * local updates, 64 lanes with an updater wave per block, and 32 and 16
 * lanes per ant where every candidate list fits; lanes_per_ant and
 * update_path, when set, restrict them.  Tuning iterations are ordinary
 * iterations (the shape never changes a decision). */
int acs_batch_iterate(acs_batch_t *b, int32_t k);

/* Launch-shape tuning: the index of the chosen candidate (-1 while still
 * tuning), the number of candidates, and per candidate its lanes per ant,
 * whether an updater wave applies the local updates (1) or the ant itself
 * (0), and the device time of its timed iteration in ms (-1 if not yet
 * timed).  The arrays hold `cap` entries; at most 4 are written. */
int acs_batch_tuning(acs_batch_t *b, int32_t *chosen, int32_t *count, int32_t *lanes,
                     int32_t *updater, double *ms, int32_t cap);

/* Multi-colony use of a batch (the model of Sec. 2: several colonies on one
 * instance with a periodic exchange of the best solution found so far along
 * a communication topology).  The batch's instances must be copies of one
 * instance (equal n; ACS_E_INVALID otherwise), each colony drawing its own
 * random numbers (params.instance + i).  From this call on, after every
 * `period`-th iteration (period >= 1; 0 turns the exchange off) colony c
 * takes the best-so-far tour and length of its source when that is strictly
 * shorter than its own; the next global update (Eq. 4) deposits on it.
 * topology 0: the source is the colony with the shortest best-so-far tour
 * (lowest index among equals); topology 1: colony c - 1 (a ring). */
int acs_batch_set_exchange(acs_batch_t *b, int32_t topology, int32_t period);

/* Number of instances, construction steps of one iteration (sum of
 * m_i (n_i - 1)), whether the iteration runs as a graph (1) or as direct
 * launches (0), and the device time of the last acs_batch_iterate. */
int acs_batch_info(acs_batch_t *b, int32_t *count, int64_t *steps_per_iteration,
                   int32_t *graph, double *last_iterate_ms);

/* Handle of instance i, for the read-back calls above (acs_best_tour,
 * acs_tours, acs_lengths, acs_pheromone_snapshot, acs_stats, ...).  It is
 * owned by the batch: do not destroy it or iterate it on its own. */
int acs_batch_instance(acs_batch_t *b, int32_t i, struct acs_t **out);

/* Best-so-far tour of instance i (as acs_best_tour). */
int acs_batch_best_tour(acs_batch_t *b, int32_t i, int32_t *tour_out, int64_t *len_out);

/* Releases the batch and every instance handle in it; NULL is a no-op. */
void acs_batch_destroy(acs_batch_t *b);

/* ------------------------------------------------------------------------
 * Learned edge prior (an addition to the paper's method).  A 4-64-64-1 MLP
 * (ReLU hidden layers, bf16 operands, fp32 accumulation on the matrix
 * cores) scores the edge from city i to its r-th nearest neighbour j
 * (r < 16) from the features (dx / s_i, dy / s_i, d_ij / s_i, r / 15),
 * s_i = d(i, 16th nearest neighbour).  max(sigmoid(z), 1e-6) then replaces
 * eta^beta of that candidate in Eq. 1 and Eq. 2 (Sec. 3); the fallback over
 * all unvisited cities keeps eta^beta.  Parameters are one device array of
 * ACS_PRIOR_PARAMS floats: W1[4][64] | b1[64] | W2[64][64] | b2[64] |
 * W3[64] | b3.  Functions taking `stream` run asynchronously on it (NULL:
 * the default stream); their pointer arguments are device pointers.
 * ------------------------------------------------------------------------ */
#define ACS_PRIOR_PARAMS 4545

/* Features of the 16 candidate edges of every city of h into X_dev
 * (n * 16 rows of 4 floats, row i * 16 + r).  Needs cl = 16. */
int acs_prior_features(struct acs_t *h, float *X_dev);

/* Logits of `rows` feature rows. */
int acs_prior_forward(const float *P_dev, const float *X_dev, int32_t rows, float *Z_dev,
                      void *stream);

/* Adds to G_dev the gradient of the mean binary cross-entropy (with logits)
 * of the rows against labels Y_dev in [0, 1], and the summed loss to
 * *loss_dev (both caller-initialised). */
int acs_prior_grad(const float *P_dev, const float *X_dev, const float *Y_dev, int32_t rows,
                   float *G_dev, float *loss_dev, void *stream);

/* One Adam step (Kingma and Ba, 2015; bias-corrected, `step` >= 1) on the
 * parameters; zeroes G_dev afterwards.  M_dev, V_dev: moment estimates. */
int acs_prior_adam(float *P_dev, float *G_dev, float *M_dev, float *V_dev, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *stream);

/* Scores of every candidate edge of h from the network, written in place
 * of eta^beta (needs cl = 16).  Later iterations of h use them. */
int acs_prior_apply(struct acs_t *h, const float *P_dev);

/* Replaces the candidate weights (eta^beta) of h by host scores[n * cl],
 * each a positive finite float. */
int acs_set_candidate_scores(struct acs_t *h, const float *scores);

/* The candidate weights h currently uses (eta^beta or scores), n * cl. */
int acs_candidate_weights(struct acs_t *h, float *out, size_t count);

#ifdef __cplusplus
}
#endif
#endif /* ACS_H */
