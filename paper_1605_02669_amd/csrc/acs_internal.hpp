// Internal interface between the C-ABI host code (acs_api.cpp) and the HIP
// kernels (acs_kernels.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct acs_params;

namespace acs {

// Record of candidate k of city i (the cl nearest neighbours of Sec. 3,
// sorted by (d, j)), one 16-byte load per lane:
//   x = neighbour j, y = d(i, j), z = bits of eta^beta(d),
//   w = bits of the pheromone tau(i, j) (the home of that directed entry).

// Device view of one colony.  Row-major matrices use the padded stride ldn.
struct Dev {
  int32_t n, m, cl, ldn;
  int32_t spm_s;
  const double *xy;        // n x 2
  const uint16_t *dist;    // dense: n x ldn exact integer distances; selective
                           //   memory: a chunk of rows while the handle is
                           //   built, NULL after (distances then come from xy)
  const uint4 *crec;       // n x cl candidate records (see above)
  const float *eta_tab;    // eta^beta indexed by distance (dmax + 1)
  float *tau;              // dense: n x ldn, home of non-candidate entries
  float *tau2;             // dense synchronous mode: the second buffer of tau
  const float *etad;       // dense: n x ldn, eta^beta(d(i, j))
  const int8_t *rpos;      // dense: n x cl, position of i in the candidate list
                           //   of its k-th candidate, -1 if i is not in it
  uint32_t *gvis;          // sequential mode: m x ceil(n / 32) visited bitmaps
  // dense memory, one colony with n - 1 > cl + kFpre: the greedy fallback's
  // prefix, the kFpre cities that follow the candidates in (d, j) order
  const uint4 *fpre;       //   n x kFpre / 2: lane l of row i holds the prefix
                           //   positions 2l and 2l + 1 as {j | d << 16, bits of
                           //   eta^beta(d)} twice
  const uint32_t *flim;    //   n: key d << 16 | j of the first city after them
  const float *femax;      //   n: largest eta^beta of the cities from flim on
  float *fbound;           //   n: per construction, fl(T * femax) with T above
                           //   every pheromone value those cities' entries of
                           //   row i hold during it
  float *ctau;             // dense: n x cl, the candidate entries' pheromone
                           //   while a construction with an updater wave runs
                           //   (their records then hold the values of the
                           //   iteration's start)
  // selective pheromone memory (Sec. 3.2): the record of city i is s pairs
  // {neighbour (-1 = empty slot), pheromone bits}; spm_tail[i] counts the
  // inserts (the most recently added slot is spm_tail[i] mod s)
  uint2 *spm;              // SPM: n x s
  const uint32_t *xnn;     // SPM: n x xl, the xl nearest cities by (d, j), as
                           //   keys d << 16 | j
  int32_t xl;              //   (xl = min(kXnn, n - 1))
  uint32_t *spm_tail;      // SPM: n
  // SPM: uniform grid of square cells over the cities for the fallback's
  // nearest-city search: cell (x, y) of side gh from (gx0, gy0), gnx x gny
  // cells, row-major; the cities of cell c are gcity[gstart[c] ..
  // gstart[c + 1]) with their coordinates in gxy (same order)
  const int32_t *gstart;   //   gnx * gny + 1
  const uint32_t *gcity;   //   n
  const double2 *gxy;      //   n
  int32_t gnx, gny;
  double gx0, gy0, gh, ginv;
  int32_t *upd_rec;        // SPM synchronous updates of one step: record
  int32_t *upd_nb;         //   ... and neighbour of update e = 2 * ant + w,
  int32_t *upd_next;       //   ... the next update of the same record (-1 end)
  int32_t *upd_head;       //   per record: first update of its list (-1 none)
  int32_t *tours;          // m x n
  int64_t *lens;           // m
  int32_t *best;           // n, best-so-far tour
  int64_t *gstate;         // [0] L_gb (-1 none), [1] L_ib, [2] ib ant
  unsigned long long *counters;  // greedy, roulette, fallback, hits, misses,
                                 // unvisited cities at fallback steps,
                                 // compare-and-swap retries, local-search moves
  uint32_t *sync;          // [0] unused, [1] error flag
  unsigned long long *bflags;  // synchronous mode: grid barrier flags, one per
                               //   block, 16 words (128 bytes) apart, from word 16
  int32_t nbflags;             //   words in bflags
  uint32_t wait_limit;         // polls before a bounded wait gives up (0: the
                               //   kernels' own limits)
};

// Per-iteration scalars.
struct Iter {
  uint32_t it, instance, key0, key1;
  uint32_t q0_24;
  float a_loc, b_loc, a_glob;
  float tau0;
  uint32_t lperiod;  // local update after every lperiod-th selected edge
  double rho;
};

// ---- instance preparation ----
// Distances of rows r0 .. r0 + rows - 1 (stored from the start of d.dist
// when `store`) and their largest value into *dmax.
hipError_t launch_dist(const Dev &d, uint32_t *dmax, int r0, int rows, bool store,
                       hipStream_t s);
// Candidate lists (and, with the selective memory, the extended neighbour
// lists) of cities r0 .. r0 + rows - 1 from the distance rows d.dist holds.
hipError_t launch_cand(const Dev &d, int32_t *cand_tmp, int r0, int rows, hipStream_t s);
hipError_t launch_nn_tour(const Dev &d, int64_t *lnn_out, hipStream_t s);
// Bounding box of the cities into box[0..3] = {xmin, ymin, xmax, ymax}.
hipError_t launch_grid_box(const Dev &d, double *box, hipStream_t s);
// The grid's cell lists (d.gnx, d.gny, d.gx0, d.gy0, d.ginv set): counts,
// starts, then the cities in cell order; cnt: gnx * gny ints of scratch.
hipError_t launch_grid(const Dev &d, int32_t *cnt, hipStream_t s);
hipError_t launch_crec(const Dev &d, const int32_t *cand_tmp, float tau0, hipStream_t s);
hipError_t launch_init_pheromone(const Dev &d, float tau0, hipStream_t s);

// ---- one iteration ----
// Construction of all m tours.  mode 0 = synchronous steps (cooperative
// persistent launch), 1 = asynchronous with atomic local updates, 2 =
// asynchronous with plain stores, 3 = sequential within each step (one
// block).  lanes: lanes per ant of the asynchronous
// dense kernels (64, 32 or 16; at least cl).  queued (asynchronous, 64
// lanes per ant): 0 the ant issues its own local updates; 1 it hands them to
// an updater wave per block.  ev0 / ev1, when not null, are recorded on s
// right before and after the construction kernel (not around the bound,
// buffer and live-pheromone copy kernels launched beside it).
hipError_t launch_construct(const Dev &d, const Iter &it, int mode, int memory, int lanes,
                            int queued, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
// Largest m a synchronous launch can keep resident for this instance.
int max_sync_ants(const Dev &d, int memory);
hipError_t launch_best_global(const Dev &d, const Iter &it, int memory,
                              hipStream_t s);
// Local search (2-opt and Or-opt descent; kind 2 adds 3-opt moves) on every
// ant's tour, dense memory, n <= kLsMaxN; rewrites tours and lengths.
constexpr int kLsMaxN = 8192;
hipError_t launch_local_search(const Dev &d, int kind, hipStream_t s);
// One iteration of many dense instances (asynchronous mode): construction of
// every (instance, ant) work item, then per-instance best and global update.
// Descriptors, iteration state and the work list are device arrays, so the
// three launches can be captured once in a graph and replayed.  mode 1:
// updates by compare-and-swap; mode 2: plain stores (lost updates).  lanes =
// 64: items are (instance, ant), one per wave; lanes = 32 or 16: items are
// (instance, first ant) of the 64 / lanes ants of one wave; lanes = 64 with
// `queued`: items are (instance, first ant) of the kBatchQAntsPerBlock ants
// of one block, whose updates an updater wave applies.
constexpr int kBatchQAntsPerBlock = 4;
// `flag` (device word): k_best_batch ORs every instance's error flag into it
// and clears the instance's flag, so one read after the iteration reports an
// exhausted bounded wait in any instance.
hipError_t launch_batch_iteration(const Dev *devs, Iter *iters, const int2 *items, int nitems,
                                  int count, int nmax, int clmax, int mode, int lanes, int queued,
                                  uint32_t *flag, hipStream_t s);
// Best-so-far exchange between `count` colonies of one instance (n cities)
// held by a batch: topology 0 from the colony with the shortest best-so-far
// tour, 1 from colony c - 1; offer (count x n) and olen (count) are device
// scratch.
hipError_t launch_exchange_batch(const Dev *devs, int count, int n, int topology,
                                 int32_t *offer, int64_t *olen, hipStream_t s);
// Learned edge prior (acs_prior.hip): parameter count and kernels.
constexpr int kPriorParams = 4545;
hipError_t launch_prior_forward(const float *P, const float *X, int rows, float *Z,
                                hipStream_t s);
hipError_t launch_prior_grad(const float *P, const float *X, const float *Y, int rows, float *G,
                             float *L, hipStream_t s);
hipError_t launch_prior_adam(float *P, float *G, float *M, float *V, int t, float lr, float b1,
                             float b2, float eps, hipStream_t s);
hipError_t launch_prior_features(const Dev &d, float *X, hipStream_t s);
hipError_t launch_prior_apply(const Dev &d, const float *P, hipStream_t s);
// Largest spm_s the GPU kernels support.
constexpr int kMaxSpmS = 16;
constexpr int kXnn = 128;  // extended neighbour list of the selective memory's fallback
constexpr int kFpre = 128;  // dense fallback prefix (two cities per lane)

// ---- host side (acs_api.cpp) ----
// Host scratch the eta^beta table takes (floats).
constexpr int kEtaHostEntries = 65536;
// Builds the instance in the device memory `ws` (ws_bytes, kept by the
// caller), runs `iterations` iterations of Alg. 1 on params->stream (NULL:
// the null stream) and copies the best-so-far tour and length out.  Creates
// no stream, event or device allocation.  eta_host: kEtaHostEntries floats of
// host scratch for the eta^beta table.  Returns an ACS_E_* code.
int solve_in(const double *coords_xy, int32_t n, const acs_params *p, int32_t iterations,
             char *ws, size_t ws_bytes, float *eta_host, int32_t *tour_out, int64_t *len_out);
// Sets the calling thread's error message; returns code.
int set_error(int code, const char *msg);

}  // namespace acs
