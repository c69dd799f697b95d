// HIP kernels for the Ant Colony System hot path on gfx950 (MI355X).
//
// Method: Skinderowicz, "The GPU-based Parallel Ant Colony System" (JPDC
// 2016), Sec. 3.  The paper maps one ant to one 32-thread block and its 32
// candidates to the threads; here one ant owns one 64-wide wavefront, the
// candidates sit one per lane, and every decision of the ant (which branch of
// Eq. 1, which candidate, the fallback) is wave-uniform, so it runs on the
// scalar unit: reductions use DPP and permlane swaps (no LDS round trips),
// the winning lane's values are read with readlane, the Philox draws are
// scalar.  The visited set is a bitmap in LDS.
//
// Data layout (dense memory).  The static record of candidate k of city i
// and the pheromone of that directed entry share one 16-byte slot,
//   crec[i][k] = {j, d(i, j), eta^beta(d) bits, tau(i, j) bits},
// so one step reads one coalesced 16-byte load per lane.  The pheromone of a
// non-candidate entry (i, j) lives in tau[i][j] (n x ldn).  Every directed
// entry therefore has exactly one home; the fallback scan only reads
// non-candidate entries, because it runs only when every candidate is
// visited.
//
// Compiled with -ffp-contract=off: every float expression is the written
// sequence of IEEE operations; fmaf is used only for the pheromone maps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "acs_internal.hpp"

namespace acs {
namespace {

constexpr uint32_t kNone = 0xffffffffu;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of the 4x32 S-box with
// multipliers 0xD2511F53 / 0xCD9E8D57, the key bumped by the Weyl constants
// 0x9E3779B9 / 0xBB67AE85 between rounds.  Counter = (step, ant, iteration,
// instance), key = the 64-bit seed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Cost d_ij (Sec. 3) as TSPLIB EUC_2D made exact: s = dx*dx + dy*dy in
// double, d = the integer with (d - 1/2)^2 <= s < (d + 1/2)^2 (0 if s < 1/4).
// The square root only seeds the search; the result is set by exact compares.
__device__ __forceinline__ uint32_t exact_dist(double xi, double yi, double xj,
                                               double yj) {
  const double dx = xi - xj, dy = yi - yj;
  const double s = dx * dx + dy * dy;
  if (s < 0.25) return 0;
  uint32_t d = (uint32_t)sqrt(s);
  while ((d + 0.5) * (d + 0.5) <= s) ++d;
  while (d > 0 && (d - 0.5) * (d - 0.5) > s) --d;
  return d;
}

// d(i, j) from the coordinates (the selective memory keeps no n x n matrix).
__device__ __forceinline__ uint32_t dist_xy(const Dev &D, int i, int j) {
  return exact_dist(D.xy[2 * i], D.xy[2 * i + 1], D.xy[2 * j], D.xy[2 * j + 1]);
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off; off >>= 1) {
    const T o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off; off >>= 1) {
    const T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Wave-wide unsigned max / min, all lanes active: quad and row permutations
// by DPP, then the row-pair and half-wave swaps of gfx950.  Returns the
// result as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_umax_u(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = max(v, max((uint32_t)a[0], (uint32_t)a[1]));
  const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = max(v, max((uint32_t)b[0], (uint32_t)b[1]));
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Maximum over lanes 0..31 (lanes 32..63 hold no candidate when cl <= 32),
// as a wave-uniform value.
__device__ __forceinline__ uint32_t half_umax_u(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = max(v, max((uint32_t)a[0], (uint32_t)a[1]));
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Wave-wide sum, every lane active (rare paths only: LDS permutes).
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
  for (int off = 32; off; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_umin_u(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = min(v, min((uint32_t)a[0], (uint32_t)a[1]));
  const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = min(v, min((uint32_t)b[0], (uint32_t)b[1]));
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Marks city c visited in an LDS bitmap without waiting for the old word
// (LDS operations of a wave take effect in issue order, so the next read of
// the word sees the bit).
__device__ __forceinline__ void mark(uint32_t *vis, int c) {
  __hip_atomic_fetch_or(vis + (c >> 5), 1u << (c & 31), __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, k);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// v_writelane: lane k of the result is s (wave-uniform), the other lanes
// keep old.  The compiler exposes it only as the LLVM intrinsic.
extern "C" __device__ int acs_writelane_i32(int s, int k, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t wrlane(uint32_t s, int k, uint32_t old) {
  return (uint32_t)acs_writelane_i32((int)s, k, (int)old);
}

// Maximum over lanes 0..L-1 (L = 16, 32 or 64) as a scalar: the row
// maxima by DPP, then one read per row.  Fewer instructions than a
// full-wave finish when only the scalar is needed.
template <int L>
__device__ __forceinline__ uint32_t rows_umax_s(uint32_t v) {
  static_assert(L == 16 || L == 32 || L == 64, "16, 32 or 64 lanes");
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  if (L == 16) return rdlane(v, 0);
  const uint32_t m01 = max(rdlane(v, 0), rdlane(v, 16));
  if (L == 32) return m01;
  return max(m01, max(rdlane(v, 32), rdlane(v, 48)));
}

// Pheromone slot of candidate k in city u's record.
__device__ __forceinline__ float *cand_tau(const Dev &D, int u, int k) {
  return reinterpret_cast<float *>(const_cast<uint4 *>(D.crec) + (size_t)u * D.cl + k) + 3;
}

// Home of the directed entry (u, v): candidate slot k of u, or tau[u][v].
__device__ __forceinline__ float *home(const Dev &D, int u, int v, int k) {
  return k >= 0 ? cand_tau(D, u, k) : D.tau + (size_t)u * D.ldn + v;
}

// Home of the directed entry (u, v) while a construction with an updater
// wave runs: slot k of u's row of ctau, or tau[u][v].
__device__ __forceinline__ float *qhome(const Dev &D, int u, int v, int k) {
  return k >= 0 ? D.ctau + (size_t)u * D.cl + k : D.tau + (size_t)u * D.ldn + v;
}

// Agent-coherent read of one pheromone value (sees every CAS performed so
// far on the device, whichever XCD performed it).
__device__ __forceinline__ float tau_load(const float *p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<const unsigned int *>(p),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Local or global map x -> fma(a, x, b), applied atomically.  `seen` is the
// value the caller believes the entry holds; a failed compare-and-swap (the
// entry changed meanwhile) retries with the value it returned.  Returns the
// number of retries.
__device__ __forceinline__ uint32_t cas_apply(float *p, unsigned int seen, float a, float b) {
  unsigned int *q = reinterpret_cast<unsigned int *>(p);
  unsigned int old = seen;
  uint32_t retries = 0;
  while (true) {
    const unsigned int nw = __float_as_uint(fmaf(a, __uint_as_float(old), b));
    const unsigned int prev = atomicCAS(q, old, nw);
    if (prev == old) break;
    old = prev;
    ++retries;
  }
  return retries;
}

// Whether the local map leaves x unchanged (in fp32).  During a
// construction an entry only receives that map, so an entry read at such a
// value still holds it, and its update can be skipped without changing any
// result.
__device__ __forceinline__ bool map_fixed(float x, float a, float b) {
  return __float_as_uint(fmaf(a, x, b)) == __float_as_uint(x);
}

// Position of v in the candidate list of u (wave-uniform), or -1.
__device__ __forceinline__ int cand_pos(const Dev &D, int u, int v, int lane) {
  const int kl = lane < D.cl ? lane : D.cl - 1;
  const uint32_t j = D.crec[(size_t)u * D.cl + kl].x;
  const uint64_t b = __ballot(lane < D.cl && j == (uint32_t)v);
  return b ? (int)__ffsll((unsigned long long)b) - 1 : -1;
}

// Grid-wide barrier for a cooperative launch, by flags.  Every wave waits for
// its own memory operations first (the local updates are compare-and-swaps
// whose results have been consumed, so they are performed at the device's
// coherence point).  One thread per block then stores the barrier's epoch
// into the block's own flag (its own 128-byte line), and the first wave of
// every block waits until every flag has reached the epoch.  No two blocks
// write the same line, so arrival costs one store instead of a
// read-modify-write queued behind every other block's on one counter, and
// no block waits for a second hop through a release word.  Readers after
// the barrier use agent-coherent loads for everything the updates touch, so
// no cache write-back or invalidation is needed.
//
// Epochs are (iteration << 32 | barrier number) and grow monotonically.  A
// block can run at most one barrier ahead of the slowest (it cannot pass the
// next barrier before the slowest block arrives there), so a waiting block
// sees every flag at its epoch or the next: it waits for "at least", and
// flags left by an earlier construction are below every epoch of a later
// one.  The wait is bounded: on exhaustion an error flag is raised, later
// barriers no longer wait, and the kernel runs to its end.
__device__ __forceinline__ uint64_t barrier_epoch(const Iter &A, uint32_t bar) {
  return ((uint64_t)A.it << 32) | bar;
}

// once any block has given up, no later barrier waits either (looked at every
// 64th poll, so a poll costs the flag loads only)
__device__ __forceinline__ bool barrier_gave_up(const Dev &D, uint32_t spins) {
  return (spins & 63) == 63 &&
         __hip_atomic_load(D.sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void grid_barrier_f(const Dev &D, uint64_t epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(D.bflags + 16 * ((size_t)blockIdx.x + 1), (unsigned long long)epoch,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < 64) {
    uint32_t spins = 0;
    while (true) {
      bool all = true;
      for (uint32_t b = threadIdx.x; b < gridDim.x; b += 64)
        all &= __hip_atomic_load(D.bflags + 16 * ((size_t)b + 1), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      if (__ballot(!all) == 0) break;
      if (barrier_gave_up(D, spins)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (D.wait_limit ? D.wait_limit : (1u << 22))) {
        if (threadIdx.x == 0)
          __hip_atomic_store(D.sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ---------------------------------------------------------------------------
// Instance preparation kernels.
// ---------------------------------------------------------------------------
// Rows r0 .. r0 + rows - 1 of the distance matrix, stored (when `store`)
// from the start of D.dist, and the largest distance into *dmax.
__global__ __launch_bounds__(256) void k_dist(Dev D, uint32_t *dmax, int r0, int rows,
                                              int store) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int i = r0 + r;
  uint32_t d = 0;
  if (r < rows && i < D.n && j < D.n && i != j) d = dist_xy(D, i, j);
  const uint32_t wmax = wave_max(d);
  if ((threadIdx.x & 63) == 0 && wmax) atomicMax(dmax, wmax);
  if (store && r < rows && i < D.n && j < D.ldn)
    const_cast<uint16_t *>(D.dist)[(size_t)r * D.ldn + j] = (uint16_t)(d > 65535u ? 65535u : d);
}

// Candidate list of city i: its cl nearest neighbours by (d, j), one wave
// per city, extracted in increasing order of the key (d << 16 | j).
// Cities r0 .. r0 + rows - 1, whose distance rows D.dist holds from its start.
__global__ __launch_bounds__(256) void k_cand(Dev D, int32_t *cand, int r0, int rows) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int i = r0 + r;
  if (r >= rows || i >= D.n) return;
  const uint16_t *row = D.dist + (size_t)r * D.ldn;
  int64_t last = -1;
  for (int k = 0; k < D.cl; ++k) {
    int64_t best = INT64_MAX;
    for (int j = lane; j < D.n; j += 64) {
      if (j == i) continue;
      const int64_t key = ((int64_t)row[j] << 16) | j;
      if (key > last && key < best) best = key;
    }
    best = wave_min(best);
    if (lane == 0) cand[(size_t)i * D.cl + k] = (int32_t)(best & 0xffff);
    last = best;
  }
}

// The xl nearest cities of every city by (d, j) (selective memory only),
// each stored as its key d << 16 | j: the fallback's nearest unvisited city
// is usually among them.  Cities r0 .. r0 + rows - 1, as k_cand.
__global__ __launch_bounds__(256) void k_xnn(Dev D, int r0, int rows) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int i = r0 + r;
  if (r >= rows || i >= D.n) return;
  const uint16_t *row = D.dist + (size_t)r * D.ldn;
  int64_t last = -1;
  for (int k = 0; k < D.xl; ++k) {
    int64_t best = INT64_MAX;
    for (int j = lane; j < D.n; j += 64) {
      if (j == i) continue;
      const int64_t key = ((int64_t)row[j] << 16) | j;
      if (key > last && key < best) best = key;
    }
    best = wave_min(best);
    if (lane == 0) const_cast<uint32_t *>(D.xnn)[(size_t)i * D.xl + k] = (uint32_t)best;
    last = best;
  }
}

// The dense fallback's prefix of city i: positions cl .. cl + kFpre - 1 of
// its neighbours in (d, j) order (the candidates are positions 0 .. cl - 1),
// the key of position cl + kFpre, and the largest eta^beta of the cities
// from that position on (eta^beta need not be monotone in fp32).
__global__ __launch_bounds__(256) void k_fpre(Dev D) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= D.n) return;
  const uint16_t *row = D.dist + (size_t)i * D.ldn;
  uint32_t *out = reinterpret_cast<uint32_t *>(const_cast<uint4 *>(D.fpre)) +
                  (size_t)i * 2 * kFpre;
  const int P = D.cl + kFpre;
  int64_t last = -1;
  for (int k = 0; k <= P; ++k) {
    int64_t best = INT64_MAX;
    for (int j = lane; j < D.n; j += 64) {
      if (j == i) continue;
      const int64_t key = ((int64_t)row[j] << 16) | j;
      if (key > last && key < best) best = key;
    }
    best = wave_min(best);
    if (lane == 0 && k >= D.cl && k < P) {
      const uint32_t d = (uint32_t)(best >> 16), j = (uint32_t)(best & 0xffff);
      out[2 * (k - D.cl)] = j | d << 16;
      out[2 * (k - D.cl) + 1] = __float_as_uint(D.eta_tab[d]);
    }
    if (lane == 0 && k == P) const_cast<uint32_t *>(D.flim)[i] = (uint32_t)best;
    last = best;
  }
  uint32_t emax = 0;
  for (int j = lane; j < D.n; j += 64) {
    const uint32_t key = (uint32_t)row[j] << 16 | (uint32_t)j;
    if (j != i && (int64_t)key >= last) emax = max(emax, __float_as_uint(D.eta_tab[row[j]]));
  }
  emax = wave_umax_u(emax);
  if (lane == 0) const_cast<float *>(D.femax)[i] = __uint_as_float(emax);
}

// Uniform grid over the cities (selective memory): the fallback's search
// for the nearest unvisited city reads only the cells around the current
// city.  Cell of a coordinate, clamped to the grid.
__device__ __forceinline__ int grid_cx(const Dev &D, double x) {
  return min(max((int)((x - D.gx0) * D.ginv), 0), D.gnx - 1);
}
__device__ __forceinline__ int grid_cy(const Dev &D, double y) {
  return min(max((int)((y - D.gy0) * D.ginv), 0), D.gny - 1);
}

// Bounding box, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_grid_box(Dev D, double *box) {
  __shared__ double sm[4][16];
  double v[4] = {INFINITY, INFINITY, -INFINITY, -INFINITY};
  for (int j = threadIdx.x; j < D.n; j += 1024) {
    const double x = D.xy[2 * j], y = D.xy[2 * j + 1];
    v[0] = fmin(v[0], x);
    v[1] = fmin(v[1], y);
    v[2] = fmax(v[2], x);
    v[3] = fmax(v[3], y);
  }
#pragma unroll
  for (int off = 32; off; off >>= 1) {
    v[0] = fmin(v[0], __shfl_xor(v[0], off, 64));
    v[1] = fmin(v[1], __shfl_xor(v[1], off, 64));
    v[2] = fmax(v[2], __shfl_xor(v[2], off, 64));
    v[3] = fmax(v[3], __shfl_xor(v[3], off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; ++q) sm[q][w] = v[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double r = sm[threadIdx.x][0];
    for (int i = 1; i < 16; ++i)
      r = threadIdx.x < 2 ? fmin(r, sm[threadIdx.x][i]) : fmax(r, sm[threadIdx.x][i]);
    box[threadIdx.x] = r;
  }
}

__global__ __launch_bounds__(256) void k_grid_count(Dev D, int32_t *cnt) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= D.n) return;
  atomicAdd(&cnt[grid_cy(D, D.xy[2 * j + 1]) * D.gnx + grid_cx(D, D.xy[2 * j])], 1);
}

// Exclusive prefix sum of the counts into gstart (one block); cnt becomes
// the fill cursor (a copy of the starts).
__global__ __launch_bounds__(1024) void k_grid_scan(Dev D, int32_t *cnt) {
  __shared__ int32_t part[1024];
  const int cells = D.gnx * D.gny;
  const int per = (cells + 1023) / 1024;
  const int c0 = min(cells, (int)threadIdx.x * per), c1 = min(cells, c0 + per);
  int32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int32_t x = part[i];
      part[i] = run;
      run += x;
    }
  }
  __syncthreads();
  int32_t *gstart = const_cast<int32_t *>(D.gstart);
  int32_t run = part[threadIdx.x];
  for (int c = c0; c < c1; ++c) {
    const int32_t x = cnt[c];
    gstart[c] = run;
    cnt[c] = run;
    run += x;
  }
  if (threadIdx.x == 0) gstart[cells] = D.n;
}

// Cities into their cells (order inside a cell is immaterial: the search
// takes the least (d, j) over every city it reads).
__global__ __launch_bounds__(256) void k_grid_fill(Dev D, int32_t *cur) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= D.n) return;
  const double x = D.xy[2 * j], y = D.xy[2 * j + 1];
  const int p = atomicAdd(&cur[grid_cy(D, y) * D.gnx + grid_cx(D, x)], 1);
  const_cast<uint32_t *>(D.gcity)[p] = (uint32_t)j;
  const_cast<double2 *>(D.gxy)[p] = make_double2(x, y);
}

// Nearest-neighbour tour from city 0 (ties: lowest index), one block; its
// length L_nn defines tau0 = 1 / (n * L_nn).
__global__ __launch_bounds__(1024) void k_nn_tour(Dev D, int64_t *lnn) {
  __shared__ uint32_t vis[2048];
  __shared__ int64_t red[16];
  const int tid = threadIdx.x;
  const int W = (D.n + 31) >> 5;
  for (int w = tid; w < W; w += 1024) vis[w] = 0;
  __syncthreads();
  if (tid == 0) vis[0] = 1u;
  __shared__ int64_t listed;
  int cur = 0;
  int64_t L = 0;
  for (int step = 1; step < D.n; ++step) {
    __syncthreads();
    // without a distance matrix: the first unvisited city of cur's list of
    // nearest cities (sorted by (d, j)) is the answer when there is one
    if (!D.dist && tid < 64) {
      int64_t key = -1;
      const uint32_t *xr = D.xnn + (size_t)cur * D.xl;
      for (int b0 = 0; b0 < D.xl; b0 += 64) {
        const int idx = b0 + tid;
        const uint32_t e = idx < D.xl ? xr[idx] : 0u;
        const uint32_t j = e & 0xffffu;
        const uint64_t ok = __ballot(idx < D.xl && !((vis[j >> 5] >> (j & 31)) & 1u));
        if (ok) {
          key = (int64_t)rdlane(e, (int)__ffsll((unsigned long long)ok) - 1);
          break;
        }
      }
      if (tid == 0) listed = key;
    }
    __syncthreads();
    int64_t best = D.dist ? -1 : listed;
    if (best < 0) {
      best = INT64_MAX;
      for (int j = tid; j < D.n; j += 1024)
        if (!((vis[j >> 5] >> (j & 31)) & 1u)) {
          const uint32_t dj = D.dist ? D.dist[(size_t)cur * D.ldn + j] : dist_xy(D, cur, j);
          const int64_t key = ((int64_t)dj << 16) | j;
          best = key < best ? key : best;
        }
      best = wave_min(best);
      if ((tid & 63) == 0) red[tid >> 6] = best;
      __syncthreads();
      best = red[0];
      for (int w = 1; w < 16; ++w) best = red[w] < best ? red[w] : best;
    }
    const int nxt = (int)(best & 0xffff);
    L += best >> 16;
    if (tid == 0) vis[nxt >> 5] |= 1u << (nxt & 31);
    cur = nxt;
  }
  if (tid == 0) *lnn = L + (D.dist ? D.dist[(size_t)cur * D.ldn] : dist_xy(D, cur, 0));
}

// Candidate records with the initial pheromone tau0 in the last word.
__global__ __launch_bounds__(256) void k_crec(Dev D, const int32_t *cand, float tau0) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D.n * D.cl) return;
  const int i = e / D.cl;
  const uint32_t c = (uint32_t)cand[e];
  const uint32_t d = dist_xy(D, i, (int)c);
  const_cast<uint4 *>(D.crec)[e] =
      make_uint4(c, d, __float_as_uint(D.eta_tab[d]), __float_as_uint(tau0));
}

// eta^beta of every entry (dense memory): one load per city in the fallback
// scan instead of a distance load followed by a table lookup.
__global__ __launch_bounds__(256) void k_etad(Dev D) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)D.n * D.ldn) return;
  const_cast<float *>(D.etad)[e] = D.eta_tab[D.dist[e]];
}

// Reverse positions: for candidate k of city i (j = cand[i][k]), the position
// of i in j's candidate list, -1 if i is not a candidate of j.
__global__ __launch_bounds__(256) void k_rpos(Dev D) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D.n * D.cl) return;
  const int i = e / D.cl;
  const uint32_t j = D.crec[e].x;
  int r = -1;
  for (int k = 0; k < D.cl && r < 0; ++k)
    if (D.crec[(size_t)j * D.cl + k].x == (uint32_t)i) r = k;
  const_cast<int8_t *>(D.rpos)[e] = (int8_t)r;
}

// A construction with an updater wave keeps the candidate entries' live
// pheromone in ctau (a record's 32 values in one 128-byte line), so the
// records the ants load are not written while it runs.  Before it, ctau
// takes the records' values; after it, each record takes back the value of
// its edge's canonical home (itself, or the same edge's slot in the smaller
// city's record when each city lists the other; see apply_entries), and a
// candidate slot whose city is not listed back passes its value to the dense
// entry (v, u).  Compare-and-swap mode only; the unsynchronised mode has no
// canonical homes and copies each slot back as it is.
__device__ __forceinline__ void ctau_out_slot(const Dev &D, size_t e, bool canonical) {
  const int u = (int)(e / (size_t)D.cl);
  const int v = (int)D.crec[e].x, kr = (int)D.rpos[e];
  const float x = canonical && kr >= 0 && u > v ? D.ctau[(size_t)v * D.cl + kr] : D.ctau[e];
  const_cast<uint4 *>(D.crec)[e].w = __float_as_uint(x);
  if (canonical && kr < 0) D.tau[(size_t)v * D.ldn + u] = x;
}

__global__ __launch_bounds__(256) void k_ctau_in(Dev D) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (size_t)D.n * D.cl) D.ctau[e] = __uint_as_float(D.crec[e].w);
}

__global__ __launch_bounds__(256) void k_ctau_out(Dev D, int canonical) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (size_t)D.n * D.cl) ctau_out_slot(D, e, canonical != 0);
}

// Before a construction, the bound that lets the dense fallback stop at its
// prefix.  During a construction an entry only ever receives the local map
// f(x) = fmaf(a, x, b) of a value one of the edge's entries held (the two
// entries of an edge start equal in every mode whose updates copy between
// them), and f(x) <= x above the map's real fixed point b / (1 - a), f(x) <=
// that point rounded up below it.  So T = max(start values, the point with a
// margin) bounds every value an entry of row i beyond the prefix holds, and
// by monotone rounding fl(T * femax) bounds their weights tau * eta^beta.
__device__ __forceinline__ void far_bound_row(const Dev &D, const Iter &A, int i, int lane) {
  const int n = D.n;
  const uint32_t lim = D.flim[i];
  const float *trow = D.tau + (size_t)i * D.ldn;
  const uint16_t *drow = D.dist + (size_t)i * D.ldn;
  uint32_t mx = 0;
  for (int j0 = 8 * lane; j0 < n; j0 += 512) {
    const float4 a = *reinterpret_cast<const float4 *>(trow + j0);
    const float4 b = *reinterpret_cast<const float4 *>(trow + j0 + 4);
    const uint4 dd = *reinterpret_cast<const uint4 *>(drow + j0);
    const float t[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    const uint32_t dw[4] = {dd.x, dd.y, dd.z, dd.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = j0 + q;
      const uint32_t key = ((dw[q >> 1] >> (16 * (q & 1))) & 0xffffu) << 16 | (uint32_t)j;
      if (j < n && j != i && key >= lim) mx = max(mx, __float_as_uint(t[q]));
    }
  }
  mx = wave_umax_u(mx);
  if (lane == 0) {
    const double fix = (double)A.b_loc / (1.0 - (double)A.a_loc);
    const float hi = (float)(fix * (1.0 + 0x1p-20));
    D.fbound[i] = fmaxf(__uint_as_float(mx), hi) * D.femax[i];
  }
}

// ctau_rows: the wave of row i also copies that row's candidate pheromone
// into ctau (k_ctau_in's work, for a construction with an updater wave).
__global__ __launch_bounds__(256) void k_far_bound(Dev D, Iter A, int ctau_rows) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= D.n) return;
  if (ctau_rows && lane < D.cl)
    D.ctau[(size_t)i * D.cl + lane] = __uint_as_float(D.crec[(size_t)i * D.cl + lane].w);
  far_bound_row(D, A, i, lane);
}

// The same for every instance of a batch that has a prefix (blockIdx.y =
// instance).
__global__ __launch_bounds__(256) void k_far_bound_batch(const Dev *devs, const Iter *iters) {
  const Dev &D = devs[blockIdx.y];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (D.fpre && i < D.n) far_bound_row(D, iters[blockIdx.y], i, threadIdx.x & 63);
}

// The same for every instance of a batch (blockIdx.y = instance).
__global__ __launch_bounds__(256) void k_ctau_in_batch(const Dev *devs) {
  const Dev D = devs[blockIdx.y];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (size_t)D.n * D.cl) D.ctau[e] = __uint_as_float(D.crec[e].w);
}

__global__ __launch_bounds__(256) void k_ctau_out_batch(const Dev *devs, int canonical) {
  const Dev D = devs[blockIdx.y];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (size_t)D.n * D.cl) ctau_out_slot(D, e, canonical != 0);
}

__global__ __launch_bounds__(256) void k_init(Dev D, float tau0) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nd = (size_t)D.n * D.ldn;
  if (D.tau && e < nd) D.tau[e] = tau0;
  if (D.spm && e < (size_t)D.n * D.spm_s) D.spm[e] = make_uint2(kNone, __float_as_uint(tau0));
  if (D.spm_tail && e < (size_t)D.n) {
    D.spm_tail[e] = (uint32_t)(D.spm_s - 1);
    D.upd_head[e] = -1;
  }
  if (D.bflags && e < (size_t)D.nbflags) D.bflags[e] = 0ull;
  if (e == 0) {
    D.gstate[0] = -1;
    D.gstate[1] = -1;
    D.gstate[2] = -1;
    D.sync[0] = 0;
    D.sync[1] = 0;
  }
  if (e < 8) D.counters[e] = 0;
}

// ---------------------------------------------------------------------------
// One step of Alg. 2 for the ant of this wave (dense memory).  `rec` is lane
// k's record of the current city (lanes >= cl hold a copy of the last one).
// Wave-uniform result.
// ---------------------------------------------------------------------------
struct Pick {
  int next;    // chosen city
  int k;       // its candidate position, -1 for the fallback
  uint32_t d;  // d(cur, next)
  float tval;  // pheromone of the entry (cur, next) as read
  int kind;    // 0 greedy (Eq. 1), 1 roulette (Eq. 2), 2 fallback
};

// Candidate-set membership and weight of this lane's candidate.
struct Cand {
  bool unv;  // member of the candidate set (an unvisited neighbour)
  float w;   // tau * eta^beta, 0 for non-members
};

__device__ __forceinline__ Cand weigh(const Dev &D, const uint32_t *vis, int lane, uint4 rec) {
  // every lane holds a valid city (lanes >= cl repeat the last candidate), so
  // the bitmap read needs no branch
  const uint32_t word = vis[rec.x >> 5];
  Cand c;
  c.unv = (lane < D.cl) & !((word >> (rec.x & 31)) & 1u);
  // tau * eta^beta >= 0, so its bit pattern orders like the value
  c.w = c.unv ? __uint_as_float(rec.w) * __uint_as_float(rec.z) : 0.f;
  return c;
}

// Philox words of 64 consecutive steps, one step per lane: lane l holds the
// draw of step base + l.  Each step then reads its words with readlane.
__device__ __forceinline__ uint4 philox_batch(const Iter &A, int ant, int base, int lane) {
  return philox10(make_uint4((uint32_t)(base + lane), (uint32_t)ant, A.it, A.instance), A.key0,
                  A.key1);
}

// q24 and u24 of step t from the batch that holds it.
__device__ __forceinline__ uint2 draw_of(uint4 batch, int t) {
  return make_uint2(rdlane(batch.x, t & 63) >> 8, rdlane(batch.y, t & 63) >> 8);
}

// Eq. 1 over the candidate set: the wave-uniform candidate position chosen,
// or -1 when the candidate set is empty (Alg. 2 then falls back).
__device__ __forceinline__ int pick_candidate(const Iter &A, int lane, int cl, Cand c, uint2 q,
                                              int &kind) {
  const bool unv = c.unv;
  const float w = c.w;
  const uint64_t umask = __ballot(unv);
  if (!umask) return -1;
  int k;
  if (q.x < A.q0_24) {
    // exploitation: maximum of tau * eta^beta, lowest position
    const uint32_t mx = cl <= 32 ? half_umax_u(__float_as_uint(w)) : wave_umax_u(__float_as_uint(w));
    const uint64_t sel = __ballot(unv && __float_as_uint(w) == mx);
    k = (int)__ffsll((unsigned long long)sel) - 1;
    kind = 0;
  } else {
    // Eq. 2 by roulette: inclusive Hillis-Steele scan over the positions
    // (offsets 1, 2, 4, ... < cl), r = u * total, first member of the
    // candidate set whose prefix sum exceeds r
    float P = w;
    for (int off = 1; off < cl; off <<= 1) {
      const float o = __shfl_up(P, off, 64);
      if (lane >= off) P = P + o;
    }
    const float total = __uint_as_float(rdlane(__float_as_uint(P), cl - 1));
    const float r = ((float)q.y * 0x1p-24f) * total;
    const uint64_t sel = __ballot(unv && P > r);
    k = sel ? (int)__ffsll((unsigned long long)sel) - 1 : 63 - (int)__clzll((long long)umask);
    kind = 1;
  }
  return uni(k);
}

// Alg. 2, empty candidate set: greedy over every unvisited city, ties ->
// lowest index.  With a prefix (D.fpre), the kFpre cities after the
// candidates come first, two per lane; when the best unvisited one beats
// D.fbound[cur] strictly, no city beyond the prefix can reach or tie it (the
// candidates are all visited), so it is the answer of the whole scan.
// Otherwise each lane scans eight consecutive cities per round.  The loads
// of round r + 1 are issued before round r is examined (every round loads,
// at an address clamped into the padded row, so the number of loads in
// flight is fixed and the wait covers round r only).
template <bool COHERENT>
__device__ __forceinline__ Pick fallback_dense(const Dev &D, const uint32_t *vis, int cur,
                                               int lane, const float *tsrc = nullptr) {
  const int n = D.n;
  Pick p;
  const float *trow = (tsrc ? tsrc : D.tau) + (size_t)cur * D.ldn;
  if (D.fpre) {
    const uint4 pe = D.fpre[(size_t)cur * (kFpre / 2) + lane];
    const float fb = D.fbound[cur];
    const uint32_t j0 = pe.x & 0xffffu, j1 = pe.z & 0xffffu;
    const float t0 = COHERENT ? tau_load(trow + j0) : trow[j0];
    const float t1 = COHERENT ? tau_load(trow + j1) : trow[j1];
    const bool u0 = !((vis[j0 >> 5] >> (j0 & 31)) & 1u);
    const bool u1 = !((vis[j1 >> 5] >> (j1 & 31)) & 1u);
    const float v0 = t0 * __uint_as_float(pe.y), v1 = t1 * __uint_as_float(pe.w);
    // this lane's best (largest weight, then lowest index)
    const bool second = u1 && (!u0 || v1 > v0 || (v1 == v0 && j1 < j0));
    const bool any = u0 || u1;
    const float bv = second ? v1 : v0;
    const uint32_t bj = second ? j1 : j0;
    // weights are >= 0, so their bit patterns order like the values
    const uint32_t mx = wave_umax_u(any ? __float_as_uint(bv) : 0u);
    if (mx > __float_as_uint(fb)) {
      const uint32_t jn = wave_umin_u(any && __float_as_uint(bv) == mx ? bj : kNone);
      const uint64_t own = __ballot(any && bj == jn);
      const int owner = uni((int)__ffsll((unsigned long long)own) - 1);
      p.k = -1;
      p.next = (int)jn;
      p.d = rdlane(second ? pe.z >> 16 : pe.x >> 16, owner);
      p.tval = __uint_as_float(rdlane(__float_as_uint(second ? t1 : t0), owner));
      p.kind = 2;
      return p;
    }
  }
  const float *erow = D.etad + (size_t)cur * D.ldn;
  const uint16_t *drow = D.dist + (size_t)cur * D.ldn;
  const int rounds = (n + 511) >> 9;
  float bv = 0.f, bt = 0.f;
  uint32_t bj = kNone, bd = 0;
  struct Round {
    float t[8], e[8];
    uint4 d;
  };
  auto fetch = [&](int r, Round &x) {
    const int j = min(8 * lane + 512 * r, D.ldn - 8);
    if (COHERENT) {
#pragma unroll
      for (int q = 0; q < 8; ++q) x.t[q] = tau_load(trow + j + q);
    } else {
      const float4 a = *reinterpret_cast<const float4 *>(trow + j);
      const float4 b = *reinterpret_cast<const float4 *>(trow + j + 4);
      x.t[0] = a.x; x.t[1] = a.y; x.t[2] = a.z; x.t[3] = a.w;
      x.t[4] = b.x; x.t[5] = b.y; x.t[6] = b.z; x.t[7] = b.w;
    }
    const float4 a = *reinterpret_cast<const float4 *>(erow + j);
    const float4 b = *reinterpret_cast<const float4 *>(erow + j + 4);
    x.e[0] = a.x; x.e[1] = a.y; x.e[2] = a.z; x.e[3] = a.w;
    x.e[4] = b.x; x.e[5] = b.y; x.e[6] = b.z; x.e[7] = b.w;
    x.d = *reinterpret_cast<const uint4 *>(drow + j);
  };
  Round cr;
  fetch(0, cr);
  for (int r = 0; r < rounds; ++r) {
    Round nr;
    fetch(min(r + 1, rounds - 1), nr);
    const int j0 = 8 * lane + 512 * r;
    uint32_t bits = (vis[min(j0, n - 1) >> 5] >> (j0 & 31)) & 0xffu;
    if (j0 >= n) bits = 0xffu;
    else if (j0 + 8 > n) bits |= (0xffu << (n - j0)) & 0xffu;
    const uint32_t dw[4] = {cr.d.x, cr.d.y, cr.d.z, cr.d.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float v = cr.t[q] * cr.e[q];
      if (!((bits >> q) & 1u) && (bj == kNone || v > bv)) {
        bv = v; bj = (uint32_t)(j0 + q); bt = cr.t[q]; bd = (dw[q >> 1] >> (16 * (q & 1))) & 0xffffu;
      }
    }
    cr = nr;
  }
  const uint32_t mx = wave_umax_u(bj == kNone ? 0u : __float_as_uint(bv));
  const uint32_t jn = wave_umin_u((bj != kNone && __float_as_uint(bv) == mx) ? bj : kNone);
  const uint64_t own = __ballot(bj == jn);
  const int owner = uni((int)__ffsll((unsigned long long)own) - 1);
  p.k = -1;
  p.next = (int)jn;
  p.d = rdlane(bd, owner);
  p.tval = __uint_as_float(rdlane(__float_as_uint(bt), owner));
  p.kind = 2;
  return p;
}

// tsrc: the dense pheromone matrix to read (default D.tau)
template <bool COHERENT>
__device__ __forceinline__ Pick select_dense(const Dev &D, const Iter &A, const uint32_t *vis,
                                             int cur, int lane, uint4 rec, Cand c, uint2 q,
                                             const float *tsrc = nullptr) {
  Pick p;
  const int k = pick_candidate(A, lane, D.cl, c, q, p.kind);
  if (k < 0) return fallback_dense<COHERENT>(D, vis, cur, lane, tsrc);
  p.k = k;
  p.next = (int)rdlane(rec.x, k);
  p.d = rdlane(rec.y, k);
  p.tval = __uint_as_float(rdlane(rec.w, k));
  return p;
}

__device__ __forceinline__ void add_counters(const Dev &D, uint32_t greedy, uint32_t roul,
                                             uint32_t fb, uint64_t fbu, uint32_t retries) {
  atomicAdd(&D.counters[0], (unsigned long long)greedy);
  atomicAdd(&D.counters[1], (unsigned long long)roul);
  atomicAdd(&D.counters[2], (unsigned long long)fb);
  atomicAdd(&D.counters[5], (unsigned long long)fbu);
  atomicAdd(&D.counters[6], (unsigned long long)retries);
}

// Tour entries are collected 64 at a time in one register (lane t % 64 holds
// entry t) and written with one coalesced store per 64 steps.
__device__ __forceinline__ void tour_put(const Dev &D, int ant, int t, int lane, int city,
                                         int &buf) {
  buf = lane == (t & 63) ? city : buf;
  if ((t & 63) == 63 || t == D.n - 1) {
    const int base = t & ~63;
    if (lane <= (t & 63)) D.tours[(size_t)ant * D.n + base + lane] = buf;
  }
}

// ---------------------------------------------------------------------------
// Synchronous construction, dense memory: persistent cooperative kernel, one
// ant per wave.  Step t is
//   SELECT (reads only, from the pheromone at the start of the step)
//   | barrier | UPDATE (Eq. 3 on both entries of each crossing, by CAS)
//   | barrier.
// The map is the same for every crossing, so the order of the updates of one
// step does not change the result: an entry crossed k times gets f^k.
// With a local-update period above 1, a step without updates leaves the
// pheromone as it is, so it needs neither barrier; the closing edges wait for
// the last step's selections before they write.
//
// With a period of 1 the pheromone is double-buffered instead, which needs
// one barrier per step: buffer 0 is (candidate records' words, tau), buffer
// 1 is (ctau, tau2), and buffer 1 starts the construction as a copy of
// buffer 0 (k_sync_buf).  Step t selects from buffer t % 2, which holds every
// update of steps < t, and applies the crossings of steps t - 1 and t to
// buffer (t + 1) % 2, which then holds every update of steps < t + 1; nobody
// reads that buffer during step t, and the barrier at the end of the step
// separates its writes from step t + 1's reads and step t's reads from step
// t + 1's writes.  The closing edges go to buffer n % 2, the final one.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float *sync_home(const Dev &D, int buf, int u, int v, int k) {
  if (buf == 0) return home(D, u, v, k);
  return k >= 0 ? D.ctau + (size_t)u * D.cl + k : D.tau2 + (size_t)u * D.ldn + v;
}

__global__ __launch_bounds__(1024) void k_construct_sync_dense(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ant = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  const bool active = ant < D.m;
  const int n = D.n, cl = D.cl;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  uint32_t *vis = smem + wv * W;
  const bool dbuf = A.lperiod == 1;

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  int tb = start;

  int cur = start;
  int64_t len = 0;
  uint32_t c_greedy = 0, c_roul = 0, c_fb = 0, c_retry = 0;
  uint64_t c_fbu = 0;
  uint32_t bar = 0;
  // the previous step's crossing (double-buffered schedule)
  int pu = -1, pv = -1, pk = -1, pk2 = -1;
  float pval = 0.f;
  for (int t = 1; t < n; ++t) {
    Pick p{};
    const int rb = dbuf ? (t & 1) : 0;
    if ((t & 63) == 0) draws = philox_batch(A, ant, t, lane);
    if (active) {
      uint4 rec = D.crec[(size_t)cur * cl + kl];
      const float *ct = rb == 0 ? cand_tau(D, cur, kl) : D.ctau + (size_t)cur * cl + kl;
      rec.w = __float_as_uint(tau_load(ct));
      const Cand c = weigh(D, vis, lane, rec);
      p = select_dense<true>(D, A, vis, cur, lane, rec, c, draw_of(draws, t),
                             rb == 0 ? D.tau : D.tau2);
      c_greedy += p.kind == 0;
      c_roul += p.kind == 1;
      if (p.kind == 2) { ++c_fb; c_fbu += (uint64_t)(n - t); }
      if (lane == 0) mark(vis, p.next);
      tour_put(D, ant, t, lane, p.next, tb);
      len += p.d;
    }
    if (dbuf) {
      // crossings of steps t - 1 and t into buffer (t + 1) % 2: lanes 0 and
      // 1 the previous crossing's two entries, lanes 2 and 3 this one's
      if (active) {
        const int k2 = cand_pos(D, p.next, cur, lane);
        const int wb = rb ^ 1;
        float *h = nullptr;
        unsigned int seen = 0;
        if (lane < 2 && pu >= 0) {
          h = lane == 0 ? sync_home(D, wb, pu, pv, pk) : sync_home(D, wb, pv, pu, pk2);
          seen = __float_as_uint(pval);
        } else if (lane == 2 || lane == 3) {
          h = lane == 2 ? sync_home(D, wb, cur, p.next, p.k) : sync_home(D, wb, p.next, cur, k2);
          seen = __float_as_uint(p.tval);
        }
        // a value the map leaves unchanged stays so under the maps that reach
        // the entry in this step: the update changes nothing
        if (h && !map_fixed(__uint_as_float(seen), A.a_loc, A.b_loc))
          c_retry += cas_apply(h, seen, A.a_loc, A.b_loc);
        pu = cur;
        pv = p.next;
        pk = p.k;
        pk2 = k2;
        pval = p.tval;
      }
      grid_barrier_f(D, barrier_epoch(A, ++bar));
    } else if (t % A.lperiod == 0) {
      grid_barrier_f(D, barrier_epoch(A, ++bar));
      if (active) {
        const int k2 = cand_pos(D, p.next, cur, lane);
        float *h = lane == 0 ? home(D, cur, p.next, p.k) : home(D, p.next, cur, k2);
        if (lane < 2 && !map_fixed(p.tval, A.a_loc, A.b_loc))
          c_retry += cas_apply(h, __float_as_uint(p.tval), A.a_loc, A.b_loc);
      }
      if (t + 1 < n) grid_barrier_f(D, barrier_epoch(A, ++bar));
    }
    if (active) cur = p.next;
  }
  if (!dbuf && (n - 1) % A.lperiod != 0) grid_barrier_f(D, barrier_epoch(A, ++bar));
  if (active) {
    // closing edge: its length and, as the last step's crossings, its update
    len += D.dist[(size_t)cur * D.ldn + start];
    const int fb = dbuf ? (n & 1) : 0;
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    float *h = lane == 0 ? sync_home(D, fb, cur, start, k1) : sync_home(D, fb, start, cur, k2);
    if (lane < 2) {
      const float seen = tau_load(h);
      c_retry += cas_apply(h, __float_as_uint(seen), A.a_loc, A.b_loc);
    }
    c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1) + rdlane(c_retry, 2) +
                                  rdlane(c_retry, 3)));
    if (lane == 0) {
      D.lens[ant] = len;
      add_counters(D, c_greedy, c_roul, c_fb, c_fbu, c_retry);
    }
  }
}

// Buffer 1 of the double-buffered synchronous schedule from buffer 0 (dir 0),
// or buffer 0 from buffer 1 (dir 1) when the construction ended in buffer 1.
__global__ __launch_bounds__(256) void k_sync_buf(Dev D, int dir) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (size_t)D.n * D.cl) {
    if (dir == 0)
      D.ctau[e] = __uint_as_float(D.crec[e].w);
    else
      const_cast<uint4 *>(D.crec)[e].w = __float_as_uint(D.ctau[e]);
  }
  if (e < (size_t)D.n * D.ldn) {
    if (dir == 0)
      D.tau2[e] = D.tau[e];
    else
      D.tau[e] = D.tau2[e];
  }
}

// ---------------------------------------------------------------------------
// Sequential construction, dense memory (Alg. 1 read literally): step by
// step, and within a step ant by ant, each ant selecting from the pheromone
// after the local updates of the ants before it in the same step.  One block
// of kSeqWaves waves.  A round gives the next kSeqWaves unresolved ants of
// the step one wave each; they select in parallel from the current
// pheromone.  An ant's choice depends on the pheromone only through the row
// of its current city, and an ant's update writes rows cur and next, so the
// round's ants up to (not including) the first whose row an earlier ant of
// the round writes have made exactly the sequential choices.  They commit
// (visited bit, tour entry, length, local update; their updates touch
// disjoint entries); the rest select again in the next round.  Every round
// commits at least its first ant.  Visited bitmaps live in global memory,
// since an ant is served by different waves over the iteration.
// ---------------------------------------------------------------------------
constexpr int kSeqWaves = 16;
// visited bitmaps in LDS when all m of them fit in this many words
constexpr int kSeqLdsWords = 36 * 1024;

// VIS_LDS: the m visited bitmaps in LDS (dynamic, m * ceil(n/32) words), else
// in global memory.  In this schedule both entries of an edge always hold
// the same value (every map is applied to both), so a committing ant stores
// the map of the value it read to both without reading the second.
template <bool VIS_LDS>
__global__ __launch_bounds__(64 * kSeqWaves) void k_construct_seq_dense(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  __shared__ int s_rows[kSeqWaves][2];  // rows the round's ant w writes (-1: none)
  __shared__ int s_cur[kSeqWaves];      // current city of the round's ant w (-1: none)
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int n = D.n, m = D.m, cl = D.cl;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  uint32_t *const vbase = VIS_LDS ? smem : D.gvis;

  for (int a = wv; a < m; a += kSeqWaves) {
    uint32_t *vis = vbase + (size_t)a * W;
    for (int w = lane; w < W; w += 64) vis[w] = 0u;
    const uint4 draws = philox_batch(A, a, 0, lane);
    const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
    if (lane == 0) {
      vis[start >> 5] |= 1u << (start & 31);
      D.tours[(size_t)a * n] = start;
      D.lens[a] = 0;
    }
  }
  __syncthreads();
  uint32_t c_greedy = 0, c_roul = 0, c_fb = 0, c_retry = 0;
  uint64_t c_fbu = 0;
  for (int t = 1; t < n; ++t) {
    const bool upd = t % (int)A.lperiod == 0;
    for (int base = 0; base < m;) {
      const int a = base + wv;
      const bool act = a < m;
      Pick p{};
      int cur = -1, kr = -1;
      if (act) {
        uint32_t *vis = vbase + (size_t)a * W;
        cur = D.tours[(size_t)a * n + t - 1];
        const uint4 draws = philox_batch(A, a, t & ~63, lane);
        const uint4 rec = D.crec[(size_t)cur * cl + kl];
        const Cand c = weigh(D, vis, lane, rec);
        p = select_dense<false>(D, A, vis, cur, lane, rec, c, draw_of(draws, t));
        // position of cur in the chosen city's list, for the second entry
        if (upd) kr = p.k >= 0 ? (int)D.rpos[(size_t)cur * cl + p.k] : cand_pos(D, p.next, cur, lane);
      }
      if (lane == 0) {
        s_cur[wv] = cur;
        s_rows[wv][0] = act && upd ? cur : -1;
        s_rows[wv][1] = act && upd ? p.next : -1;
      }
      __syncthreads();
      // the round commits its ants before the first one whose row an earlier
      // ant of the round writes (every wave finds the same K): lane v holds
      // ant v's current city and the rows it writes
      const int vl = lane < kSeqWaves ? lane : kSeqWaves - 1;
      const int lc = s_cur[vl], lr0 = s_rows[vl][0], lr1 = s_rows[vl][1];
      bool bad = false;
#pragma unroll
      for (int u = 0; u + 1 < kSeqWaves; ++u) {
        const int r0 = (int)rdlane((uint32_t)lr0, u), r1 = (int)rdlane((uint32_t)lr1, u);
        bad |= lane > u && lane < kSeqWaves && lc >= 0 && (lc == r0 || lc == r1);
      }
      const uint64_t badm = __ballot(bad);
      const int K = badm ? (int)__ffsll((unsigned long long)badm) - 1 : kSeqWaves;
      if (act && wv < K) {
        c_greedy += p.kind == 0;
        c_roul += p.kind == 1;
        if (p.kind == 2) { ++c_fb; c_fbu += (uint64_t)(n - t); }
        if (lane == 0) {
          __hip_atomic_fetch_or(vbase + (size_t)a * W + (p.next >> 5), 1u << (p.next & 31),
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          D.tours[(size_t)a * n + t] = p.next;
          D.lens[a] += p.d;
        }
        if (upd && lane < 2) {
          float *h = lane == 0 ? home(D, cur, p.next, p.k) : home(D, p.next, cur, kr);
          *h = fmaf(A.a_loc, p.tval, A.b_loc);
        }
      }
      __syncthreads();
      base += K;
    }
  }
  // closing edges: lengths and updates (edges shared by several ants get the
  // map once per ant, in any order)
  for (int a = wv; a < m; a += kSeqWaves) {
    const int cur = D.tours[(size_t)a * n + n - 1], start = D.tours[(size_t)a * n];
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    float *h = lane == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (lane < 2) c_retry += cas_apply(h, __float_as_uint(tau_load(h)), A.a_loc, A.b_loc);
    if (lane == 0) D.lens[a] += D.dist[(size_t)cur * D.ldn + start];
  }
  c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1)));
  if (lane == 0) add_counters(D, c_greedy, c_roul, c_fb, c_fbu, c_retry);
}

// ---------------------------------------------------------------------------
// Asynchronous construction, dense memory: one launch per iteration, one ant
// per wave, no waiting for the other ants.  Each crossing gets the local
// update of Eq. 3 as a compare-and-swap of the exact map on both directed
// entries of the crossed edge.
//
// The steps of one ant form a dependent chain, so the latency of a step sets
// the iteration time, and the wave waits for its memory operations in issue
// order.  The step is therefore arranged so that nothing slow is issued
// right before the wait for the next record:
//   1. wait for the record of the current city cur (issued at the end of the
//      previous step); check the compare-and-swaps issued one step earlier
//      and repeat any that found the entry changed;
//   2. issue the two compare-and-swaps of the previous move (prev, cur): the
//      forward entry with the pheromone the selection read as its expected
//      value, the reverse entry with the value cur's record holds (or the
//      forward value when prev is not a candidate of cur);
//   3. select the next city (Alg. 2) while those are in flight;
//   4. issue the load of the next city's record.
// ATOMIC = false is the paper's unsynchronised variant (ACS-GPU-Alt,
// Sec. 3.1.2): each entry gets the map of the value the ant read, by a plain
// (not read-modify-write) store, and updates that race with it are lost.
// ---------------------------------------------------------------------------
template <bool ATOMIC>
__device__ __forceinline__ void ant_async_dense(const Dev &D, const Iter &A, int ant,
                                                uint32_t *vis, int lane) {
  uint32_t uleft = A.lperiod;  // steps until the next local update
  const int n = D.n, cl = D.cl, ldn = D.ldn;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  const float al = A.a_loc, bl = A.b_loc;

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  int tb = start;
  uint4 rec = D.crec[(size_t)start * cl + kl];

  int cur = start, prev = -1;
  float *fwd = nullptr;  // home of the forward entry of the previous move
  float fval = 0.f;      // its value as read by the selection
  int64_t len = 0;
  // decisions by kind, 21 bits each: greedy | roulette << 21 | fallback << 42
  uint64_t c_kind = 0;
  uint32_t c_retry = 0;
  uint64_t c_fbu = 0;
  // compare-and-swap in flight on lanes 0 (forward) and 1 (reverse)
  float *pptr = nullptr;
  unsigned int pexp = 0, pret = 0;
  bool pend = false;

  // steps in chunks of 64: a chunk's draws come from one Philox batch and
  // its tour entries leave in one store, so no step tests for either
  for (int t0 = 0; t0 <= n; t0 += 64) {
  if (t0 > 0) draws = philox_batch(A, ant, t0, lane);
  uint32_t clen = 0;  // at most 64 distances below 2^16 each
  const int tend = min(t0 + 64, n + 1);
  for (int t = t0 > 0 ? t0 : 1; t < tend; ++t) {
    // 1. the record of cur is needed now; so are last step's CAS results
    if (pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
    pend = false;
    const Cand c = weigh(D, vis, lane, rec);
    // the weights are complete here, before the updates below are issued, so
    // no later wait for this record also waits for those updates
    __asm__ volatile("" ::"v"(c.w), "v"((int)c.unv));
    // 2. updates of the previous move (prev, cur), selected at step t - 1
    if (t > 1 && --uleft == 0) {
      uleft = A.lperiod;
      const uint64_t b = __ballot(lane < cl && rec.x == (uint32_t)prev);
      const int kr = b ? uni((int)__ffsll((unsigned long long)b) - 1) : -1;
      const float rval = kr >= 0 ? __uint_as_float(rdlane(rec.w, kr)) : fval;
      if (ATOMIC) {
        if (lane == 0) {
          pptr = fwd;
          pexp = __float_as_uint(fval);
          pend = true;
        } else if (lane == 1) {
          pptr = home(D, cur, prev, kr);
          pexp = __float_as_uint(rval);
          pend = true;
        }
        if (pend && map_fixed(__uint_as_float(pexp), al, bl)) pend = false;
        if (pend)
          pret = atomicCAS(reinterpret_cast<unsigned int *>(pptr), pexp,
                           __float_as_uint(fmaf(al, __uint_as_float(pexp), bl)));
      } else if (lane < 2 && !map_fixed(lane == 0 ? fval : rval, al, bl)) {
        float *h = lane == 0 ? fwd : home(D, cur, prev, kr);
        __hip_atomic_store(h, fmaf(al, lane == 0 ? fval : rval, bl), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (t == n) break;
    // 3. selection
    const Pick p = select_dense<false>(D, A, vis, cur, lane, rec, c, draw_of(draws, t));
    c_kind += 1ull << (21 * p.kind);
    if (p.kind == 2) c_fbu += (uint64_t)(n - t);
    if (lane == 0) mark(vis, p.next);
    tb = lane == t - t0 ? p.next : tb;
    clen += p.d;
    // 4. record of the next city
    rec = D.crec[(size_t)p.next * cl + kl];
    fwd = home(D, cur, p.next, p.k);
    fval = p.tval;
    prev = cur;
    cur = p.next;
  }
  len += clen;
  // tour entries t0 .. min(t0 + 63, n - 1) of this chunk
  if (t0 < n && lane <= min(63, n - 1 - t0)) D.tours[(size_t)ant * n + t0 + lane] = tb;
  }
  if (pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
  // closing edge: both entries, read fresh (once per ant)
  {
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    float *h = lane == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (lane < 2) {
      if (ATOMIC)
        c_retry += cas_apply(h, __float_as_uint(tau_load(h)), al, bl);
      else
        __hip_atomic_store(h, fmaf(al, tau_load(h), bl), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  len += D.dist[(size_t)cur * ldn + start];
  c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1)));
  if (lane == 0) {
    D.lens[ant] = len;
    const uint32_t m21 = (1u << 21) - 1;
    add_counters(D, (uint32_t)c_kind & m21, (uint32_t)(c_kind >> 21) & m21,
                 (uint32_t)(c_kind >> 42) & m21, c_fbu, c_retry);
  }
}

template <bool ATOMIC>
__global__ __launch_bounds__(256) void k_construct_async_dense(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ant = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  if (ant >= D.m) return;  // the whole wave leaves; no block-level sync below
  ant_async_dense<ATOMIC>(D, A, ant, smem + wv * ((D.n + 31) >> 5), lane);
}

// ---------------------------------------------------------------------------
// Local updates handed to an updater wave.  gfx950 counts loads, stores and
// atomics of a wave in one in-order counter, so a wave that waits for its
// next record also waits for every update it issued before that load.  The
// ant wave therefore issues no update: the crossing selected at step t goes
// into lane t % 64 of an entry held in registers, and every kQGroup steps one
// LDS store of those lanes hands the group to the block's updater wave,
// which applies Eq. 3 to both directed entries of each crossed edge.  An
// update thus lands a few steps after its crossing (at most a group plus
// the updater's sleep), where an ant that applied it itself would have
// waited for it.
// Each ant wave owns a ring of kQRing entries indexed by step (single
// producer, single consumer): the entry of step t sits at t % kQRing; the
// ant publishes head = the first step not yet written, the updater tail =
// the first step not yet read.  LDS instructions of one wave take effect in
// issue order, so a published head covers entries already written, and a
// published tail frees entries already read.  Every wait is bounded: on
// exhaustion the error flag (2) is raised and the ant applies its entries
// itself, so every wave still reaches its end.
//
// Entry of the crossing u -> v: {u | v << 16, k, x, kr}: k the position of v
// in u's candidate list (-1 if none), x the pheromone of (u, v) as the ant
// read it, kr the position of u in v's list: -2 = look it up in the reverse
// table (v is the k-th candidate of u), -3 = search v's list (v is not a
// candidate of u), else kr itself (-1: u is not a candidate of v).  Steps
// without an update hold x = kNoEntry in the first word.
// ---------------------------------------------------------------------------
constexpr int kQAnts = 8;     // at most this many ant waves per block
constexpr int kQGroup = 16;   // steps per hand-over (divides 64)
constexpr int kQRing = 256;   // ring entries per ant wave (power of 2, >= 64 + kQGroup)
constexpr uint32_t kQSpin = 1u << 22;
constexpr uint32_t kQIdle = 1u << 20;
constexpr uint32_t kNoEntry = 0xffffffffu;
// fourth word of a buffer resource for untyped dword loads (gfx9 family)
constexpr int kBufWord3 = 0x00020000;
// cache policy of a buffer load that reads what the device's coherence point
// holds (sc1), for values other waves update during the launch
constexpr int kCoherent = 16;

struct QRing {
  uint4 *ent;      // [ant wave][kQRing]
  uint32_t *head;  // per ant wave: first step not yet written
  uint32_t *tail;  // per ant wave: first step not yet read by the updater
  uint32_t *done;  // ant waves that have written their last entry
};

__device__ __forceinline__ uint32_t lds_ld(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Eq. 3 on both directed entries of the crossings held by the lanes of the
// wave (one entry per lane, all lanes active).
// Compare-and-swap mode: one entry of the edge is its canonical home and
// receives the exact map by compare-and-swap (x, the value the ant read, as
// the first expected value; a compare-and-swap that finds another value
// retries with it); the other entry gets the value just written by a
// device-coherent store, for readers at the other endpoint.  The canonical home is a
// candidate slot: the one in the record of the smaller city when each city
// lists the other, else the only one; k_ctau_out copies every canonical
// value to its other entry when the construction ends, so both entries
// then hold exactly the result of all the maps.  An edge with both entries
// in the dense matrix (a fallback move between cities that do not list each
// other) gets both compare-and-swaps.  Candidate entries live in ctau
// meanwhile (see k_ctau_in).
// Unsynchronised mode (ACS-GPU-Alt, Sec. 3.1.2): each entry is read and its
// map stored back, both device-coherent but not as one atomic operation;
// updates landing in between are lost.  (The value the ant read is several
// steps old by now: storing its map would undo the updates made since.)
// Returns this lane's retries.
template <bool ATOMIC>
__device__ __forceinline__ uint32_t apply_entries(const Dev &D, const Iter &A, uint4 e,
                                                  int lane) {
  const bool valid = e.x != kNoEntry;
  const int u = (int)(e.x & 0xffffu), v = (int)(e.x >> 16), k = (int)e.y;
  int kr = (int)e.w;
  const float al = A.a_loc, bl = A.b_loc;
  // compare-and-swap mode: the value the ant read is one the edge's entries
  // have held; if the map leaves it unchanged (map_fixed), they hold it now
  // and neither is written.  Tested first, so that such an entry needs
  // neither the reverse position nor the fallback's search.
  const bool fixed = ATOMIC && valid && map_fixed(__uint_as_float(e.z), al, bl);
  // after a fallback move: the whole wave searches v's list, once per entry
  uint64_t need = __ballot(valid && !fixed && kr == -3);
  while (need) {
    const int l = (int)__ffsll((unsigned long long)need) - 1;
    need &= need - 1;
    const int r = cand_pos(D, (int)rdlane((uint32_t)v, l), (int)rdlane((uint32_t)u, l), lane);
    if (lane == l) kr = r;
  }
  if (!valid || fixed) return 0;
  if (kr == -2) kr = (int)D.rpos[(size_t)u * D.cl + k];
  float *pf = qhome(D, u, v, k);
  float *pr = qhome(D, v, u, kr);
  if (ATOMIC) {
    const bool both_dense = k < 0 && kr < 0;
    const bool fwd_canon = k >= 0 && (kr < 0 || u < v);
    float *pc = fwd_canon || both_dense ? pf : pr;
    float *po = fwd_canon || both_dense ? pr : pf;
    unsigned int seen = e.z, nw;
    uint32_t r = 0;
    while (true) {
      nw = __float_as_uint(fmaf(al, __uint_as_float(seen), bl));
      const unsigned int old = atomicCAS(reinterpret_cast<unsigned int *>(pc), seen, nw);
      if (old == seen) break;
      seen = old;
      ++r;
    }
    // the value the first entry held just before its update is a fresh
    // guess for the second
    if (both_dense) return r + cas_apply(po, seen, al, bl);
    __hip_atomic_store(po, __uint_as_float(nw), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return r;
  }
  const float xf = tau_load(pf), xr = tau_load(pr);
  if (!map_fixed(xf, al, bl))
    __hip_atomic_store(pf, fmaf(al, xf, bl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!map_fixed(xr, al, bl))
    __hip_atomic_store(pr, fmaf(al, xr, bl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

template <bool ATOMIC>
__device__ __forceinline__ uint32_t spm_apply_entries(const Dev &D, const Iter &A, uint4 e,
                                                      uint32_t &hits, uint32_t &misses);

// Hands the entries of steps [g0, g1) (lanes g0 - t0 .. g1 - t0 - 1 of `e`)
// to the updater, or, once the updater has stopped draining, applies them in
// place.  `head` (= g0 on entry), `tail` (last tail seen) and `direct` are
// the wave's own.  SPM: the entries are the selective memory's (see
// spm_apply_entries; hits and misses count its updates).  Returns this
// lane's retries.
template <bool ATOMIC, bool SPM = false>
__device__ __forceinline__ uint32_t group_push(const Dev &D, const Iter &A, const QRing &q, int w,
                                               uint32_t &head, uint32_t &tail, bool &direct,
                                               int lane, uint4 e, int t0, int g1,
                                               uint32_t &hits, uint32_t &misses) {
  const bool mine = lane + t0 >= (int)head && lane + t0 < g1;
  if (!direct && (uint32_t)g1 - tail > (uint32_t)kQRing) {
    uint32_t spins = 0;
    while (true) {
      tail = (uint32_t)uni((int)lds_ld(q.tail + w));
      if ((uint32_t)g1 - tail <= (uint32_t)kQRing) break;
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (D.wait_limit ? D.wait_limit : kQSpin)) {
        if (lane == 0)
          __hip_atomic_store(D.sync + 1, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        direct = true;
        break;
      }
    }
  }
  if (direct) {
    head = (uint32_t)g1;
    const uint4 own = mine ? e : make_uint4(kNoEntry, 0u, 0u, 0u);
    if (SPM) return spm_apply_entries<ATOMIC>(D, A, own, hits, misses);
    return apply_entries<ATOMIC>(D, A, own, lane);
  }
  if (mine) q.ent[(size_t)w * kQRing + ((lane + t0) & (kQRing - 1))] = e;
  head = (uint32_t)g1;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (lane == 0) lds_st(q.head + w, head);
  return 0;
}

// The updater wave: applies the entries of every ant wave of its block until
// all `na` ant waves are done and every entry is applied.  One pass takes
// the pending entries of all rings at once, up to 64 (ring after ring, each
// from its tail), and applies them together, so the updates of different
// rings share their memory round trips.  With nothing pending it sleeps, so
// it takes few issue slots from the ant waves that share its SIMD.
template <bool ATOMIC, bool SPM = false, int NR = kQAnts>
__device__ __forceinline__ void ring_updater(const Dev &D, const Iter &A, const QRing &q,
                                             int lane, int na) {
  static_assert((kQRing & (kQRing - 1)) == 0 && kQRing >= 64 + kQGroup, "ring size");
  uint32_t tl[NR];  // the updater's own tails (wave-uniform)
#pragma unroll
  for (int w = 0; w < NR; ++w) tl[w] = 0;
  uint32_t retries = 0, idle = 0, hits = 0, misses = 0;
  while (true) {
    // read `done` before the heads: an ant wave publishes its last head
    // before it counts itself done
    const uint32_t done = (uint32_t)uni((int)lds_ld(q.done));
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    uint32_t taken = 0;  // lanes given an entry so far
    uint4 e = make_uint4(kNoEntry, 0u, 0u, 0u);
#pragma unroll
    for (int w = 0; w < NR; ++w) {
      if (w >= na) break;
      const uint32_t h = (uint32_t)uni((int)lds_ld(q.head + w));
      const uint32_t c = min(h - tl[w], 64u - taken);
      if ((uint32_t)lane >= taken && (uint32_t)lane < taken + c)
        e = q.ent[(size_t)w * kQRing + ((tl[w] + (uint32_t)lane - taken) & (kQRing - 1))];
      tl[w] += c;
      taken += c;
    }
    if (taken) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
      for (int w = 0; w < NR; ++w)
        if (w < na && lane == 0) lds_st(q.tail + w, tl[w]);
      if (SPM)
        retries += spm_apply_entries<ATOMIC>(D, A, e, hits, misses);
      else
        retries += apply_entries<ATOMIC>(D, A, e, lane);
      idle = 0;
      continue;
    }
    if (done == (uint32_t)na) break;
    __builtin_amdgcn_s_sleep(32);
    if (++idle > (D.wait_limit ? D.wait_limit : kQIdle)) {
      if (lane == 0)
        __hip_atomic_store(D.sync + 1, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  if (retries) atomicAdd(&D.counters[6], (unsigned long long)retries);
  if (SPM) {
    hits = (uint32_t)uni((int)wave_sum_u(hits));
    misses = (uint32_t)uni((int)wave_sum_u(misses));
    if (lane == 0 && (hits | misses)) {
      atomicAdd(&D.counters[3], (unsigned long long)hits);
      atomicAdd(&D.counters[4], (unsigned long long)misses);
    }
  }
}

// ---------------------------------------------------------------------------
// Asynchronous construction, dense memory, local updates through the
// block's updater wave.  The step holds only what Alg. 2 needs: weigh the
// current city's record, choose (Eq. 1 or Eq. 2 over the candidate set, the
// fallback when it is empty), mark, issue the next record's load, and note
// the crossing in the lane of its step; every kQGroup steps the noted
// crossings go to the ring.  Records and their live pheromone (ctau) come by
// buffer loads (the lane's offset fixed, the row's a scalar; a read outside
// the table returns zeros instead of faulting).  HALF: every candidate list
// fits lanes 0..31.  EVERY: every step has a local update (period 1), so
// the per-step test drops out.  Decisions are the same as those of
// ant_async_dense.
// ---------------------------------------------------------------------------
template <bool ATOMIC, bool HALF, bool EVERY = false>
__device__ __forceinline__ void ant_queued(const Dev &D, const Iter &A, int ant, uint32_t *vis,
                                           int lane, const QRing &q, int qw) {
  const int n = D.n, cl = D.cl;
  const int W = (n + 31) >> 5;
  const uint64_t clmask = cl >= 64 ? ~0ull : (1ull << cl) - 1;
  const int dumw = lane % W;  // this lane's word for the visited-bit store
  const int koff = (lane < cl ? lane : cl - 1) * 16;
  const int rowb = cl * 16;  // bytes per record row
  const __amdgpu_buffer_rsrc_t crs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint4 *>(D.crec), 0, n * rowb, kBufWord3);
  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc(D.ctau, 0, n * cl * 4, kBufWord3);
  // a record's fields and the live pheromone of its slot (the record's own
  // pheromone word is the value of the iteration's start), the latter read
  // device-coherently
  auto load_rec = [&](int city) {
    const auto r = __builtin_amdgcn_raw_buffer_load_b128(crs, koff, city * rowb, 0);
    const uint32_t t =
        __builtin_amdgcn_raw_buffer_load_b32(trs, koff >> 2, city * cl * 4, kCoherent);
    return make_uint4(r[0], r[1], r[2], t);
  };

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  uint4 rec = load_rec(start);

  uint32_t qhead = 0, qtail = 0, c_retry = 0, c_roul = 0, c_fb = 0, unused = 0;
  bool qdirect = false;
  uint64_t c_fbu = 0;
  int64_t len = 0;
  int cur = start;
  // steps in chunks of 64: lane l holds step t0 + l's draw, tour entry and
  // crossing, so a chunk's draws come from one Philox batch and its tour
  // entries leave in one store; its crossings leave kQGroup at a time
  for (int t0 = 0; t0 < n; t0 += 64) {
    if (t0 > 0) draws = philox_batch(A, ant, t0, lane);
    const int lt = lane + t0;
    // bit t - t0 of `upd`: step t has a local update (after every
    // lperiod-th selected edge); of `greedy`: step t takes Eq. 1's argmax
    const uint64_t upd = __builtin_amdgcn_ballot_w64(lt % (int)A.lperiod == 0);
    const uint64_t greedy = __builtin_amdgcn_ballot_w64((draws.x >> 8) < A.q0_24);
    // lane t - t0 holds step t's crossing (x = kNoEntry: no update) and
    // tour entry; every crossing is a candidate move (kr = -2) unless the
    // fallback made it
    uint4 e = make_uint4(kNoEntry, 0u, 0u, (uint32_t)-2);
    int tb = start;
    uint32_t clen = 0;  // at most 64 distances below 2^16 each
    const int tend = min(t0 + 64, n);
    for (int g0 = t0 > 0 ? t0 : 1; g0 < tend;) {
      const int g1 = min((g0 & ~(kQGroup - 1)) + kQGroup, tend);
      uint64_t sb = 1ull << (g0 - t0);  // bit t - t0
      for (int t = g0; t < g1; ++t, sb <<= 1) {
        const int tl = t - t0;
        // lanes >= cl repeat candidate cl - 1 (same city, same weight), so
        // they never change a maximum or a prefix sum of positions < cl; the
        // candidate mask leaves them out of every choice
        const uint32_t word = vis[__builtin_amdgcn_ubfe(rec.x, 5, 11)];
        const bool unv = !__builtin_amdgcn_ubfe(word, rec.x, 1);
        const uint64_t umask = __builtin_amdgcn_ballot_w64(unv) & clmask;
        int next, k;
        uint32_t d, tv;
        if (__builtin_expect(umask == 0, 0)) {
          const Pick p = fallback_dense<false>(D, vis, cur, lane);
          next = p.next;
          k = -1;
          d = p.d;
          tv = __float_as_uint(p.tval);
          if (EVERY || (upd & sb)) e.w = wrlane((uint32_t)-3, tl, e.w);
          ++c_fb;
          c_fbu += (uint64_t)(n - t);
        } else {
          // tau * eta^beta >= 0, so its bit pattern orders like the value
          const float w = unv ? __uint_as_float(rec.w) * __uint_as_float(rec.z) : 0.f;
          if (greedy & sb) {
            // Eq. 1: maximum weight, lowest position
            const uint32_t wb = __float_as_uint(w);
            const uint32_t mx = rows_umax_s<HALF ? 32 : 64>(wb);
            k = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(wb == mx) & umask);
          } else {
            // Eq. 2 by roulette: inclusive Hillis-Steele scan over the
            // positions (offsets 1, 2, 4, ... < cl), r = u * total, first
            // member of the candidate set whose prefix sum exceeds r
            float P = w;
            for (int off = 1; off < cl; off <<= 1) {
              const float o = __shfl_up(P, off, 64);
              if (lane >= off) P = P + o;
            }
            const float total = __uint_as_float(rdlane(__float_as_uint(P), cl - 1));
            const float r = ((float)(rdlane(draws.y, tl) >> 8) * 0x1p-24f) * total;
            const uint64_t sel = __builtin_amdgcn_ballot_w64(P > r) & umask;
            k = sel ? (int)__builtin_ctzll(sel) : 63 - (int)__builtin_clzll(umask);
            ++c_roul;
          }
          next = (int)rdlane(rec.x, k);
          d = rdlane(rec.y, k);
          tv = rdlane(rec.w, k);
        }
        rec = load_rec(next);
        // one lane marks the city (lane k holds it as its candidate)
        if (lane == (k < 0 ? 0 : k))
          __hip_atomic_fetch_or(vis + (next >> 5), 1u << (next & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
        tb = (int)wrlane((uint32_t)next, tl, (uint32_t)tb);
        if (EVERY || (upd & sb)) {
          e.x = wrlane((uint32_t)cur | ((uint32_t)next << 16), tl, e.x);
          e.y = wrlane((uint32_t)k, tl, e.y);
          e.z = wrlane(tv, tl, e.z);
        }
        clen += d;
        cur = next;
      }
      c_retry += group_push<ATOMIC>(D, A, q, qw, qhead, qtail, qdirect, lane, e, t0, g1, unused,
                                    unused);
      g0 = g1;
    }
    len += clen;
    if (lane < tend - t0) D.tours[(size_t)ant * n + lt] = tb;
  }
  // closing edge (cur, start), every ant, as step n: both positions
  // searched, the value read fresh
  {
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    const uint32_t x = rdlane(__float_as_uint(tau_load(qhome(D, cur, start, k1))), 0);
    const uint4 ce =
        make_uint4((uint32_t)cur | ((uint32_t)start << 16), (uint32_t)k1, x, (uint32_t)k2);
    c_retry += group_push<ATOMIC>(D, A, q, qw, qhead, qtail, qdirect, lane, ce, n, n + 1, unused,
                                  unused);
    len += D.dist[(size_t)cur * D.ldn + start];
  }
  c_retry = (uint32_t)uni((int)wave_sum_u(c_retry));
  if (lane == 0) {
    D.lens[ant] = len;
    add_counters(D, (uint32_t)(n - 1) - c_roul - c_fb, c_roul, c_fb, c_fbu, c_retry);
  }
}

// One instance, updates through the block's updater wave: waves 0..na-1 are
// ants blockIdx.x * na + wave, wave na (the last) applies their entries.  The
// host picks na so that every compute unit holds about the same number of
// ants (the slowest unit sets the iteration time).  Dynamic LDS: the rings
// of the na ant waves, then their visited bitmaps.
template <bool ATOMIC, bool HALF, bool EVERY>
__global__ __launch_bounds__(64 * (kQAnts + 1)) void k_construct_async_dense_q(Dev D, Iter A) {
  extern __shared__ uint4 qsm[];
  __shared__ uint32_t qhd[kQAnts], qtl[kQAnts], qdone;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int na = (int)(blockDim.x >> 6) - 1;
  if (threadIdx.x < kQAnts) {
    qhd[threadIdx.x] = 0;
    qtl[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) qdone = 0;
  __syncthreads();
  const QRing q{qsm, qhd, qtl, &qdone};
  if (wv == na) {
    ring_updater<ATOMIC>(D, A, q, lane, na);
    return;
  }
  uint32_t *vis = reinterpret_cast<uint32_t *>(qsm + (size_t)na * kQRing) +
                  wv * ((D.n + 31) >> 5);
  const int ant = uni(blockIdx.x * na + wv);
  if (ant < D.m) ant_queued<ATOMIC, HALF, EVERY>(D, A, ant, vis, lane, q, wv);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (lane == 0) atomicAdd(&qdone, 1u);
}

// Many instances in one launch, updates through each block's updater wave:
// block b runs ants bitems[b].y .. bitems[b].y + kBatchQAnts - 1 of
// instance bitems[b].x (one instance per block, so the updater wave works
// with one descriptor), wave kBatchQAnts applies their entries.
constexpr int kBatchQAnts = kBatchQAntsPerBlock;

template <bool ATOMIC, bool HALF>
__global__ __launch_bounds__(64 * (kBatchQAnts + 1)) void k_construct_async_batch_q(
    const Dev *devs, const Iter *iters, const int2 *bitems, int nb, int wmax) {
  extern __shared__ uint4 qsm[];
  __shared__ uint32_t qhd[kBatchQAnts], qtl[kBatchQAnts], qdone;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  if (threadIdx.x < kBatchQAnts) {
    qhd[threadIdx.x] = 0;
    qtl[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) qdone = 0;
  __syncthreads();
  const int b = blockIdx.x;  // the grid has exactly nb blocks
  const int2 item = bitems[b];
  const int inst = uni(item.x);
  const Dev D = devs[inst];
  const Iter A = iters[inst];
  const QRing q{qsm, qhd, qtl, &qdone};
  if (wv == kBatchQAnts) {
    ring_updater<ATOMIC>(D, A, q, lane, kBatchQAnts);
    return;
  }
  uint32_t *vis = reinterpret_cast<uint32_t *>(qsm + (size_t)kBatchQAnts * kQRing) +
                  wv * wmax;
  const int ant = uni(item.y + wv);
  if (ant < D.m) ant_queued<ATOMIC, HALF>(D, A, ant, vis, lane, q, wv);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (lane == 0) atomicAdd(&qdone, 1u);
}

// Many instances in one launch: wave w builds the tour of ant items[w].y of
// instance items[w].x, whose descriptor and iteration state live in device
// memory (so the launch can be replayed from a graph).  The work list is
// ordered by decreasing n, so the longest chains start first.
template <bool ATOMIC>
__global__ __launch_bounds__(256) void k_construct_async_batch(const Dev *devs, const Iter *iters,
                                                               const int2 *items, int nitems,
                                                               int wmax) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int w = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  if (w >= nitems) return;
  const int2 item = items[w];
  const int inst = uni(item.x);
  const Dev D = devs[inst];
  const Iter A = iters[inst];
  ant_async_dense<ATOMIC>(D, A, uni(item.y), smem + wv * wmax, lane);
}

// ---------------------------------------------------------------------------
// Asynchronous construction with several ants per wave: a group of L lanes
// (L = 32 or 16, L >= cl) carries one ant, so a wave advances 64 / L ants in
// lockstep.  The rule is the same as above, computed group by group: the
// argmax and the roulette scan over candidate positions in the same order
// (so the choice of L never changes a decision), reductions confined to the
// group's rows (DPP within a row of 16, the row-pair swap for L = 32),
// group-local lane reads by ds_bpermute.  All ants of a wave belong to one
// instance and step together (same n); a group whose ant index is past m
// leaves at the start.
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ uint32_t grp_umax(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  if (L == 32) {
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = max(v, max((uint32_t)a[0], (uint32_t)a[1]));
  }
  return v;
}

template <int L>
__device__ __forceinline__ uint32_t grp_umin(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  if (L == 32) {
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min(v, min((uint32_t)a[0], (uint32_t)a[1]));
  }
  return v;
}

// This group's bits of a wave ballot.
template <int L>
__device__ __forceinline__ uint32_t grp_bits(uint64_t ballot, int base) {
  const uint32_t b = (uint32_t)(ballot >> base);
  return L == 32 ? b : (b & 0xffffu);
}

// Value of v on lane k of this group.
__device__ __forceinline__ uint32_t grp_read(uint32_t v, int base, int k) {
  return (uint32_t)__shfl((int)v, base + k, 64);
}

template <int L, bool ATOMIC>
__device__ __forceinline__ void ants_async_dense(const Dev &D, const Iter &A, int first,
                                                 uint32_t *vis_wave, int lane) {
  const int gi = lane / L, gl = lane % L, base = gi * L;
  const int ant = first + gi;
  if (ant >= D.m) return;  // the whole group leaves
  const int n = D.n, cl = D.cl, ldn = D.ldn;
  const int W = (n + 31) >> 5;
  const int kl = gl < cl ? gl : cl - 1;
  const float al = A.a_loc, bl = A.b_loc;
  uint32_t *vis = vis_wave + gi * W;

  for (int w = gl; w < W; w += L) vis[w] = 0u;
  uint4 draws = philox10(make_uint4((uint32_t)gl, (uint32_t)ant, A.it, A.instance), A.key0, A.key1);
  const int start = (int)__umulhi(grp_read(draws.z, base, 0), (uint32_t)n);
  if (gl == 0) vis[start >> 5] |= 1u << (start & 31);
  int tb = start;
  uint4 rec = D.crec[(size_t)start * cl + kl];

  int cur = start, prev = -1;
  float *fwd = nullptr;
  float fval = 0.f;
  int64_t len = 0;
  uint64_t c_kind = 0;  // greedy | roulette << 21 | fallback << 42
  uint32_t c_retry = 0;
  uint64_t c_fbu = 0;
  float *pptr = nullptr;
  unsigned int pexp = 0, pret = 0;
  bool pend = false;
  uint32_t uleft = A.lperiod;

  // chunks of L steps: one Philox batch and one tour store per chunk
  for (int t0 = 0; t0 <= n; t0 += L) {
  if (t0 > 0)
    draws = philox10(make_uint4((uint32_t)(t0 + gl), (uint32_t)ant, A.it, A.instance), A.key0,
                     A.key1);
  // the chunk's greedy draws (lane gl: step t0 + gl) as one ballot
  const uint32_t gbits = grp_bits<L>(__ballot((draws.x >> 8) < A.q0_24), base);
  uint32_t clen = 0;
  const int tend = min(t0 + L, n + 1);
  for (int t = t0 > 0 ? t0 : 1; t < tend; ++t) {
    if (ATOMIC && pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
    pend = false;
    const uint32_t word = vis[rec.x >> 5];
    const bool unv = (gl < cl) & !((word >> (rec.x & 31)) & 1u);
    const float w = unv ? __uint_as_float(rec.w) * __uint_as_float(rec.z) : 0.f;
    __asm__ volatile("" ::"v"(w), "v"((int)unv));
    if (t > 1 && --uleft == 0) {
      uleft = A.lperiod;
      const uint32_t b = grp_bits<L>(__ballot(gl < cl && rec.x == (uint32_t)prev), base);
      const int kr = b ? __builtin_ctz(b) : -1;
      const float rval = kr >= 0 ? __uint_as_float(grp_read(rec.w, base, kr)) : fval;
      if (gl < 2 && !map_fixed(gl == 0 ? fval : rval, al, bl)) {
        float *h = gl == 0 ? fwd : home(D, cur, prev, kr);
        const float seen = gl == 0 ? fval : rval;
        if (ATOMIC) {
          pptr = h;
          pexp = __float_as_uint(seen);
          pend = true;
          pret = atomicCAS(reinterpret_cast<unsigned int *>(h), pexp,
                           __float_as_uint(fmaf(al, seen, bl)));
        } else {
          __hip_atomic_store(h, fmaf(al, seen, bl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    if (t == n) break;
    const uint32_t umask = grp_bits<L>(__ballot(unv), base);
    int next, kind, k = -1;
    uint32_t d;
    float tval;
    if (umask) {
      if ((gbits >> (t - t0)) & 1u) {
        const uint32_t mx = grp_umax<L>(__float_as_uint(w));
        k = __builtin_ctz(grp_bits<L>(__ballot(unv && __float_as_uint(w) == mx), base));
        kind = 0;
      } else {
        float P = w;
        for (int off = 1; off < cl; off <<= 1) {
          const float o = __shfl_up(P, off, L);
          if (gl >= off) P = P + o;
        }
        const float total = __uint_as_float(grp_read(__float_as_uint(P), base, cl - 1));
        const uint32_t u24 = grp_read(draws.y, base, t - t0) >> 8;
        const float r = ((float)u24 * 0x1p-24f) * total;
        const uint32_t sel = grp_bits<L>(__ballot(unv && P > r), base);
        k = sel ? __builtin_ctz(sel) : 31 - __builtin_clz(umask);
        kind = 1;
      }
      next = (int)grp_read(rec.x, base, k);
      d = grp_read(rec.y, base, k);
      tval = __uint_as_float(grp_read(rec.w, base, k));
    } else {
      // Alg. 2's fallback over every unvisited city, ties -> lowest index;
      // first over the prefix (as in fallback_dense, 128 / L cities per lane)
      const float *trow = D.tau + (size_t)cur * ldn;
      const float *erow = D.etad + (size_t)cur * ldn;
      const uint16_t *drow = D.dist + (size_t)cur * ldn;
      float bv = 0.f, bt = 0.f;
      uint32_t bj = kNone, bd = 0;
      bool found = false;
      if (D.fpre) {
        const uint4 *fr = D.fpre + (size_t)cur * (kFpre / 2);
        const float fb = D.fbound[cur];
        uint4 pe[64 / L];
#pragma unroll
        for (int r = 0; r < 64 / L; ++r) pe[r] = fr[gl + L * r];
#pragma unroll
        for (int r = 0; r < 64 / L; ++r) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const uint32_t x = q ? pe[r].z : pe[r].x;
            const uint32_t j = x & 0xffffu;
            const float tq = trow[j];
            const float v = tq * __uint_as_float(q ? pe[r].w : pe[r].y);
            if (!((vis[j >> 5] >> (j & 31)) & 1u) &&
                (bj == kNone || v > bv || (v == bv && j < bj))) {
              bv = v; bj = j; bt = tq; bd = x >> 16;
            }
          }
        }
        found = grp_umax<L>(bj == kNone ? 0u : __float_as_uint(bv)) > __float_as_uint(fb);
        if (!found) { bv = 0.f; bj = kNone; }
      }
#pragma unroll 2
      for (int j0 = 4 * gl; !found && j0 < n; j0 += 4 * L) {
        const float4 tv = *reinterpret_cast<const float4 *>(trow + j0);
        const float4 ev = *reinterpret_cast<const float4 *>(erow + j0);
        const ushort4 dv = *reinterpret_cast<const ushort4 *>(drow + j0);
        const float tq[4] = {tv.x, tv.y, tv.z, tv.w};
        const float eq[4] = {ev.x, ev.y, ev.z, ev.w};
        const uint32_t dq[4] = {dv.x, dv.y, dv.z, dv.w};
        uint32_t bits = (vis[j0 >> 5] >> (j0 & 31)) & 0xfu;
        if (j0 + 4 > n) bits |= (0xfu << (n - j0)) & 0xfu;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float v = tq[q] * eq[q];
          if (!((bits >> q) & 1u) && (bj == kNone || v > bv)) {
            bv = v; bj = (uint32_t)(j0 + q); bt = tq[q]; bd = dq[q];
          }
        }
      }
      const uint32_t mx = grp_umax<L>(bj == kNone ? 0u : __float_as_uint(bv));
      const uint32_t jn = grp_umin<L>((bj != kNone && __float_as_uint(bv) == mx) ? bj : kNone);
      const int owner = __builtin_ctz(grp_bits<L>(__ballot(bj == jn), base));
      next = (int)jn;
      d = grp_read(bd, base, owner);
      tval = __uint_as_float(grp_read(__float_as_uint(bt), base, owner));
      kind = 2;
    }
    c_kind += 1ull << (21 * kind);
    if (kind == 2) c_fbu += (uint64_t)(n - t);
    if (gl == 0) mark(vis, next);
    tb = gl == t - t0 ? next : tb;
    clen += d;
    rec = D.crec[(size_t)next * cl + kl];
    fwd = home(D, cur, next, k);
    fval = tval;
    prev = cur;
    cur = next;
  }
  len += clen;
  if (t0 < n && gl <= min(L - 1, n - 1 - t0)) D.tours[(size_t)ant * n + t0 + gl] = tb;
  }
  if (ATOMIC && pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
  {
    const uint32_t b1 = grp_bits<L>(__ballot(gl < cl && D.crec[(size_t)cur * cl + kl].x ==
                                                         (uint32_t)start), base);
    const uint32_t b2 = grp_bits<L>(__ballot(gl < cl && D.crec[(size_t)start * cl + kl].x ==
                                                         (uint32_t)cur), base);
    const int k1 = b1 ? __builtin_ctz(b1) : -1, k2 = b2 ? __builtin_ctz(b2) : -1;
    float *h = gl == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (gl < 2) {
      if (ATOMIC)
        c_retry += cas_apply(h, __float_as_uint(tau_load(h)), al, bl);
      else
        __hip_atomic_store(h, fmaf(al, tau_load(h), bl), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  len += D.dist[(size_t)cur * ldn + start];
  c_retry += grp_read(c_retry, base, 1);
  if (gl == 0) {
    D.lens[ant] = len;
    const uint32_t m21 = (1u << 21) - 1;
    add_counters(D, (uint32_t)c_kind & m21, (uint32_t)(c_kind >> 21) & m21,
                 (uint32_t)(c_kind >> 42) & m21, c_fbu, c_retry);
  }
}

// Batch of instances, L lanes per ant: wave w runs ants witems[w].y ..
// witems[w].y + 64 / L - 1 of instance witems[w].x.
template <int L, bool ATOMIC>
__global__ __launch_bounds__(256) void k_construct_async_batch_g(const Dev *devs,
                                                                 const Iter *iters,
                                                                 const int2 *witems, int nw,
                                                                 int wmax) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int w = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  if (w >= nw) return;
  const int2 item = witems[w];
  const int inst = uni(item.x);
  const Dev D = devs[inst];
  const Iter A = iters[inst];
  ants_async_dense<L, ATOMIC>(D, A, uni(item.y), smem + wv * (64 / L) * wmax, lane);
}

// One instance, L lanes per ant.
template <int L, bool ATOMIC>
__global__ __launch_bounds__(256) void k_construct_async_dense_g(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int first = uni((blockIdx.x * (blockDim.x >> 6) + wv) * (64 / L));
  if (first >= D.m) return;
  ants_async_dense<L, ATOMIC>(D, A, first, smem + wv * (64 / L) * ((D.n + 31) >> 5), lane);
}

// ---------------------------------------------------------------------------
// Selective pheromone memory (Sec. 3.2, Alg. 3).  The record of city c is s
// pairs {neighbour, pheromone}; a wave holds it with slot i on lane i.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint2 pair_load_coherent(const uint2 *p) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

__device__ __forceinline__ void pair_store_coherent(uint2 *p, uint2 v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     ((unsigned long long)v.y << 32) | v.x, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long pack(uint2 v) {
  return ((unsigned long long)v.y << 32) | v.x;
}

template <bool COHERENT>
__device__ __forceinline__ uint2 spm_record(const Dev &D, int c, int lane) {
  const int i = lane < D.spm_s ? lane : D.spm_s - 1;
  const uint2 *p = D.spm + (size_t)c * D.spm_s + i;
  return COHERENT ? pair_load_coherent(p) : *p;
}

// Pheromone of (c, j) for this lane's j: the value of the first slot of c's
// record holding j, else tau0 (every trail not stored is at the minimum).
__device__ __forceinline__ float spm_tau(uint2 pr, int s, uint32_t j, float tau0) {
  float t = tau0;
  for (int i = s - 1; i >= 0; --i) {
    const uint32_t node = rdlane(pr.x, i);
    const uint32_t val = rdlane(pr.y, i);
    t = j == node ? __uint_as_float(val) : t;
  }
  return t;
}

__device__ __forceinline__ Cand weigh_spm(const Dev &D, const uint32_t *vis, int lane, uint4 rec,
                                          uint2 pr, float tau0) {
  const uint32_t word = vis[rec.x >> 5];
  Cand c;
  c.unv = (lane < D.cl) & !((word >> (rec.x & 31)) & 1u);
  const float t = spm_tau(pr, D.spm_s, rec.x, tau0);
  c.w = c.unv ? t * __uint_as_float(rec.z) : 0.f;
  return c;
}

// Alg. 2's fallback with the selective memory.  Every trail outside cur's
// record holds tau0 and tau0 * eta^beta strictly decreases with d (checked
// when the handle is created), so among the unvisited cities outside the
// record the nearest one by (d, j) has the largest value and the lowest
// index among equals.  The result is the best of that city and the
// unvisited cities of the record, ties -> lowest index: exactly the greedy
// argmax over all unvisited cities.
__device__ __forceinline__ Pick fallback_spm(const Dev &D, uint32_t *vis, int cur, int lane,
                                             uint2 pr, float tau0, int unvisited) {
  const int s = D.spm_s;
  // every load that does not depend on another goes out first: the first
  // 128 keys of cur's extended list (two per lane), cur's coordinates and
  // those of the record's cities
  const uint32_t *xr = D.xnn + (size_t)cur * D.xl;
  const uint32_t e0 = lane < D.xl ? xr[lane] : kNone;
  const uint32_t e1 = lane + 64 < D.xl ? xr[lane + 64] : kNone;
  const double xc = D.xy[2 * cur], yc = D.xy[2 * cur + 1];
  const bool in_rec = lane < s && pr.x != kNone;
  const uint32_t rj = in_rec ? pr.x : 0u;
  const double2 rxy = reinterpret_cast<const double2 *>(D.xy)[rj];
  const bool rec_unv = in_rec && !((vis[rj >> 5] >> (rj & 31)) & 1u);
  // hide the record's unvisited cities from the search of the others
  if (rec_unv) atomicOr(&vis[rj >> 5], 1u << (rj & 31));
  // the extended neighbour list is sorted by (d, j), so its first city that
  // is neither visited nor in the record is the nearest such city overall
  uint32_t key = kNone;
  {
    const uint32_t j0 = e0 & 0xffffu, j1 = e1 & 0xffffu;
    const uint64_t ok0 = __ballot(e0 != kNone && !((vis[j0 >> 5] >> (j0 & 31)) & 1u));
    const uint64_t ok1 = __ballot(e1 != kNone && !((vis[j1 >> 5] >> (j1 & 31)) & 1u));
    if (ok0)
      key = rdlane(e0, (int)__ffsll((unsigned long long)ok0) - 1);
    else if (ok1)
      key = rdlane(e1, (int)__ffsll((unsigned long long)ok1) - 1);
  }
  for (int b0 = 128; key == kNone && b0 < D.xl; b0 += 64) {
    // lists longer than 128 (not built today)
    const int idx = b0 + lane;
    const uint32_t e = idx < D.xl ? xr[idx] : kNone;
    const uint32_t j = e & 0xffffu;
    const uint64_t ok = __ballot(e != kNone && !((vis[j >> 5] >> (j & 31)) & 1u));
    if (ok) key = rdlane(e, (int)__ffsll((unsigned long long)ok) - 1);
  }
  // (when every unvisited city is in the record there is nothing to find)
  const int rec_left = __popcll(__ballot(rec_unv));
  if (key == kNone && unvisited > rec_left) {
    // every listed city is taken: search the grid ring by ring around cur's
    // cell (ring r: the cells at Chebyshev distance r).  Every city of ring
    // r lies at least lb(r) = (r - 1) * gh + (cur's distance to its cell's
    // nearest edge) from cur, so once lb(r) >= d + 1/2 for the best d found
    // no farther city can reach d, let alone beat it (ties go to the lower
    // index, so cities at the best d are still read).  Each lane keeps the
    // least key over the cities it reads; a city is looked at more closely
    // only when its s = dx*dx + dy*dy is below (d + 1/2)^2, which is exactly
    // when its distance is at most d.
    const int cx = grid_cx(D, xc), cy = grid_cy(D, yc);
    const double fx = xc - (D.gx0 + cx * D.gh), fy = yc - (D.gy0 + cy * D.gh);
    // the margin covers rounding in the cell of a coordinate
    const double margin = 1e-9 * (fabs(D.gx0) + fabs(D.gy0) + D.gh * (double)(D.gnx + D.gny));
    const double edge = fmax(0.0, fmin(fmin(fx, D.gh - fx), fmin(fy, D.gh - fy))) - margin;
    // Every city of rings 0..r lies within (r + 1) * gh * sqrt(2) of cur.
    // Where that is below d_last - 1/2 (d_last: the list's last distance),
    // each such city is nearer than d_last, so it is on the list, and so
    // visited or in the record: the search starts at the first ring that
    // can hold anything else.
    const uint32_t klast = D.xl <= 128 ? rdlane(D.xl - 1 < 64 ? e0 : e1, (D.xl - 1) & 63) : 0u;
    const double reach = ((double)(klast >> 16) - 0.5 - margin) / (D.gh * 1.4142135623730951);
    const int rfirst = reach > 1.0 ? (int)ceil(reach - 1.0) : 0;
    uint32_t lkey = kNone;
    double bound = INFINITY;  // (d + 1/2)^2 for the best key so far
    const int rmax = max(D.gnx, D.gny);
    for (int r = rfirst; r <= rmax; ++r) {
      if (key != kNone && r >= 1) {
        const double lb = (double)(r - 1) * D.gh + edge;
        if (lb > 0.0 && lb * lb >= bound) break;
      }
      const int ncell = r == 0 ? 1 : 8 * r;
      for (int q = lane; q < ncell; q += 64) {
        int ix, iy;
        if (r == 0) {
          ix = cx;
          iy = cy;
        } else if (q < 2 * r + 1) {  // top row
          ix = cx - r + q;
          iy = cy - r;
        } else if (q < 4 * r + 2) {  // bottom row
          ix = cx - r + (q - 2 * r - 1);
          iy = cy + r;
        } else if (q < 6 * r + 1) {  // left column without the corners
          ix = cx - r;
          iy = cy - r + 1 + (q - 4 * r - 2);
        } else {                     // right column without the corners
          ix = cx + r;
          iy = cy - r + 1 + (q - 6 * r - 1);
        }
        if (ix < 0 || iy < 0 || ix >= D.gnx || iy >= D.gny) continue;
        const int c = iy * D.gnx + ix;
        const int p1 = D.gstart[c + 1];
        // four cities of the cell per round, their loads issued together
        for (int p = D.gstart[c]; p < p1; p += 4) {
          uint32_t jq[4];
          double2 cq[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int pu = min(p + u, p1 - 1);
            jq[u] = D.gcity[pu];
            cq[u] = D.gxy[pu];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t j = jq[u];
            if (p + u >= p1 || ((vis[j >> 5] >> (j & 31)) & 1u)) continue;
            const double dx = xc - cq[u].x, dy = yc - cq[u].y;
            if (dx * dx + dy * dy < bound) {
              const uint32_t d = exact_dist(xc, yc, cq[u].x, cq[u].y);
              const uint32_t kk = (d << 16) | j;
              if (kk < lkey) lkey = kk;
            }
          }
        }
      }
      key = wave_umin_u(lkey);
      if (key != kNone) {
        const double b = (double)(key >> 16) + 0.5;
        bound = b * b;
      }
    }
  }
  if (rec_unv) atomicAnd(&vis[rj >> 5], ~(1u << (rj & 31)));
  // record candidates on lanes < s, the off-record candidate on its own
  const uint32_t rd = rec_unv ? exact_dist(xc, yc, rxy.x, rxy.y) : 0u;
  const bool off = key != kNone;
  const float re = D.eta_tab[rd];
  const float oe = D.eta_tab[off ? key >> 16 : 0u];
  const float rv = rec_unv ? __uint_as_float(pr.y) * re : 0.f;
  const float ov = off ? tau0 * oe : 0.f;
  const uint64_t any_rec = __ballot(rec_unv);
  uint32_t mx = any_rec ? wave_umax_u(rec_unv ? __float_as_uint(rv) : 0u) : 0u;
  if (off && (!any_rec || __float_as_uint(ov) > mx)) mx = __float_as_uint(ov);
  const bool rec_win = rec_unv && __float_as_uint(rv) == mx;
  uint32_t jn = wave_umin_u(rec_win ? rj : kNone);
  const bool off_win = off && __float_as_uint(ov) == mx && (key & 0xffffu) < jn;
  Pick p;
  p.k = -1;
  p.kind = 2;
  if (off_win) {
    jn = key & 0xffffu;
    p.d = key >> 16;
    p.tval = tau0;
  } else {
    const int owner = uni((int)__ffsll((unsigned long long)__ballot(rec_win && rj == jn)) - 1);
    p.d = rdlane(rd, owner);
    p.tval = __uint_as_float(rdlane(pr.y, owner));
  }
  p.next = (int)jn;
  return p;
}

// Alg. 3 on a record held by the wave (slot i on lane i, insert counter
// `tail`): the trail for neighbour nb gets the map x -> fma(a, x, b); a
// missing trail gets the map applied to tau0 in the slot after the most
// recently added one, which overwrites the least recently added trail.
__device__ __forceinline__ void spm_update_wave(uint2 &pr, uint32_t &tail, int s, int lane,
                                                int nb, float a, float b, float tau0,
                                                uint32_t &hits, uint32_t &misses) {
  const uint64_t hit = __ballot(lane < s && pr.x == (uint32_t)nb);
  if (hit) {
    const int i = (int)__ffsll((unsigned long long)hit) - 1;
    if (lane == i) pr.y = __float_as_uint(fmaf(a, __uint_as_float(pr.y), b));
    ++hits;
  } else {
    tail += 1;
    const int slot = (int)(tail % (uint32_t)s);
    if (lane == slot) pr = make_uint2((uint32_t)nb, __float_as_uint(fmaf(a, tau0, b)));
    ++misses;
  }
}

// Synchronous step updates of record r: every registered update of this step
// whose record is r, in increasing update index e = 2 * ant + w (ant
// ascending, the ant's own record before the next city's).  The updates of
// r form a list (in arrival order); up to 64 of them are gathered onto the
// lanes and applied smallest e first.  A longer list (more than 64 updates
// of one record in one step) is found by scanning every registration.
__device__ __forceinline__ void spm_apply_step(const Dev &D, int r, int ne, float a, float b,
                                               float tau0, int lane, uint32_t &hits,
                                               uint32_t &misses) {
  const int s = D.spm_s;
  uint2 pr = spm_record<true>(D, r, lane);
  uint32_t tail = __hip_atomic_load(D.spm_tail + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int cnt = 0, mine = INT_MAX;
  int e = __hip_atomic_load(D.upd_head + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (e >= 0 && cnt <= 64) {
    if (lane == cnt) mine = e;
    ++cnt;
    e = __hip_atomic_load(D.upd_next + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (cnt <= 64) {
    for (int i = 0; i < cnt; ++i) {
      const int emin = (int)wave_umin_u((uint32_t)mine);
      if (mine == emin) mine = INT_MAX;
      const int nb = __hip_atomic_load(D.upd_nb + emin, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
      spm_update_wave(pr, tail, s, lane, nb, a, b, tau0, hits, misses);
    }
  } else {
    for (int e0 = 0; e0 < ne; e0 += 64) {
      const int ee = e0 + lane;
      int rr = -1, nbv = 0;
      if (ee < ne) {
        rr = __hip_atomic_load(D.upd_rec + ee, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nbv = __hip_atomic_load(D.upd_nb + ee, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      uint64_t mask = __ballot(rr == r);
      while (mask) {
        const int l = (int)__ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        spm_update_wave(pr, tail, s, lane, (int)rdlane((uint32_t)nbv, l), a, b, tau0, hits,
                        misses);
      }
    }
  }
  if (lane < s) pair_store_coherent(D.spm + (size_t)r * s + lane, pr);
  if (lane == 0) {
    __hip_atomic_store(D.spm_tail + r, tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(D.upd_head + r, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Registers update e (record r, neighbour nb) for this step by pushing it
// onto r's list.  Returns true for the update that found the list empty:
// its wave applies the record's list after the barrier.
__device__ __forceinline__ bool spm_register(const Dev &D, int e, int r, int nb) {
  __hip_atomic_store(D.upd_rec + e, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(D.upd_nb + e, nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int old = __hip_atomic_exchange(D.upd_head + r, e, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(D.upd_next + e, old, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return old < 0;
}

// The UPDATE phase of one synchronous step with the selective memory: the
// wave of ant `ant` applies the lists of the records it leads (lead0: its
// own record r0, lead1: the next city's record r1).
__device__ __forceinline__ void spm_sync_updates(const Dev &D, bool lead0, bool lead1, int r0,
                                                 int r1, float a, float b, float tau0, int lane,
                                                 uint32_t &hits, uint32_t &misses) {
  const int ne = 2 * D.m;
  if (lead0) spm_apply_step(D, r0, ne, a, b, tau0, lane, hits, misses);
  if (lead1) spm_apply_step(D, r1, ne, a, b, tau0, lane, hits, misses);
}

__device__ __forceinline__ void add_spm_counters(const Dev &D, uint32_t hits, uint32_t misses) {
  atomicAdd(&D.counters[3], (unsigned long long)hits);
  atomicAdd(&D.counters[4], (unsigned long long)misses);
}

// ---------------------------------------------------------------------------
// Synchronous construction with the selective memory.  Per step:
//   SELECT (coherent reads) and registration of the step's 2m updates
//   | barrier | each record's updates applied in (ant, record i then j)
//   order by the wave that leads it | barrier.
// The closing edges are one more such round.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_construct_sync_spm(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ant = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  const bool active = ant < D.m;
  const int n = D.n, cl = D.cl;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  uint32_t *vis = smem + wv * W;
  const float tau0 = A.tau0;

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  int tb = start;

  int cur = start;
  int64_t len = 0;
  uint32_t c_greedy = 0, c_roul = 0, c_fb = 0, hits = 0, misses = 0;
  uint64_t c_fbu = 0;
  uint32_t bar = 0;
  for (int t = 1; t <= n; ++t) {
    int next = start;
    if ((t & 63) == 0) draws = philox_batch(A, ant, t, lane);
    if (active && t < n) {
      const uint4 rec = D.crec[(size_t)cur * cl + kl];
      const uint2 pr = spm_record<true>(D, cur, lane);
      const Cand c = weigh_spm(D, vis, lane, rec, pr, tau0);
      Pick p;
      const int k = pick_candidate(A, lane, cl, c, draw_of(draws, t), p.kind);
      if (k >= 0) {
        p.next = (int)rdlane(rec.x, k);
        p.d = rdlane(rec.y, k);
      } else {
        p = fallback_spm(D, vis, cur, lane, pr, tau0, n - t);
      }
      c_greedy += p.kind == 0;
      c_roul += p.kind == 1;
      if (p.kind == 2) { ++c_fb; c_fbu += (uint64_t)(n - t); }
      if (lane == 0) mark(vis, p.next);
      tour_put(D, ant, t, lane, p.next, tb);
      len += p.d;
      next = p.next;
    }
    if (active && t == n) len += dist_xy(D, cur, start);
    // t < n: the step's crossing (every lperiod-th step); t == n: the closing edge
    if (t == n || t % A.lperiod == 0) {
      bool lead = false;
      if (active && lane < 2)
        lead = spm_register(D, 2 * ant + lane, lane == 0 ? cur : next, lane == 0 ? next : cur);
      const uint64_t leads = __ballot(lead);
      grid_barrier_f(D, barrier_epoch(A, ++bar));
      if (active)
        spm_sync_updates(D, leads & 1u, (leads >> 1) & 1u, cur, next, A.a_loc, A.b_loc, tau0,
                         lane, hits, misses);
      if (t < n) grid_barrier_f(D, barrier_epoch(A, ++bar));
    }
    cur = next;
  }
  if (active && lane == 0) {
    D.lens[ant] = len;
    add_counters(D, c_greedy, c_roul, c_fb, c_fbu, 0);
    add_spm_counters(D, hits, misses);
  }
}

// ---------------------------------------------------------------------------
// Asynchronous construction with the selective memory: no barriers; each
// crossing's two record updates are lock-free.  A trail already in the
// record gets the map by a 64-bit compare-and-swap of its {neighbour, value}
// pair (a pair that changed meanwhile is re-examined); a missing trail takes
// the next slot of the record by an atomic increment of its insert counter
// and is written there as one 64-bit store.  Two ants inserting the same
// trail at the same moment can both succeed (a duplicate; reads take the
// first slot).  The updates of a move are issued at the start of the next
// step and checked one step later, like the dense kernel's.
// ---------------------------------------------------------------------------
struct SpmOp {
  uint2 *pair;         // hit: the pair's slot
  uint32_t *tail;      // miss: the record's insert counter
  unsigned long long expect, desired;
  uint32_t ret_lo, ret_hi;
  int nb, rec;
  bool hit, live;
};

__device__ __forceinline__ void spm_async_issue(const Dev &D, SpmOp &op, uint2 pr, int r, int nb,
                                                int lane, int owner, float a, float b,
                                                float tau0, uint32_t &hits, uint32_t &misses) {
  const int s = D.spm_s;
  const uint64_t hm = __ballot(lane < s && pr.x == (uint32_t)nb);
  if (lane != owner) return;
  op.live = true;
  op.nb = nb;
  op.rec = r;
  if (hm) {
    const int i = (int)__ffsll((unsigned long long)hm) - 1;
    const uint32_t v = rdlane(pr.y, i);
    op.hit = true;
    op.pair = D.spm + (size_t)r * s + i;
    op.expect = ((unsigned long long)v << 32) | (uint32_t)nb;
    op.desired = ((unsigned long long)__float_as_uint(fmaf(a, __uint_as_float(v), b)) << 32) |
                 (uint32_t)nb;
    const unsigned long long got = atomicCAS(reinterpret_cast<unsigned long long *>(op.pair),
                                             op.expect, op.desired);
    op.ret_lo = (uint32_t)got;
    op.ret_hi = (uint32_t)(got >> 32);
    ++hits;
  } else {
    op.hit = false;
    op.tail = D.spm_tail + r;
    op.ret_lo = atomicAdd(op.tail, 1u);
    ++misses;
  }
}

// Finishes an issued update: a miss writes its pair into the slot it took;
// a hit whose pair changed is redone against the record's current state.
__device__ __forceinline__ uint32_t spm_async_finish(const Dev &D, SpmOp &op, float a, float b,
                                                     float tau0) {
  if (!op.live) return 0;
  op.live = false;
  const int s = D.spm_s;
  if (!op.hit) {
    const uint32_t slot = (op.ret_lo + 1u) % (uint32_t)s;
    pair_store_coherent(D.spm + (size_t)op.rec * s + slot,
                        make_uint2((uint32_t)op.nb, __float_as_uint(fmaf(a, tau0, b))));
    return 0;
  }
  if ((((unsigned long long)op.ret_hi << 32) | op.ret_lo) == op.expect) return 0;
  // the pair changed: look for the trail again and apply the map
  uint32_t retries = 1;
  while (true) {
    int found = -1;
    uint2 cur_pair = make_uint2(0, 0);
    for (int i = 0; i < s; ++i) {
      const uint2 q = pair_load_coherent(D.spm + (size_t)op.rec * s + i);
      if (found < 0 && q.x == (uint32_t)op.nb) { found = i; cur_pair = q; }
    }
    if (found < 0) {
      const uint32_t t = atomicAdd(D.spm_tail + op.rec, 1u);
      pair_store_coherent(D.spm + (size_t)op.rec * s + (t + 1u) % (uint32_t)s,
                          make_uint2((uint32_t)op.nb, __float_as_uint(fmaf(a, tau0, b))));
      return retries;
    }
    const unsigned long long ex = pack(cur_pair);
    const unsigned long long de =
        ((unsigned long long)__float_as_uint(fmaf(a, __uint_as_float(cur_pair.y), b)) << 32) |
        (uint32_t)op.nb;
    if (atomicCAS(reinterpret_cast<unsigned long long *>(D.spm + (size_t)op.rec * s + found), ex,
                  de) == ex)
      return retries;
    ++retries;
  }
}

// The unsynchronised variant of Alg. 3 (ACS-GPU-Alt): the owner lane writes
// the changed pair of the record the wave read (pr, insert counter tl) and,
// for a new trail, the advanced insert counter, with plain (not
// read-modify-write) device-coherent stores; updates that race with it are
// lost.
__device__ __forceinline__ void spm_racy_issue(const Dev &D, uint2 pr, uint32_t tl, int r, int nb,
                                               int lane, int owner, float a, float b, float tau0,
                                               uint32_t &hits, uint32_t &misses) {
  const int s = D.spm_s;
  const uint64_t hm = __ballot(lane < s && pr.x == (uint32_t)nb);
  if (lane != owner) return;
  if (hm) {
    const int i = (int)__ffsll((unsigned long long)hm) - 1;
    const uint32_t v = rdlane(pr.y, i);
    pair_store_coherent(D.spm + (size_t)r * s + i,
                        make_uint2((uint32_t)nb, __float_as_uint(fmaf(a, __uint_as_float(v), b))));
    ++hits;
  } else {
    const uint32_t slot = (tl + 1u) % (uint32_t)s;
    pair_store_coherent(D.spm + (size_t)r * s + slot,
                        make_uint2((uint32_t)nb, __float_as_uint(fmaf(a, tau0, b))));
    __hip_atomic_store(D.spm_tail + r, tl + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++misses;
  }
}

// The wave keeps the record of its current city in registers (pr, tl).  Its
// own update of that record (the reverse entry of the move that reached the
// city) is applied to the copy before the copy is read, so an ant always
// sees its own updates, as in Alg. 1; with one ant the result is exactly the
// sequential one.  The memory operations of the update are issued after the
// weights are formed (see the dense kernel for why).
template <bool ATOMIC>
__global__ __launch_bounds__(256) void k_construct_async_spm(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ant = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  if (ant >= D.m) return;
  const int n = D.n, cl = D.cl, s = D.spm_s;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  uint32_t *vis = smem + wv * W;
  const float al = A.a_loc, bl = A.b_loc, tau0 = A.tau0;

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  int tb = start;
  uint4 rec = D.crec[(size_t)start * cl + kl];
  uint2 pr = spm_record<false>(D, start, lane);
  uint32_t tl = D.spm_tail[start];
  uint2 pr_prev = pr;
  uint32_t tl_prev = tl;

  int cur = start, prev = -1;
  int64_t len = 0;
  uint64_t c_kind = 0;  // greedy | roulette << 21 | fallback << 42
  uint32_t c_retry = 0, hits = 0, misses = 0;
  uint64_t c_fbu = 0;
  SpmOp op{};
  op.live = false;
  uint32_t uleft = A.lperiod;

  // chunks of 64 steps: one Philox batch and one tour store per chunk
  for (int t0 = 0; t0 <= n; t0 += 64) {
  if (t0 > 0) draws = philox_batch(A, ant, t0, lane);
  uint32_t clen = 0;
  const int tend = min(t0 + 64, n + 1);
  for (int t = t0 > 0 ? t0 : 1; t < tend; ++t) {
    if (ATOMIC) c_retry += spm_async_finish(D, op, al, bl, tau0);
    bool upd = false;
    if (t > 1 && --uleft == 0) {
      uleft = A.lperiod;
      upd = true;
    }
    // record of cur as it was read, then with this ant's reverse update
    const uint2 pr_read = pr;
    const uint32_t tl_read = tl;
    if (upd) {
      uint32_t h0 = 0, m0 = 0;
      spm_update_wave(pr, tl, s, lane, prev, al, bl, tau0, h0, m0);
    }
    const Cand c = weigh_spm(D, vis, lane, rec, pr, tau0);
    __asm__ volatile("" ::"v"(c.w), "v"((int)c.unv));
    if (upd) {
      // forward entry of the previous move in prev's record (lane 0),
      // reverse entry in cur's record (lane 1)
      if (ATOMIC) {
        spm_async_issue(D, op, pr_prev, prev, cur, lane, 0, al, bl, tau0, hits, misses);
        spm_async_issue(D, op, pr_read, cur, prev, lane, 1, al, bl, tau0, hits, misses);
      } else {
        spm_racy_issue(D, pr_prev, tl_prev, prev, cur, lane, 0, al, bl, tau0, hits, misses);
        spm_racy_issue(D, pr_read, tl_read, cur, prev, lane, 1, al, bl, tau0, hits, misses);
      }
    }
    if (t == n) break;
    Pick p;
    const int k = pick_candidate(A, lane, cl, c, draw_of(draws, t), p.kind);
    if (k >= 0) {
      p.next = (int)rdlane(rec.x, k);
      p.d = rdlane(rec.y, k);
    } else {
      p = fallback_spm(D, vis, cur, lane, pr, tau0, n - t);
    }
    c_kind += 1ull << (21 * p.kind);
    if (p.kind == 2) c_fbu += (uint64_t)(n - t);
    if (lane == 0) mark(vis, p.next);
    tb = lane == t - t0 ? p.next : tb;
    clen += p.d;
    rec = D.crec[(size_t)p.next * cl + kl];
    pr_prev = pr;
    tl_prev = tl;
    pr = spm_record<false>(D, p.next, lane);
    tl = D.spm_tail[p.next];
    prev = cur;
    cur = p.next;
  }
  len += clen;
  if (t0 < n && lane <= min(63, n - 1 - t0)) D.tours[(size_t)ant * n + t0 + lane] = tb;
  }
  if (ATOMIC) c_retry += spm_async_finish(D, op, al, bl, tau0);
  // closing edge, read fresh: record cur (neighbour start), record start
  {
    const uint2 q0 = spm_record<true>(D, cur, lane);
    if (ATOMIC) {
      spm_async_issue(D, op, q0, cur, start, lane, 0, al, bl, tau0, hits, misses);
      c_retry += spm_async_finish(D, op, al, bl, tau0);
    } else {
      const uint32_t t0 = __hip_atomic_load(D.spm_tail + cur, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      spm_racy_issue(D, q0, t0, cur, start, lane, 0, al, bl, tau0, hits, misses);
    }
    const uint2 q1 = spm_record<true>(D, start, lane);
    if (ATOMIC) {
      spm_async_issue(D, op, q1, start, cur, lane, 0, al, bl, tau0, hits, misses);
      c_retry += spm_async_finish(D, op, al, bl, tau0);
    } else {
      const uint32_t t1 = __hip_atomic_load(D.spm_tail + start, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      spm_racy_issue(D, q1, t1, start, cur, lane, 0, al, bl, tau0, hits, misses);
    }
  }
  len += dist_xy(D, cur, start);
  c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1)));
  hits = (uint32_t)uni((int)(rdlane(hits, 0) + rdlane(hits, 1)));
  misses = (uint32_t)uni((int)(rdlane(misses, 0) + rdlane(misses, 1)));
  if (lane == 0) {
    D.lens[ant] = len;
    const uint32_t m21 = (1u << 21) - 1;
    add_counters(D, (uint32_t)c_kind & m21, (uint32_t)(c_kind >> 21) & m21,
                 (uint32_t)(c_kind >> 42) & m21, c_fbu, c_retry);
    add_spm_counters(D, hits, misses);
  }
}

// ---------------------------------------------------------------------------
// Asynchronous construction with the selective memory, updates through the
// block's updater wave (as the dense k_construct_async_dense_q): the ant
// wave issues no update, so its record loads never wait behind an atomic.
// Entry of city r: {r, nbA, nbB, 0}: Alg. 3 on r's record for neighbour nbA
// (the edge that reached r), then for nbB (the edge that left it); kNone
// marks an edge without an update (local-update period).  One entry per
// visited city keeps the two updates of a record in their order, and the
// updates of different entries concern different records of one ant, so an
// ant's updates land in the order Alg. 1 applies them.  The start city's
// entry (its departure, then the closing edge) goes last.
// ---------------------------------------------------------------------------
template <bool ATOMIC>
__device__ __forceinline__ uint32_t spm_apply_entries(const Dev &D, const Iter &A, uint4 e,
                                                      uint32_t &hits, uint32_t &misses) {
  if (e.x == kNoEntry) return 0;
  const int r = (int)e.x, s = D.spm_s;
  uint2 *rec = D.spm + (size_t)r * s;
  const float a = A.a_loc, b = A.b_loc;
  const uint32_t ins = __float_as_uint(fmaf(a, A.tau0, b));  // a new trail: the map of tau0
  uint32_t retries = 0;
  for (int u = 0; u < 2; ++u) {
    const uint32_t nb = u == 0 ? e.y : e.z;
    if (nb == kNone) continue;
    while (true) {
      // the record as it is now; the first slot holding nb is its trail
      int found = -1;
      uint2 cur = make_uint2(0u, 0u);
      for (int i = 0; i < s; ++i) {
        const uint2 x = pair_load_coherent(rec + i);
        if (found < 0 && x.x == nb) {
          found = i;
          cur = x;
        }
      }
      if (found < 0) {
        // miss: the slot after the most recently added one
        uint32_t t;
        if (ATOMIC) {
          t = atomicAdd(D.spm_tail + r, 1u);
        } else {
          t = __hip_atomic_load(D.spm_tail + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(D.spm_tail + r, t + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        pair_store_coherent(rec + (t + 1u) % (uint32_t)s, make_uint2(nb, ins));
        ++misses;
        break;
      }
      const uint2 nw = make_uint2(nb, __float_as_uint(fmaf(a, __uint_as_float(cur.y), b)));
      if (!ATOMIC) {
        pair_store_coherent(rec + found, nw);
        ++hits;
        break;
      }
      if (atomicCAS(reinterpret_cast<unsigned long long *>(rec + found), pack(cur), pack(nw)) ==
          pack(cur)) {
        ++hits;
        break;
      }
      ++retries;  // the pair changed meanwhile: look again
    }
  }
  return retries;
}

// Trail of this lane's candidate j from the record pairs on lanes 0..S-1:
// slot I is broadcast over each row of 16 lanes by DPP (row_newbcast), from
// the last slot to the first, so the first slot holding j is the one kept.
template <int I>
__device__ __forceinline__ void spm_trail_rows(uint2 pr, uint32_t j, float &t) {
  if constexpr (I >= 0) {
    const uint32_t node = (uint32_t)__builtin_amdgcn_mov_dpp((int)pr.x, 0x150 + I, 0xF, 0xF, true);
    const uint32_t val = (uint32_t)__builtin_amdgcn_mov_dpp((int)pr.y, 0x150 + I, 0xF, 0xF, true);
    t = j == node ? __uint_as_float(val) : t;
    spm_trail_rows<I - 1>(pr, j, t);
  }
}

// The ant of k_construct_async_spm_q.  Records come by buffer loads: the
// candidates' {j, d, eta^beta} on lanes 0..cl-1, the selective record's
// pairs on lanes 0..s-1 and its insert counter.  Before the record of cur is
// read, the ant applies its own update of the edge that reached cur to its
// copy (Alg. 1 order): only a miss matters there, which replaces the slot
// after the most recently added one by prev (visited, so its trail is never
// read).  S: s when known at compile time (0: D.spm_s).  L: lanes holding
// the candidates (16, 32 or 64).
template <bool ATOMIC, int S, int L>
__device__ __forceinline__ void spm_ant_queued(const Dev &D, const Iter &A, int ant,
                                               uint32_t *vis, int lane, const QRing &q, int qw) {
  const int n = D.n, cl = D.cl, s = S ? S : D.spm_s;
  const int W = (n + 31) >> 5;
  const uint64_t clmask = cl >= 64 ? ~0ull : (1ull << cl) - 1;
  const int koff = (lane < cl ? lane : cl - 1) * 16;
  const int rowb = cl * 16;
  const int soff = (lane < s ? lane : s - 1) * 8;
  const float tau0 = A.tau0;
  const __amdgpu_buffer_rsrc_t crs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint4 *>(D.crec), 0, n * rowb, kBufWord3);
  const __amdgpu_buffer_rsrc_t srs =
      __builtin_amdgcn_make_buffer_rsrc(D.spm, 0, n * s * 8, kBufWord3);
  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc(D.spm_tail, 0, n * 4, kBufWord3);
  auto load_rec = [&](int city) {
    const auto r = __builtin_amdgcn_raw_buffer_load_b96(crs, koff, city * rowb, 0);
    return make_uint3(r[0], r[1], r[2]);
  };
  auto load_pair = [&](int city) {
    const auto r = __builtin_amdgcn_raw_buffer_load_b64(srs, soff, city * s * 8, kCoherent);
    return make_uint2(r[0], r[1]);
  };
  auto load_tail = [&](int city) {
    return __builtin_amdgcn_raw_buffer_load_b32(trs, 0, city * 4, kCoherent);
  };

  for (int w = lane; w < W; w += 64) vis[w] = 0u;
  uint4 draws = philox_batch(A, ant, 0, lane);
  const int start = (int)__umulhi(rdlane(draws.z, 0), (uint32_t)n);
  if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
  uint3 rec = load_rec(start);
  uint2 pr = load_pair(start);
  uint32_t tlv = load_tail(start);

  uint32_t qhead = 0, qtail = 0, c_retry = 0, hits = 0, misses = 0, c_roul = 0, c_fb = 0;
  bool qdirect = false;
  uint64_t c_fbu = 0;
  int64_t len = 0;
  int cur = start, prev = -1;
  bool arrived_upd = false;    // the edge that reached cur gets a local update
  uint32_t nb_start = kNone;   // the start city's departure update (applied last)
  const uint32_t lp = A.lperiod;
  for (int t0 = 0; t0 < n; t0 += 64) {
    if (t0 > 0) draws = philox_batch(A, ant, t0, lane);
    const uint64_t upd = __builtin_amdgcn_ballot_w64((uint32_t)(lane + t0) % lp == 0);
    const uint64_t greedy = __builtin_amdgcn_ballot_w64((draws.x >> 8) < A.q0_24);
    // lane t - t0: step t's entry (x = kNoEntry: none) and tour entry
    uint4 e = make_uint4(kNoEntry, 0u, 0u, 0u);
    int tb = start;
    uint32_t clen = 0;
    const int tend = min(t0 + 64, n);
    for (int g0 = t0 > 0 ? t0 : 1; g0 < tend;) {
      const int g1 = min((g0 & ~(kQGroup - 1)) + kQGroup, tend);
      uint64_t sb = 1ull << (g0 - t0);  // bit t - t0
      for (int t = g0; t < g1; ++t, sb <<= 1) {
        const int tl = t - t0;
        if (arrived_upd) {
          const uint64_t hit =
              __builtin_amdgcn_ballot_w64(lane < s && pr.x == (uint32_t)prev);
          if (!hit) {
            const uint32_t tu = (uint32_t)uni((int)tlv) + 1u;
            const int slot = (int)(S ? (tu % (uint32_t)S) : (tu % (uint32_t)s));
            if (lane == slot) pr.x = (uint32_t)prev;
          }
        }
        // the candidates' trails: the first slot holding j, else tau0.  With
        // every candidate in lanes 0..15 a DPP row broadcast hands slot i to
        // them (no scalar round trip); otherwise a lane read per slot.
        float tj = tau0;
        if constexpr (L == 16 && S != 0) {
          spm_trail_rows<S - 1>(pr, rec.x, tj);
        } else {
#pragma unroll
          for (int i = (S ? S : kMaxSpmS) - 1; i >= 0; --i) {
            if (S == 0 && i >= s) continue;
            const uint32_t node = rdlane(pr.x, i);
            const uint32_t val = rdlane(pr.y, i);
            tj = rec.x == node ? __uint_as_float(val) : tj;
          }
        }
        const uint32_t word = vis[__builtin_amdgcn_ubfe(rec.x, 5, 11)];
        const bool unv = !__builtin_amdgcn_ubfe(word, rec.x, 1);
        const uint64_t umask = __builtin_amdgcn_ballot_w64(unv) & clmask;
        int next, k;
        uint32_t d;
        if (__builtin_expect(umask == 0, 0)) {
          const Pick p = fallback_spm(D, vis, cur, lane, pr, tau0, n - t);
          next = p.next;
          k = -1;
          d = p.d;
          ++c_fb;
          c_fbu += (uint64_t)(n - t);
        } else {
          const float w = unv ? tj * __uint_as_float(rec.z) : 0.f;
          if (greedy & sb) {
            // Eq. 1: maximum weight, lowest position
            const uint32_t wb = __float_as_uint(w);
            const uint32_t mx = rows_umax_s<L>(wb);
            k = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(wb == mx) & umask);
          } else {
            // Eq. 2 by roulette, as in ant_queued
            float P = w;
            for (int off = 1; off < cl; off <<= 1) {
              const float o = __shfl_up(P, off, 64);
              if (lane >= off) P = P + o;
            }
            const float total = __uint_as_float(rdlane(__float_as_uint(P), cl - 1));
            const float r = ((float)(rdlane(draws.y, tl) >> 8) * 0x1p-24f) * total;
            const uint64_t sel = __builtin_amdgcn_ballot_w64(P > r) & umask;
            k = sel ? (int)__builtin_ctzll(sel) : 63 - (int)__builtin_clzll(umask);
            ++c_roul;
          }
          next = (int)rdlane(rec.x, k);
          d = rdlane(rec.y, k);
        }
        rec = load_rec(next);
        pr = load_pair(next);
        tlv = load_tail(next);
        if (lane == (k < 0 ? 0 : k))
          __hip_atomic_fetch_or(vis + (next >> 5), 1u << (next & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
        const bool up = (upd & sb) != 0;
        if (t == 1) {
          nb_start = up ? (uint32_t)next : kNone;
        } else if (arrived_upd || up) {
          e.x = wrlane((uint32_t)cur, tl, e.x);
          e.y = wrlane(arrived_upd ? (uint32_t)prev : kNone, tl, e.y);
          e.z = wrlane(up ? (uint32_t)next : kNone, tl, e.z);
        }
        tb = (int)wrlane((uint32_t)next, tl, (uint32_t)tb);
        clen += d;
        arrived_upd = up;
        prev = cur;
        cur = next;
      }
      c_retry += group_push<ATOMIC, true>(D, A, q, qw, qhead, qtail, qdirect, lane, e, t0, g1,
                                          hits, misses);
      g0 = g1;
    }
    len += clen;
    if (lane < tend - t0) D.tours[(size_t)ant * n + t0 + lane] = tb;
  }
  // closing edge (cur, start), always updated: cur's entry, then start's
  {
    const uint4 ce = lane == 0 ? make_uint4((uint32_t)cur, arrived_upd ? (uint32_t)prev : kNone,
                                            (uint32_t)start, 0u)
                               : make_uint4((uint32_t)start, nb_start, (uint32_t)cur, 0u);
    c_retry += group_push<ATOMIC, true>(D, A, q, qw, qhead, qtail, qdirect, lane, ce, n, n + 2,
                                        hits, misses);
    len += dist_xy(D, cur, start);
  }
  c_retry = (uint32_t)uni((int)wave_sum_u(c_retry));
  hits = (uint32_t)uni((int)wave_sum_u(hits));
  misses = (uint32_t)uni((int)wave_sum_u(misses));
  if (lane == 0) {
    D.lens[ant] = len;
    add_counters(D, (uint32_t)(n - 1) - c_roul - c_fb, c_roul, c_fb, c_fbu, c_retry);
    if (hits | misses) add_spm_counters(D, hits, misses);
  }
}

// One instance, selective memory, updates through the block's updater wave
// (waves 0..na-1 are ants, wave na applies their entries); LDS as in
// k_construct_async_dense_q.  S and L as in spm_ant_queued (the host picks
// them from s and cl).
template <bool ATOMIC, int S, int L>
__global__ __launch_bounds__(64 * (kQAnts + 1)) void k_construct_async_spm_q(Dev D, Iter A) {
  extern __shared__ uint4 qsm[];
  __shared__ uint32_t qhd[kQAnts], qtl[kQAnts], qdone;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int na = (int)(blockDim.x >> 6) - 1;
  if (threadIdx.x < kQAnts) {
    qhd[threadIdx.x] = 0;
    qtl[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) qdone = 0;
  __syncthreads();
  const QRing q{qsm, qhd, qtl, &qdone};
  if (wv == na) {
    ring_updater<ATOMIC, true>(D, A, q, lane, na);
    return;
  }
  uint32_t *vis = reinterpret_cast<uint32_t *>(qsm + (size_t)na * kQRing) +
                  wv * ((D.n + 31) >> 5);
  const int ant = uni(blockIdx.x * na + wv);
  if (ant < D.m) spm_ant_queued<ATOMIC, S, L>(D, A, ant, vis, lane, q, wv);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (lane == 0) atomicAdd(&qdone, 1u);
}

// ---------------------------------------------------------------------------
// Iteration best, best-so-far and the global update (Alg. 1, Eq. 4), one
// block.  Every directed entry of the best tour is touched exactly once, so
// plain read-modify-writes suffice.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void argmin_len(const Dev &D, int64_t &bl, int &ba) {
  __shared__ int64_t sl[16];
  __shared__ int sa[16];
  bl = INT64_MAX;
  ba = INT_MAX;
  for (int a = threadIdx.x; a < D.m; a += blockDim.x)
    if (D.lens[a] < bl) { bl = D.lens[a]; ba = a; }
#pragma unroll
  for (int off = 32; off; off >>= 1) {
    const int64_t ol = __shfl_xor(bl, off, 64);
    const int oa = __shfl_xor(ba, off, 64);
    if (ol < bl || (ol == bl && oa < ba)) { bl = ol; ba = oa; }
  }
  if ((threadIdx.x & 63) == 0) { sl[threadIdx.x >> 6] = bl; sa[threadIdx.x >> 6] = ba; }
  __syncthreads();
  bl = sl[0];
  ba = sa[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
    if (sl[w] < bl || (sl[w] == bl && sa[w] < ba)) { bl = sl[w]; ba = sa[w]; }
}

// ---------------------------------------------------------------------------
// Local search after the construction (the paper's further research asks
// how a local search heuristic such as 3-opt changes convergence): a
// first-improvement descent over 2-opt and Or-opt moves, each creating an
// edge from the examined city a to one of its candidates, with a FIFO queue
// of cities to examine.  For a popped city the moves are tried in a fixed
// order and the first that shortens the tour is applied:
//   1. 2-opt on a's successor b: candidates c (k ascending) while
//      d(a,c) < d(a,b), e = succ(c): (a,b),(c,e) -> (a,c),(b,e);
//   2. 2-opt on a's predecessor b: while d(a,c) < d(b,a), e = pred(c);
//   3. Or-opt, L = 1, 2, 3: the segment of a and the L - 1 cities after it,
//      p before it, x after it; per candidate c (k ascending): (A) the
//      segment between c and succ(c), a next to c; (B) reversed between
//      pred(c) and c;
//   4. (kind 2) 3-opt, the four reconnections that replace (a,b), (c,d) and
//      (e,f) of a [b..c] [d..e] f by three new edges (see ls_three_opt).
// The cities at the ends of the changed edges are then queued (in the order
// listed per move) unless queued already; at most 50 n moves are applied.
// A 2-opt move reverses the forward path between its two cities when that
// path holds at most half the cities, else the rest of the tour; an Or-opt
// move shifts the shorter of the blocks between the segment's old and new
// places by L positions and writes the segment into the gap.  One wave per
// tour, its lanes evaluate the candidates of a move kind at once and the
// lowest-order improving one is taken, which is the move a sequential scan
// in that order finds.  Tour, positions and queue live in LDS as 16-bit
// indices (n <= kLsMaxN); the queue flags are a bitmap.
// ---------------------------------------------------------------------------
struct LsTour {
  uint16_t *t, *pos, *q;
  uint32_t *inq;
  int n;
};

__device__ __forceinline__ int ls_wrap(int i, int n) { return ((i % n) + n) % n; }
__device__ __forceinline__ int ls_at(const LsTour &w, int i) { return w.t[ls_wrap(i, w.n)]; }
__device__ __forceinline__ void ls_put(const LsTour &w, int i, int c) {
  i = ls_wrap(i, w.n);
  w.t[i] = (uint16_t)c;
  w.pos[c] = (uint16_t)i;
}
__device__ __forceinline__ int ls_dist(const Dev &D, int u, int v) {
  return (int)D.dist[(size_t)u * D.ldn + v];
}

// queues city c (wave-uniform) unless it is queued; qh, qn wave-uniform
__device__ __forceinline__ void ls_push(const LsTour &w, int c, int qh, int &qn, int lane) {
  const uint32_t word = w.inq[c >> 5];
  if ((word >> (c & 31)) & 1u) return;
  if (lane == 0) {
    w.inq[c >> 5] = word | (1u << (c & 31));
    w.q[(qh + qn) % w.n] = (uint16_t)c;
  }
  ++qn;
}

// the forward path from city u to city v reversed, or the rest of the tour
__device__ __forceinline__ void ls_reverse(const LsTour &w, int u, int v, int lane) {
  const int n = w.n;
  int i = w.pos[u], j = w.pos[v];
  int len = (j - i + n) % n + 1;
  if (2 * len > n) {
    const int i2 = (j + 1) % n, j2 = (i - 1 + n) % n;
    i = i2;
    j = j2;
    len = n - len;
  }
  for (int s = lane; s < len / 2; s += 64) {
    const int a = ls_at(w, i + s), b = ls_at(w, j - s);
    ls_put(w, i + s, b);
    ls_put(w, j - s, a);
  }
}

// block move: positions from .. from + cnt - 1 to from + by .. (by = -L or
// +L), chunks of 64 ordered so no chunk reads what an earlier chunk wrote
__device__ __forceinline__ void ls_shift(const LsTour &w, int from, int cnt, int by, int lane) {
  if (by < 0) {
    for (int r0 = 0; r0 < cnt; r0 += 64) {
      const int r = r0 + lane;
      const int c = r < cnt ? ls_at(w, from + r) : 0;
      if (r < cnt) ls_put(w, from + r + by, c);
    }
  } else {
    for (int r0 = ((cnt - 1) / 64) * 64; r0 >= 0; r0 -= 64) {
      const int r = r0 + lane;
      const int c = r < cnt ? ls_at(w, from + r) : 0;
      if (r < cnt) ls_put(w, from + r + by, c);
    }
  }
}

// Or-opt: the L cities at positions i .. i + L - 1 (seg, in order) between
// c and succ(c) (side 0) or reversed between pred(c) and c (side 1)
__device__ __forceinline__ void ls_oropt(const LsTour &w, int i, int L, int c, int side,
                                         const int seg[3], int lane) {
  const int n = w.n;
  if (side == 0) {
    const int nb = (w.pos[c] - (i + L) % n + n) % n + 1, nc = n - L - nb;
    if (nb <= nc) {
      ls_shift(w, i + L, nb, -L, lane);
      if (lane < L) ls_put(w, i + nb + lane, seg[lane]);
    } else {
      const int e0 = (w.pos[c] + 1) % n;
      ls_shift(w, e0, nc, L, lane);
      if (lane < L) ls_put(w, e0 + lane, seg[lane]);
    }
  } else {
    const int c0 = w.pos[c];
    const int nc = (i - 1 - c0 + 2 * n) % n + 1, nb = n - L - nc;
    if (nc <= nb) {
      ls_shift(w, c0, nc, L, lane);
      if (lane < L) ls_put(w, c0 + lane, seg[L - 1 - lane]);
    } else {
      ls_shift(w, i + L, nb, -L, lane);
      if (lane < L) ls_put(w, i + nb + lane, seg[L - 1 - lane]);
    }
  }
}

// the cities at positions i .. j (forward, j reached from i) in reverse order
__device__ __forceinline__ void ls_reverse_at(const LsTour &w, int i, int j, int lane) {
  const int n = w.n;
  const int len = (j - i + n) % n + 1;
  for (int s = lane; s < len / 2; s += 64) {
    const int a = ls_at(w, i + s), b = ls_at(w, j - s);
    ls_put(w, i + s, b);
    ls_put(w, j - s, a);
  }
}

// 3-opt for the popped city a at position pa (local search kind 2): with
// b = succ(a), the tour a [B = b..c] [C = d..e] f becomes a C B, a C B',
// a C' B or a B' C' f (reconnections 0 to 3, tried in that order).  The
// first new edge joins a to a candidate x with d(a,x) < d(a,b), x = d, d, e,
// c for the four, in candidate order; the second joins b (c for C B') to one
// of its candidates y, in candidate order, while the partial gain stays
// positive.  The move a sequential scan finds is the lowest (reconnection,
// x, y).  The wave takes one x at a time with all four reconnections at once
// (their loads in one round, the lanes taking y), keeps the first improving
// move of the most preferred reconnection seen, and stops early once
// reconnection 0 has one.  Returns true if a move was applied.
__device__ __forceinline__ bool ls_three_opt(const Dev &D, const LsTour &w, int a, int pa,
                                          int64_t &len, int qh, int &qn, int lane) {
  const int n = w.n, cl = D.cl;
  const int kl = lane < cl ? lane : cl - 1;
  const bool cand = lane < cl;
  const int b = uni(ls_at(w, pa + 1));
  const int dab = ls_dist(D, a, b);
  const uint4 ra = D.crec[(size_t)a * cl + kl];
  const uint4 rb = D.crec[(size_t)b * cl + kl];
  // a's candidates closer than b: a prefix (the lists are sorted by distance)
  const uint64_t far = __ballot(lane >= cl || !((int)ra.y < dab));
  const int nx = far ? (int)__ffsll((unsigned long long)far) - 1 : 64;
  const int yb = (int)rb.x, dyb = (int)rb.y;  // b's candidates
  const int oyb = (w.pos[yb] - pa + n) % n;
  int best = 4, bod = 0, boe = 0, bc = 0, bd = 0, be = 0, bf = 0, bdelta = 0;
  for (int kx = 0; kx < nx && best > 0; ++kx) {
    const int x = (int)rdlane(ra.x, kx), dax = (int)rdlane(ra.y, kx);
    const int ox = (w.pos[x] - pa + n) % n;
    const int px = uni(ls_at(w, pa + ox - 1)), sx = uni(ls_at(w, pa + ox + 1));
    const int g01 = dab - dax + ls_dist(D, px, x);  // x = d: removed (c, d), c = pred(x)
    const int g23 = dab - dax + ls_dist(D, x, sx);  // x = e or c: removed (x, succ(x))
    const uint4 rc = D.crec[(size_t)px * cl + kl];  // candidates of c for C B'
    const int yc = (int)rc.x, dyc = (int)rc.y;
    const int oyc = (w.pos[yc] - pa + n) % n;
#pragma unroll
    for (int type = 0; type < 4; ++type) {
      if (type >= best) break;
      int od, oe;
      bool ok;
      if (type == 0) {
        od = ox, oe = oyb;
        ok = cand && dyb < g01 && ox >= 2 && oyb >= ox;
      } else if (type == 1) {
        od = ox, oe = oyc;
        ok = cand && dyc < g01 && ox >= 2 && oyc > ox;
      } else if (type == 2) {
        od = oyb, oe = ox;
        ok = cand && dyb < g23 && ox >= 3 && oyb >= 2 && oyb < ox;
      } else {
        od = ox + 1, oe = oyb;
        ok = cand && dyb < g23 && ox >= 2 && ox <= n - 3 && oyb > ox + 1;
      }
      const int c = ls_at(w, pa + od - 1), d = ls_at(w, pa + od);
      const int e = ls_at(w, pa + oe), f = ls_at(w, pa + oe + 1);
      const int removed = dab + ls_dist(D, c, d) + ls_dist(D, e, f);
      int added;
      if (type == 0) added = ls_dist(D, a, d) + ls_dist(D, e, b) + ls_dist(D, c, f);
      else if (type == 1) added = ls_dist(D, a, d) + ls_dist(D, c, e) + ls_dist(D, b, f);
      else if (type == 2) added = ls_dist(D, a, e) + ls_dist(D, b, d) + ls_dist(D, c, f);
      else added = ls_dist(D, a, c) + ls_dist(D, b, e) + ls_dist(D, d, f);
      const uint64_t imp = __ballot(ok && added - removed < 0);
      if (imp) {
        const int k = (int)__ffsll((unsigned long long)imp) - 1;
        best = type;
        bod = (int)rdlane((uint32_t)od, k), boe = (int)rdlane((uint32_t)oe, k);
        bc = (int)rdlane((uint32_t)c, k), bd = (int)rdlane((uint32_t)d, k);
        be = (int)rdlane((uint32_t)e, k), bf = (int)rdlane((uint32_t)f, k);
        bdelta = (int)rdlane((uint32_t)(added - removed), k);
      }
    }
  }
  if (best == 4) return false;
  len += bdelta;
  // positions pa + 1 .. pa + oe hold B (od - 1 cities) then C
  const int p0 = (pa + 1) % n, pe = (pa + boe) % n;
  const int nb = bod - 1, nc = boe - bod + 1;
  if (best == 3) {
    ls_reverse_at(w, p0, (p0 + nb - 1) % n, lane);
    ls_reverse_at(w, (p0 + nb) % n, pe, lane);
  } else {
    ls_reverse_at(w, p0, pe, lane);                                 // C' B'
    if (best <= 1) ls_reverse_at(w, p0, (p0 + nc - 1) % n, lane);   // C
    if (best != 1) ls_reverse_at(w, (p0 + nc) % n, pe, lane);       // B
  }
  ls_push(w, a, qh, qn, lane);
  ls_push(w, b, qh, qn, lane);
  ls_push(w, bc, qh, qn, lane);
  ls_push(w, bd, qh, qn, lane);
  ls_push(w, be, qh, qn, lane);
  ls_push(w, bf, qh, qn, lane);
  return true;
}

// One block (one wave) per ant.  Dynamic LDS: t, pos, q (n 16-bit entries
// each) and the queue bitmap.  kind 2 adds the 3-opt move.
__global__ __launch_bounds__(64) void k_local_search(Dev D, int kind) {
  extern __shared__ uint32_t lsm[];
  const int ant = blockIdx.x, lane = threadIdx.x, n = D.n, cl = D.cl;
  const int np2 = (n + 1) & ~1;  // 16-bit arrays padded to whole words
  LsTour w;
  w.t = reinterpret_cast<uint16_t *>(lsm);
  w.pos = w.t + np2;
  w.q = w.pos + np2;
  w.inq = reinterpret_cast<uint32_t *>(w.q + np2);
  w.n = n;
  const int W = (n + 31) >> 5;
  const int32_t *tour = D.tours + (size_t)ant * n;
  for (int p = lane; p < n; p += 64) {
    const int c = tour[p];
    w.t[p] = (uint16_t)c;
    w.pos[c] = (uint16_t)p;
    w.q[p] = (uint16_t)c;
  }
  for (int k = lane; k < W; k += 64) w.inq[k] = k < W - 1 || (n & 31) == 0 ? ~0u
                                                            : (1u << (n & 31)) - 1u;
  int qh = 0, qn = n;
  int64_t len = D.lens[ant];
  uint32_t moves = 0;
  const uint32_t cap = 50u * (uint32_t)n;
  const int kl = lane < cl ? lane : cl - 1;
  while (qn > 0 && moves < cap) {
    const int a = uni(w.q[qh]);
    qh = (qh + 1) % n;
    --qn;
    if (lane == 0) w.inq[a >> 5] &= ~(1u << (a & 31));
    const uint4 rec = D.crec[(size_t)a * cl + kl];
    const int c = (int)rec.x, dac = (int)rec.y;
    const bool cand = lane < cl;
    const int pa = w.pos[a];
    // moves 1 to 3 all read the tour as it stands, so their distances are
    // loaded together (one round of memory latency); the first improving
    // move in the order above is then applied
    const int bs = uni(ls_at(w, pa + 1)), bp = uni(ls_at(w, pa - 1));  // succ, pred of a
    const int pc = w.pos[c];
    const int e = ls_at(w, pc + 1), f = ls_at(w, pc - 1);  // succ, pred of c
    const int dab = ls_dist(D, a, bs), dba = ls_dist(D, bp, a);
    const int dbe = ls_dist(D, bs, e), dce = ls_dist(D, c, e);
    const int dbf = ls_dist(D, bp, f), dfc = ls_dist(D, f, c);
    const int off = (pc - pa + n) % n;
    int sl[3], xl[3], gl[3], dse[3], dfs[3];  // Or-opt, L = 1, 2, 3
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sl[i] = uni(ls_at(w, pa + i));      // the segment's last city
      xl[i] = uni(ls_at(w, pa + i + 1));  // the city after it
      gl[i] = dba + ls_dist(D, sl[i], xl[i]) - ls_dist(D, bp, xl[i]);
      dse[i] = ls_dist(D, sl[i], e);
      dfs[i] = ls_dist(D, f, sl[i]);
    }
    bool done = false;
    // 1. 2-opt on the successor
    {
      const bool ok = cand && dac < dab && c != bs && e != a;
      const int delta = dac + dbe - dab - dce;
      const uint64_t imp = __ballot(ok && delta < 0);
      if (imp) {
        const int k = (int)__ffsll((unsigned long long)imp) - 1;
        const int cc = (int)rdlane((uint32_t)c, k), ee = (int)rdlane((uint32_t)e, k);
        len += (int)rdlane((uint32_t)delta, k);
        ls_reverse(w, bs, cc, lane);
        ls_push(w, a, qh, qn, lane);
        ls_push(w, bs, qh, qn, lane);
        ls_push(w, cc, qh, qn, lane);
        ls_push(w, ee, qh, qn, lane);
        done = true;
      }
    }
    // 2. 2-opt on the predecessor
    if (!done) {
      const bool ok = cand && dac < dba && c != bp && f != a;
      const int delta = dac + dbf - dba - dfc;
      const uint64_t imp = __ballot(ok && delta < 0);
      if (imp) {
        const int k = (int)__ffsll((unsigned long long)imp) - 1;
        const int cc = (int)rdlane((uint32_t)c, k), ee = (int)rdlane((uint32_t)f, k);
        len += (int)rdlane((uint32_t)delta, k);
        ls_reverse(w, a, ee, lane);
        ls_push(w, a, qh, qn, lane);
        ls_push(w, bp, qh, qn, lane);
        ls_push(w, cc, qh, qn, lane);
        ls_push(w, ee, qh, qn, lane);
        done = true;
      }
    }
    // 3. Or-opt of the segment a .. (L cities)
    for (int L = 1; L <= 3 && !done; ++L) {
      if (n < L + 3) break;
      const int sL = sl[L - 1], x = xl[L - 1], g = gl[L - 1];
      const bool out = cand && off >= L;
      const bool okA = out && c != bp, okB = out && c != x;
      const int dA = dac + dse[L - 1] - dce - g;
      const int dB = dfs[L - 1] + dac - dfc - g;
      const uint64_t impA = __ballot(okA && dA < 0), impB = __ballot(okB && dB < 0);
      if (impA | impB) {
        const int k = (int)__ffsll((unsigned long long)(impA | impB)) - 1;
        const int side = ((impA >> k) & 1ull) ? 0 : 1;
        const int cc = (int)rdlane((uint32_t)c, k);
        const int ef = (int)rdlane((uint32_t)(side == 0 ? e : f), k);
        len += (int)rdlane((uint32_t)(side == 0 ? dA : dB), k);
        const int seg[3] = {sl[0], sl[1], sl[2]};
        ls_oropt(w, pa, L, cc, side, seg, lane);
        ls_push(w, bp, qh, qn, lane);
        ls_push(w, x, qh, qn, lane);
        ls_push(w, a, qh, qn, lane);
        ls_push(w, sL, qh, qn, lane);
        if (side == 0) {
          ls_push(w, cc, qh, qn, lane);
          ls_push(w, ef, qh, qn, lane);
        } else {
          ls_push(w, ef, qh, qn, lane);
          ls_push(w, cc, qh, qn, lane);
        }
        done = true;
      }
    }
    // 4. 3-opt
    if (!done && kind >= 2 && n >= 6) done = ls_three_opt(D, w, a, pa, len, qh, qn, lane);
    if (done) ++moves;
  }
  int32_t *out = D.tours + (size_t)ant * n;
  for (int p = lane; p < n; p += 64) out[p] = w.t[p];
  if (lane == 0) {
    D.lens[ant] = len;
    if (moves) atomicAdd(&D.counters[7], (unsigned long long)moves);
  }
}

__global__ __launch_bounds__(1024) void k_best(Dev D) {
  __shared__ int s_better;
  int64_t bl;
  int ba;
  argmin_len(D, bl, ba);
  if (threadIdx.x == 0) {
    const int64_t lgb = D.gstate[0];
    s_better = (lgb < 0 || bl < lgb) ? 1 : 0;
    D.gstate[0] = s_better ? bl : lgb;
    D.gstate[1] = bl;
    D.gstate[2] = ba;
  }
  __syncthreads();
  const int n = D.n;
  if (s_better)
    for (int p = threadIdx.x; p < n; p += blockDim.x) D.best[p] = D.tours[(size_t)ba * n + p];
}

// Eq. 4 on the best-so-far tour, dense memory: one wave per tour edge finds
// both candidate positions with one coalesced load of each row; the 2n
// directed entries are distinct, so plain read-modify-writes suffice.
__global__ __launch_bounds__(256) void k_global_dense(Dev D, Iter A) {
  const int lane = threadIdx.x & 63;
  const int p = uni(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int n = D.n;
  if (p >= n) return;
  const float ag = A.a_glob;
  const float bg = (float)(A.rho / (double)D.gstate[0]);
  const int u = D.best[p], v = D.best[p + 1 < n ? p + 1 : 0];
  const int ku = cand_pos(D, u, v, lane), kv = cand_pos(D, v, u, lane);
  if (lane < 2) {
    float *h = lane == 0 ? home(D, u, v, ku) : home(D, v, u, kv);
    *h = fmaf(ag, *h, bg);
  }
}

// Eq. 4 with the selective memory, in the order of the tour: edge p updates
// record u_p then record v_p.  City best[p] is touched by edges p-1 and p
// (edges 0 and n-1 for p = 0), so one wave per tour position applies its
// record's two updates in that order and no record is shared.
__global__ __launch_bounds__(256) void k_global_spm(Dev D, Iter A) {
  const int lane = threadIdx.x & 63;
  const int p = uni(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int n = D.n, s = D.spm_s;
  if (p >= n) return;
  const float ag = A.a_glob;
  const float bg = (float)(A.rho / (double)D.gstate[0]);
  const int r = D.best[p];
  const int nb1 = p >= 1 ? D.best[p - 1] : D.best[1];
  const int nb2 = p >= 1 ? D.best[p + 1 < n ? p + 1 : 0] : D.best[n - 1];
  uint2 pr = spm_record<false>(D, r, lane);
  uint32_t tail = D.spm_tail[r];
  uint32_t hits = 0, misses = 0;
  spm_update_wave(pr, tail, s, lane, nb1, ag, bg, A.tau0, hits, misses);
  spm_update_wave(pr, tail, s, lane, nb2, ag, bg, A.tau0, hits, misses);
  if (lane < s) D.spm[(size_t)r * s + lane] = pr;
  if (lane == 0) {
    D.spm_tail[r] = tail;
    add_spm_counters(D, hits, misses);
  }
}

// Batched iteration end: block b handles instance b (iteration best and
// best-so-far), then advances that instance's iteration counter and moves
// its error flag (an exhausted bounded wait) into the batch's flag.
__global__ __launch_bounds__(1024) void k_best_batch(const Dev *devs, Iter *iters,
                                                     uint32_t *flag) {
  __shared__ int s_better;
  const Dev D = devs[blockIdx.x];
  int64_t bl;
  int ba;
  argmin_len(D, bl, ba);
  if (threadIdx.x == 0) {
    const uint32_t f = atomicExch(D.sync + 1, 0u);
    if (f) atomicOr(flag, f);
    const int64_t lgb = D.gstate[0];
    s_better = (lgb < 0 || bl < lgb) ? 1 : 0;
    D.gstate[0] = s_better ? bl : lgb;
    D.gstate[1] = bl;
    D.gstate[2] = ba;
    iters[blockIdx.x].it += 1;
  }
  __syncthreads();
  const int n = D.n;
  if (s_better)
    for (int p = threadIdx.x; p < n; p += blockDim.x) D.best[p] = D.tours[(size_t)ba * n + p];
}

// Batched global update (dense): grid (edges / 256, instances).
__global__ __launch_bounds__(256) void k_global_batch(const Dev *devs, const Iter *iters) {
  const Dev D = devs[blockIdx.y];
  const Iter A = iters[blockIdx.y];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = D.n;
  if (p >= n) return;
  const float ag = A.a_glob;
  const float bg = (float)(A.rho / (double)D.gstate[0]);
  const int u = D.best[p], v = D.best[p + 1 < n ? p + 1 : 0];
  int ku = -1, kv = -1;
  for (int k = 0; k < D.cl; ++k) {
    if (D.crec[(size_t)u * D.cl + k].x == (uint32_t)v) ku = k;
    if (D.crec[(size_t)v * D.cl + k].x == (uint32_t)u) kv = k;
  }
  float *h1 = home(D, u, v, ku);
  float *h2 = home(D, v, u, kv);
  *h1 = fmaf(ag, *h1, bg);
  *h2 = fmaf(ag, *h2, bg);
}

// Best-so-far exchange between the colonies of a batch that all solve one
// instance (the multi-colony model of the paper's Sec. 2: periodic exchange
// of the best solution found so far along a communication topology).  Every
// colony first offers its best-so-far tour and length (block per colony);
// then every colony takes its source's offer when it is strictly shorter
// than its own: topology 0, the source is the colony with the shortest
// offer (lowest index among equals); topology 1, colony c - 1 (a ring).
// Reading every offer before any colony changes keeps the exchange
// independent of the order the blocks run in.
__global__ __launch_bounds__(256) void k_offer_batch(const Dev *devs, int n, int32_t *offer,
                                                     int64_t *olen) {
  const Dev D = devs[blockIdx.x];
  for (int p = threadIdx.x; p < n; p += blockDim.x) offer[(size_t)blockIdx.x * n + p] = D.best[p];
  if (threadIdx.x == 0) olen[blockIdx.x] = D.gstate[0];
}

__global__ __launch_bounds__(256) void k_accept_batch(const Dev *devs, int count, int n,
                                                      int topology, const int32_t *offer,
                                                      const int64_t *olen) {
  const int c = blockIdx.x;
  int src = (c + count - 1) % count;
  if (topology == 0) {
    src = -1;
    for (int i = 0; i < count; ++i)
      if (olen[i] >= 0 && (src < 0 || olen[i] < olen[src])) src = i;
  }
  if (src < 0 || olen[src] < 0) return;
  const Dev D = devs[c];
  const int64_t own = olen[c];
  if (own >= 0 && olen[src] >= own) return;
  for (int p = threadIdx.x; p < n; p += blockDim.x) D.best[p] = offer[(size_t)src * n + p];
  if (threadIdx.x == 0) D.gstate[0] = olen[src];
}

size_t lds_bytes(const Dev &D, int block) {
  return (size_t)(block / 64) * ((D.n + 31) / 32) * sizeof(uint32_t);
}

constexpr int kSyncBlock = 1024;
// the host sizes the barrier flags (Dev::bflags) for 16 ants per block
static_assert(kSyncBlock == 64 * 16, "one synchronous block holds 16 ants");
constexpr int kAsyncBlock = 256;

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers.
// ---------------------------------------------------------------------------
hipError_t launch_dist(const Dev &d, uint32_t *dmax, int r0, int rows, bool store,
                       hipStream_t s) {
  dim3 grid((d.ldn + 63) / 64, (rows + 3) / 4);
  hipLaunchKernelGGL(k_dist, grid, dim3(256), 0, s, d, dmax, r0, rows, store ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_grid_box(const Dev &d, double *box, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_box, dim3(1), dim3(1024), 0, s, d, box);
  return hipGetLastError();
}

hipError_t launch_grid(const Dev &d, int32_t *cnt, hipStream_t s) {
  const size_t cells = (size_t)d.gnx * d.gny;
  hipError_t e = hipMemsetAsync(cnt, 0, cells * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  const dim3 g((d.n + 255) / 256);
  hipLaunchKernelGGL(k_grid_count, g, dim3(256), 0, s, d, cnt);
  hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, s, d, cnt);
  hipLaunchKernelGGL(k_grid_fill, g, dim3(256), 0, s, d, cnt);
  return hipGetLastError();
}

hipError_t launch_cand(const Dev &d, int32_t *cand_tmp, int r0, int rows, hipStream_t s) {
  hipLaunchKernelGGL(k_cand, dim3((rows + 3) / 4), dim3(256), 0, s, d, cand_tmp, r0, rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !d.xnn) return e;
  hipLaunchKernelGGL(k_xnn, dim3((rows + 3) / 4), dim3(256), 0, s, d, r0, rows);
  return hipGetLastError();
}

hipError_t launch_nn_tour(const Dev &d, int64_t *lnn_out, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_tour, dim3(1), dim3(1024), 0, s, d, lnn_out);
  return hipGetLastError();
}

hipError_t launch_crec(const Dev &d, const int32_t *cand_tmp, float tau0, hipStream_t s) {
  const int total = d.n * d.cl;
  hipLaunchKernelGGL(k_crec, dim3((total + 255) / 256), dim3(256), 0, s, d, cand_tmp, tau0);
  return hipGetLastError();
}

hipError_t launch_init_pheromone(const Dev &d, float tau0, hipStream_t s) {
  if (d.fpre) {
    hipLaunchKernelGGL(k_fpre, dim3((d.n + 3) / 4), dim3(256), 0, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (d.rpos) {
    hipLaunchKernelGGL(k_rpos, dim3((d.n * d.cl + 255) / 256), dim3(256), 0, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (d.etad) {
    const size_t total = (size_t)d.n * d.ldn;
    hipLaunchKernelGGL(k_etad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  size_t total = d.tau ? (size_t)d.n * d.ldn : (size_t)d.n;
  if (d.spm && total < (size_t)d.n * d.spm_s) total = (size_t)d.n * d.spm_s;
  if (total < 8) total = 8;
  if (total < (size_t)d.nbflags) total = (size_t)d.nbflags;
  hipLaunchKernelGGL(k_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, tau0);
  return hipGetLastError();
}

// Ant waves per block of the kernels with an updater wave: the m ants spread
// evenly over the compute units, two or more blocks per unit, at most
// kQAnts per block.
static hipError_t queued_ants_per_block(int m, int *na) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  const int per_cu = (m + cus - 1) / cus;
  const int bpc = std::max(2, (per_cu + kQAnts - 1) / kQAnts);
  *na = std::max(1, std::min(kQAnts, (m + cus * bpc - 1) / (cus * bpc)));
  return hipSuccess;
}

hipError_t launch_construct(const Dev &d, const Iter &it, int mode, int memory, int lanes,
                            int queued, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  // ev0 / ev1 (optional) bracket the construction kernel itself, so that
  // their interval leaves out the bound, buffer and copy kernels beside it
  auto mark = [s](hipEvent_t e) { return e ? hipEventRecord(e, s) : hipSuccess; };
  // the fallback prefix's bound holds where every update maps an entry's own
  // value or a value its edge's other entry held from an equal start; the
  // unsynchronised ants that issue their own updates write f(forward value)
  // into a reverse entry that may differ from it, so they scan whole rows
  const bool queued_dense = memory == 0 && lanes == 64 && queued && (mode == 1 || mode == 2);
  const bool far = memory == 0 && d.fpre && (mode != 2 || (lanes == 64 && queued));
  if (far) {
    hipLaunchKernelGGL(k_far_bound, dim3((d.n + 3) / 4), dim3(256), 0, s, d, it,
                       queued_dense ? 1 : 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (mode == 3) {
    const size_t words = (size_t)d.m * ((d.n + 31) / 32);
    const hipError_t me = mark(ev0);
    if (me != hipSuccess) return me;
    if (words <= (size_t)kSeqLdsWords)
      hipLaunchKernelGGL(k_construct_seq_dense<true>, dim3(1), dim3(64 * kSeqWaves),
                         words * sizeof(uint32_t), s, d, it);
    else
      hipLaunchKernelGGL(k_construct_seq_dense<false>, dim3(1), dim3(64 * kSeqWaves), 0, s, d,
                         it);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : mark(ev1);
  }
  if (mode == 0) {
    const int apb = kSyncBlock / 64;
    const int grid = (d.m + apb - 1) / apb;
    Dev dd = d;
    Iter a = it;
    void *args[] = {&dd, &a};
    const void *fn = memory == 0 ? reinterpret_cast<const void *>(&k_construct_sync_dense)
                                 : reinterpret_cast<const void *>(&k_construct_sync_spm);
    const bool dbuf = memory == 0 && it.lperiod == 1;
    const dim3 gb((unsigned)(((size_t)d.n * d.ldn + 255) / 256));
    if (dbuf) {
      hipLaunchKernelGGL(k_sync_buf, gb, dim3(256), 0, s, d, 0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const hipError_t me = mark(ev0);
    if (me != hipSuccess) return me;
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kSyncBlock), args,
                                              lds_bytes(d, kSyncBlock), s);
    if (e == hipSuccess) e = mark(ev1);
    if (e != hipSuccess || !dbuf || (d.n & 1) == 0) return e;
    hipLaunchKernelGGL(k_sync_buf, gb, dim3(256), 0, s, d, 1);
    return hipGetLastError();
  }
  const int apb = kAsyncBlock / 64;
  const int grid = (d.m + apb - 1) / apb;
  const size_t lds = lds_bytes(d, kAsyncBlock);
  const bool atomic = mode == 1;
  if (memory == 0 && lanes == 64 && queued) {
    int na = 0;
    const hipError_t qe = queued_ants_per_block(d.m, &na);
    if (qe != hipSuccess) return qe;
    const dim3 gq((d.m + na - 1) / na), bq(64 * (na + 1));
    const size_t lq = (size_t)na * kQRing * sizeof(uint4) +
                      (size_t)na * ((d.n + 31) / 32) * sizeof(uint32_t);
    const bool half = d.cl <= 32;
    const dim3 gc((d.n * d.cl + 255) / 256);
    if (!far) hipLaunchKernelGGL(k_ctau_in, gc, dim3(256), 0, s, d);
    const hipError_t me = mark(ev0);
    if (me != hipSuccess) return me;
    const bool every = it.lperiod == 1;
#define ACS_DENSE_Q(AT, HF, EV)                                                        \
    if (atomic == AT && half == HF && every == EV)                                      \
      hipLaunchKernelGGL((k_construct_async_dense_q<AT, HF, EV>), gq, bq, lq, s, d, it);
    ACS_DENSE_Q(true, true, true)
    ACS_DENSE_Q(true, true, false)
    ACS_DENSE_Q(true, false, true)
    ACS_DENSE_Q(true, false, false)
    ACS_DENSE_Q(false, true, true)
    ACS_DENSE_Q(false, true, false)
    ACS_DENSE_Q(false, false, true)
    ACS_DENSE_Q(false, false, false)
#undef ACS_DENSE_Q
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = mark(ev1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ctau_out, gc, dim3(256), 0, s, d, atomic ? 1 : 0);
    return hipGetLastError();
  }
  const hipError_t me = mark(ev0);
  if (me != hipSuccess) return me;
  if (memory == 0 && lanes < 64) {
    const int g = 64 / lanes;
    const dim3 gg((d.m + apb * g - 1) / (apb * g));
    const size_t lg = lds * g;
    Dev dr = d;
    dr.fpre = nullptr;
    if (lanes == 32 && atomic)
      hipLaunchKernelGGL((k_construct_async_dense_g<32, true>), gg, dim3(kAsyncBlock), lg, s, d, it);
    else if (lanes == 32)
      hipLaunchKernelGGL((k_construct_async_dense_g<32, false>), gg, dim3(kAsyncBlock), lg, s, dr, it);
    else if (atomic)
      hipLaunchKernelGGL((k_construct_async_dense_g<16, true>), gg, dim3(kAsyncBlock), lg, s, d, it);
    else
      hipLaunchKernelGGL((k_construct_async_dense_g<16, false>), gg, dim3(kAsyncBlock), lg, s, dr, it);
  } else if (memory == 0) {
    if (atomic) {
      hipLaunchKernelGGL(k_construct_async_dense<true>, dim3(grid), dim3(kAsyncBlock), lds, s, d,
                         it);
    } else {
      Dev dd = d;
      dd.fpre = nullptr;
      hipLaunchKernelGGL(k_construct_async_dense<false>, dim3(grid), dim3(kAsyncBlock), lds, s,
                         dd, it);
    }
  } else if (queued) {
    int na = 0;
    const hipError_t e = queued_ants_per_block(d.m, &na);
    if (e != hipSuccess) return e;
    const dim3 gq((d.m + na - 1) / na), bq(64 * (na + 1));
    const size_t lq = (size_t)na * kQRing * sizeof(uint4) +
                      (size_t)na * ((d.n + 31) / 32) * sizeof(uint32_t);
    // the common shapes get kernels with s and the candidate lanes fixed
    const int sk = d.spm_s == 8 ? 8 : 0;
    const int lk = sk == 0 ? 64 : d.cl <= 16 ? 16 : d.cl <= 32 ? 32 : 64;
#define ACS_SPM_Q(AT, SS, LL) \
    if (atomic == AT && sk == SS && lk == LL) \
      hipLaunchKernelGGL((k_construct_async_spm_q<AT, SS, LL>), gq, bq, lq, s, d, it);
    ACS_SPM_Q(true, 8, 16)
    ACS_SPM_Q(true, 8, 32)
    ACS_SPM_Q(true, 8, 64)
    ACS_SPM_Q(true, 0, 64)
    ACS_SPM_Q(false, 8, 16)
    ACS_SPM_Q(false, 8, 32)
    ACS_SPM_Q(false, 8, 64)
    ACS_SPM_Q(false, 0, 64)
#undef ACS_SPM_Q
  } else {
    if (atomic)
      hipLaunchKernelGGL(k_construct_async_spm<true>, dim3(grid), dim3(kAsyncBlock), lds, s, d,
                         it);
    else
      hipLaunchKernelGGL(k_construct_async_spm<false>, dim3(grid), dim3(kAsyncBlock), lds, s, d,
                         it);
  }
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : mark(ev1);
}

int max_sync_ants(const Dev &d, int memory) {
  int per_cu = 0;
  const void *fn = memory == 0 ? reinterpret_cast<const void *>(&k_construct_sync_dense)
                               : reinterpret_cast<const void *>(&k_construct_sync_spm);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSyncBlock,
                                                   lds_bytes(d, kSyncBlock)) != hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus * (kSyncBlock / 64);
}

hipError_t launch_local_search(const Dev &d, int kind, hipStream_t s) {
  const int np2 = (d.n + 1) & ~1;
  const size_t lds = (size_t)3 * np2 * sizeof(uint16_t) + (size_t)((d.n + 31) / 32) * 4;
  hipLaunchKernelGGL(k_local_search, dim3(d.m), dim3(64), lds, s, d, kind);
  return hipGetLastError();
}

hipError_t launch_best_global(const Dev &d, const Iter &it, int memory, hipStream_t s) {
  hipLaunchKernelGGL(k_best, dim3(1), dim3(1024), 0, s, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (memory == 0)
    hipLaunchKernelGGL(k_global_dense, dim3((d.n + 3) / 4), dim3(256), 0, s, d, it);
  else
    hipLaunchKernelGGL(k_global_spm, dim3((d.n + 3) / 4), dim3(256), 0, s, d, it);
  return hipGetLastError();
}

hipError_t launch_exchange_batch(const Dev *devs, int count, int n, int topology,
                                 int32_t *offer, int64_t *olen, hipStream_t s) {
  hipLaunchKernelGGL(k_offer_batch, dim3(count), dim3(256), 0, s, devs, n, offer, olen);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_accept_batch, dim3(count), dim3(256), 0, s, devs, count, n, topology,
                     offer, olen);
  return hipGetLastError();
}

hipError_t launch_batch_iteration(const Dev *devs, Iter *iters, const int2 *items, int nitems,
                                  int count, int nmax, int clmax, int mode, int lanes, int queued,
                                  uint32_t *flag, hipStream_t s) {
  const int apb = kAsyncBlock / 64;
  const int wmax = (nmax + 31) / 32;
  if (mode == 1) {
    // instances without a prefix (and the unsynchronised mode, see
    // launch_construct) have fpre null and scan whole rows
    hipLaunchKernelGGL(k_far_bound_batch, dim3((nmax + 3) / 4, count), dim3(256), 0, s, devs,
                       iters);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (lanes == 64 && queued) {
    const size_t lq = (size_t)kBatchQAnts * kQRing * sizeof(uint4) +
                      (size_t)kBatchQAnts * wmax * sizeof(uint32_t);
    const dim3 gq(nitems), bq(64 * (kBatchQAnts + 1));
    const bool half = clmax <= 32;
    const dim3 gc((nmax * clmax + 255) / 256, count);
    hipLaunchKernelGGL(k_ctau_in_batch, gc, dim3(256), 0, s, devs);
    if (mode == 1 && half)
      hipLaunchKernelGGL((k_construct_async_batch_q<true, true>), gq, bq, lq, s, devs, iters,
                         items, nitems, wmax);
    else if (mode == 1)
      hipLaunchKernelGGL((k_construct_async_batch_q<true, false>), gq, bq, lq, s, devs, iters,
                         items, nitems, wmax);
    else if (half)
      hipLaunchKernelGGL((k_construct_async_batch_q<false, true>), gq, bq, lq, s, devs, iters,
                         items, nitems, wmax);
    else
      hipLaunchKernelGGL((k_construct_async_batch_q<false, false>), gq, bq, lq, s, devs, iters,
                         items, nitems, wmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ctau_out_batch, gc, dim3(256), 0, s, devs, mode == 1 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_best_batch, dim3(count), dim3(1024), 0, s, devs, iters, flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_global_batch, dim3((nmax + 255) / 256, count), dim3(256), 0, s, devs,
                       iters);
    return hipGetLastError();
  }
  const size_t lds = (size_t)apb * (64 / lanes) * wmax * sizeof(uint32_t);
  const dim3 grid((nitems + apb - 1) / apb), blk(kAsyncBlock);
  const bool atomic = mode == 1;
  if (lanes == 64 && atomic)
    hipLaunchKernelGGL(k_construct_async_batch<true>, grid, blk, lds, s, devs, iters, items,
                       nitems, wmax);
  else if (lanes == 64)
    hipLaunchKernelGGL(k_construct_async_batch<false>, grid, blk, lds, s, devs, iters, items,
                       nitems, wmax);
  else if (lanes == 32 && atomic)
    hipLaunchKernelGGL((k_construct_async_batch_g<32, true>), grid, blk, lds, s, devs, iters,
                       items, nitems, wmax);
  else if (lanes == 32)
    hipLaunchKernelGGL((k_construct_async_batch_g<32, false>), grid, blk, lds, s, devs, iters,
                       items, nitems, wmax);
  else if (atomic)
    hipLaunchKernelGGL((k_construct_async_batch_g<16, true>), grid, blk, lds, s, devs, iters,
                       items, nitems, wmax);
  else
    hipLaunchKernelGGL((k_construct_async_batch_g<16, false>), grid, blk, lds, s, devs, iters,
                       items, nitems, wmax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_best_batch, dim3(count), dim3(1024), 0, s, devs, iters, flag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_global_batch, dim3((nmax + 255) / 256, count), dim3(256), 0, s, devs,
                     iters);
  return hipGetLastError();
}

}  // namespace acs
