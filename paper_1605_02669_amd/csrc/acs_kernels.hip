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

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, k);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pheromone slot of candidate k in city u's record.
__device__ __forceinline__ float *cand_tau(const Dev &D, int u, int k) {
  return reinterpret_cast<float *>(const_cast<uint4 *>(D.crec) + (size_t)u * D.cl + k) + 3;
}

// Home of the directed entry (u, v): candidate slot k of u, or tau[u][v].
__device__ __forceinline__ float *home(const Dev &D, int u, int v, int k) {
  return k >= 0 ? cand_tau(D, u, k) : D.tau + (size_t)u * D.ldn + v;
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

// Position of v in the candidate list of u (wave-uniform), or -1.
__device__ __forceinline__ int cand_pos(const Dev &D, int u, int v, int lane) {
  const int kl = lane < D.cl ? lane : D.cl - 1;
  const uint32_t j = D.crec[(size_t)u * D.cl + kl].x;
  const uint64_t b = __ballot(lane < D.cl && j == (uint32_t)v);
  return b ? (int)__ffsll((unsigned long long)b) - 1 : -1;
}

// Grid-wide barrier for a cooperative launch.  Every wave waits for its own
// memory operations first (the local updates are compare-and-swaps whose
// results have been consumed, so they are performed at the device's
// coherence point); one thread per block then arrives on a monotonically
// growing counter and waits for all blocks.  Readers after the barrier use
// agent-coherent loads for everything the updates touch, so no cache
// write-back or invalidation is needed.  The wait is bounded: on exhaustion
// an error flag is raised, later barriers no longer wait, and the kernel
// runs to its end.
__device__ __forceinline__ void grid_barrier(uint32_t *sync, uint32_t target) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while (__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      // once any block has given up, no later barrier waits either
      if (__hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 22)) {
        __hip_atomic_store(sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
__global__ __launch_bounds__(256) void k_dist(Dev D, uint32_t *dmax) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  uint32_t d = 0;
  if (i < D.n && j < D.n && i != j)
    d = exact_dist(D.xy[2 * i], D.xy[2 * i + 1], D.xy[2 * j], D.xy[2 * j + 1]);
  const uint32_t wmax = wave_max(d);
  if ((threadIdx.x & 63) == 0 && wmax) atomicMax(dmax, wmax);
  if (i < D.n && j < D.ldn) const_cast<uint16_t *>(D.dist)[(size_t)i * D.ldn + j] =
      (uint16_t)(d > 65535u ? 65535u : d);
}

// Candidate list of city i: its cl nearest neighbours by (d, j), one wave
// per city, extracted in increasing order of the key (d << 16 | j).
__global__ __launch_bounds__(256) void k_cand(Dev D, int32_t *cand) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= D.n) return;
  const uint16_t *row = D.dist + (size_t)i * D.ldn;
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
  int cur = 0;
  int64_t L = 0;
  for (int step = 1; step < D.n; ++step) {
    __syncthreads();
    const uint16_t *row = D.dist + (size_t)cur * D.ldn;
    int64_t best = INT64_MAX;
    for (int j = tid; j < D.n; j += 1024)
      if (!((vis[j >> 5] >> (j & 31)) & 1u)) {
        const int64_t key = ((int64_t)row[j] << 16) | j;
        best = key < best ? key : best;
      }
    best = wave_min(best);
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    best = red[0];
    for (int w = 1; w < 16; ++w) best = red[w] < best ? red[w] : best;
    const int nxt = (int)(best & 0xffff);
    L += best >> 16;
    if (tid == 0) vis[nxt >> 5] |= 1u << (nxt & 31);
    cur = nxt;
  }
  if (tid == 0) *lnn = L + D.dist[(size_t)cur * D.ldn];
}

// Candidate records with the initial pheromone tau0 in the last word.
__global__ __launch_bounds__(256) void k_crec(Dev D, const int32_t *cand, float tau0) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D.n * D.cl) return;
  const int i = e / D.cl;
  const uint32_t c = (uint32_t)cand[e];
  const uint32_t d = D.dist[(size_t)i * D.ldn + c];
  const_cast<uint4 *>(D.crec)[e] =
      make_uint4(c, d, __float_as_uint(D.eta_tab[d]), __float_as_uint(tau0));
}

__global__ __launch_bounds__(256) void k_init(Dev D, float tau0) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nd = (size_t)D.n * D.ldn;
  if (D.tau && e < nd) D.tau[e] = tau0;
  if (D.spm_node && e < (size_t)D.n * D.spm_s) {
    D.spm_node[e] = -1;
    D.spm_val[e] = tau0;
  }
  if (D.spm_tail && e < (size_t)D.n) D.spm_tail[e] = D.spm_s - 1;
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

template <bool COHERENT>
__device__ __forceinline__ Pick select_dense(const Dev &D, const Iter &A, const uint32_t *vis,
                                             int cur, int lane, uint4 rec, Cand c, uint2 q) {
  const int n = D.n, cl = D.cl;
  const bool unv = c.unv;
  const float w = c.w;
  const uint64_t umask = __ballot(unv);
  Pick p;
  if (umask) {
    int k;
    if (q.x < A.q0_24) {
      // Eq. 1, exploitation: maximum of tau * eta^beta, lowest position
      const uint32_t mx = wave_umax_u(__float_as_uint(w));
      const uint64_t sel = __ballot(unv && __float_as_uint(w) == mx);
      k = (int)__ffsll((unsigned long long)sel) - 1;
      p.kind = 0;
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
      p.kind = 1;
    }
    k = uni(k);
    p.k = k;
    p.next = (int)rdlane(rec.x, k);
    p.d = rdlane(rec.y, k);
    p.tval = __uint_as_float(rdlane(rec.w, k));
    return p;
  }
  // Alg. 2, empty candidate set: greedy over every unvisited city, ties ->
  // lowest index.  Each lane scans four consecutive cities per round.
  const float *trow = D.tau + (size_t)cur * D.ldn;
  const uint16_t *drow = D.dist + (size_t)cur * D.ldn;
  float bv = 0.f, bt = 0.f;
  uint32_t bj = kNone, bd = 0;
  for (int j0 = 4 * lane; j0 < n; j0 += 256) {
    uint32_t bits = (vis[j0 >> 5] >> (j0 & 31)) & 0xfu;
    if (j0 + 4 > n) bits |= (0xfu << (n - j0)) & 0xfu;
    if (bits != 0xfu) {
      float tq[4];
      if (COHERENT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) tq[q] = tau_load(trow + j0 + q);
      } else {
        const float4 tv = *reinterpret_cast<const float4 *>(trow + j0);
        tq[0] = tv.x; tq[1] = tv.y; tq[2] = tv.z; tq[3] = tv.w;
      }
      const ushort4 dv = *reinterpret_cast<const ushort4 *>(drow + j0);
      const uint32_t dq[4] = {dv.x, dv.y, dv.z, dv.w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (!((bits >> q) & 1u)) {
          const float v = tq[q] * D.eta_tab[dq[q]];
          if (bj == kNone || v > bv) { bv = v; bj = (uint32_t)(j0 + q); bt = tq[q]; bd = dq[q]; }
        }
    }
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
// ---------------------------------------------------------------------------
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
  for (int t = 1; t < n; ++t) {
    Pick p{};
    if ((t & 63) == 0) draws = philox_batch(A, ant, t, lane);
    if (active) {
      uint4 rec = D.crec[(size_t)cur * cl + kl];
      rec.w = __float_as_uint(tau_load(cand_tau(D, cur, kl)));
      const Cand c = weigh(D, vis, lane, rec);
      p = select_dense<true>(D, A, vis, cur, lane, rec, c, draw_of(draws, t));
      c_greedy += p.kind == 0;
      c_roul += p.kind == 1;
      if (p.kind == 2) { ++c_fb; c_fbu += (uint64_t)(n - t); }
      if (lane == 0) vis[p.next >> 5] |= 1u << (p.next & 31);
      tour_put(D, ant, t, lane, p.next, tb);
      len += p.d;
    }
    grid_barrier(D.sync, (++bar) * gridDim.x);
    if (active) {
      const int k2 = cand_pos(D, p.next, cur, lane);
      float *h = lane == 0 ? home(D, cur, p.next, p.k) : home(D, p.next, cur, k2);
      if (lane < 2) c_retry += cas_apply(h, __float_as_uint(p.tval), A.a_loc, A.b_loc);
      cur = p.next;
    }
    if (t + 1 < n) grid_barrier(D.sync, (++bar) * gridDim.x);
  }
  if (active) {
    // closing edge: its length and, as the last step's crossings, its update
    len += D.dist[(size_t)cur * D.ldn + start];
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    float *h = lane == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (lane < 2) {
      const float seen = tau_load(h);
      c_retry += cas_apply(h, __float_as_uint(seen), A.a_loc, A.b_loc);
    }
    c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1)));
    if (lane == 0) {
      D.lens[ant] = len;
      add_counters(D, c_greedy, c_roul, c_fb, c_fbu, c_retry);
    }
  }
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
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_construct_async_dense(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ant = uni(blockIdx.x * (blockDim.x >> 6) + wv);
  if (ant >= D.m) return;  // the whole wave leaves; no block-level sync below
  const int n = D.n, cl = D.cl, ldn = D.ldn;
  const int W = (n + 31) >> 5;
  const int kl = lane < cl ? lane : cl - 1;
  uint32_t *vis = smem + wv * W;
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
  uint32_t c_greedy = 0, c_roul = 0, c_fb = 0, c_retry = 0;
  uint64_t c_fbu = 0;
  // compare-and-swap in flight on lanes 0 (forward) and 1 (reverse)
  float *pptr = nullptr;
  unsigned int pexp = 0, pret = 0;
  bool pend = false;

  for (int t = 1; t <= n; ++t) {
    // 1. the record of cur is needed now; so are last step's CAS results
    if (pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
    pend = false;
    const Cand c = weigh(D, vis, lane, rec);
    // the weights are complete here, before the updates below are issued, so
    // no later wait for this record also waits for those updates
    __asm__ volatile("" ::"v"(c.w), "v"((int)c.unv));
    // 2. updates of the previous move (prev, cur)
    if (t > 1) {
      const uint64_t b = __ballot(lane < cl && rec.x == (uint32_t)prev);
      const int kr = b ? uni((int)__ffsll((unsigned long long)b) - 1) : -1;
      const float rval = kr >= 0 ? __uint_as_float(rdlane(rec.w, kr)) : fval;
      if (lane == 0) {
        pptr = fwd;
        pexp = __float_as_uint(fval);
        pend = true;
      } else if (lane == 1) {
        pptr = home(D, cur, prev, kr);
        pexp = __float_as_uint(rval);
        pend = true;
      }
      if (pend)
        pret = atomicCAS(reinterpret_cast<unsigned int *>(pptr), pexp,
                         __float_as_uint(fmaf(al, __uint_as_float(pexp), bl)));
    }
    if (t == n) break;
    // 3. selection
    if ((t & 63) == 0) draws = philox_batch(A, ant, t, lane);
    const Pick p = select_dense<false>(D, A, vis, cur, lane, rec, c, draw_of(draws, t));
    c_greedy += p.kind == 0;
    c_roul += p.kind == 1;
    if (p.kind == 2) { ++c_fb; c_fbu += (uint64_t)(n - t); }
    if (lane == 0) vis[p.next >> 5] |= 1u << (p.next & 31);
    tour_put(D, ant, t, lane, p.next, tb);
    len += p.d;
    // 4. record of the next city
    rec = D.crec[(size_t)p.next * cl + kl];
    fwd = home(D, cur, p.next, p.k);
    fval = p.tval;
    prev = cur;
    cur = p.next;
  }
  if (pend && pret != pexp) c_retry += 1 + cas_apply(pptr, pret, al, bl);
  // closing edge: both entries, read fresh (once per ant)
  {
    const int k1 = cand_pos(D, cur, start, lane);
    const int k2 = cand_pos(D, start, cur, lane);
    float *h = lane == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (lane < 2) c_retry += cas_apply(h, __float_as_uint(tau_load(h)), al, bl);
  }
  len += D.dist[(size_t)cur * ldn + start];
  c_retry = (uint32_t)uni((int)(rdlane(c_retry, 0) + rdlane(c_retry, 1)));
  if (lane == 0) {
    D.lens[ant] = len;
    add_counters(D, c_greedy, c_roul, c_fb, c_fbu, c_retry);
  }
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

__global__ __launch_bounds__(1024) void k_best_global_dense(Dev D, Iter A) {
  __shared__ int s_better;
  __shared__ int64_t s_lgb;
  int64_t bl;
  int ba;
  argmin_len(D, bl, ba);
  if (threadIdx.x == 0) {
    const int64_t lgb = D.gstate[0];
    s_better = (lgb < 0 || bl < lgb) ? 1 : 0;
    s_lgb = s_better ? bl : lgb;
    D.gstate[0] = s_lgb;
    D.gstate[1] = bl;
    D.gstate[2] = ba;
    D.sync[0] = 0;  // barrier counter for the next construction
  }
  __syncthreads();
  const int n = D.n;
  if (s_better)
    for (int p = threadIdx.x; p < n; p += blockDim.x) D.best[p] = D.tours[(size_t)ba * n + p];
  __syncthreads();
  const float ag = A.a_glob;
  const float bg = (float)(A.rho / (double)s_lgb);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
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
}

size_t lds_bytes(const Dev &D, int block) {
  return (size_t)(block / 64) * ((D.n + 31) / 32) * sizeof(uint32_t);
}

constexpr int kSyncBlock = 1024;
constexpr int kAsyncBlock = 256;

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers.
// ---------------------------------------------------------------------------
hipError_t launch_dist(const Dev &d, uint32_t *dmax, hipStream_t s) {
  dim3 grid((d.ldn + 63) / 64, (d.n + 3) / 4);
  hipLaunchKernelGGL(k_dist, grid, dim3(256), 0, s, d, dmax);
  return hipGetLastError();
}

hipError_t launch_cand(const Dev &d, int32_t *cand_tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_cand, dim3((d.n + 3) / 4), dim3(256), 0, s, d, cand_tmp);
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
  size_t total = (size_t)d.n * d.ldn;
  if (total < (size_t)d.n * d.spm_s) total = (size_t)d.n * d.spm_s;
  if (total < 8) total = 8;
  hipLaunchKernelGGL(k_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, tau0);
  return hipGetLastError();
}

hipError_t launch_construct(const Dev &d, const Iter &it, int mode, int memory, hipStream_t s) {
  if (memory != 0) return hipErrorInvalidValue;
  if (mode == 0) {
    const int apb = kSyncBlock / 64;
    const int grid = (d.m + apb - 1) / apb;
    Dev dd = d;
    Iter a = it;
    void *args[] = {&dd, &a};
    return hipLaunchCooperativeKernel(reinterpret_cast<void *>(&k_construct_sync_dense),
                                      dim3(grid), dim3(kSyncBlock), args, lds_bytes(d, kSyncBlock), s);
  }
  const int apb = kAsyncBlock / 64;
  const int grid = (d.m + apb - 1) / apb;
  hipLaunchKernelGGL(k_construct_async_dense, dim3(grid), dim3(kAsyncBlock),
                     lds_bytes(d, kAsyncBlock), s, d, it);
  return hipGetLastError();
}

int max_sync_ants(const Dev &d, int memory) {
  if (memory != 0) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(&k_construct_sync_dense), kSyncBlock,
          lds_bytes(d, kSyncBlock)) != hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus * (kSyncBlock / 64);
}

hipError_t launch_best_global(const Dev &d, const Iter &it, int memory, hipStream_t s) {
  if (memory != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_best_global_dense, dim3(1), dim3(1024), 0, s, d, it);
  return hipGetLastError();
}

}  // namespace acs
