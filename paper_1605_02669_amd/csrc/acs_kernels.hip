// HIP kernels for the Ant Colony System hot path on gfx950 (MI355X).
//
// Method: Skinderowicz, "The GPU-based Parallel Ant Colony System" (JPDC
// 2016), Sec. 3.  Layout and mapping are designed for CDNA4: one group of
// LANES lanes (16, 32 or 64 of a 64-wide wavefront) per ant, the candidate
// set evaluated one candidate per lane, the visited set as a bitmap in LDS,
// the argmax and the roulette prefix sums as group-level reductions in a
// fixed order, and the local update as a compare-and-swap loop applying the
// exact map of Eq. 3.
//
// Pheromone homes (dense memory): the value of the directed entry (i, j)
// lives in tau_nn[i][k] when j is the k-th candidate of i, otherwise in
// tau[i][j].  Reads of the candidate set are then one coalesced row of
// tau_nn; the fallback scan only ever reads non-candidate entries of tau
// (it runs only when every candidate is visited), so each entry has exactly
// one home and every update goes to it.
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

template <int LANES>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
  for (int off = LANES / 2; off; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, LANES));
  return v;
}

template <int LANES>
__device__ __forceinline__ int group_min_i(int v) {
#pragma unroll
  for (int off = LANES / 2; off; off >>= 1) v = min(v, __shfl_xor(v, off, LANES));
  return v;
}

// Local or global map x -> fma(a, x, b) applied atomically to one entry.
__device__ __forceinline__ void cas_map(float *p, float a, float b) {
  unsigned int *q = reinterpret_cast<unsigned int *>(p);
  unsigned int old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (true) {
    const unsigned int nw = __float_as_uint(fmaf(a, __uint_as_float(old), b));
    const unsigned int prev = atomicCAS(q, old, nw);
    if (prev == old) break;
    old = prev;
  }
}

// Home of the directed pheromone entry (u, v) when the candidate position of
// v in u's list is already known (k >= 0) or not in it (k < 0).
__device__ __forceinline__ float *home(const Dev &D, int u, int v, int k) {
  return k >= 0 ? D.tau_nn + (size_t)u * D.cl + k : D.tau + (size_t)u * D.ldn + v;
}

// Position of v in the candidate list of u, or -1: one probe per lane.
template <int LANES>
__device__ __forceinline__ int cand_pos(const Dev &D, int u, int v, int g, uint64_t gmask,
                                        int gbase) {
  bool hit = false;
  for (int k0 = 0; k0 < D.cl; k0 += LANES) {
    const int k = k0 + g;
    hit = k < D.cl && D.crec[(size_t)u * D.cl + k].x == (uint32_t)v;
    const uint64_t b = __ballot(hit) & gmask;
    if (b) return k0 + (__ffsll((unsigned long long)b) - 1 - gbase);
  }
  return -1;
}

// Grid-wide barrier for a cooperative launch: every wave publishes its
// writes at agent scope, one arrival per block on a monotonically growing
// counter, and every wave acquires after the wait.  The wait is bounded: on
// exhaustion an error flag is raised and the kernel runs on, so it always
// terminates.
__device__ __forceinline__ void grid_barrier(uint32_t *sync, uint32_t target) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while (__hip_atomic_load(sync, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
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
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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

__global__ __launch_bounds__(256) void k_crec(Dev D, const int32_t *cand) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D.n * D.cl) return;
  const int i = e / D.cl;
  const uint32_t c = (uint32_t)cand[e];
  const uint32_t d = D.dist[(size_t)i * D.ldn + c];
  uint32_t inv = kNone;
  for (int q = 0; q < D.cl; ++q)
    if (cand[(size_t)c * D.cl + q] == i) { inv = (uint32_t)q; break; }
  const_cast<uint4 *>(D.crec)[e] = make_uint4(c, d, __float_as_uint(D.eta_tab[d]), inv);
}

__global__ __launch_bounds__(256) void k_init(Dev D, float tau0) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nd = (size_t)D.n * D.ldn;
  if (D.tau && e < nd) D.tau[e] = tau0;
  if (D.tau_nn && e < (size_t)D.n * D.cl) D.tau_nn[e] = tau0;
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
// Construction, dense pheromone memory (Alg. 1 steps, Alg. 2 per ant).
// One group of LANES lanes per ant; lane g < cl evaluates candidate g.
// SYNC = true: persistent cooperative kernel, every step is
//   SELECT (reads only) | grid barrier | UPDATE (Eq. 3 by CAS) | grid barrier.
// SYNC = false: no barriers, the update follows each ant's own move.
// ---------------------------------------------------------------------------
template <int LANES, bool SYNC>
__global__ __launch_bounds__(256) void k_construct_dense(Dev D, Iter A) {
  extern __shared__ uint32_t smem[];
  const int apb = blockDim.x / LANES;
  const int lane = threadIdx.x & 63;
  const int g = threadIdx.x & (LANES - 1);
  const int grp = threadIdx.x / LANES;
  const int gbase = lane & ~(LANES - 1);
  const uint64_t gmask =
      LANES == 64 ? ~0ull : (((1ull << (LANES & 63)) - 1ull) << gbase);
  const int ant = blockIdx.x * apb + grp;
  const bool active = ant < D.m;
  const int n = D.n, cl = D.cl, ldn = D.ldn;
  const int W = (n + 31) >> 5;
  uint32_t *vis = smem + grp * W;

  for (int w = g; w < W; w += LANES) vis[w] = 0u;
  const uint4 r0 = philox10(make_uint4(0u, (uint32_t)ant, A.it, A.instance), A.key0, A.key1);
  const int start = (int)__umulhi(r0.z, (uint32_t)n);
  if (g == 0) vis[start >> 5] |= 1u << (start & 31);
  if (g == 0 && active) D.tours[(size_t)ant * n] = start;

  int cur = start;
  int64_t len = 0;
  uint32_t c_greedy = 0, c_roul = 0, c_fb = 0;
  uint64_t c_fbu = 0;  // unvisited cities scanned by fallbacks
  uint32_t bar = 0;  // barriers passed (sync)

  for (int t = 1; t < n; ++t) {
    int next = 0, kstar = -1;
    uint32_t dnext = 0, inv = kNone;
    if (active) {
      uint4 rec = make_uint4(0, 0, 0, kNone);
      float tn = 0.f;
      if (g < cl) {
        rec = D.crec[(size_t)cur * cl + g];
        tn = D.tau_nn[(size_t)cur * cl + g];
      }
      const uint4 rnd = philox10(make_uint4((uint32_t)t, (uint32_t)ant, A.it, A.instance), A.key0, A.key1);
      bool unv = false;
      float w = 0.f;
      if (g < cl) {
        unv = !((vis[rec.x >> 5] >> (rec.x & 31)) & 1u);
        w = unv ? tn * __uint_as_float(rec.z) : 0.f;
      }
      const uint64_t umask = __ballot(unv) & gmask;
      if (umask) {
        if ((rnd.x >> 8) < A.q0_24) {
          // Eq. 1, exploitation: argmax of tau * eta^beta, lowest position
          const float mv = group_max<LANES>(unv ? w : -1.f);
          const uint64_t sel = __ballot(unv && w == mv) & gmask;
          kstar = __ffsll((unsigned long long)sel) - 1 - gbase;
          ++c_greedy;
        } else {
          // Eq. 2 by roulette: Hillis-Steele inclusive scan over positions
          float P = w;
          for (int off = 1; off < cl; off <<= 1) {
            const float o = __shfl_up(P, off, LANES);
            if (g >= off) P = P + o;
          }
          const float total = __shfl(P, cl - 1, LANES);
          const float u = (float)(rnd.y >> 8) * 0x1p-24f;
          const float r = u * total;
          const uint64_t sel = __ballot(unv && P > r) & gmask;
          kstar = sel ? __ffsll((unsigned long long)sel) - 1 - gbase
                      : 63 - __clzll((long long)umask) - gbase;
          ++c_roul;
        }
        next = (int)__shfl(rec.x, kstar, LANES);
        dnext = __shfl(rec.y, kstar, LANES);
        inv = __shfl(rec.w, kstar, LANES);
      } else {
        // Alg. 2, empty candidate set: greedy over every unvisited city,
        // ties -> lowest index.  Four consecutive cities per lane.
        const float *trow = D.tau + (size_t)cur * ldn;
        const uint16_t *drow = D.dist + (size_t)cur * ldn;
        float bv = -1.f;
        int bj = INT_MAX;
        for (int j0 = 4 * g; j0 < n; j0 += 4 * LANES) {
          uint32_t bits = (vis[j0 >> 5] >> (j0 & 31)) & 0xfu;
          if (j0 + 4 > n) bits |= (0xfu << (n - j0)) & 0xfu;
          if (bits != 0xfu) {
            const float4 tv = *reinterpret_cast<const float4 *>(trow + j0);
            const ushort4 dv = *reinterpret_cast<const ushort4 *>(drow + j0);
            const float tq[4] = {tv.x, tv.y, tv.z, tv.w};
            const uint32_t dq[4] = {dv.x, dv.y, dv.z, dv.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (!((bits >> q) & 1u)) {
                const float v = tq[q] * D.eta_tab[dq[q]];
                if (v > bv) { bv = v; bj = j0 + q; }
              }
          }
        }
        const float mv = group_max<LANES>(bv);
        next = group_min_i<LANES>(bv == mv ? bj : INT_MAX);
        dnext = drow[next];
        ++c_fb;
        c_fbu += (uint64_t)(n - t);
      }
      if (g == 0) {
        vis[next >> 5] |= 1u << (next & 31);
        D.tours[(size_t)ant * n + t] = next;
      }
      len += dnext;
    }
    if (SYNC) grid_barrier(D.sync, (++bar) * gridDim.x);
    if (active) {
      // Eq. 3 on both directed entries of the crossed edge.
      int k2;
      if (kstar >= 0) k2 = inv == kNone ? -1 : (int)inv;
      else k2 = cand_pos<LANES>(D, next, cur, g, gmask, gbase);
      // lanes 0 and 1 update the two directed entries concurrently
      float *h = g == 0 ? home(D, cur, next, kstar) : home(D, next, cur, k2);
      if (g < 2) cas_map(h, A.a_loc, A.b_loc);
      cur = next;
    }
    if (SYNC && t + 1 < n) grid_barrier(D.sync, (++bar) * gridDim.x);
  }
  if (active) {
    // closing edge: length and local update (the last step's crossings)
    len += D.dist[(size_t)cur * ldn + start];
    const int k1 = cand_pos<LANES>(D, cur, start, g, gmask, gbase);
    const int k2 = cand_pos<LANES>(D, start, cur, g, gmask, gbase);
    float *h = g == 0 ? home(D, cur, start, k1) : home(D, start, cur, k2);
    if (g < 2) cas_map(h, A.a_loc, A.b_loc);
    if (g == 0) {
      D.lens[ant] = len;
      atomicAdd(&D.counters[0], (unsigned long long)c_greedy);
      atomicAdd(&D.counters[1], (unsigned long long)c_roul);
      atomicAdd(&D.counters[2], (unsigned long long)c_fb);
      atomicAdd(&D.counters[5], (unsigned long long)c_fbu);
    }
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

template <int LANES, bool SYNC>
hipError_t launch_dense(const Dev &D, const Iter &A, hipStream_t s) {
  const int block = SYNC ? 256 : 64;
  const int apb = block / LANES;
  const int grid = (D.m + apb - 1) / apb;
  const size_t lds = (size_t)apb * ((D.n + 31) / 32) * sizeof(uint32_t);
  if (SYNC) {
    Dev d = D;
    Iter a = A;
    void *args[] = {&d, &a};
    return hipLaunchCooperativeKernel(reinterpret_cast<void *>(&k_construct_dense<LANES, true>),
                                      dim3(grid), dim3(block), args, lds, s);
  }
  hipLaunchKernelGGL((k_construct_dense<LANES, false>), dim3(grid), dim3(block), lds, s, D, A);
  return hipGetLastError();
}

template <int LANES>
int max_sync_dense(const Dev &D) {
  const int block = 256;
  const size_t lds = (size_t)(block / LANES) * ((D.n + 31) / 32) * sizeof(uint32_t);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(&k_construct_dense<LANES, true>), block, lds) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus * (block / LANES);
}

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

hipError_t launch_crec(const Dev &d, const int32_t *cand_tmp, hipStream_t s) {
  const int total = d.n * d.cl;
  hipLaunchKernelGGL(k_crec, dim3((total + 255) / 256), dim3(256), 0, s, d, cand_tmp);
  return hipGetLastError();
}

hipError_t launch_init_pheromone(const Dev &d, float tau0, hipStream_t s) {
  size_t total = (size_t)d.n * d.ldn;
  if (total < (size_t)d.n * d.cl) total = (size_t)d.n * d.cl;
  if (total < (size_t)d.n * d.spm_s) total = (size_t)d.n * d.spm_s;
  if (total < 8) total = 8;
  hipLaunchKernelGGL(k_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, tau0);
  return hipGetLastError();
}

hipError_t launch_construct(const Dev &d, const Iter &it, int mode, int memory, hipStream_t s) {
  if (memory != 0) return hipErrorInvalidValue;
  const bool sync = mode == 0;
  if (d.cl <= 16) return sync ? launch_dense<16, true>(d, it, s) : launch_dense<16, false>(d, it, s);
  if (d.cl <= 32) return sync ? launch_dense<32, true>(d, it, s) : launch_dense<32, false>(d, it, s);
  return sync ? launch_dense<64, true>(d, it, s) : launch_dense<64, false>(d, it, s);
}

int max_sync_ants(const Dev &d, int memory) {
  if (memory != 0) return 0;
  if (d.cl <= 16) return max_sync_dense<16>(d);
  if (d.cl <= 32) return max_sync_dense<32>(d);
  return max_sync_dense<64>(d);
}

hipError_t launch_best_global(const Dev &d, const Iter &it, int memory, hipStream_t s) {
  if (memory != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_best_global_dense, dim3(1), dim3(1024), 0, s, d, it);
  return hipGetLastError();
}

}  // namespace acs
