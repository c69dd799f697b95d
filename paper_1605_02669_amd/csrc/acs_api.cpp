// C-ABI of libacs: argument checks, device memory layout, instance
// preparation, the iteration loop and read-back.  The arithmetic of the
// method runs in the HIP kernels of acs_kernels.hip; this file only
// validates, allocates, launches and copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/acs.h"
#include "acs_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? ACS_E_NOMEM : ACS_E_DEVICE, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                   \
  } while (0)

std::mutex g_live_mu;
std::unordered_set<const void *> g_live;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device buffers of one handle, as offsets into one allocation.
struct Layout {
  size_t xy, dist, crec, cand, eta, tau, tau2, etad, rpos, ctau, gvis, fpre, flim, femax, fbound, bflags, spm, spm_tail, xnn, gbox, gstart, gcnt, gcity, gxy, upd_rec, upd_nb, upd_next, upd_head, tours, lens,
      best, gstate, counters, sync, dmax, lnn, total;
  size_t dist_rows;  // rows of the distance matrix `dist` holds at a time
};

constexpr int kEtaEntries = acs::kEtaHostEntries;  // eta^beta for every 16-bit distance

// Cells per side of the selective memory's search grid (about two cities
// per cell); the grid has at most (side + 1)^2 cells.
int grid_side(int n) {
  return std::min(256, std::max(1, (int)std::ceil(std::sqrt((double)n / 2.0))));
}

// The dense fallback first scans the kFpre cities after the candidates; it
// needs the city after them too.
bool fallback_prefix(int n, int cl) { return n - 1 > cl + acs::kFpre; }

Layout make_layout(int n, int m, int cl, int ldn, int memory, int s, int mode) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  L.xy = take(sizeof(double) * 2 * (size_t)n);
  // dense memory: the whole distance matrix; the selective memory keeps none
  // (Sec. 3.2: O(n s) pheromone memory) and builds its neighbour lists from
  // chunks of rows placed where the tours go
  const size_t tour_bytes = sizeof(int32_t) * (size_t)m * n;
  if (memory == ACS_DENSE) {
    L.dist_rows = (size_t)n;
    L.dist = take(sizeof(uint16_t) * (size_t)n * ldn);
  } else {
    L.dist_rows = std::min<size_t>((size_t)n, std::max<size_t>(64, tour_bytes /
                                                                     (sizeof(uint16_t) * ldn)));
  }
  L.crec = take(sizeof(uint4) * (size_t)n * cl);
  L.cand = take(sizeof(int32_t) * (size_t)n * cl);
  L.eta = take(sizeof(float) * kEtaEntries);
  if (memory == ACS_DENSE) {
    L.tau = take(sizeof(float) * (size_t)n * ldn);
    L.etad = take(sizeof(float) * (size_t)n * ldn);
    L.rpos = take(sizeof(int8_t) * (size_t)n * cl);
    L.ctau = take(sizeof(float) * (size_t)n * cl);
    if (mode == ACS_SEQUENTIAL) L.gvis = take(sizeof(uint32_t) * (size_t)m * ((n + 31) / 32));
    if (mode == ACS_SYNC) L.tau2 = take(sizeof(float) * (size_t)n * ldn);
    if (fallback_prefix(n, cl)) {
      L.fpre = take(sizeof(uint32_t) * 2 * (size_t)n * acs::kFpre);
      L.flim = take(sizeof(uint32_t) * (size_t)n);
      L.femax = take(sizeof(float) * (size_t)n);
      L.fbound = take(sizeof(float) * (size_t)n);
    }
  } else {
    L.spm = take(sizeof(uint32_t) * 2 * (size_t)n * s);
    L.spm_tail = take(sizeof(uint32_t) * (size_t)n);
    L.xnn = take(sizeof(uint32_t) * (size_t)n * std::min(acs::kXnn, n - 1));
    const size_t cells = (size_t)(grid_side(n) + 1) * (grid_side(n) + 1);
    L.gbox = take(sizeof(double) * 4);
    L.gstart = take(sizeof(int32_t) * (cells + 1));
    L.gcnt = take(sizeof(int32_t) * cells);
    L.gcity = take(sizeof(uint32_t) * (size_t)n);
    L.gxy = take(sizeof(double) * 2 * (size_t)n);
    L.upd_rec = take(sizeof(int32_t) * 2 * (size_t)m);
    L.upd_nb = take(sizeof(int32_t) * 2 * (size_t)m);
    L.upd_next = take(sizeof(int32_t) * 2 * (size_t)m);
    L.upd_head = take(sizeof(int32_t) * (size_t)n);
  }
  if (mode == ACS_SYNC) L.bflags = take(sizeof(uint64_t) * 16 * (size_t)((m + 15) / 16 + 1));
  if (memory == ACS_DENSE) {
    L.tours = take(tour_bytes);
  } else {
    L.tours = take(std::max(tour_bytes, sizeof(uint16_t) * L.dist_rows * ldn));
    L.dist = L.tours;
  }
  L.lens = take(sizeof(int64_t) * (size_t)m);
  L.best = take(sizeof(int32_t) * (size_t)n);
  L.gstate = take(sizeof(int64_t) * 4);
  L.counters = take(sizeof(unsigned long long) * 8);
  L.sync = take(sizeof(uint32_t) * 4);
  L.dmax = take(sizeof(uint32_t));
  L.lnn = take(sizeof(int64_t));
  L.total = off;
  return L;
}

int check_params(int32_t n, const acs_params *p) {
  if (!p) return fail(ACS_E_INVALID, "params is NULL");
  if (p->struct_size != sizeof(acs_params))
    return fail(ACS_E_INVALID, "params.struct_size %u != %zu", p->struct_size, sizeof(acs_params));
  if (n < 3) return fail(ACS_E_INVALID, "n = %d < 3", n);
  if (p->cl < 1) return fail(ACS_E_INVALID, "cl must be >= 1");
  if (!(p->q0 >= 0.0 && p->q0 <= 1.0)) return fail(ACS_E_INVALID, "q0 not in [0, 1]");
  if (!(p->phi > 0.0 && p->phi < 1.0)) return fail(ACS_E_INVALID, "phi not in (0, 1)");
  if (!(p->rho > 0.0 && p->rho < 1.0)) return fail(ACS_E_INVALID, "rho not in (0, 1)");
  if (!(p->beta >= 0.0) || !std::isfinite(p->beta)) return fail(ACS_E_INVALID, "beta invalid");
  if (!std::isfinite(p->tau0)) return fail(ACS_E_INVALID, "tau0 not finite");
  if (p->memory != ACS_DENSE && p->memory != ACS_SPM) return fail(ACS_E_INVALID, "bad memory");
  if (p->memory == ACS_SPM && p->spm_s < 1) return fail(ACS_E_INVALID, "spm_s must be >= 1");
  if (p->mode != ACS_SYNC && p->mode != ACS_ASYNC_ATOMIC && p->mode != ACS_ASYNC_RACY &&
      p->mode != ACS_SEQUENTIAL)
    return fail(ACS_E_INVALID, "bad mode");
  if (p->mode == ACS_SEQUENTIAL && p->memory != ACS_DENSE)
    return fail(ACS_E_UNSUPPORTED, "the sequential mode needs dense memory");
  if (p->local_update_period < 1) return fail(ACS_E_INVALID, "local_update_period must be >= 1");
  if (n > 65535) return fail(ACS_E_UNSUPPORTED, "n = %d > 65535", n);
  const uint32_t cl = std::min<uint32_t>(p->cl, (uint32_t)n - 1);
  if (cl > 64) return fail(ACS_E_UNSUPPORTED, "cl = %u > 64", cl);
  if (p->memory == ACS_SPM && p->spm_s > (uint32_t)acs::kMaxSpmS)
    return fail(ACS_E_UNSUPPORTED, "spm_s = %u > %d", p->spm_s, acs::kMaxSpmS);
  const uint32_t lpa = p->lanes_per_ant;
  if (lpa != 0 && lpa != 64 && lpa != 32 && lpa != 16)
    return fail(ACS_E_INVALID, "lanes_per_ant = %u not in {0, 16, 32, 64}", lpa);
  if (lpa != 0 && lpa < cl)
    return fail(ACS_E_UNSUPPORTED, "lanes_per_ant = %u < cl = %u", lpa, cl);
  if (lpa != 0 && lpa != 64 &&
      ((p->mode != ACS_ASYNC_ATOMIC && p->mode != ACS_ASYNC_RACY) || p->memory != ACS_DENSE))
    return fail(ACS_E_UNSUPPORTED, "lanes_per_ant < 64 needs an asynchronous mode and dense memory");
  if (p->update_path > 2) return fail(ACS_E_INVALID, "update_path = %u not in {0, 1, 2}",
                                      p->update_path);
  if (p->local_search > 2)
    return fail(ACS_E_INVALID, "local_search = %u not in {0, 1, 2}", p->local_search);
  if (p->local_search && (p->memory != ACS_DENSE || n > acs::kLsMaxN))
    return fail(ACS_E_UNSUPPORTED, "the local search needs dense memory and n <= %d",
                acs::kLsMaxN);
  return ACS_OK;
}

// eta^beta for integer distance d (eta = 1/d; a zero distance reads as 1/2).
float eta_beta(double beta, uint32_t d) {
  if (d == 0) return (float)std::pow(2.0, beta);
  return (float)(1.0 / std::pow((double)d, beta));
}

}  // namespace

struct acs_t {
  acs_params p{};
  int n = 0, m = 0, cl = 0, ldn = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char *ws = nullptr;
  bool own_ws = false;
  Layout L{};
  acs::Dev dev{};
  acs::Iter base{};
  int64_t lnn = 0;
  float tau0 = 0.f;
  uint32_t iter = 0;
  double construct_ms = 0.0, iterate_ms = 0.0;
  int construct_launches = 0;
  std::vector<hipEvent_t> ev;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  bool timed = true;  // events around every construction (not for a fixed workspace)
};

namespace {

bool live(const acs_t *h) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return h && g_live.count(h);
}

// Waits for the handle's stream and frees what the handle owns (its stream,
// events and workspace, where it created them).
void release_resources(acs_t *h) {
  // (a handle on the null stream has work queued once it has a workspace)
  if (h->stream || h->ws) (void)hipStreamSynchronize(h->stream);
  for (auto e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  if (h->ev_begin) (void)hipEventDestroy(h->ev_begin);
  if (h->ev_end) (void)hipEventDestroy(h->ev_end);
  h->ev_begin = h->ev_end = nullptr;
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  h->ws = nullptr;
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  h->stream = nullptr;
}

void release(acs_t *h) {
  if (!h) return;
  release_resources(h);
  delete h;
}

int sync_and_check(acs_t *h) {
  HIP_TRY(hipStreamSynchronize(h->stream));
  uint32_t flags[2] = {0, 0};
  HIP_TRY(hipMemcpy(flags, h->ws + h->L.sync, sizeof flags, hipMemcpyDeviceToHost));
  if (flags[1])
    return fail(ACS_E_DEVICE, "a bounded device wait was exhausted (flag %u: 1 grid barrier, "
                              "2 update ring)", flags[1]);
  return ACS_OK;
}

int build(acs_t *h, const double *xy, float *eta_host) {
  const int n = h->n;
  HIP_TRY(hipMemcpyAsync(h->ws + h->L.xy, xy, sizeof(double) * 2 * n, hipMemcpyHostToDevice,
                         h->stream));
  HIP_TRY(hipMemsetAsync(h->ws + h->L.dmax, 0, sizeof(uint32_t), h->stream));
  uint32_t *dmax_d = reinterpret_cast<uint32_t *>(h->ws + h->L.dmax);
  const bool dense = h->p.memory == ACS_DENSE;
  // dense: the whole matrix; selective memory: only the largest distance
  HIP_TRY(acs::launch_dist(h->dev, dmax_d, 0, n, dense, h->stream));
  uint32_t dmax = 0;
  HIP_TRY(hipMemcpyAsync(&dmax, dmax_d, sizeof dmax, hipMemcpyDeviceToHost, h->stream));
  double box[4] = {0, 0, 0, 0};
  if (!dense) {
    double *box_d = reinterpret_cast<double *>(h->ws + h->L.gbox);
    HIP_TRY(acs::launch_grid_box(h->dev, box_d, h->stream));
    HIP_TRY(hipMemcpyAsync(box, box_d, sizeof box, hipMemcpyDeviceToHost, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (dmax > 65535u)
    return fail(ACS_E_UNSUPPORTED, "largest distance %u exceeds 65535", dmax);
  if (!dense) {
    // square cells of side (largest extent) / side over the bounding box
    const int g = grid_side(n);
    const double wx = box[2] - box[0], wy = box[3] - box[1];
    const double ext = std::max(wx, wy);
    acs::Dev &dv = h->dev;
    dv.gx0 = box[0];
    dv.gy0 = box[1];
    dv.gh = ext > 0.0 ? ext / g : 1.0;
    dv.ginv = 1.0 / dv.gh;
    dv.gnx = std::min(g + 1, (int)std::floor(wx * dv.ginv) + 1);
    dv.gny = std::min(g + 1, (int)std::floor(wy * dv.ginv) + 1);
    HIP_TRY(acs::launch_grid(dv, reinterpret_cast<int32_t *>(h->ws + h->L.gcnt), h->stream));
  }

  int32_t *cand = reinterpret_cast<int32_t *>(h->ws + h->L.cand);
  if (dense) {
    HIP_TRY(acs::launch_cand(h->dev, cand, 0, n, h->stream));
  } else {
    // the neighbour lists of the selective memory from chunks of distance
    // rows, computed in the region the tours take later
    const int rows = (int)h->L.dist_rows;
    for (int r0 = 0; r0 < n; r0 += rows) {
      const int nr = std::min(rows, n - r0);
      HIP_TRY(acs::launch_dist(h->dev, dmax_d, r0, nr, true, h->stream));
      HIP_TRY(acs::launch_cand(h->dev, cand, r0, nr, h->stream));
    }
    h->dev.dist = nullptr;
  }
  int64_t *lnn_d = reinterpret_cast<int64_t *>(h->ws + h->L.lnn);
  HIP_TRY(acs::launch_nn_tour(h->dev, lnn_d, h->stream));
  HIP_TRY(hipMemcpyAsync(&h->lnn, lnn_d, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->lnn <= 0) return fail(ACS_E_INVALID, "nearest-neighbour tour has length %lld",
                               (long long)h->lnn);

  // Host constants of the method (scalars and the per-distance eta table).
  const acs_params &p = h->p;
  h->tau0 = p.tau0 > 0.0 ? (float)p.tau0 : (float)(1.0 / ((double)n * (double)h->lnn));
  std::vector<float> eta_vec;
  if (!eta_host) {
    eta_vec.resize(kEtaEntries);
    eta_host = eta_vec.data();
  }
  float *eta = eta_host;
  std::fill(eta, eta + kEtaEntries, 0.f);
  for (uint32_t d = 0; d <= dmax; ++d) eta[d] = eta_beta(p.beta, d);
  if (p.memory == ACS_SPM) {
    // the selective memory's fallback relies on tau0 * eta^beta(d) strictly
    // decreasing in d (every trail outside a record holds tau0)
    for (uint32_t d = 0; d < dmax; ++d)
      if (!(h->tau0 * eta[d] > h->tau0 * eta[d + 1]))
        return fail(ACS_E_UNSUPPORTED,
                    "tau0 * eta^beta is not strictly decreasing at d = %u (selective memory)", d);
  }
  HIP_TRY(hipMemcpyAsync(h->ws + h->L.eta, eta, sizeof(float) * kEtaEntries,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(acs::launch_crec(h->dev, cand, h->tau0, h->stream));
  HIP_TRY(acs::launch_init_pheromone(h->dev, h->tau0, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));

  acs::Iter &b = h->base;
  b.it = 0;
  b.instance = p.instance;
  b.key0 = (uint32_t)p.seed;
  b.key1 = (uint32_t)(p.seed >> 32);
  b.q0_24 = (uint32_t)std::ceil(p.q0 * 16777216.0);
  b.a_loc = (float)(1.0 - p.phi);
  b.b_loc = (float)(p.phi * (double)h->tau0);
  b.a_glob = (float)(1.0 - p.rho);
  b.tau0 = h->tau0;
  b.lperiod = p.local_update_period;
  b.rho = p.rho;
  return ACS_OK;
}

// Sets up the fresh handle *h for the instance.  With fixed_ws (device
// memory of fixed_bytes the caller keeps) nothing is created: the handle
// runs on params.stream (NULL: the null stream), untimed, in that memory.
// Otherwise the stream, events and workspace are the handle's own (or the
// caller's, from params).  eta_host: host buffer of kEtaEntries floats for
// the eta^beta table, NULL for a temporary one.  On failure the caller
// releases what the handle holds.
int init_handle(acs_t *h, const double *coords_xy, int32_t n, const acs_params *p, char *fixed_ws,
                size_t fixed_bytes, float *eta_host) {
  int rc = check_params(n, p);
  if (rc) return rc;
  if (!coords_xy) return fail(ACS_E_INVALID, "coords is NULL");
  for (int i = 0; i < 2 * n; ++i)
    if (!std::isfinite(coords_xy[i])) return fail(ACS_E_INVALID, "coordinate %d not finite", i);
  const int m = p->m ? (int)p->m : n;
  if (m < 1) return fail(ACS_E_INVALID, "m < 1");

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(ACS_E_DEVICE, "no HIP device available");

  h->p = *p;
  h->n = n;
  h->m = m;
  h->cl = (int)std::min<uint32_t>(p->cl, (uint32_t)n - 1);
  h->ldn = (int)align_up((size_t)n, 64);
  h->L = make_layout(n, m, h->cl, h->ldn, (int)p->memory, (int)p->spm_s, (int)p->mode);

  if (fixed_ws) {
    // caller-owned device memory: no stream, event or workspace is created
    if (fixed_bytes < h->L.total)
      return fail(ACS_E_BUFSIZE, "workspace of %zu bytes < %zu needed", fixed_bytes, h->L.total);
    h->stream = reinterpret_cast<hipStream_t>(p->stream);
    h->ws = fixed_ws;
    h->timed = false;
  } else {
    if (p->stream) {
      h->stream = reinterpret_cast<hipStream_t>(p->stream);
    } else {
      if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(ACS_E_DEVICE, "stream creation failed");
      h->own_stream = true;
    }
    if (p->workspace) {
      if (p->workspace_bytes < h->L.total)
        return fail(ACS_E_BUFSIZE, "workspace of %zu bytes < %zu needed", p->workspace_bytes,
                    h->L.total);
      h->ws = reinterpret_cast<char *>(p->workspace);
    } else {
      hipError_t e = hipMalloc(&h->ws, h->L.total);
      if (e != hipSuccess) {
        h->ws = nullptr;
        // the failed allocation is also this thread's last HIP error, which
        // the launch checks of later calls would otherwise report as theirs
        (void)hipGetLastError();
        return fail(ACS_E_NOMEM, "hipMalloc(%zu): %s", h->L.total, hipGetErrorString(e));
      }
      h->own_ws = true;
    }
    if (hipEventCreate(&h->ev_begin) != hipSuccess || hipEventCreate(&h->ev_end) != hipSuccess)
      return fail(ACS_E_DEVICE, "event creation failed");
  }

  acs::Dev &d = h->dev;
  char *w = h->ws;
  d.n = n;
  d.m = m;
  d.cl = h->cl;
  d.ldn = h->ldn;
  d.spm_s = (int)p->spm_s;
  d.xy = reinterpret_cast<const double *>(w + h->L.xy);
  d.dist = reinterpret_cast<const uint16_t *>(w + h->L.dist);
  d.crec = reinterpret_cast<const uint4 *>(w + h->L.crec);
  d.eta_tab = reinterpret_cast<const float *>(w + h->L.eta);
  if (p->memory == ACS_DENSE) {
    d.tau = reinterpret_cast<float *>(w + h->L.tau);
    d.etad = reinterpret_cast<const float *>(w + h->L.etad);
    d.rpos = reinterpret_cast<const int8_t *>(w + h->L.rpos);
    d.ctau = reinterpret_cast<float *>(w + h->L.ctau);
    if (p->mode == ACS_SEQUENTIAL) d.gvis = reinterpret_cast<uint32_t *>(w + h->L.gvis);
    if (p->mode == ACS_SYNC) d.tau2 = reinterpret_cast<float *>(w + h->L.tau2);
    if (fallback_prefix(n, h->cl)) {
      d.fpre = reinterpret_cast<const uint4 *>(w + h->L.fpre);
      d.flim = reinterpret_cast<const uint32_t *>(w + h->L.flim);
      d.femax = reinterpret_cast<const float *>(w + h->L.femax);
      d.fbound = reinterpret_cast<float *>(w + h->L.fbound);
    }
  } else {
    d.spm = reinterpret_cast<uint2 *>(w + h->L.spm);
    d.spm_tail = reinterpret_cast<uint32_t *>(w + h->L.spm_tail);
    d.xnn = reinterpret_cast<const uint32_t *>(w + h->L.xnn);
    d.xl = std::min(acs::kXnn, n - 1);
    d.gstart = reinterpret_cast<const int32_t *>(w + h->L.gstart);
    d.gcity = reinterpret_cast<const uint32_t *>(w + h->L.gcity);
    d.gxy = reinterpret_cast<const double2 *>(w + h->L.gxy);
    d.upd_rec = reinterpret_cast<int32_t *>(w + h->L.upd_rec);
    d.upd_nb = reinterpret_cast<int32_t *>(w + h->L.upd_nb);
    d.upd_next = reinterpret_cast<int32_t *>(w + h->L.upd_next);
    d.upd_head = reinterpret_cast<int32_t *>(w + h->L.upd_head);
  }
  d.tours = reinterpret_cast<int32_t *>(w + h->L.tours);
  d.lens = reinterpret_cast<int64_t *>(w + h->L.lens);
  d.best = reinterpret_cast<int32_t *>(w + h->L.best);
  d.gstate = reinterpret_cast<int64_t *>(w + h->L.gstate);
  d.counters = reinterpret_cast<unsigned long long *>(w + h->L.counters);
  d.sync = reinterpret_cast<uint32_t *>(w + h->L.sync);
  d.wait_limit = p->wait_limit;
  if (p->mode == ACS_SYNC) {
    d.bflags = reinterpret_cast<unsigned long long *>(w + h->L.bflags);
    d.nbflags = 16 * ((m + 15) / 16 + 1);
  }

  if (p->mode == ACS_SYNC) {
    const int cap = acs::max_sync_ants(d, (int)p->memory);
    if (m > cap)
      return fail(ACS_E_UNSUPPORTED, "m = %d ants exceed the %d one synchronous launch holds",
                  m, cap);
  }
  return build(h, coords_xy, eta_host);
}

// How the asynchronous kernels with one ant per wave apply local updates
// (acs_internal.hpp, launch_construct): 0 the ant itself, 1 an updater wave
// per block (the default).
int queued_kind(const acs_t *h) { return h->p.update_path == 1 ? 0 : 1; }

// k iterations of Alg. 1 on the handle (see acs_iterate).
int iterate_handle(acs_t *h, int32_t k) {
  if (k < 0) return fail(ACS_E_INVALID, "k < 0");
  if (k == 0) return ACS_OK;
  while (h->timed && (int)h->ev.size() < 2 * k) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    h->ev.push_back(e);
  }
  // a bounded wait that ran out in an earlier call was reported by it
  HIP_TRY(hipMemsetAsync(h->ws + h->L.sync, 0, 2 * sizeof(uint32_t), h->stream));
  if (h->timed) HIP_TRY(hipEventRecord(h->ev_begin, h->stream));
  for (int i = 0; i < k; ++i) {
    acs::Iter it = h->base;
    it.it = h->iter + (uint32_t)i;
    HIP_TRY(acs::launch_construct(h->dev, it, (int)h->p.mode, (int)h->p.memory,
                                  h->p.lanes_per_ant ? (int)h->p.lanes_per_ant : 64,
                                  queued_kind(h), h->stream,
                                  h->timed ? h->ev[2 * i] : nullptr,
                                  h->timed ? h->ev[2 * i + 1] : nullptr));
    if (h->p.local_search)
      HIP_TRY(acs::launch_local_search(h->dev, (int)h->p.local_search, h->stream));
    HIP_TRY(acs::launch_best_global(h->dev, it, (int)h->p.memory, h->stream));
  }
  if (h->timed) HIP_TRY(hipEventRecord(h->ev_end, h->stream));
  int rc = sync_and_check(h);
  h->iter += (uint32_t)k;
  if (rc || !h->timed) return rc;
  double cms = 0.0;
  for (int i = 0; i < k; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
    cms += ms;
  }
  float total = 0.f;
  HIP_TRY(hipEventElapsedTime(&total, h->ev_begin, h->ev_end));
  h->construct_ms = cms;
  h->construct_launches = k;
  h->iterate_ms = total;
  return ACS_OK;
}

// Best-so-far tour and length of the handle (see acs_best_tour).
int best_handle(acs_t *h, int32_t *tour_out, int64_t *len_out) {
  int64_t g[3];
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(g, h->ws + h->L.gstate, sizeof g, hipMemcpyDeviceToHost));
  if (g[0] < 0) return fail(ACS_E_STATE, "no iteration has run yet");
  if (len_out) *len_out = g[0];
  if (tour_out)
    HIP_TRY(hipMemcpy(tour_out, h->ws + h->L.best, sizeof(int32_t) * h->n, hipMemcpyDeviceToHost));
  return ACS_OK;
}

}  // namespace

namespace acs {

int solve_in(const double *coords_xy, int32_t n, const acs_params *p, int32_t iterations,
             char *ws, size_t ws_bytes, float *eta_host, int32_t *tour_out, int64_t *len_out) {
  if (iterations < 1) return fail(ACS_E_INVALID, "iterations = %d < 1", iterations);
  if (!tour_out || !len_out) return fail(ACS_E_INVALID, "NULL output");
  acs_t h;
  int rc = init_handle(&h, coords_xy, n, p, ws, ws_bytes, eta_host);
  if (!rc) rc = iterate_handle(&h, iterations);
  if (!rc) rc = best_handle(&h, tour_out, len_out);
  const std::string keep = rc ? g_err : std::string();
  release_resources(&h);
  if (rc) g_err = keep;
  return rc;
}

int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

}  // namespace acs

extern "C" {

int acs_default_params(acs_params *p) {
  if (!p) return fail(ACS_E_INVALID, "params is NULL");
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof(acs_params);
  p->m = 0;
  p->cl = 32;
  p->memory = ACS_DENSE;
  p->spm_s = 8;
  p->mode = ACS_SYNC;
  p->local_update_period = 1;
  p->beta = 2.0;
  p->q0 = 0.9;
  p->phi = 0.1;
  p->rho = 0.1;
  p->tau0 = 0.0;
  p->seed = 0;
  return ACS_OK;
}

int acs_workspace_bytes(int32_t n, const acs_params *p, size_t *out) {
  int rc = check_params(n, p);
  if (rc) return rc;
  if (!out) return fail(ACS_E_INVALID, "out is NULL");
  const int m = p->m ? (int)p->m : n;
  const int cl = (int)std::min<uint32_t>(p->cl, (uint32_t)n - 1);
  const int ldn = (int)align_up((size_t)n, 64);
  *out = make_layout(n, m, cl, ldn, (int)p->memory, (int)p->spm_s, (int)p->mode).total;
  return ACS_OK;
}

int acs_create(const double *coords_xy, int32_t n, const acs_params *p, acs_t **out) {
  if (!out) return fail(ACS_E_INVALID, "out is NULL");
  *out = nullptr;
  acs_t *h = new (std::nothrow) acs_t;
  if (!h) return fail(ACS_E_NOMEM, "host allocation failed");
  const int rc = init_handle(h, coords_xy, n, p, nullptr, 0, nullptr);
  if (rc) {
    std::string keep = g_err;
    release(h);
    g_err = keep;
    return rc;
  }
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.insert(h);
  }
  *out = h;
  return ACS_OK;
}

int acs_iterate(acs_t *h, int32_t k) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  return iterate_handle(h, k);
}

int acs_best_tour(acs_t *h, int32_t *tour_out, int64_t *len_out) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  return best_handle(h, tour_out, len_out);
}

int acs_pheromone_snapshot(acs_t *h, float *out, size_t count) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (h->p.memory != ACS_DENSE) return fail(ACS_E_UNSUPPORTED, "not a dense handle");
  const size_t n = (size_t)h->n, ldn = (size_t)h->ldn, cl = (size_t)h->cl;
  if (!out || count < n * n) return fail(ACS_E_BUFSIZE, "need %zu floats", n * n);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy2D(out, n * sizeof(float), h->ws + h->L.tau, ldn * sizeof(float),
                      n * sizeof(float), n, hipMemcpyDeviceToHost));
  std::vector<uint32_t> rec(n * cl * 4);
  HIP_TRY(hipMemcpy(rec.data(), h->ws + h->L.crec, rec.size() * sizeof(uint32_t),
                    hipMemcpyDeviceToHost));
  // candidate entries live in the last word of the candidate records
  for (size_t e = 0; e < n * cl; ++e) {
    float v;
    std::memcpy(&v, &rec[4 * e + 3], sizeof v);
    out[(e / cl) * n + rec[4 * e]] = v;
  }
  return ACS_OK;
}

int acs_spm_snapshot(acs_t *h, int32_t *nodes, float *vals, int32_t *tail) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (h->p.memory != ACS_SPM) return fail(ACS_E_UNSUPPORTED, "not an SPM handle");
  if (!nodes || !vals || !tail) return fail(ACS_E_INVALID, "NULL output");
  const size_t s = h->p.spm_s, ns = (size_t)h->n * s;
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<uint32_t> pairs(2 * ns), cnt((size_t)h->n);
  HIP_TRY(hipMemcpy(pairs.data(), h->ws + h->L.spm, pairs.size() * sizeof(uint32_t),
                    hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(cnt.data(), h->ws + h->L.spm_tail, cnt.size() * sizeof(uint32_t),
                    hipMemcpyDeviceToHost));
  for (size_t e = 0; e < ns; ++e) {
    nodes[e] = (int32_t)pairs[2 * e];
    std::memcpy(&vals[e], &pairs[2 * e + 1], sizeof(float));
  }
  // the record keeps an insert counter; the most recently added slot is it mod s
  for (size_t i = 0; i < (size_t)h->n; ++i) tail[i] = (int32_t)(cnt[i] % s);
  return ACS_OK;
}

int acs_tours(acs_t *h, int32_t *out, size_t count) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  const size_t need = (size_t)h->m * h->n;
  if (!out || count < need) return fail(ACS_E_BUFSIZE, "need %zu ints", need);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(out, h->ws + h->L.tours, need * sizeof(int32_t), hipMemcpyDeviceToHost));
  return ACS_OK;
}

int acs_lengths(acs_t *h, int64_t *out, size_t count) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (!out || count < (size_t)h->m) return fail(ACS_E_BUFSIZE, "need %d values", h->m);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(out, h->ws + h->L.lens, (size_t)h->m * sizeof(int64_t),
                    hipMemcpyDeviceToHost));
  return ACS_OK;
}

int acs_candidates(acs_t *h, int32_t *out, size_t count) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  const size_t need = (size_t)h->n * h->cl;
  if (!out || count < need) return fail(ACS_E_BUFSIZE, "need %zu ints", need);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(out, h->ws + h->L.cand, need * sizeof(int32_t), hipMemcpyDeviceToHost));
  return ACS_OK;
}

int acs_stats(acs_t *h, acs_stats_t *out) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (!out) return fail(ACS_E_INVALID, "out is NULL");
  if (out->struct_size != sizeof(acs_stats_t))
    return fail(ACS_E_INVALID, "stats.struct_size %u != %zu", out->struct_size,
                sizeof(acs_stats_t));
  HIP_TRY(hipStreamSynchronize(h->stream));
  int64_t g[3];
  unsigned long long c[8];
  HIP_TRY(hipMemcpy(g, h->ws + h->L.gstate, sizeof g, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(c, h->ws + h->L.counters, sizeof c, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->struct_size = sizeof(acs_stats_t);
  out->iteration = h->iter;
  out->best_length = g[0];
  out->iter_best_length = g[1];
  out->iter_best_ant = (int32_t)g[2];
  out->n = h->n;
  out->m = h->m;
  out->cl = h->cl;
  out->nn_length = h->lnn;
  out->tau0 = h->tau0;
  out->greedy = (int64_t)c[0];
  out->roulette = (int64_t)c[1];
  out->fallback = (int64_t)c[2];
  out->spm_hits = (int64_t)c[3];
  out->spm_misses = (int64_t)c[4];
  out->fallback_unvisited = (int64_t)c[5];
  out->cas_retries = (int64_t)c[6];
  out->ls_moves = (int64_t)c[7];
  out->steps = out->greedy + out->roulette + out->fallback;
  out->construct_ms = h->construct_ms;
  out->construct_launches = h->construct_launches;
  out->iterate_ms = h->iterate_ms;
  return ACS_OK;
}

void acs_destroy(acs_t *h) {
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    if (!h || !g_live.count(h)) return;
    g_live.erase(h);
  }
  release(h);
}

const char *acs_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many independent instances, one launch per iteration.
// ---------------------------------------------------------------------------
struct acs_batch_t {
  int count = 0;
  std::vector<acs_t *> inst;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char *ws = nullptr;
  bool own_ws = false;
  acs::Dev *d_devs = nullptr;
  acs::Iter *d_iters = nullptr;
  uint32_t *d_flag = nullptr;  // OR of the instances' error flags (see k_best_batch)
  int nmax = 0, clmax = 0, mode = ACS_ASYNC_ATOMIC;
  int64_t steps_per_iteration = 0;
  // One launch configuration per candidate lanes-per-ant value: its work
  // list and its captured iteration.  The first iterations time each of
  // them once (after one untimed warm-up iteration); the fastest is kept.
  struct Variant {
    int lanes = 64;
    bool queued = false;  // 64 lanes, updates through an updater wave per block
    int2 *d_items = nullptr;
    int nitems = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double ms = -1.0;
  };
  std::vector<Variant> var;
  int chosen = -1;     // index into var once tuned
  int tuning_step = 0; // iterations spent on tuning so far
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double iterate_ms = 0.0;
  // best-so-far exchange between the instances (colonies of one instance)
  int xtopology = 0, xperiod = 0;
  int64_t iters_done = 0;
  int32_t *d_offer = nullptr;
  int64_t *d_olen = nullptr;
};

namespace {

std::unordered_set<const void *> g_live_batches;

bool live_batch(const acs_batch_t *b) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return b && g_live_batches.count(b);
}

void release_batch(acs_batch_t *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (acs_t *h : b->inst) acs_destroy(h);
  for (auto &v : b->var) {
    if (v.exec) (void)hipGraphExecDestroy(v.exec);
    if (v.graph) (void)hipGraphDestroy(v.graph);
  }
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  if (b->own_ws && b->ws) (void)hipFree(b->ws);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

struct BatchLayout {
  std::vector<size_t> off;
  size_t devs, iters, items, flag, offer, olen, total;
};

int batch_layout(const int32_t *n, int32_t count, const acs_params *p, BatchLayout *L,
                 int *nitems) {
  size_t off = 0;
  *nitems = 0;
  L->off.resize((size_t)count);
  for (int i = 0; i < count; ++i) {
    size_t bytes = 0;
    const int rc = acs_workspace_bytes(n[i], p, &bytes);
    if (rc) return rc;
    L->off[(size_t)i] = off;
    off = align_up(off + bytes, 256);
    const int m = p->m ? (int)p->m : n[i];
    // work lists: 64 lanes per ant, 64 with the updater, 32 and 16 lanes
    *nitems += m + (m + acs::kBatchQAntsPerBlock - 1) / acs::kBatchQAntsPerBlock + (m + 1) / 2 +
               (m + 3) / 4;
  }
  L->devs = off;
  off = align_up(off + sizeof(acs::Dev) * (size_t)count, 256);
  L->iters = off;
  off = align_up(off + sizeof(acs::Iter) * (size_t)count, 256);
  L->items = off;
  off = align_up(off + sizeof(int2) * (size_t)*nitems, 256);
  L->flag = off;
  off = align_up(off + sizeof(uint32_t), 256);
  int nmax = 0;
  for (int i = 0; i < count; ++i) nmax = std::max(nmax, (int)n[i]);
  L->offer = off;
  off = align_up(off + sizeof(int32_t) * (size_t)count * nmax, 256);
  L->olen = off;
  off = align_up(off + sizeof(int64_t) * (size_t)count, 256);
  L->total = off;
  return ACS_OK;
}

int check_batch_args(const int32_t *n, int32_t count, const acs_params *p) {
  if (count < 1) return fail(ACS_E_INVALID, "count < 1");
  if (!n || !p) return fail(ACS_E_INVALID, "NULL argument");
  if (p->mode != ACS_ASYNC_ATOMIC && p->mode != ACS_ASYNC_RACY)
    return fail(ACS_E_UNSUPPORTED, "batches run in an asynchronous mode");
  if (p->memory != ACS_DENSE) return fail(ACS_E_UNSUPPORTED, "batches use the dense memory");
  if (p->local_search)
    return fail(ACS_E_UNSUPPORTED, "the local search runs on one instance, not in batches");
  for (int i = 0; i < count; ++i) {
    const int rc = check_params(n[i], p);
    if (rc) return rc;
  }
  return ACS_OK;
}

}  // namespace

extern "C" {

int acs_batch_workspace_bytes(const int32_t *n, int32_t count, const acs_params *p, size_t *out) {
  int rc = check_batch_args(n, count, p);
  if (rc) return rc;
  if (!out) return fail(ACS_E_INVALID, "out is NULL");
  BatchLayout L;
  int nitems = 0;
  rc = batch_layout(n, count, p, &L, &nitems);
  if (rc) return rc;
  *out = L.total;
  return ACS_OK;
}

int acs_batch_create(const double *const *coords, const int32_t *n, int32_t count,
                     const acs_params *p, acs_batch_t **out) {
  if (!out) return fail(ACS_E_INVALID, "out is NULL");
  *out = nullptr;
  int rc = check_batch_args(n, count, p);
  if (rc) return rc;
  if (!coords) return fail(ACS_E_INVALID, "coords is NULL");
  for (int i = 0; i < count; ++i)
    if (!coords[i]) return fail(ACS_E_INVALID, "coords[%d] is NULL", i);
  BatchLayout L;
  int nitems = 0;
  rc = batch_layout(n, count, p, &L, &nitems);
  if (rc) return rc;

  acs_batch_t *b = new (std::nothrow) acs_batch_t;
  if (!b) return fail(ACS_E_NOMEM, "host allocation failed");
  b->count = count;
  b->mode = (int)p->mode;
  auto bail = [&](int code) {
    std::string keep = g_err;
    release_batch(b);
    g_err = keep;
    return code;
  };
  if (p->stream) {
    b->stream = reinterpret_cast<hipStream_t>(p->stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(ACS_E_DEVICE, "stream creation failed"));
    b->own_stream = true;
  }
  if (p->workspace) {
    if (p->workspace_bytes < L.total)
      return bail(fail(ACS_E_BUFSIZE, "workspace of %zu bytes < %zu needed", p->workspace_bytes,
                       L.total));
    b->ws = reinterpret_cast<char *>(p->workspace);
  } else {
    hipError_t e = hipMalloc(&b->ws, L.total);
    if (e != hipSuccess) {
      b->ws = nullptr;
      (void)hipGetLastError();  // not the last error of later calls (see acs_create)
      return bail(fail(ACS_E_NOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e)));
    }
    b->own_ws = true;
  }
  if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess)
    return bail(fail(ACS_E_DEVICE, "event creation failed"));

  std::vector<acs::Dev> devs((size_t)count);
  std::vector<acs::Iter> iters((size_t)count);
  for (int i = 0; i < count; ++i) {
    acs_params pi = *p;
    pi.instance = p->instance + (uint32_t)i;
    pi.stream = b->stream;
    pi.workspace = b->ws + L.off[(size_t)i];
    size_t bytes = 0;
    acs_workspace_bytes(n[i], &pi, &bytes);
    pi.workspace_bytes = bytes;
    acs_t *h = nullptr;
    rc = acs_create(coords[i], n[i], &pi, &h);
    if (rc) return bail(rc);
    b->inst.push_back(h);
    devs[(size_t)i] = h->dev;
    // the unsynchronised mode's fallbacks scan whole rows (see launch_construct)
    if (p->mode != ACS_ASYNC_ATOMIC) devs[(size_t)i].fpre = nullptr;
    iters[(size_t)i] = h->base;
    b->nmax = std::max(b->nmax, n[i]);
    b->steps_per_iteration += (int64_t)h->m * (h->n - 1);
  }
  // candidate lanes per ant: the requested one, else every width that holds
  // the largest candidate list (64 always; 32 and 16 when cl fits)
  int clmax = 0;
  for (acs_t *h : b->inst) clmax = std::max(clmax, h->cl);
  b->clmax = clmax;
  // candidates (lanes per ant, updater wave): 64 lanes with updates issued
  // by the ant (update_path 1) or handed to an updater wave (update_path 2),
  // both unless one is asked for; 32 and 16 lanes issue their own
  std::vector<std::pair<int, bool>> widths;
  for (int w : {64, 32, 16}) {
    if (p->lanes_per_ant ? w != (int)p->lanes_per_ant : w < clmax) continue;
    if (w == 64) {
      if (p->update_path != 2) widths.push_back({64, false});
      if (p->update_path != 1) widths.push_back({64, true});
    } else {
      widths.push_back({w, false});
    }
  }
  // work lists: instances by decreasing n, so the longest chains start
  // first; a wave's ants always belong to one instance
  std::vector<int> order((size_t)count);
  for (int i = 0; i < count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return n[a] > n[c]; });
  b->d_devs = reinterpret_cast<acs::Dev *>(b->ws + L.devs);
  b->d_iters = reinterpret_cast<acs::Iter *>(b->ws + L.iters);
  b->d_flag = reinterpret_cast<uint32_t *>(b->ws + L.flag);
  b->d_offer = reinterpret_cast<int32_t *>(b->ws + L.offer);
  b->d_olen = reinterpret_cast<int64_t *>(b->ws + L.olen);
  int2 *d_items = reinterpret_cast<int2 *>(b->ws + L.items);
  std::vector<int2> items;
  items.reserve((size_t)nitems);
  for (const auto &wq : widths) {
    acs_batch_t::Variant v;
    v.lanes = wq.first;
    v.queued = wq.second;
    v.d_items = d_items + items.size();
    const int g = v.queued ? acs::kBatchQAntsPerBlock : 64 / v.lanes;
    for (int i : order)
      for (int a = 0; a < b->inst[(size_t)i]->m; a += g) items.push_back(make_int2(i, a));
    v.nitems = (int)(items.size() - (size_t)(v.d_items - d_items));
    b->var.push_back(v);
  }
  if (items.size() > (size_t)nitems)
    return bail(fail(ACS_E_STATE, "batch work lists exceed their reserved space"));
  if (hipMemcpyAsync(b->d_devs, devs.data(), sizeof(acs::Dev) * devs.size(),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipMemcpyAsync(b->d_iters, iters.data(), sizeof(acs::Iter) * iters.size(),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipMemcpyAsync(d_items, items.data(), sizeof(int2) * items.size(),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(fail(ACS_E_DEVICE, "copy of batch descriptors failed"));

  // each variant's iteration captured once as a graph (plain kernels only,
  // no memset nodes); a variant whose capture fails is launched directly
  for (auto &v : b->var) {
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) continue;
    const hipError_t le = acs::launch_batch_iteration(b->d_devs, b->d_iters, v.d_items, v.nitems,
                                                      b->count, b->nmax, b->clmax, b->mode, v.lanes,
                                                      v.queued ? 1 : 0, b->d_flag, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (le == hipSuccess && ce == hipSuccess && g) {
      v.graph = g;
      if (hipGraphInstantiate(&v.exec, g, nullptr, nullptr, 0) != hipSuccess) v.exec = nullptr;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  (void)hipGetLastError();
  if (b->var.size() == 1) b->chosen = 0;
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live_batches.insert(b);
  }
  *out = b;
  return ACS_OK;
}

int acs_batch_iterate(acs_batch_t *b, int32_t k) {
  if (!live_batch(b)) return fail(ACS_E_STATE, "invalid batch handle");
  if (k < 0) return fail(ACS_E_INVALID, "k < 0");
  if (k == 0) return ACS_OK;
  auto launch = [&](const acs_batch_t::Variant &v) -> hipError_t {
    if (v.exec) return hipGraphLaunch(v.exec, b->stream);
    return acs::launch_batch_iteration(b->d_devs, b->d_iters, v.d_items, v.nitems, b->count,
                                       b->nmax, b->clmax, b->mode, v.lanes, v.queued ? 1 : 0,
                                       b->d_flag, b->stream);
  };
  // the best-so-far exchange after every xperiod-th iteration of the batch
  auto exchange = [&]() -> hipError_t {
    ++b->iters_done;
    if (b->xperiod <= 0 || b->iters_done % b->xperiod != 0) return hipSuccess;
    return acs::launch_exchange_batch(b->d_devs, b->count, b->nmax, b->xtopology, b->d_offer,
                                      b->d_olen, b->stream);
  };
  // cleared outside the captured graphs (a memset node is not captured)
  HIP_TRY(hipMemsetAsync(b->d_flag, 0, sizeof(uint32_t), b->stream));
  double total_ms = 0.0;
  int i = 0;
  // tuning: one untimed warm-up iteration, then one timed iteration per
  // variant (each a full iteration of every instance), then the fastest
  while (b->chosen < 0 && i < k) {
    const int v = b->tuning_step - 1;
    HIP_TRY(hipEventRecord(b->e0, b->stream));
    HIP_TRY(launch(b->var[(size_t)(v < 0 ? 0 : v)]));
    HIP_TRY(hipEventRecord(b->e1, b->stream));
    HIP_TRY(exchange());
    HIP_TRY(hipStreamSynchronize(b->stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, b->e0, b->e1));
    total_ms += ms;
    if (v >= 0) b->var[(size_t)v].ms = ms;
    ++b->tuning_step;
    ++i;
    if (b->tuning_step > (int)b->var.size()) {
      int best = 0;
      for (int j = 1; j < (int)b->var.size(); ++j)
        if (b->var[(size_t)j].ms < b->var[(size_t)best].ms) best = j;
      b->chosen = best;
    }
  }
  if (i < k) {
    HIP_TRY(hipEventRecord(b->e0, b->stream));
    for (; i < k; ++i) {
      HIP_TRY(launch(b->var[(size_t)b->chosen]));
      HIP_TRY(exchange());
    }
    HIP_TRY(hipEventRecord(b->e1, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, b->e0, b->e1));
    total_ms += ms;
  }
  const double ms = total_ms;
  b->iterate_ms = ms;
  for (acs_t *h : b->inst) {
    h->iter += (uint32_t)k;
    h->iterate_ms = ms;
    h->construct_ms = 0.0;
    h->construct_launches = 0;
  }
  uint32_t flag = 0;
  HIP_TRY(hipMemcpy(&flag, b->d_flag, sizeof flag, hipMemcpyDeviceToHost));
  if (flag)
    return fail(ACS_E_DEVICE, "a bounded device wait was exhausted in a batch instance (flag %u: "
                              "1 grid barrier, 2 update ring); local updates may be missing", flag);
  return ACS_OK;
}

int acs_batch_set_exchange(acs_batch_t *b, int32_t topology, int32_t period) {
  if (!live_batch(b)) return fail(ACS_E_STATE, "invalid batch handle");
  if (topology != 0 && topology != 1)
    return fail(ACS_E_INVALID, "topology = %d not in {0, 1}", topology);
  if (period < 0) return fail(ACS_E_INVALID, "period = %d < 0", period);
  for (acs_t *h : b->inst)
    if (h->n != b->inst[0]->n)
      return fail(ACS_E_INVALID, "the exchange needs colonies of one instance (n %d and %d)",
                  b->inst[0]->n, h->n);
  b->xtopology = topology;
  b->xperiod = period;
  b->iters_done = 0;
  return ACS_OK;
}

int acs_batch_info(acs_batch_t *b, int32_t *count, int64_t *steps_per_iteration,
                   int32_t *graph, double *last_iterate_ms) {
  if (!live_batch(b)) return fail(ACS_E_STATE, "invalid batch handle");
  if (count) *count = b->count;
  if (steps_per_iteration) *steps_per_iteration = b->steps_per_iteration;
  if (graph) *graph = b->var[(size_t)(b->chosen < 0 ? 0 : b->chosen)].exec ? 1 : 0;
  if (last_iterate_ms) *last_iterate_ms = b->iterate_ms;
  return ACS_OK;
}

int acs_batch_tuning(acs_batch_t *b, int32_t *chosen, int32_t *count, int32_t *lanes,
                     int32_t *updater, double *ms, int32_t cap) {
  if (!live_batch(b)) return fail(ACS_E_STATE, "invalid batch handle");
  if (chosen) *chosen = b->chosen;
  if (count) *count = (int32_t)b->var.size();
  for (int j = 0; j < (int)b->var.size() && j < cap; ++j) {
    if (lanes) lanes[j] = b->var[(size_t)j].lanes;
    if (updater) updater[j] = b->var[(size_t)j].queued ? 1 : 0;
    if (ms) ms[j] = b->var[(size_t)j].ms;
  }
  return ACS_OK;
}

int acs_batch_instance(acs_batch_t *b, int32_t i, acs_t **out) {
  if (!live_batch(b)) return fail(ACS_E_STATE, "invalid batch handle");
  if (i < 0 || i >= b->count || !out) return fail(ACS_E_INVALID, "instance %d out of range", i);
  *out = b->inst[(size_t)i];
  return ACS_OK;
}

int acs_batch_best_tour(acs_batch_t *b, int32_t i, int32_t *tour_out, int64_t *len_out) {
  acs_t *h = nullptr;
  const int rc = acs_batch_instance(b, i, &h);
  if (rc) return rc;
  return acs_best_tour(h, tour_out, len_out);
}

// ---------------------------------------------------------------------------
// Learned edge prior.
// ---------------------------------------------------------------------------
int acs_prior_features(acs_t *h, float *X_dev) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (!X_dev) return fail(ACS_E_INVALID, "X is NULL");
  if (h->cl != 16) return fail(ACS_E_UNSUPPORTED, "the prior uses cl = 16 (handle has %d)", h->cl);
  HIP_TRY(acs::launch_prior_features(h->dev, X_dev, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACS_OK;
}

int acs_prior_forward(const float *P_dev, const float *X_dev, int32_t rows, float *Z_dev,
                      void *stream) {
  if (!P_dev || !X_dev || !Z_dev || rows < 0) return fail(ACS_E_INVALID, "bad argument");
  if (rows == 0) return ACS_OK;
  HIP_TRY(acs::launch_prior_forward(P_dev, X_dev, rows, Z_dev,
                                    reinterpret_cast<hipStream_t>(stream)));
  return ACS_OK;
}

int acs_prior_grad(const float *P_dev, const float *X_dev, const float *Y_dev, int32_t rows,
                   float *G_dev, float *loss_dev, void *stream) {
  if (!P_dev || !X_dev || !Y_dev || !G_dev || !loss_dev || rows < 1)
    return fail(ACS_E_INVALID, "bad argument");
  HIP_TRY(acs::launch_prior_grad(P_dev, X_dev, Y_dev, rows, G_dev, loss_dev,
                                 reinterpret_cast<hipStream_t>(stream)));
  return ACS_OK;
}

int acs_prior_adam(float *P_dev, float *G_dev, float *M_dev, float *V_dev, int32_t step, float lr,
                   float beta1, float beta2, float eps, void *stream) {
  if (!P_dev || !G_dev || !M_dev || !V_dev || step < 1) return fail(ACS_E_INVALID, "bad argument");
  HIP_TRY(acs::launch_prior_adam(P_dev, G_dev, M_dev, V_dev, step, lr, beta1, beta2, eps,
                                 reinterpret_cast<hipStream_t>(stream)));
  return ACS_OK;
}

int acs_prior_apply(acs_t *h, const float *P_dev) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (!P_dev) return fail(ACS_E_INVALID, "P is NULL");
  if (h->cl != 16) return fail(ACS_E_UNSUPPORTED, "the prior uses cl = 16 (handle has %d)", h->cl);
  HIP_TRY(acs::launch_prior_apply(h->dev, P_dev, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACS_OK;
}

int acs_set_candidate_scores(acs_t *h, const float *scores) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  if (!scores) return fail(ACS_E_INVALID, "scores is NULL");
  const size_t cnt = (size_t)h->n * h->cl;
  for (size_t e = 0; e < cnt; ++e)
    if (!(scores[e] > 0.f) || !std::isfinite(scores[e]))
      return fail(ACS_E_INVALID, "score %zu is not a positive finite number", e);
  std::vector<uint32_t> rec(cnt * 4);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(rec.data(), h->ws + h->L.crec, rec.size() * sizeof(uint32_t),
                    hipMemcpyDeviceToHost));
  for (size_t e = 0; e < cnt; ++e) std::memcpy(&rec[4 * e + 2], &scores[e], sizeof(float));
  HIP_TRY(hipMemcpy(h->ws + h->L.crec, rec.data(), rec.size() * sizeof(uint32_t),
                    hipMemcpyHostToDevice));
  return ACS_OK;
}

int acs_candidate_weights(acs_t *h, float *out, size_t count) {
  if (!live(h)) return fail(ACS_E_STATE, "invalid handle");
  const size_t cnt = (size_t)h->n * h->cl;
  if (!out || count < cnt) return fail(ACS_E_BUFSIZE, "need %zu floats", cnt);
  std::vector<uint32_t> rec(cnt * 4);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(rec.data(), h->ws + h->L.crec, rec.size() * sizeof(uint32_t),
                    hipMemcpyDeviceToHost));
  for (size_t e = 0; e < cnt; ++e) std::memcpy(&out[e], &rec[4 * e + 2], sizeof(float));
  return ACS_OK;
}

void acs_batch_destroy(acs_batch_t *b) {
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    if (!b || !g_live_batches.count(b)) return;
    g_live_batches.erase(b);
  }
  release_batch(b);
}


}  // extern "C"
