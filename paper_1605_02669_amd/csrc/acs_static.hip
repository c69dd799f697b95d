// acs_solve_static: the whole method (instance preparation, iterations of
// Alg. 1, best-so-far read-back) for callers that cannot allocate device
// memory.  Its device workspace is one file-scope array of this library,
// `scratch`, which every GPU the library runs on holds for the life of the
// process; the call allocates nothing.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/acs.h"
#include "acs_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)ACS_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Calls are serialised: every call on a device uses that device's one array.
std::mutex g_mu;
// Device address of `scratch` per device (the array's name is a host-side
// stand-in, not a device address); looked up once per device with that
// device current.
void *g_scratch[kMaxDevices];
// Host scratch for the eta^beta table.
float g_eta[acs::kEtaHostEntries];

int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return acs::set_error(ACS_E_DEVICE, "no current HIP device");
  if (dev >= kMaxDevices) return acs::set_error(ACS_E_UNSUPPORTED, "device index above 63");
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[256];
      snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
               hipGetErrorString(e));
      return acs::set_error(ACS_E_DEVICE, msg);
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return ACS_OK;
}

}  // namespace

extern "C" int acs_solve_static(const double *coords_xy, int32_t n, const acs_params *p,
                                int32_t iterations, int32_t *tour_out, int64_t *len_out) {
  if (!p) return acs::set_error(ACS_E_INVALID, "params is NULL");
  if (p->workspace)
    return acs::set_error(ACS_E_INVALID,
                          "params.workspace must be NULL: acs_solve_static uses its own");
  size_t need = 0;
  int rc = acs_workspace_bytes(n, p, &need);
  if (rc) return rc;
  if (need > kScratchBytes) {
    char msg[256];
    snprintf(msg, sizeof msg,
             "n = %d needs %zu bytes of device workspace; the static workspace holds %zu",
             (int)n, need, kScratchBytes);
    return acs::set_error(ACS_E_BUFSIZE, msg);
  }
  std::lock_guard<std::mutex> lock(g_mu);
  void *ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return acs::solve_in(coords_xy, n, p, iterations, static_cast<char *>(ws), kScratchBytes, g_eta,
                       tour_out, len_out);
}
