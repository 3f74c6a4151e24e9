// mc_static.hip -- min_time over a static device scratch, for callers that cannot
// allocate device memory.
//
// The workspace of mc_min_time (visited set, counters, tables, frontiers, trace buffer)
// lives here in one file-scope device array.  Each device holds its own copy of the
// array, from the first call on that device until the process ends.  Its device address
// is looked up once per device with hipGetSymbolAddress and cached; the array's name is
// a host-side stand-in and is never passed to a kernel or a copy.  The call creates no
// pinned memory, events or streams and allocates no device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mctune.h"
#include "mc_model.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on the first call on the device).
int scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return MC_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MC_E_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return MC_OK;
}

}  // namespace

extern "C" {

int mc_min_time_static(const mc_desc* d, const mc_opts* o, void* stream, uint32_t* t_min,
                       uint32_t* argmin, size_t cap, size_t* n_argmin, mc_stats* st) {
  if (!d || !t_min || !n_argmin) return MC_E_INVAL;
  size_t need = 0;
  int rc = mc_workspace_bytes(d, o, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return MC_E_NOMEM;
  void* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  return mc::min_time_in_place(d, o, ws, kScratchBytes, stream, t_min, argmin, cap, n_argmin,
                               st);
}

}  // extern "C"
