// mc_host_pool.h -- process-wide pools of pinned host staging blocks and HIP events.
// A tuning query loads a model, runs and frees it; allocating and freeing pinned host
// memory and events each time costs driver calls of tens of microseconds (freeing
// pinned memory can wait for the device).  Blocks and events are kept per device and
// reused; they are released to the driver only when the process ends.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mc {

// A pinned host block of at least `bytes` (rounded up to a power of two, at least
// 4 KiB), or nullptr.  Return it with pinned_put and the same size.
void* pinned_get(size_t bytes);
void pinned_put(void* p, size_t bytes);

// A timing event of the current device, or nullptr.  Return it with event_put.
hipEvent_t event_get();
void event_put(hipEvent_t e);

}  // namespace mc
