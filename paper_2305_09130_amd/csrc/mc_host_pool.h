// mc_host_pool.h -- process-wide pools of pinned host staging blocks, HIP events and
// streams.  A tuning query loads a model, runs and frees it; allocating and freeing pinned
// host memory, events and streams each time costs driver calls of tens of microseconds
// (freeing pinned memory can wait for the device).  They are kept per device and reused;
// they are released to the driver only when the process ends.
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

// A non-blocking stream of the current device at the default priority, or nullptr.
// Return it, with no work left in it, with stream_put.
hipStream_t stream_get();
void stream_put(hipStream_t s);

}  // namespace mc
