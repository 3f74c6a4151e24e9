// mc_host_pool.cpp -- pools of pinned host blocks and events (see mc_host_pool.h).
#include "mc_host_pool.h"

#include <map>
#include <mutex>
#include <utility>
#include <vector>

namespace mc {
namespace {

std::mutex g_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_blocks;  // (device, class) -> free
std::map<int, std::vector<hipEvent_t>> g_events;                 // device -> free
std::map<int, std::vector<hipStream_t>> g_streams;               // device -> free

size_t size_class(size_t bytes) {
  size_t c = 4096;
  while (c < bytes) c <<= 1;
  return c;
}

int device() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  return d;
}

}  // namespace

void* pinned_get(size_t bytes) {
  const size_t c = size_class(bytes);
  const int d = device();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = g_blocks[{d, c}];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pinned_put(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_blocks[{device(), size_class(bytes)}].push_back(p);
}

hipEvent_t event_get() {
  const int d = device();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = g_events[d];
    if (!v.empty()) {
      hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void event_put(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_events[device()].push_back(e);
}

hipStream_t stream_get() {
  const int d = device();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = g_streams[d];
    if (!v.empty()) {
      hipStream_t s = v.back();
      v.pop_back();
      return s;
    }
  }
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return s;
}

void stream_put(hipStream_t s) {
  if (!s) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_streams[device()].push_back(s);
}

}  // namespace mc
