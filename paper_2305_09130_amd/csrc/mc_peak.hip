// mc_peak.hip -- random-access peak probes of the device (measurement only).
//
// The visited set of the explorer is a hash table far larger than the 256 MB
// Infinity Cache for the large workloads, so its ceiling is the rate at which the chip
// serves independent random accesses to HBM, not the streaming bandwidth.  These
// kernels measure that ceiling on the same buffer sizes:
//   * random 64-bit compare-and-swap (the claim of a visited-set slot): every lane
//     issues kIlp independent CAS to uniformly random words per round;
//   * random 64-byte line reads (one HBM access granule per random touch): four lanes
//     read the four 16-byte quarters of one uniformly random line, kIlp lines in
//     flight per lane group.
// Addresses come from a 64-bit finalizer of (lane, round), so every access of a
// launch is independent of the values returned.  Each kernel folds what it read into
// one word per wavefront (an atomic XOR), so nothing is optimised away and almost no
// bytes are written besides the CAS themselves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcpeak.h"

namespace {

constexpr int kIlp = 4;

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  // the 64-bit finalizer of MurmurHash3 (Appleby)
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__device__ __forceinline__ unsigned long long wave_xor(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o);
  return v;
}

__global__ __launch_bounds__(256) void k_random_cas(unsigned long long* buf,
                                                    unsigned long long mask, uint32_t rounds,
                                                    unsigned long long seed,
                                                    unsigned long long* sink) {
  const unsigned long long gid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long acc = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    unsigned long long old[kIlp];
#pragma unroll
    for (int j = 0; j < kIlp; ++j) {
      const unsigned long long h = mix64(seed ^ (gid * (unsigned long long)(rounds * kIlp) +
                                                 (unsigned long long)(r * kIlp + j)));
      // a key never equal to the cleared value ~0
      const unsigned long long key = h >> 1;
      old[j] = atomicCAS(buf + (h & mask), ~0ull, key);
    }
#pragma unroll
    for (int j = 0; j < kIlp; ++j) acc ^= old[j];
  }
  acc = wave_xor(acc);
  if ((threadIdx.x & 63u) == 0u) atomicXor(sink, acc);
}

__global__ __launch_bounds__(256) void k_random_read(const uint4* __restrict__ buf,
                                                     unsigned long long line_mask,
                                                     uint32_t rounds, unsigned long long seed,
                                                     unsigned long long* sink) {
  const unsigned long long gid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long grp = gid >> 2;  // four lanes share one 64-byte line
  const uint32_t quarter = (uint32_t)(gid & 3u);
  uint32_t acc = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    uint4 v[kIlp];
#pragma unroll
    for (int j = 0; j < kIlp; ++j) {
      const unsigned long long h = mix64(seed ^ (grp * (unsigned long long)(rounds * kIlp) +
                                                 (unsigned long long)(r * kIlp + j)));
      v[j] = buf[(h & line_mask) * 4u + quarter];
    }
#pragma unroll
    for (int j = 0; j < kIlp; ++j) acc ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
  }
  const unsigned long long a = wave_xor((unsigned long long)acc);
  if ((threadIdx.x & 63u) == 0u) atomicXor(sink, a);
}

bool pow2(unsigned long long x) { return x && !(x & (x - 1)); }

}  // namespace

extern "C" {

int mcp_random_cas(void* buf, uint64_t n_words, uint32_t grid, uint32_t rounds, uint64_t seed,
                   void* sink, void* stream, uint64_t* n_ops) {
  if (!buf || !sink || !pow2(n_words) || !grid || !rounds) return MCP_E_INVAL;
  hipLaunchKernelGGL(k_random_cas, dim3(grid), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<unsigned long long*>(buf), n_words - 1, rounds, seed,
                     reinterpret_cast<unsigned long long*>(sink));
  if (hipGetLastError() != hipSuccess) return MCP_E_DEVICE;
  if (n_ops) *n_ops = (uint64_t)grid * 256u * rounds * kIlp;
  return MCP_OK;
}

int mcp_random_read(const void* buf, uint64_t n_lines, uint32_t grid, uint32_t rounds,
                    uint64_t seed, void* sink, void* stream, uint64_t* n_lines_read) {
  if (!buf || !sink || !pow2(n_lines) || !grid || !rounds) return MCP_E_INVAL;
  hipLaunchKernelGGL(k_random_read, dim3(grid), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint4*>(buf),
                     n_lines - 1, rounds, seed, reinterpret_cast<unsigned long long*>(sink));
  if (hipGetLastError() != hipSuccess) return MCP_E_DEVICE;
  if (n_lines_read) *n_lines_read = (uint64_t)grid * 64u * rounds * kIlp;
  return MCP_OK;
}

}  // extern "C"
