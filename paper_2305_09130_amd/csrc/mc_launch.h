// mc_launch.h -- host-side launch helpers of the exploration kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mc_device.h"

namespace mc {

constexpr uint32_t kLevelBlock = 128;

struct QueryArgs {
  Ctrl* ctrl;
  uint32_t* tc;             // per-configuration least terminal clock
  const CfgRec* cfgs;
  unsigned char* table;
  unsigned long long mask;  // slots - 1
  Layout L;
  uint32_t n_cfg;
  uint32_t prune;           // check(T): drop states with clock > T
  uint32_t T;
  uint32_t max_clock;       // bound of the packed clock field
};

struct LevelArgs {
  QueryArgs q;
  uint32_t in_idx, out_idx, clr_idx;  // rotating frontier counters
  uint32_t fcap;
};

// One model of a persistent launch (device memory, written by the host).
struct ModelDev {
  Ctrl* ctrl;
  uint32_t* tc;
  const CfgRec* cfgs;
  Seed* seeds;
  unsigned char* table;
  unsigned long long mask;  // slots - 1
  Layout L;
  uint32_t n_cfg;
  uint32_t prune;
  uint32_t T;
  uint32_t max_clock;
  uint32_t pad[2];
};

// Partitions of a persistent launch: (model index, configuration), largest first.
struct PartQueue {
  const ModelDev* models;
  const uint2* parts;
  uint32_t n_parts;
  uint32_t batch_items;  // states generated per super-step batch before waiting (target)
  unsigned int* head;
};

template <int W>
hipError_t launch_seed(hipStream_t st, const QueryArgs& q, Seed* seeds, void* front0);
template <int W>
hipError_t launch_level(hipStream_t st, uint32_t grid, const LevelArgs& la, const void* fin,
                        void* fout);
hipError_t launch_super(hipStream_t st, uint32_t grid, uint32_t block, const PartQueue& pq);
hipError_t launch_seed_models(hipStream_t st, const ModelDev* models, uint32_t n);
hipError_t launch_reset_models(hipStream_t st, const ModelDev* models, uint32_t n,
                               unsigned int* head);
template <int W>
hipError_t launch_find(hipStream_t st, const QueryArgs& q, const unsigned long long* key);
template <int W>
hipError_t launch_chase(hipStream_t st, const QueryArgs& q, unsigned long long* out, uint32_t cap);
hipError_t launch_clear(hipStream_t st, void* p, unsigned long long bytes);
hipError_t launch_reset(hipStream_t st, Ctrl* ctrl, uint32_t* tc, uint32_t n_cfg);
hipError_t launch_simulate(hipStream_t st, const QueryArgs& q, unsigned long long seed);

}  // namespace mc
