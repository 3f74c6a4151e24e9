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
  uint32_t hkeep;           // bits of the key hash kept (0 = all; testing only)
};

// Keys each thread of the persistent kernel inserts per round trip: 1 or 2 as asked,
// else (0) 2 for keys of one or two words and 1 for four-word keys, whose two-key
// kernel needs more registers than three wavefronts per SIMD allow.
inline uint32_t lane_items_for(uint32_t asked, uint32_t W) {
  return asked == 1u || asked == 2u ? asked : (W == 4u ? 1u : 2u);
}

// Library error code (MC_E_*) of a device error flag (kDevErr*).
inline int dev_error_code(unsigned int e) {
  switch (e) {
    case 0: return MC_OK;
    case kDevErrTableFull: return MC_E_TABLE_FULL;
    case kDevErrOverflow: return MC_E_OVERFLOW;
    case kDevErrSplit: return MC_E_INTERNAL;
    case kDevErrAbort: return MC_E_ABORTED;
    default: return MC_E_DEVICE;
  }
}

struct LevelArgs {
  QueryArgs q;
  uint32_t in_idx, out_idx, clr_idx;  // rotating frontier counters
  uint32_t fcap;
  const unsigned int* abort;  // host-set stop request (pinned host word), or null
};

// Saved frontier of a partition explored across several launches.
struct PartState {
  unsigned long long k[4];
  uint32_t slot, depth;
  uint32_t status;  // 0 not started, 1 in progress (one saved frontier state), 2 done
  uint32_t pad;
};
static_assert(sizeof(PartState) == 48, "PartState layout");

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
  uint32_t n_parts;   // partitions of the model (entries of pstate)
  uint32_t bb;        // branch and bound: prune at min(T, ctrl->bound), every new
                      // terminal lowers ctrl->bound
  PartState* pstate;  // one per partition when partitions may yield, else null
  uint32_t hkeep;     // bits of the key hash kept (0 = all; testing only)
  uint32_t refloor;   // a continued exploration: every state with clock < refloor was
                      // inserted before, and one found again is still expanded, so the
                      // walk reaches the new states past it (0 = a fresh exploration)
};

// One partition of a persistent launch: rounds [r0, r1) of one configuration's subgraph
// (r1 = kRoundsToEnd: through its terminal).  After r full rounds the subgraph of a
// configuration passes through the single state (c, r*d, n - r*m, every unit idle), so a
// block of whole rounds can be explored from that state on its own.
struct Part {
  uint32_t model, cfg, r0, r1;  // r0 = r1 = kRunSlice: a run slice [j0, j1)
  uint32_t pidx;  // index of the partition within its model (its PartState)
  uint32_t j0, j1;  // a run slice's states; else j1 > 0 caps the runs from SELECT
  uint32_t pad;
};
static_assert(sizeof(Part) == 32, "Part layout");

// Partitions of a persistent launch, largest first.
struct PartQueue {
  const ModelDev* models;
  const Part* parts;
  uint32_t n_parts;
  uint32_t batch_items;  // states generated per super-step batch before waiting (target)
  unsigned int* head;
  uint32_t slice;        // super-step levels per partition before it yields (0 = no limit)
  uint32_t reverse;      // take the partitions smallest first
  Part* yielded;         // partitions that yielded, for the next launch
  unsigned int* n_yielded;
  // host-set stop request (a pinned host word read at system scope), or null: a
  // partition taken after it is set is not explored, so the launch drains quickly and
  // every workgroup still exits normally
  const unsigned int* abort;
};

template <int W>
hipError_t launch_seed(hipStream_t st, const QueryArgs& q, Seed* seeds, void* front0);
template <int W>
hipError_t launch_level(hipStream_t st, uint32_t grid, const LevelArgs& la, const void* fin,
                        void* fout);
// All models of the queue have key width W (1, 2, 4).  items: keys per lane per insert
// round trip, as for lane_items_for.  general: some configuration of some model of the
// queue has waves or two-operation periods (ModelHost::general); false selects the
// engine built for uniform phases only.  hetero: some model runs on units of unequal
// speed (ModelHost::hetero), which selects the build with determined ADVANCE chains.
hipError_t launch_super(hipStream_t st, uint32_t W, uint32_t grid, uint32_t block,
                        uint32_t items, const PartQueue& pq, bool general, bool hetero);

// Runs up to three launches (one per key width) concurrently on sub-streams forked from
// and joined back into a main stream with events; usable inside stream capture.
struct Fork {
  hipStream_t sub[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[3] = {nullptr, nullptr, nullptr};
  hipError_t create() {
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&sub[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    }
    return e;
  }
  void destroy() {
    for (int i = 0; i < 3; ++i) {
      if (sub[i]) (void)hipStreamDestroy(sub[i]);
      if (join[i]) (void)hipEventDestroy(join[i]);
      sub[i] = nullptr;
      join[i] = nullptr;
    }
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
  }
};

// queue[w] (w = 0, 1, 2 for key widths 1, 2, 4) with n_parts == 0 are skipped
hipError_t launch_super_fork(hipStream_t main, Fork& f, const PartQueue (&queue)[3],
                             const uint32_t (&grid)[3], uint32_t block, uint32_t items,
                             bool general, bool hetero);
hipError_t launch_seed_models(hipStream_t st, const ModelDev* models, uint32_t n);
hipError_t launch_reset_models(hipStream_t st, const ModelDev* models, uint32_t n,
                               unsigned int* head, uint32_t n_heads);
// Counters and clocks kept, partition bookkeeping reset: before a launch that continues
// an exploration on the same visited set.
hipError_t launch_resume_models(hipStream_t st, const ModelDev* models, uint32_t n,
                                unsigned int* head, uint32_t n_heads);
// *out += states of the visited set (slots slots) with clock <= T; *out is not cleared.
template <int W>
hipError_t launch_count_le(hipStream_t st, const unsigned char* table, unsigned long long slots,
                           const Layout& L, const CfgRec* cfgs, uint32_t T,
                           unsigned long long* out);
template <int W>
hipError_t launch_find(hipStream_t st, const QueryArgs& q, const unsigned long long* key);
template <int W>
hipError_t launch_chase(hipStream_t st, const QueryArgs& q, unsigned long long* out, uint32_t cap);
hipError_t launch_clear(hipStream_t st, void* p, unsigned long long bytes);
hipError_t launch_reset(hipStream_t st, Ctrl* ctrl, uint32_t* tc, uint32_t n_cfg);
hipError_t launch_simulate(hipStream_t st, const QueryArgs& q, unsigned long long seed);

// ---- swarm search (Sec. 5) ----------------------------------------------------------
// One member of a swarm (device record, 80 bytes; mirrored by mc_swarm_member).
struct SwarmMember {
  unsigned long long walks, trails, steps;
  unsigned long long best_walk_start;  // member step at which the best trail's walk began
  unsigned long long first_step;       // member step at which its first trail ended (~0: none)
  unsigned long long start_ticks, first_ticks;  // device clock (100 MHz) at start / first trail
  uint32_t best_clock, best_cfg;       // kNoClock / kParentNone without trails
  uint32_t first_clock, first_cfg;     // the member's first trail
  uint32_t pad[2];
};
static_assert(sizeof(SwarmMember) == 80, "SwarmMember layout");

struct SwarmArgs {
  const CfgRec* cfgs;
  uint32_t n_cfg, m;
  unsigned long long seed;    // base seed; member i uses splitmix64(seed + i)
  unsigned long long budget;  // member steps before no new walk starts
  uint32_t members, bits_log2;
  uint32_t prune, T;          // over-time property with threshold T, else non-termination
  uint32_t* bits;             // members x 2^bits_log2 bits, zero
  SwarmMember* out;           // members records
  uint8_t speed[kMaxCU];      // speed of each unit (1 = full speed)
};
hipError_t launch_swarm(hipStream_t st, const SwarmArgs& a);
// Replays the walk of member seed `mseed` that began at member step `start`, writing the
// rows (cfg, clock, pending, rem[0..m-1]) of its states root first into `rows` (at most
// `cap` rows; ctrl->trace_len gets the number written, ctrl->error kDevErrTrace if more).
hipError_t launch_swarm_replay(hipStream_t st, const SwarmArgs& a, Ctrl* ctrl,
                               unsigned long long mseed, unsigned long long start,
                               uint32_t* rows, uint32_t cap);

}  // namespace mc
