// mc_model.h -- host-side model logic shared by the library's host code and kernels:
// descriptor validation, per-configuration operation tables, packed-key layout and
// the exact sizes of the lock-step round structure used to size device memory.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mctune.h"

namespace mc {

constexpr int kMaxCU = (int)MC_MAX_CU;
// key fields: cfg, pending, clock, rem_0..rem_{m-1}; with Layout::shared_rem the
// fields after the clock are the busy-unit mask and the one remaining time they share
constexpr int kFields = 3 + kMaxCU;
constexpr int kFCfg = 0, kFPending = 1, kFClock = 2, kFRem = 3;
constexpr int kMaxPhases = 4;

constexpr uint32_t kParentNone = 0xFFFFFFFFu;  // no parent recorded (empty slot)
constexpr uint32_t kParentRoot = 0xFFFFFFFEu;  // the root has no parent
constexpr uint64_t kEmptyWord = ~0ull;         // empty slot (word 0)
constexpr uint32_t kNoClock = 0xFFFFFFFFu;

// Packed key layout.  Fields never straddle a 64-bit word; the configuration index
// sits in the low bits of word 0 and all-ones never encodes a valid configuration,
// so no valid key has word 0 equal to kEmptyWord.
struct Layout {
  uint8_t word[kFields];
  uint8_t shift[kFields];
  uint8_t width[kFields];
  uint8_t m;
  uint8_t W;  // key words: 1, 2 or 4
  uint8_t used_bits;
  uint8_t hetero;            // units of unequal speed
  uint8_t shared_rem;        // equal units: busy mask + one remaining time (kFRem, kFRem + 1)
  uint8_t speed[kMaxCU];     // cycles per cycle of work of each unit (1 = full speed)
  // equal units: the clock is not stored (width 0).  Every run proceeds in lock-step
  // rounds, so a state's clock follows from its other fields and its configuration's
  // n and d: ceil((n - pending - busy)/m) * d, plus d - rem while units are busy
  // (implied_clock).  Decoding then needs the configuration records.
  uint8_t clock_implied;
  uint8_t pad_[3];
  uint32_t n_cfg;            // configurations; the root carries cfg = n_cfg
};

// One configuration: workgroup count, duration and the timed operation phases of one
// wave (operations of zero latency add no end and are dropped).  A workgroup is
// `waves` back-to-back repetitions of the wave, each lasting dw with bw ends.  Phase j
// of a wave holds cnt[j] ends on a grid that starts at t0[j] (a phase may start after
// the previous phase's last end when its first operation is longer than its period):
//   la[j] = 0: one operation per period, ends at t0[j] + k*lat[j], k = 1..cnt[j];
//   la[j] > 0: two operations per period lat[j], ends at t0[j] + k*lat[j] + la[j] and
//              t0[j] + (k+1)*lat[j], k = 0..cnt[j]/2 - 1 (cnt[j] even).
// i0[j] = ends of the wave before phase j.
struct CfgRec {
  uint32_t n;      // workgroups
  uint32_t d;      // workgroup duration = last operation end = waves * dw
  uint32_t b;      // number of distinct operation ends = waves * bw
  uint32_t nph;    // timed phases of one wave
  uint32_t cnt[kMaxPhases];
  uint32_t lat[kMaxPhases];
  uint32_t t0[kMaxPhases];
  uint32_t i0[kMaxPhases];
  uint32_t la[kMaxPhases];
  uint32_t waves;  // repetitions of the wave, >= 1
  uint32_t dw;     // duration of one wave
  uint32_t bw;     // operation ends of one wave
  uint32_t tc;     // ceil(n/m) * d: clock of every terminal of this configuration
  uint32_t pad[4];
};
static_assert(sizeof(CfgRec) == 128, "CfgRec layout");

// Cut points of a configuration's determined part on units of unequal speed: instants t
// at which every unit is busy, work is pending and no workgroup ends (so the state at t
// has a single predecessor chain and lies on every run), with the state's depth from the
// root and the states counted up to it.
struct ChainCut {
  uint64_t t = 0, depth = 0, states = 0;
};
constexpr uint64_t kCutSpacing = 32;  // least distance between recorded cut points, in states
constexpr size_t kMaxCuts = 4096;     // most cut points recorded per configuration
constexpr uint64_t kMaxPeriodLcm = 1u << 12;  // longest period (in workgroups of speed 1)
                                              // that the walk repeats rather than walks

struct ModelHost {
  mc_desc desc{};
  std::vector<uint32_t> params;  // n_cfg * 4
  std::vector<CfgRec> cfgs;
  Layout layout{};
  uint32_t m = 0, n_cfg = 0, W = 1;
  bool general = false;          // some configuration has waves or two-operation periods,
                                 // or the units have unequal speeds
  bool hetero = false;           // units of unequal speed (no closed-form counts)
  uint32_t speed[kMaxCU] = {1, 1, 1, 1, 1, 1, 1, 1};
  uint64_t states = 0;           // exact reachable count, root included
  uint64_t max_depth = 0;        // longest path (edges)
  uint32_t max_clock = 0;
  uint32_t max_n = 0, max_d = 0;
  std::vector<uint64_t> cfg_states;  // reachable states per configuration subgraph
  // unequal units: cut points per configuration walked; configuration c uses those of
  // cut_of[c] (the first configuration whose record, but for its terminal clock, equals its
  // own: their walks are the same)
  std::vector<std::vector<ChainCut>> cut_cands;
  std::vector<uint32_t> cut_of;
  uint64_t frontier_bound = 0;   // widest BFS level
};

// Validates d and fills h.  Returns MC_OK or MC_E_INVAL with a message in err.
int build_model(const mc_desc* d, ModelHost* h, std::string* err);

// One partition of a model's exploration: rounds [r0, r1) of configuration cfg
// (r1 = kRoundsToEnd: through the terminal), with its expected state count.
constexpr uint32_t kRoundsToEnd = 0xFFFFFFFFu;
constexpr uint32_t kMinBlockRounds = 8;     // shortest block worth a partition of its own,
constexpr uint32_t kMinBlockStates = 2048;  // unless fewer rounds already hold this many
// A run slice: states j0 <= j < j1 of every lock-step run of a configuration with a
// single round (n <= m workgroups all start at clock 0, so run j of every choice of
// units is (c, E_j, 0, d - E_j on the chosen units)); the partition that holds the
// configuration's SELECT closure then explores its runs only up to j1 of its plan
// (its `j1`, 0 = whole runs).
constexpr uint32_t kRunSlice = 0xFFFFFFFEu;
// A chain slice (units of unequal speed; Part::r0 = kChainSlice): the configuration's
// states with clock in [j0, r1] along its determined part (r1 = kNoClock: to the end,
// tails included).  It starts at the SELECT state when j0 = 0, else at the state at
// clock j0, an instant of the determined part at which no workgroup ends (j1 = that
// state's depth), and ends on the state at clock r1, another such instant, which the
// next slice starts from.
constexpr uint32_t kChainSlice = 0xFFFFFFFDu;
constexpr uint32_t kMinSlice = 1024, kMaxSlice = 8192;
struct PartPlan {
  uint32_t cfg, r0, r1;
  uint64_t states;
  uint32_t j0 = 0, j1 = 0;
};

// Partitions of a model.  Each configuration's subgraph is cut into blocks of whole
// rounds of about `target` states each (target 0: never cut).  Block k starts at the
// state reached after r0 full rounds, (c, r0 d, n - r0 m, all units idle), which every
// path of the configuration passes through.  A cut needs the configuration index, the
// pending count and the clock in key word 0: two blocks then share no word-0 value
// except their common boundary state.  Under the same condition a configuration with a
// single round whose runs are longer than a slice is cut into run slices: each spans
// every run of the configuration over about max(1024, min(8192, target) / runs) states
// of each (every state of a slice has a clock no other partition's states have).
// With clock_max, the blocks and run slices of rounds that start after clock_max are left
// out (a query that drops every state past clock_max explores nothing there).
void plan_parts(const ModelHost& h, uint64_t target, std::vector<PartPlan>* out,
                uint64_t clock_max = ~0ull);

// Whether key word 0 alone tells apart the states of different rounds and of different
// positions along a round's runs (configuration, pending count and either the clock or,
// when the clock is implied, the busy mask and time left): the condition for cutting a
// configuration into blocks of rounds and run slices explored by separate workgroups,
// which then share no word-0 value except their common boundary states.
bool word0_orders_rounds(const ModelHost& h);

// Whether an exploration pruned at some T can be continued to a larger T' on the same
// visited set: units that all work alike (every configuration passes through the state
// after r full rounds, (c, r d, n - r m, all idle)) and a key whose word 0 holds the
// pending count and the clock (so a partition may start at that state); or units of
// unequal speed, which continue from the cuts of their chain slices (or from SELECT).
bool resumable(const ModelHost& h);

// Partitions that continue a resumable model's exploration after every state with clock
// <= T_done was inserted, from rounds r0 = floor(T_done / d) of each configuration not yet
// at its terminals (its start state is in the set; re-exploring round r0 finds its states
// up to T_done present and inserts the rest).  A configuration that the fresh plan `fresh`
// cuts into round blocks keeps the blocks that end past round r0, the one holding r0
// starting there, so the continuation is as parallel as the fresh exploration; any other
// configuration continues as one partition.  Never more partitions than the fresh plan
// has (or than configurations, if that is more).  On units of unequal speed it keeps the
// chain slices that end past T_done and restarts uncut configurations from SELECT.
void plan_resume(const ModelHost& h, uint64_t T_done, const std::vector<PartPlan>& fresh,
                 std::vector<PartPlan>* out);

// Default target states per partition for a launch exploring `states` states in total
// on models of m units.
uint64_t auto_part_states(uint64_t states, uint32_t m = 2u);

// Operation ends of one workgroup of configuration r at or before time x.
uint64_t ends_le(const CfgRec& r, uint64_t x);

// Sizes of one configuration's subgraph on units of unequal speed (sp[0..m-1]): states
// with clock <= T (an upper bound: tails that meet are counted twice), the longest path
// from the SELECT state, the latest terminal clock.  With `cuts`, also records cut
// points of the determined part at least kCutSpacing states apart (at most kMaxCuts:
// beyond that every other one is dropped and the spacing doubles).
struct ChainCount {
  uint64_t states = 0, depth = 0, max_clock = 0;
};
ChainCount walk_unequal(const CfgRec& r, const uint32_t* sp, uint32_t m, uint64_t T,
                        std::vector<ChainCut>* cuts = nullptr);
// Time of the k-th operation end (0-based, k < r.b) of one workgroup.
uint64_t end_at_host(const CfgRec& r, uint64_t k);

// The recorded cut points (in order) thinned to about `target` states apart: each one
// kept is the first at least `target` states past the previous one kept.
void chain_cuts(const std::vector<ChainCut>& cands, uint64_t target,
                std::vector<ChainCut>* out);

// An upper bound (exact for every configuration whose last round is not partial) on the
// number of states with clock <= T, root included: what a check(T) inserts.  Sizes its
// visited set only.
uint64_t count_le_bound(const ModelHost& h, uint64_t T);

uint64_t binom(uint32_t n, uint32_t k);
uint32_t bit_length(uint64_t x);

// Packed key of a state on the host.  fields: cfg, pending, clock, then the time left
// on every unit (packed as a busy mask and one shared time when the layout says so; an
// implied clock is not stored).
void encode_key_host(const Layout& L, const uint32_t* fields, uint64_t* words);
// The inverse; cfgs (the configuration records) give an implied clock.
void decode_key_host(const Layout& L, const uint64_t* words, uint32_t* fields,
                     const CfgRec* cfgs);

// min_time of a descriptor over a caller's device workspace, with no pinned staging and
// no runtime objects created (mc_api.hip): the query path of mc_min_time_static.
int min_time_in_place(const mc_desc* d, const mc_opts* o, void* dev_ws, size_t ws_bytes,
                      void* stream, uint32_t* t_min, uint32_t* argmin, size_t cap,
                      size_t* n_argmin, mc_stats* st);

}  // namespace mc
