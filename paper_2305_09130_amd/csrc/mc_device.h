// mc_device.h -- device-side building blocks of the explorer: packed keys, operation
// tables, the lock-free visited set and wavefront compaction helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_model.h"

namespace mc {

// Device counters of one query (one per model; zeroed before every query).
struct Ctrl {
  unsigned long long states;     // states claimed in the visited set (root included)
  unsigned long long terminals;  // terminal states claimed
  unsigned long long edges;      // successor generations
  unsigned long long dups;       // inserts that found the state present
  unsigned long long probes;     // slots probed
  unsigned long long max_depth;  // deepest claimed state
  unsigned int error;            // kDevErr* (first error wins)
  unsigned int violated;         // some terminal with clock <= T
  unsigned int queue_head;       // next partition of the persistent engine
  unsigned int levels;           // level-engine launches with a non-empty frontier
  unsigned int fcount[3];        // level-engine frontier sizes (rotating)
  unsigned int root_slot;
  unsigned int trace_len;
  unsigned int target_slot;
  unsigned int sim_t, sim_cfg;
  unsigned int max_probe;        // longest probe sequence of one insert
  unsigned int crit_part;        // partition with the longest exploration time
  unsigned long long supersteps; // super-steps (persistent engine)
  unsigned long long chunks;     // insert batches (persistent engine)
  unsigned long long crit_ticks; // longest partition time, 100 MHz ticks
  unsigned int parts_done;       // partitions explored to the end (resumable queues)
  unsigned int bound;            // branch-and-bound min_time: least terminal clock found
                                 // so far (starts at the query's T)
  unsigned int pad[6];
};
static_assert(sizeof(Ctrl) == 160, "Ctrl layout");

constexpr unsigned int kDevErrTableFull = 1;
constexpr unsigned int kDevErrOverflow = 2;
constexpr unsigned int kDevErrPublish = 3;
constexpr unsigned int kDevErrTrace = 4;
constexpr unsigned int kDevErrSplit = 5;  // a round block did not end on its predicted state
constexpr unsigned int kDevErrAbort = 6;  // the host asked the query to stop

constexpr uint32_t kMaxProbeIters = 1u << 16;

// A visited set of S slots holds the keys of all its slots first (8W bytes each), then
// their links (a parent and a jump word, 8 bytes each): 8W + 8 bytes per slot.

template <int W>
struct Key {
  unsigned long long w[W];
};

// A queued state: key, its visited-set slot and its depth (path length from the root).
template <int W>
struct Entry {
  unsigned long long k[W];
  uint32_t slot;
  uint32_t depth;
};

struct Seed {
  unsigned long long k[4];
  uint32_t slot;
  uint32_t depth;
  uint32_t pad[2];
};
static_assert(sizeof(Seed) == 48, "Seed layout");

struct St {
  uint32_t cfg, pending, clock;
  uint32_t rem[kMaxCU];
};

// ---- packed keys ----------------------------------------------------------------

template <int W>
__device__ __forceinline__ unsigned long long key_word(const Key<W>& k, int i) {
  unsigned long long r = k.w[0];
#pragma unroll
  for (int j = 1; j < W; ++j) r = (i == j) ? k.w[j] : r;
  return r;
}

template <int W>
__device__ __forceinline__ uint32_t key_get(const Key<W>& k, const Layout& L, int f) {
  const unsigned long long v = key_word<W>(k, L.word[f]) >> L.shift[f];
  return (uint32_t)(v & ((1ull << L.width[f]) - 1ull));
}

template <int W>
__device__ __forceinline__ void key_put(Key<W>& k, const Layout& L, int f, uint32_t v) {
  const unsigned long long x = (unsigned long long)v << L.shift[f];
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (L.word[f] == j) k.w[j] |= x;
}

// Clock of a state on equal units from its other fields: the units run lock-step
// rounds of d cycles, so after `done` = n - pending - busy workgroups ended or started
// together, ceil(done / m) rounds lie behind (the ceiling counts a last round of fewer
// than m workgroups once they have ended), and a busy round is d - rem cycles in.
// The root (cfg = n_cfg) is at clock 0.
__device__ __forceinline__ uint32_t implied_clock(uint32_t cfg, uint32_t pending, uint32_t mask,
                                                  uint32_t rem, const Layout& L,
                                                  const CfgRec* cfgs) {
  if (cfg >= L.n_cfg) return 0u;
  const uint2 nd = *reinterpret_cast<const uint2*>(&cfgs[cfg]);  // n, d
  const uint32_t done = nd.x - pending - (uint32_t)__popc(mask);
  const uint32_t rounds = (done + L.m - 1u) / L.m;
  return rounds * nd.y + (mask ? nd.y - rem : 0u);
}

// cfgs: the configuration records (read only when the layout implies the clock)
template <int W>
__device__ __forceinline__ St decode(const Key<W>& k, const Layout& L, const CfgRec* cfgs) {
  St s;
  s.cfg = key_get<W>(k, L, kFCfg);
  s.pending = key_get<W>(k, L, kFPending);
  if (L.shared_rem) {
    const uint32_t mask = key_get<W>(k, L, kFRem), rem = key_get<W>(k, L, kFRem + 1);
#pragma unroll
    for (int i = 0; i < kMaxCU; ++i) s.rem[i] = ((mask >> i) & 1u) ? rem : 0u;
    s.clock = L.clock_implied ? implied_clock(s.cfg, s.pending, mask, rem, L, cfgs)
                              : key_get<W>(k, L, kFClock);
  } else {
    s.clock = key_get<W>(k, L, kFClock);
#pragma unroll
    for (int i = 0; i < kMaxCU; ++i) s.rem[i] = (i < L.m) ? key_get<W>(k, L, kFRem + i) : 0u;
  }
  return s;
}

template <int W>
__device__ __forceinline__ Key<W> encode(const St& s, const Layout& L) {
  Key<W> k;
#pragma unroll
  for (int j = 0; j < W; ++j) k.w[j] = 0ull;
  key_put<W>(k, L, kFCfg, s.cfg);
  key_put<W>(k, L, kFPending, s.pending);
  if (!L.clock_implied) key_put<W>(k, L, kFClock, s.clock);
  if (L.shared_rem) {  // every busy unit has the same time left
    uint32_t mask = 0, rem = 0;
#pragma unroll
    for (int i = 0; i < kMaxCU; ++i)
      if (i < L.m && s.rem[i]) {
        mask |= 1u << i;
        rem = s.rem[i];
      }
    key_put<W>(k, L, kFRem, mask);
    key_put<W>(k, L, kFRem + 1, rem);
  } else {
#pragma unroll
    for (int i = 0; i < kMaxCU; ++i)
      if (i < L.m) key_put<W>(k, L, kFRem + i, s.rem[i]);
  }
  return k;
}

__device__ __forceinline__ unsigned long long fmix64(unsigned long long x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

template <int W>
__device__ __forceinline__ unsigned long long key_hash(const Key<W>& k) {
  unsigned long long h = k.w[0] * 0x9e3779b97f4a7c15ull;
#pragma unroll
  for (int j = 1; j < W; ++j) h ^= (k.w[j] + (unsigned long long)j) * 0xd6e8feb86659fd93ull;
  return fmix64(h);
}

__device__ __forceinline__ bool is_terminal(const St& s, int m) {
  if (s.pending) return false;
  bool idle = true;
#pragma unroll
  for (int i = 0; i < kMaxCU; ++i) idle &= (i >= m) || (s.rem[i] == 0u);
  return idle;
}

// ---- operation ends of one workgroup (phases of CfgRec) ----------------------------

// Uniform phases (one operation per period, back to back from 0, a single wave): the
// operation lists of the reduction and matmul kinds.  Bit-for-bit the general helpers
// below on such configurations, with fewer live registers.
__device__ __forceinline__ uint32_t ends_upto_uniform(const CfgRec& r, uint32_t e) {
  if (e >= r.d) return r.b;
  uint32_t res = r.b;
  bool found = false;
#pragma unroll
  for (int j = kMaxPhases - 1; j >= 0; --j) {
    if (j < (int)r.nph && e >= r.t0[j] && !found) {
      res = r.i0[j] + (e - r.t0[j]) / r.lat[j];
      found = true;
    }
  }
  return res;
}

__device__ __forceinline__ uint32_t end_at_uniform(const CfgRec& r, uint32_t k) {
  uint32_t res = r.d;
  bool found = false;
#pragma unroll
  for (int j = 0; j < kMaxPhases; ++j) {
    if (j < (int)r.nph && !found && k < r.i0[j] + r.cnt[j]) {
      res = r.t0[j] + (k - r.i0[j] + 1u) * r.lat[j];
      found = true;
    }
  }
  return res;
}

// number of operation ends of one wave at times <= e, 0 <= e <= dw
__device__ __forceinline__ uint32_t wave_ends_upto(const CfgRec& r, uint32_t e) {
  uint32_t res = 0;
  bool found = false;
#pragma unroll
  for (int j = kMaxPhases - 1; j >= 0; --j) {
    if (j < (int)r.nph && e >= r.t0[j] && !found) {
      const uint32_t rel = e - r.t0[j], reps = rel / r.lat[j];
      uint32_t k = reps;
      if (r.la[j]) k = 2u * reps + (rel - reps * r.lat[j] >= r.la[j] ? 1u : 0u);
      res = r.i0[j] + (k < r.cnt[j] ? k : r.cnt[j]);
      found = true;
    }
  }
  return res;
}

// number of operation ends at times <= e, for 0 <= e
__device__ __forceinline__ uint32_t ends_upto(const CfgRec& r, uint32_t e) {
  if (e >= r.d) return r.b;
  if (r.waves > 1u) {
    const uint32_t w = e / r.dw;
    return w * r.bw + wave_ends_upto(r, e - w * r.dw);
  }
  return wave_ends_upto(r, e);
}

// time of the k-th operation end of one wave (0-based), k < bw
__device__ __forceinline__ uint32_t wave_end_at(const CfgRec& r, uint32_t k) {
  uint32_t res = r.dw;
  bool found = false;
#pragma unroll
  for (int j = 0; j < kMaxPhases; ++j) {
    if (j < (int)r.nph && !found && k < r.i0[j] + r.cnt[j]) {
      const uint32_t q = k - r.i0[j];
      res = r.t0[j] + (q + 1u) * r.lat[j];
      if (r.la[j]) res = r.t0[j] + (q >> 1) * r.lat[j] + ((q & 1u) ? r.lat[j] : r.la[j]);
      found = true;
    }
  }
  return res;
}

// time of the k-th operation end (0-based), k < b
__device__ __forceinline__ uint32_t end_at(const CfgRec& r, uint32_t k) {
  if (r.waves > 1u) {
    const uint32_t w = k / r.bw;
    return w * r.dw + wave_end_at(r, k - w * r.bw);
  }
  return wave_end_at(r, k);
}

// The super-step engine is compiled twice: GEN = false for models whose
// configurations all have uniform phases, GEN = true for the rest.
template <bool GEN>
__device__ __forceinline__ uint32_t ends_upto_t(const CfgRec& r, uint32_t e) {
  if constexpr (GEN) return ends_upto(r, e);
  else return ends_upto_uniform(r, e);
}
template <bool GEN>
__device__ __forceinline__ uint32_t end_at_t(const CfgRec& r, uint32_t k) {
  if constexpr (GEN) return end_at(r, k);
  else return end_at_uniform(r, k);
}

// Workgroup duration on unit u: a unit of speed s runs every operation s times as long
// (its operation ends are s*E, its workgroup lasts s*d).  The uniform-phase build only
// runs models whose units all have speed 1.
template <bool GEN>
__device__ __forceinline__ uint32_t unit_dur(const CfgRec& r, const uint8_t* speed, int u) {
  if constexpr (GEN) return (uint32_t)speed[u] * r.d;
  else return r.d;
}

// One ADVANCE step: the clock moves to the next operation end of any busy unit, on that
// unit's own grid s*E (speed null: every unit at speed 1).
template <bool GEN = true>
__device__ __forceinline__ void advance_once(St& s, const CfgRec& r, int m,
                                             const uint8_t* speed = nullptr) {
  uint32_t delta = 0xFFFFFFFFu;
#pragma unroll
  for (int i = 0; i < kMaxCU; ++i) {
    if (i < m && s.rem[i]) {
      uint32_t di;
      if (GEN && speed && speed[i] != 1u) {
        // elapsed e < sp*d; the next end sp*E[k] > e has E[k] > floor(e / sp)
        const uint32_t sp = speed[i];
        const uint32_t e = sp * r.d - s.rem[i];
        di = sp * end_at_t<GEN>(r, ends_upto_t<GEN>(r, e / sp)) - e;
      } else {
        const uint32_t e = r.d - s.rem[i];
        di = end_at_t<GEN>(r, ends_upto_t<GEN>(r, e)) - e;
      }
      delta = di < delta ? di : delta;
    }
  }
  s.clock += delta;
#pragma unroll
  for (int i = 0; i < kMaxCU; ++i)
    if (i < m && s.rem[i]) s.rem[i] -= delta;
}

// ---- visited set ----------------------------------------------------------------

// The key region starts at base; the link region of a set of mask + 1 slots follows it.
// Every writer of a link stores both words.  On units alike only the key region is
// cleared: a state's links are read only where they were written (the trace tells the
// states that store none from their keys).
template <int W>
__device__ __forceinline__ unsigned long long* slot_key(unsigned char* base, unsigned long long s) {
  return reinterpret_cast<unsigned long long*>(base + s * (8ull * W));
}
template <int W>
__device__ __forceinline__ uint32_t* slot_parent(unsigned char* base, unsigned long long mask,
                                                 unsigned long long s) {
  return reinterpret_cast<uint32_t*>(base + (mask + 1ull) * (8ull * W) + s * 8ull);
}
// jump word: first predecessor of the lock-step run a state belongs to (else 0xFFFFFFFF)
template <int W>
__device__ __forceinline__ uint32_t* slot_jump(unsigned char* base, unsigned long long mask,
                                               unsigned long long s) {
  return reinterpret_cast<uint32_t*>(base + (mask + 1ull) * (8ull * W) + s * 8ull + 4ull);
}
// both links of a slot in one 8-byte store
template <int W>
__device__ __forceinline__ void set_links(unsigned char* base, unsigned long long mask,
                                          unsigned long long s, uint32_t parent, uint32_t jump) {
  *reinterpret_cast<unsigned long long*>(base + (mask + 1ull) * (8ull * W) + s * 8ull) =
      (unsigned long long)parent | ((unsigned long long)jump << 32);
}

constexpr int kScopeWG = __HIP_MEMORY_SCOPE_WORKGROUP;
constexpr int kScopeAgent = __HIP_MEMORY_SCOPE_AGENT;
constexpr int kScopeSystem = __HIP_MEMORY_SCOPE_SYSTEM;

enum { kInsNew = 1, kInsDup = 0, kInsFail = -1 };

// Open addressing in windows of consecutive slots whose keys share one 64-byte line (8, 4
// or 2 slots for 1-, 2- and 4-word keys); windows are visited in a double-hashing sequence
// (odd step, so every window is reached) and the slots of a window in a circular order
// that starts at a slot the key's hash picks (keys that share a home window then start
// apart: with windows of four slots, 1.38 probes per new key instead of 1.90 when every
// key starts at the window's first slot, at the load 0.43 of the largest workload).  Every
// probe is a 64-bit compare-and-swap of word 0 from empty to the key's word 0, issued
// without reading the slot first: a probe of an empty slot claims it in one round trip,
// and a failed one returns the slot's word 0, which is all a read would have told.
// Wider keys are claimed on word 0; the winner then stores the other words.  No valid
// key has a word equal to the all-ones of a cleared slot (the key layout keeps a zero
// bit in every word), and every word is stored once, so a lane that finds its own word 0
// in a slot waits until none of the other words reads all-ones and then compares them:
// each word is read and written as an atomic at the insert's scope, which makes it
// coherent by itself, and no release/acquire pair (on gfx950 an L2 writeback at agent
// scope) is needed.  One slot is handled per loop iteration and waiting never spins
// inside an iteration: every lane of the wavefront runs the same loop, and a winner
// stores its words in the iteration it won, so a waiting lane cannot starve a winner of
// its own wavefront.  SCOPE is the widest set of threads that may insert the same key:
// the workgroup in the super-step engine (one configuration's subgraph, or a block of
// its rounds, per workgroup; the configuration index in word 0), the device in the
// level engine.  The slot claimed is always the first empty one of the key's sequence,
// so a lookup stops at the first empty slot.
template <int W>
struct Win {
  static constexpr int n = 8 / W;                       // slots per window (one 64-byte line)
  static constexpr int log2 = W == 1 ? 3 : W == 2 ? 2 : 1;
};
static_assert(Win<1>::n == 8 && Win<2>::n == 4 && Win<4>::n == 2, "window sizes");

// Home window wi, odd window step, and the first slot j0 within every window (from
// the hash's top log2(slots per window) bits, which neither wi nor step use for tables of
// at most 2^31 slots: step takes bits 33 to 32 + log2(windows)).
// The key's hash with only its low `hkeep` bits kept (hkeep 0: all), remixed: a testing
// aid that crowds keys into 2^hkeep probe sequences.
__device__ __forceinline__ unsigned long long keep_hash(unsigned long long h, uint32_t hkeep) {
  return hkeep ? fmix64((h & ((1ull << hkeep) - 1ull)) + 0x9e3779b97f4a7c15ull) : h;
}

template <int W>
__device__ __forceinline__ void probe_start(unsigned long long h, unsigned long long mask,
                                            unsigned long long& wi, unsigned long long& step,
                                            int& j0) {
  const unsigned long long nwin_mask = (mask + 1ull) / Win<W>::n - 1ull;
  wi = h & nwin_mask;
  step = ((h >> 33) | 1ull) & nwin_mask;
  step |= 1ull;
  j0 = (int)(h >> (64 - Win<W>::log2)) & (Win<W>::n - 1);
}

// the t-th slot of window wi in the circular order from j0
template <int W>
__device__ __forceinline__ unsigned long long win_slot(unsigned long long wi, int j0, int t) {
  return wi * Win<W>::n + (unsigned long long)((j0 + t) & (Win<W>::n - 1));
}

template <int W, int SCOPE>
__device__ __forceinline__ int table_insert(unsigned char* base, unsigned long long mask,
                                            const Key<W>& k, uint32_t& slot_out,
                                            uint32_t& probes, uint32_t hkeep = 0u) {
  constexpr int KW = Win<W>::n;
  unsigned long long wi, step;
  int j0;
  probe_start<W>(keep_hash(key_hash<W>(k), hkeep), mask, wi, step, j0);
  const unsigned long long nwin_mask = (mask + 1ull) / KW - 1ull;
  const unsigned long long max_iters =
      (mask + 1ull) * 2ull < kMaxProbeIters ? (mask + 1ull) * 2ull : kMaxProbeIters;
  int j = 0;  // slots of the window probed so far
  bool waiting = false;
  for (unsigned long long it = 0; it < max_iters; ++it) {
    const unsigned long long s = win_slot<W>(wi, j0, j);
    unsigned long long* p = slot_key<W>(base, s);
    bool advance = false;
    if (waiting) {
      bool ready = true, eq = true;
#pragma unroll
      for (int q = 1; q < W; ++q) {
        const unsigned long long v = __hip_atomic_load(p + q, __ATOMIC_RELAXED, SCOPE);
        ready &= v != kEmptyWord;
        eq &= v == k.w[q];
      }
      if (ready) {
        if (eq) {
          slot_out = (uint32_t)s;
          return kInsDup;
        }
        waiting = false;
        advance = true;
      }
    } else {
      ++probes;
      const unsigned long long old = atomicCAS(p, kEmptyWord, k.w[0]);
      if (old == kEmptyWord) {
#pragma unroll
        for (int q = 1; q < W; ++q) __hip_atomic_store(p + q, k.w[q], __ATOMIC_RELAXED, SCOPE);
        slot_out = (uint32_t)s;
        return kInsNew;
      }
      if (old == k.w[0]) {
        if (W == 1) {
          slot_out = (uint32_t)s;
          return kInsDup;
        }
        waiting = true;
      } else {
        advance = true;
      }
    }
    if (advance && ++j == KW) {
      j = 0;
      wi = (wi + step) & nwin_mask;
    }
  }
  return kInsFail;
}

// N independent inserts per lane, stepped together so that their round trips overlap:
// every iteration first issues the compare-and-swaps of all keys not waiting, then the
// reads of the other words of the slots waited on, and only then looks at the results.
// Same protocol, sequence and guarantees as table_insert, one state machine per key.
template <int W, int SCOPE, int N>
__device__ __forceinline__ void table_insert_n(unsigned char* base, unsigned long long mask,
                                               const unsigned long long (&key)[N][W],
                                               const bool (&act)[N], uint32_t (&slot)[N],
                                               int (&res)[N], uint32_t& probes,
                                               uint32_t hkeep = 0u) {
  constexpr int KW = Win<W>::n;
  const unsigned long long nwin_mask = (mask + 1ull) / KW - 1ull;
  const unsigned long long max_iters =
      (mask + 1ull) * 2ull < kMaxProbeIters ? (mask + 1ull) * 2ull : kMaxProbeIters;
  unsigned long long wi[N], step[N], old[N];
  int j[N], j0[N];
  bool waiting[N], done[N], ready[N], eq[N];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    res[n] = kInsFail;
    slot[n] = kParentNone;
    done[n] = !act[n];
    waiting[n] = false;
    j[n] = 0;
    j0[n] = 0;
    wi[n] = step[n] = 0ull;
    if (act[n]) {
      Key<W> k;
#pragma unroll
      for (int q = 0; q < W; ++q) k.w[q] = key[n][q];
      probe_start<W>(keep_hash(key_hash<W>(k), hkeep), mask, wi[n], step[n], j0[n]);
    }
  }
  for (unsigned long long it = 0; it < max_iters; ++it) {
    bool any = false;
#pragma unroll
    for (int n = 0; n < N; ++n) {  // claims
      if (done[n] || waiting[n]) continue;
      ++probes;
      old[n] = atomicCAS(slot_key<W>(base, win_slot<W>(wi[n], j0[n], j[n])), kEmptyWord,
                         key[n][0]);
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {  // other words of the slots waited on
      ready[n] = eq[n] = true;
      if (done[n] || !waiting[n]) continue;
      const unsigned long long* p = slot_key<W>(base, win_slot<W>(wi[n], j0[n], j[n]));
#pragma unroll
      for (int q = 1; q < W; ++q) {
        const unsigned long long v = __hip_atomic_load(p + q, __ATOMIC_RELAXED, SCOPE);
        ready[n] &= v != kEmptyWord;
        eq[n] &= v == key[n][q];
      }
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {  // results
      if (done[n]) continue;
      any = true;
      const unsigned long long s = win_slot<W>(wi[n], j0[n], j[n]);
      bool advance = false;
      if (waiting[n]) {
        if (ready[n]) {
          if (eq[n]) {
            slot[n] = (uint32_t)s;
            res[n] = kInsDup;
            done[n] = true;
            continue;
          }
          waiting[n] = false;
          advance = true;
        }
      } else if (old[n] == kEmptyWord) {
        unsigned long long* p = slot_key<W>(base, s);
#pragma unroll
        for (int q = 1; q < W; ++q) __hip_atomic_store(p + q, key[n][q], __ATOMIC_RELAXED, SCOPE);
        slot[n] = (uint32_t)s;
        res[n] = kInsNew;
        done[n] = true;
        continue;
      } else if (old[n] == key[n][0]) {
        if (W == 1) {
          slot[n] = (uint32_t)s;
          res[n] = kInsDup;
          done[n] = true;
          continue;
        }
        waiting[n] = true;
      } else {
        advance = true;
      }
      if (advance && ++j[n] == KW) {
        j[n] = 0;
        wi[n] = (wi[n] + step[n]) & nwin_mask;
      }
    }
    if (!any) break;
  }
}

// Lookup only (after the exploration finished; plain loads).
template <int W>
__device__ __forceinline__ uint32_t table_find(unsigned char* base, unsigned long long mask,
                                               const Key<W>& k, uint32_t hkeep = 0u) {
  constexpr int KW = Win<W>::n;
  unsigned long long wi, step;
  int j0;
  probe_start<W>(keep_hash(key_hash<W>(k), hkeep), mask, wi, step, j0);
  const unsigned long long nwin_mask = (mask + 1ull) / KW - 1ull;
  for (unsigned long long it = 0; it <= nwin_mask; ++it) {
    for (int j = 0; j < KW; ++j) {
      const unsigned long long s = win_slot<W>(wi, j0, j);
      const unsigned long long* p = slot_key<W>(base, s);
      if (p[0] == kEmptyWord) return kParentNone;
      bool eq = true;
#pragma unroll
      for (int q = 0; q < W; ++q) eq &= p[q] == k.w[q];
      if (eq) return (uint32_t)s;
    }
    wi = (wi + step) & nwin_mask;
  }
  return kParentNone;
}

// ---- wavefront helpers ------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
  const uint32_t l = lane_id();
  return (uint32_t)__popcll(mask & ((1ull << l) - 1ull));
}

// Wavefront-aggregated append: one atomic per wavefront; returns this lane's position
// (valid only where pred).  Must be reached by every lane of the wavefront.
__device__ __forceinline__ uint32_t wave_append(bool pred, unsigned int* counter) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return 0u;
  const int leader = __ffsll((long long)mask) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(counter, (unsigned int)__popcll(mask));
  base = __shfl(base, leader);
  return base + lanes_below(mask);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(v, o);
    v = x > v ? x : v;
  }
  return v;
}

// Records the first error of a query (later ones keep it).
__device__ __forceinline__ void set_error(Ctrl* ctrl, unsigned int e) { atomicCAS(&ctrl->error, 0u, e); }

// splitmix64 (Steele, Lea, Flood 2014)
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace mc
