// mc_walks.hip -- seeded walks of the MI355X explicit-state checker.
//
//   k_simulate      one seeded random run from the root (simulation mode, the T_ini of
//                   the tuning loop)
//   k_swarm         swarm search: many independent bitstate walkers, one per lane
//   k_swarm_replay  one member's walk again, state by state (its counterexample)
#include <hip/hip_runtime.h>

#include "mc_launch.h"

namespace mc {

// ---- simulation mode ------------------------------------------------------------------
//
// One run from the root, choosing uniformly among the successors at every step with
// the choice of step t drawn from splitmix64(seed ^ splitmix64(t)); successors are
// ordered by configuration (SELECT) and by unit index (DISPATCH).  A lock-step ADVANCE
// run has one successor per step; it is taken in one jump that counts its steps.

// Units of unequal speed with no DISPATCH enabled until clock H (the first workgroup end
// while work is pending, else the last): the ADVANCE steps up to H are one per distinct
// operation end of the busy units in (clock, H].  The wavefront counts them a window at a
// time: lane l takes the (l mod p)-th next end of unit l / p (p = 64 / m); the window
// closes at the least last-slot end of any unit (no end of any unit below it is missing),
// an end counts unless a unit of lower index ends at the same time, and the state moves
// to the window's close.  Returns the steps; x is left at clock H.
__device__ uint32_t jump_unequal(St& x, const CfgRec& r, int m, const uint8_t* speed,
                                 uint32_t H) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t per = 64u / (uint32_t)m;
  const uint32_t u = lane / per, k = lane - u * per;
  uint32_t steps = 0;
  while (x.clock < H) {
    uint32_t v = 0xFFFFFFFFu;
    if (u < (uint32_t)m && x.rem[u]) {
      const uint32_t sp = speed[u];
      const uint32_t e = sp * r.d - x.rem[u];
      const uint32_t kk = ends_upto(r, e / sp) + k;
      if (kk < r.b) {
        const uint32_t tau = x.clock + sp * end_at(r, kk) - e;
        if (tau <= H) v = tau;
      }
    }
    uint32_t lim = (k + 1u == per) ? v : 0xFFFFFFFFu;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t y = __shfl_xor(lim, o);
      lim = y < lim ? y : lim;
    }
    lim = lim < H ? lim : H;
    bool first = v <= lim;
    for (uint32_t j = 0; j < u && first; ++j) {
      // does unit j (busy until clock + rem_j) end an operation at time v?
      if (x.rem[j] == 0u || v > x.clock + x.rem[j]) continue;
      const uint32_t sj = speed[j];
      const uint32_t diff = v - x.clock + (sj * r.d - x.rem[j]);
      if (diff % sj) continue;
      const uint32_t q = diff / sj;
      if (q && ends_upto(r, q) != ends_upto(r, q - 1u)) first = false;
    }
    steps += (uint32_t)__popcll(__ballot(first));
    const uint32_t dt = lim - x.clock;
#pragma unroll
    for (int i = 0; i < kMaxCU; ++i) x.rem[i] = x.rem[i] > dt ? x.rem[i] - dt : 0u;
    x.clock = lim;
  }
  return steps;
}

__global__ void k_simulate(QueryArgs a, unsigned long long seed) {
  // every lane of the wavefront follows the same run; jump_unequal splits its windows
  if (blockIdx.x != 0 || threadIdx.x >= 64) return;
  const int m = a.L.m;
  const uint8_t* speed = a.L.speed;
  unsigned long long step = 0;
  const uint32_t c = (uint32_t)(splitmix64(seed ^ splitmix64(step)) % a.n_cfg);
  ++step;
  const CfgRec r = a.cfgs[c];
  St x{};
  x.cfg = c;
  x.pending = r.n;
  for (;;) {
    uint32_t freem = 0, busy = 0, brem = 0, bsp = 0;
    bool same = true;
    for (int u = 0; u < m; ++u) {
      if (x.rem[u] == 0u) {
        freem |= 1u << u;
      } else {
        if (busy && (x.rem[u] != brem || speed[u] != bsp)) same = false;
        brem = x.rem[u];
        bsp = speed[u];
        busy |= 1u << u;
      }
    }
    if (x.pending && freem) {
      const uint32_t nfree = (uint32_t)__popc(freem);
      uint32_t pick = (uint32_t)(splitmix64(seed ^ splitmix64(step)) % nfree);
      ++step;
      for (int u = 0; u < m; ++u) {
        if ((freem >> u) & 1u) {
          if (pick == 0u) {
            x.rem[u] = unit_dur<true>(r, speed, u);
            x.pending -= 1u;
            break;
          }
          --pick;
        }
      }
      continue;
    }
    if (!busy) break;
    if (same) {
      // busy units in lock step (equal speed and time left): one step per end to go
      const uint32_t e0 = bsp * r.d - brem;
      step += r.b - ends_upto(r, e0 / bsp);
      x.clock += brem;
      for (int u = 0; u < m; ++u) x.rem[u] = 0u;
    } else {
      // no DISPATCH before the first workgroup end (work pending) or the last
      uint32_t H = x.pending ? 0xFFFFFFFFu : 0u;
      for (int u = 0; u < m; ++u) {
        if (!x.rem[u]) continue;
        const uint32_t t = x.clock + x.rem[u];
        H = x.pending ? (t < H ? t : H) : (t > H ? t : H);
      }
      step += jump_unequal(x, r, m, speed, H);
    }
  }
  if (threadIdx.x == 0) {
    a.ctrl->sim_t = x.clock;
    a.ctrl->sim_cfg = c;
  }
}

// ---- swarm search (Sec. 5) -----------------------------------------------------------
//
// Swarm model checking runs many independent, incomplete searches: each member keeps a
// bit array of its own (bitstate hashing) instead of storing states, and reports the
// counterexamples it meets within a bounded number of model steps.  Against G(!FIN)
// every run reaching a terminal is a counterexample whose clock is a model time;
// against the over-time property with threshold T only terminals with clock <= T are.
// Member i (one lane) uses seed splitmix64(seed + i) and makes walks from the root: at
// its step t (counted over all its walks) it takes successor number
// splitmix64(seed_i ^ splitmix64(t)) mod k of the k successors (configurations in order
// at the root, free units in index order for DISPATCH).  With a threshold a walk ends
// at the first state with clock > T.  At every state it reaches (not the root) with
// other than exactly one successor it hashes (cfg, clock, pending, rem_0..rem_{m-1})
// with a splitmix64 chain to bit positions h mod B and (h >> 32) mod B: both set, the
// walk ends (the state was visited); else both are set.  A new terminal ends the walk
// as a counterexample (a trail).  A new walk starts only while t < budget.  The
// interior states of a lock-step run (one successor each, no bitstate lookup) are
// crossed in one jump that counts their steps, and, with a threshold, stops exactly at
// the first of them past T.

__device__ __forceinline__ unsigned long long swarm_hash(const St& x, int m) {
  unsigned long long h = splitmix64((unsigned long long)x.cfg);
  h = splitmix64(h ^ x.clock);
  h = splitmix64(h ^ x.pending);
  for (int u = 0; u < m; ++u) h = splitmix64(h ^ x.rem[u]);
  return h;
}

// successor count of a non-root state, its free and busy units, and whether the busy
// units are in lock step (equal speed and remaining time)
struct SwarmView {
  uint32_t k, freem, busy, brem, bsp;
  bool same;
};
__device__ __forceinline__ SwarmView swarm_view(const St& x, int m, const uint8_t* speed) {
  SwarmView v{0u, 0u, 0u, 0u, 1u, true};
  for (int u = 0; u < m; ++u) {
    if (x.rem[u] == 0u) {
      v.freem |= 1u << u;
    } else {
      if (v.busy && (x.rem[u] != v.brem || speed[u] != v.bsp)) v.same = false;
      v.brem = x.rem[u];
      v.bsp = speed[u];
      v.busy |= 1u << u;
    }
  }
  v.k = (x.pending && v.freem) ? (uint32_t)__popc(v.freem) : (v.busy ? 1u : 0u);
  return v;
}

__device__ __forceinline__ void swarm_dispatch(St& x, const CfgRec& r, uint32_t freem,
                                               uint32_t pick, int m, const uint8_t* speed) {
  for (int u = 0; u < m; ++u) {
    if ((freem >> u) & 1u) {
      if (pick == 0u) {
        x.rem[u] = unit_dur<true>(r, speed, u);
        x.pending -= 1u;
        return;
      }
      --pick;
    }
  }
}

// A walk's ADVANCE chain on units that are not in lock step: from x on every state has
// one successor (no work pending, or no unit free) until a unit falls idle while work is
// pending, or no unit is busy.  Each busy unit keeps the index and time of its next
// operation end and its workgroup's end, so a step is the least next end and one
// operation-end lookup per unit that ends there.  t counts one model step per state, as
// one ADVANCE at a time would.  With a threshold it stops on the first state past T and
// returns true (the walk ends there).  x is left on the chain's last state.
__device__ bool swarm_advance_run(St& x, const CfgRec& r, int m, const uint8_t* speed,
                                  bool prune, uint32_t T, unsigned long long& t) {
  uint32_t nx[kMaxCU], kk[kMaxCU], wend[kMaxCU], sp[kMaxCU];
  uint32_t busy = 0;
#pragma unroll
  for (int u = 0; u < kMaxCU; ++u) {
    nx[u] = 0xFFFFFFFFu;
    kk[u] = 0u;
    wend[u] = 0u;
    sp[u] = 1u;
    if (u < m && x.rem[u]) {
      sp[u] = speed[u];
      // elapsed e < sp*d; the next end sp*E[k] > e has E[k] > floor(e / sp)
      const uint32_t e = sp[u] * r.d - x.rem[u];
      kk[u] = ends_upto(r, e / sp[u]);
      wend[u] = x.clock + x.rem[u];
      nx[u] = x.clock + sp[u] * end_at(r, kk[u]) - e;
      busy |= 1u << u;
    }
  }
  bool past = false;
  for (;;) {
    uint32_t tmin = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u) tmin = nx[u] < tmin ? nx[u] : tmin;
    x.clock = tmin;
    ++t;
    bool freed = false;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u) {
      if (nx[u] != tmin) continue;
      if (++kk[u] == r.b) {
        busy &= ~(1u << u);
        nx[u] = 0xFFFFFFFFu;
        freed = true;
      } else {
        nx[u] = wend[u] - sp[u] * r.d + sp[u] * end_at(r, kk[u]);
      }
    }
    if (prune && x.clock > T) {
      past = true;
      break;
    }
    if (!busy || (freed && x.pending)) break;
  }
#pragma unroll
  for (int u = 0; u < kMaxCU; ++u) x.rem[u] = ((busy >> u) & 1u) ? wend[u] - x.clock : 0u;
  return past;
}

__global__ __launch_bounds__(256) void k_swarm(SwarmArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.members) return;
  const int m = (int)a.m;
  const unsigned long long seed = splitmix64(a.seed + i);
  const unsigned long long B = 1ull << a.bits_log2;
  uint32_t* bits = a.bits + (unsigned long long)i * (B >> 5);
  SwarmMember rec;
  rec.walks = rec.trails = rec.best_walk_start = 0ull;
  rec.first_step = ~0ull;
  rec.first_ticks = 0ull;
  rec.best_clock = rec.first_clock = kNoClock;
  rec.best_cfg = rec.first_cfg = kParentNone;
  rec.pad[0] = rec.pad[1] = 0u;
  rec.start_ticks = __builtin_amdgcn_s_memrealtime();
  unsigned long long t = 0;
  while (t < a.budget) {
    ++rec.walks;
    const unsigned long long start = t;
    const uint32_t c = (uint32_t)(splitmix64(seed ^ splitmix64(t)) % a.n_cfg);
    ++t;
    const CfgRec r = a.cfgs[c];
    St x{};
    x.cfg = c;
    x.pending = r.n;
    for (;;) {  // x was just reached by a transition
      if (a.prune && x.clock > a.T) break;
      const SwarmView v = swarm_view(x, m, a.speed);
      if (v.k != 1u) {
        const unsigned long long h = swarm_hash(x, m);
        const unsigned long long p0 = h & (B - 1ull), p1 = (h >> 32) & (B - 1ull);
        const uint32_t w0 = bits[p0 >> 5], w1 = bits[p1 >> 5];
        const uint32_t m0 = 1u << (p0 & 31ull), m1 = 1u << (p1 & 31ull);
        if ((w0 & m0) && (w1 & m1)) break;  // visited
        bits[p0 >> 5] = w0 | m0;
        bits[p1 >> 5] = bits[p1 >> 5] | m1;
      }
      if (v.k == 0u) {  // a new terminal: a trail
        ++rec.trails;
        if (rec.first_step == ~0ull) {
          rec.first_step = t;
          rec.first_ticks = __builtin_amdgcn_s_memrealtime();
          rec.first_clock = x.clock;
          rec.first_cfg = x.cfg;
        }
        if (rec.best_clock == kNoClock || x.clock < rec.best_clock) {
          rec.best_clock = x.clock;
          rec.best_cfg = x.cfg;
          rec.best_walk_start = start;
        }
        break;
      }
      if (x.pending && v.freem) {  // DISPATCH
        const uint32_t pick = (uint32_t)(splitmix64(seed ^ splitmix64(t)) % v.k);
        ++t;
        swarm_dispatch(x, r, v.freem, pick, m, a.speed);
        continue;
      }
      if (v.same) {  // a lock-step run to its end, one transition per operation end
        // ends of the busy units' grid bsp*E after the elapsed time e0
        const uint32_t e0 = v.bsp * r.d - v.brem;
        const uint32_t idx0 = ends_upto(r, e0 / v.bsp);
        if (a.prune && x.clock + v.brem > a.T) {
          // stop at the first state of the run past T
          const uint32_t idx = ends_upto(r, (a.T - x.clock + e0) / v.bsp);
          t += (unsigned long long)(idx - idx0 + 1u);
          break;
        }
        t += (unsigned long long)(r.b - idx0);
        x.clock += v.brem;
        for (int u = 0; u < m; ++u) x.rem[u] = 0u;
        continue;
      }
      if (swarm_advance_run(x, r, m, a.speed, a.prune != 0u, a.T, t)) break;
    }
  }
  rec.steps = t;
  a.out[i] = rec;
}

// One thread: the walk of one member from member step `start`, to its terminal.
__global__ void k_swarm_replay(SwarmArgs a, Ctrl* ctrl, unsigned long long seed,
                               unsigned long long start, uint32_t* rows, uint32_t cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = (int)a.m;
  const uint32_t S = 3u + (uint32_t)m;
  uint32_t n = 0;
  bool bad = false;
  auto put = [&](const St& x, bool root) {
    if (n >= cap) {
      bad = true;
      return;
    }
    uint32_t* row = rows + (unsigned long long)n * S;
    row[0] = root ? kParentNone : x.cfg;
    row[1] = root ? 0u : x.clock;
    row[2] = root ? 0u : x.pending;
    for (int u = 0; u < m; ++u) row[3 + u] = root ? 0u : x.rem[u];
    ++n;
  };
  St x{};
  put(x, true);
  unsigned long long t = start;
  const uint32_t c = (uint32_t)(splitmix64(seed ^ splitmix64(t)) % a.n_cfg);
  ++t;
  const CfgRec r = a.cfgs[c];
  x.cfg = c;
  x.pending = r.n;
  put(x, false);
  for (;;) {
    const SwarmView v = swarm_view(x, m, a.speed);
    if (v.k == 0u || bad) break;
    if (x.pending && v.freem) {
      const uint32_t pick = (uint32_t)(splitmix64(seed ^ splitmix64(t)) % v.k);
      ++t;
      swarm_dispatch(x, r, v.freem, pick, m, a.speed);
    } else {
      advance_once(x, r, m, a.speed);
      ++t;
    }
    put(x, false);
  }
  if (bad) set_error(ctrl, kDevErrTrace);
  ctrl->trace_len = n;
}

// ---- launch helpers (host) ------------------------------------------------------------

hipError_t launch_swarm(hipStream_t st, const SwarmArgs& a) {
  hipLaunchKernelGGL(k_swarm, dim3((a.members + 255u) / 256u), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_swarm_replay(hipStream_t st, const SwarmArgs& a, Ctrl* ctrl,
                               unsigned long long mseed, unsigned long long start,
                               uint32_t* rows, uint32_t cap) {
  hipLaunchKernelGGL(k_swarm_replay, dim3(1), dim3(64), 0, st, a, ctrl, mseed, start, rows, cap);
  return hipGetLastError();
}

hipError_t launch_simulate(hipStream_t st, const QueryArgs& q, unsigned long long seed) {
  hipLaunchKernelGGL(k_simulate, dim3(1), dim3(64), 0, st, q, seed);
  return hipGetLastError();
}

}  // namespace mc
