// mc_kernels.hip -- exploration kernels of the MI355X explicit-state checker.
//
//   k_clear      fill the visited set with empty slots (16-byte vector stores)
//   k_reset      zero the per-query counters and the per-configuration clocks
//   k_seed       root and SELECT successors (the nondeterministic parameter choice)
//   k_level      plain level-synchronous BFS: one launch expands one BFS level
//   k_superstep  persistent engine: one configuration's subgraph per workgroup;
//                each super-step expands a frontier state's zero-time DISPATCH
//                closure and the lock-step ADVANCE runs that follow it in one
//                parallel batch of visited-set inserts
//   k_find / k_chase   counterexample: locate the terminal, follow parent slots
//   k_simulate   one seeded random run (simulation mode)
#include <hip/hip_runtime.h>

#include "mc_launch.h"

namespace mc {



__global__ void k_clear(uint4* p, unsigned long long n16) {
  const uint4 v = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += stride)
    p[i] = v;
}

__global__ void k_reset(Ctrl* ctrl, uint32_t* tc, uint32_t n_cfg) {
  if (blockIdx.x == 0) {
    unsigned int* c = reinterpret_cast<unsigned int*>(ctrl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) c[i] = 0u;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_cfg; i += gridDim.x * blockDim.x)
    tc[i] = kNoClock;
}

__device__ __forceinline__ void set_error(Ctrl* ctrl, unsigned int e) { atomicCAS(&ctrl->error, 0u, e); }

// Root and its SELECT successors.  The root carries the reserved configuration code
// n_cfg.  Writes the per-configuration start states (seeds) and level 1 of the BFS.
template <int W>
__global__ __launch_bounds__(256) void k_seed(QueryArgs a, Seed* seeds, Entry<W>* front0) {
  __shared__ uint32_t s_root;
  uint32_t probes = 0;
  if (threadIdx.x == 0) {
    St r{};
    r.cfg = a.n_cfg;
    const Key<W> k = encode<W>(r, a.L);
    uint32_t slot = kParentNone;
    const int res = table_insert<W, kScopeAgent>(a.table, a.mask, k, slot, probes);
    if (res != kInsNew) set_error(a.ctrl, kDevErrTableFull);
    else *slot_parent<W>(a.table, slot) = kParentRoot;
    s_root = slot;
    a.ctrl->root_slot = slot;
    a.ctrl->fcount[0] = a.n_cfg;
    a.ctrl->levels = 2;   // root level and the SELECT level
    a.ctrl->max_depth = 1;
    atomicAdd(&a.ctrl->states, 1ull + a.n_cfg);
    atomicAdd(&a.ctrl->edges, (unsigned long long)a.n_cfg);
  }
  __syncthreads();
  for (uint32_t c = threadIdx.x; c < a.n_cfg; c += blockDim.x) {
    St s{};
    s.cfg = c;
    s.pending = a.cfgs[c].n;
    const Key<W> k = encode<W>(s, a.L);
    uint32_t slot = kParentNone;
    const int res = table_insert<W, kScopeAgent>(a.table, a.mask, k, slot, probes);
    if (res != kInsNew) {
      set_error(a.ctrl, kDevErrTableFull);
      slot = kParentNone;
    } else {
      *slot_parent<W>(a.table, slot) = s_root;
    }
    Seed sd;
#pragma unroll
    for (int j = 0; j < 4; ++j) sd.k[j] = j < W ? k.w[j] : 0ull;
    sd.slot = slot;
    sd.depth = 1;
    sd.pad[0] = sd.pad[1] = 0;
    seeds[c] = sd;
    if (front0) {
      Entry<W> e;
#pragma unroll
      for (int j = 0; j < W; ++j) e.k[j] = k.w[j];
      e.slot = slot;
      e.depth = 1;
      front0[c] = e;
    }
  }
  const unsigned long long p = wave_sum(probes);
  if (lane_id() == 0 && p) atomicAdd(&a.ctrl->probes, p);
}

// Per-block counter reduction: one atomic per wavefront.
__device__ __forceinline__ void flush_counters(Ctrl* ctrl, unsigned long long states,
                                               unsigned long long terms, unsigned long long edges,
                                               unsigned long long dups, unsigned long long probes,
                                               unsigned long long depth) {
  states = wave_sum(states);
  terms = wave_sum(terms);
  edges = wave_sum(edges);
  dups = wave_sum(dups);
  probes = wave_sum(probes);
  depth = wave_max(depth);
  if (lane_id() == 0) {
    if (states) atomicAdd(&ctrl->states, states);
    if (terms) atomicAdd(&ctrl->terminals, terms);
    if (edges) atomicAdd(&ctrl->edges, edges);
    if (dups) atomicAdd(&ctrl->dups, dups);
    if (probes) atomicAdd(&ctrl->probes, probes);
    if (depth) atomicMax(&ctrl->max_depth, depth);
  }
}

// ---- plain level-synchronous BFS ----------------------------------------------------
//
// One launch expands the frontier of one level.  Phase 1: each thread decodes one
// frontier state and generates its successors (one per free unit while work is
// pending, else the single ADVANCE successor); the successors are compacted into an
// LDS staging buffer with a wavefront ballot and a lanes-below population count.
// Phase 2: each thread inserts one staged successor into the visited set; new
// non-terminal states are appended to the next frontier with one atomic per
// wavefront; terminals update the configuration's least clock.


template <int W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_level(LevelArgs a, const Entry<W>* __restrict__ fin,
                                                 Entry<W>* __restrict__ fout) {
  constexpr int STAGE = BLOCK * kMaxCU;
  __shared__ unsigned long long s_key[STAGE][W];
  __shared__ uint32_t s_par[STAGE];
  __shared__ uint32_t s_dep[STAGE];
  __shared__ uint32_t s_cnt;
  const QueryArgs& q = a.q;
  uint32_t n_in = __hip_atomic_load(&q.ctrl->fcount[a.in_idx], __ATOMIC_RELAXED, kScopeAgent);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    q.ctrl->fcount[a.clr_idx] = 0u;
    if (n_in) atomicAdd(&q.ctrl->levels, 1u);
  }
  if (__hip_atomic_load(&q.ctrl->error, __ATOMIC_RELAXED, kScopeAgent)) n_in = 0;  // stop
  if (n_in > a.fcap) n_in = a.fcap;  // appends beyond the capacity were dropped (error set)
  const int m = q.L.m;
  unsigned long long n_states = 0, n_terms = 0, n_edges = 0, n_dups = 0, depth_max = 0;
  uint32_t probes = 0;
  for (uint32_t base = blockIdx.x * BLOCK; base < n_in; base += gridDim.x * BLOCK) {
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < n_in;
    St x{};
    uint32_t pslot = 0, pdepth = 0;
    CfgRec r{};
    if (valid) {
      const Entry<W> e = fin[i];
      Key<W> k;
#pragma unroll
      for (int j = 0; j < W; ++j) k.w[j] = e.k[j];
      x = decode<W>(k, q.L);
      pslot = e.slot;
      pdepth = e.depth;
      r = q.cfgs[x.cfg];
    }
    uint32_t freem = 0, busy = 0;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u) {
      if (u < m && x.rem[u] == 0u) freem |= 1u << u;
      if (u < m && x.rem[u] != 0u) busy |= 1u << u;
    }
    const bool dispatch = valid && x.pending > 0 && freem != 0;
    const bool advance = valid && !dispatch && busy != 0;
    St adv = x;
    if (advance) advance_once(adv, r, m);
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j) {
      bool has = false;
      St y = x;
      if (dispatch && ((freem >> j) & 1u)) {
        y.rem[j] = r.d;
        y.pending -= 1u;
        has = true;
      } else if (advance && j == 0) {
        y = adv;
        has = true;
      }
      if (has && q.prune && y.clock > q.T) has = false;
      if (has && y.clock > q.max_clock) {
        set_error(q.ctrl, kDevErrOverflow);
        has = false;
      }
      const unsigned long long bm = __ballot(has);
      uint32_t wbase = 0;
      if (bm) {
        const int leader = __ffsll((long long)bm) - 1;
        if ((int)lane_id() == leader) wbase = atomicAdd(&s_cnt, (unsigned int)__popcll(bm));
        wbase = __shfl(wbase, leader);
      }
      if (has) {
        const uint32_t pos = wbase + lanes_below(bm);
        const Key<W> k = encode<W>(y, q.L);
#pragma unroll
        for (int w = 0; w < W; ++w) s_key[pos][w] = k.w[w];
        s_par[pos] = pslot;
        s_dep[pos] = pdepth + 1u;
      }
    }
    __syncthreads();
    const uint32_t n_st = s_cnt;
    for (uint32_t t0 = 0; t0 < n_st; t0 += BLOCK) {
      const uint32_t t = t0 + threadIdx.x;
      bool fresh = false, term = false;
      Key<W> k;
      uint32_t slot = kParentNone, dep = 0;
      if (t < n_st) {
#pragma unroll
        for (int w = 0; w < W; ++w) k.w[w] = s_key[t][w];
        dep = s_dep[t];
        ++n_edges;
        const int res = table_insert<W, kScopeAgent>(q.table, q.mask, k, slot, probes);
        if (res == kInsFail) {
          set_error(q.ctrl, kDevErrTableFull);
        } else if (res == kInsNew) {
          fresh = true;
          *slot_parent<W>(q.table, slot) = s_par[t];
          ++n_states;
          depth_max = dep > depth_max ? dep : depth_max;
          const St y = decode<W>(k, q.L);
          term = is_terminal(y, m);
          if (term) {
            ++n_terms;
            atomicMin(&q.tc[y.cfg], y.clock);
            if (q.prune) q.ctrl->violated = 1u;
          }
        } else {
          ++n_dups;
        }
      }
      const bool push = fresh && !term;
      const uint32_t pos = wave_append(push, &q.ctrl->fcount[a.out_idx]);
      if (push) {
        if (pos < a.fcap) {
          Entry<W> e;
#pragma unroll
          for (int w = 0; w < W; ++w) e.k[w] = k.w[w];
          e.slot = slot;
          e.depth = dep;
          fout[pos] = e;
        } else {
          set_error(q.ctrl, kDevErrOverflow);
        }
      }
    }
    __syncthreads();
  }
  flush_counters(q.ctrl, n_states, n_terms, n_edges, n_dups, probes, depth_max);
}

// ---- persistent super-step engine ------------------------------------------------------
//
// After SELECT the state graph is a disjoint union of one subgraph per configuration
// (the configuration index never changes), so each workgroup takes a whole subgraph
// from a queue (largest first) and explores it with workgroup-local synchronisation
// only.  A super-step expands one frontier state f:
//   * its DISPATCH closure: every set S of f's free units with |S| <= k* =
//     min(pending, #free) started (zero time; all dispatch orders reach the same set,
//     so the closure is enumerated as subsets; parent of S = S minus its highest unit);
//   * from every leaf (|S| = k*), the run of ADVANCE steps up to the next workgroup
//     completion.  When the busy units of the leaf are in lock step (same remaining
//     time) the j-th state of the run is E[i0 + j] on every busy unit, computed
//     directly per lane; otherwise the leaf contributes one ADVANCE step and the next
//     super-step continues from it.
// All states of the super-step are inserted in one parallel batch; run ends that are
// new and non-terminal form the next frontier.  Every state of the subgraph is still
// generated and inserted once per generation; only the exploration order differs from
// the level engine.


template <int W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_superstep(SuperArgs a) {
  constexpr int FCAP = 256;
  constexpr int NW = BLOCK / 64;
  __shared__ uint32_t s_mask_slot[256];
  __shared__ uint8_t s_leaf[256];
  __shared__ uint32_t s_chunk_slot[BLOCK];
  __shared__ unsigned long long s_fkey[2][FCAP][W];
  __shared__ uint32_t s_fslot[2][FCAP];
  __shared__ uint32_t s_fdep[2][FCAP];
  __shared__ uint32_t s_fcount[2];
  __shared__ uint32_t s_wcnt[NW];
  __shared__ uint32_t s_part, s_carry, s_stop;
  const QueryArgs& q = a.q;
  const int m = q.L.m;
  const uint32_t tid = threadIdx.x;
  unsigned long long n_states = 0, n_terms = 0, n_edges = 0, n_dups = 0, depth_max = 0;
  uint32_t probes = 0;

  if (tid == 0) s_stop = 0u;
  for (;;) {
    if (tid == 0) {
      s_part = atomicAdd(&q.ctrl->queue_head, 1u);
      if (__hip_atomic_load(&q.ctrl->error, __ATOMIC_RELAXED, kScopeAgent)) s_stop = 1u;
    }
    __syncthreads();
    const uint32_t part = s_part;
    if (part >= a.n_parts || s_stop) break;
    const uint32_t c = a.order[part];
    const CfgRec r = q.cfgs[c];
    if (tid == 0) {
      const Seed sd = a.seeds[c];
#pragma unroll
      for (int w = 0; w < W; ++w) s_fkey[0][0][w] = sd.k[w];
      s_fslot[0][0] = sd.slot;
      s_fdep[0][0] = sd.depth;
      s_fcount[0] = sd.slot == kParentNone ? 0u : 1u;
      s_fcount[1] = 0u;
    }
    __syncthreads();
    int cur = 0;
    while (s_fcount[cur] > 0u && !s_stop) {
      const uint32_t nf = s_fcount[cur] < (uint32_t)FCAP ? s_fcount[cur] : (uint32_t)FCAP;
      for (uint32_t fi = 0; fi < nf; ++fi) {
        Key<W> fk;
#pragma unroll
        for (int w = 0; w < W; ++w) fk.w[w] = s_fkey[cur][fi][w];
        const uint32_t fslot = s_fslot[cur][fi];
        const uint32_t fdep = s_fdep[cur][fi];
        const St x = decode<W>(fk, q.L);
        uint32_t freem = 0, busy = 0, brem = 0;
        bool bsame = true;
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u) {
          if (u < m) {
            if (x.rem[u] == 0u) {
              freem |= 1u << u;
            } else {
              if (busy && x.rem[u] != brem) bsame = false;
              brem = x.rem[u];
              busy |= 1u << u;
            }
          }
        }
        const uint32_t nfree = (uint32_t)__popc(freem);
        const uint32_t kstar = x.pending < nfree ? x.pending : nfree;
        if (kstar == 0u && busy == 0u) continue;  // terminal: no successors
        const uint32_t nclos = kstar ? (1u << nfree) - 1u : 0u;
        // leaves of the closure in ascending mask order
        uint32_t nleaf = 1u;
        if (kstar) {
          const uint32_t mk = tid + 1u;
          const bool isleaf = mk <= nclos && (uint32_t)__popc(mk) == kstar;
          const unsigned long long bm = __ballot(isleaf);
          if (lane_id() == 0) s_wcnt[tid >> 6] = (uint32_t)__popcll(bm);
          __syncthreads();
          uint32_t off = 0;
          for (uint32_t w = 0; w < (tid >> 6); ++w) off += s_wcnt[w];
          if (isleaf) s_leaf[off + lanes_below(bm)] = (uint8_t)mk;
          nleaf = 0;
          for (int w = 0; w < NW; ++w) nleaf += s_wcnt[w];
          __syncthreads();
        }
        // lock step: round start (no unit busy before the dispatches) or a pure run
        const bool lock = kstar ? (busy == 0u) : bsame;
        const uint32_t e0 = kstar ? 0u : r.d - brem;
        const uint32_t idx0 = lock ? ends_upto(r, e0) : 0u;
        const uint32_t len = lock ? r.b - idx0 : 1u;
        const uint32_t total = nclos + nleaf * len;
        if (tid == 0) s_carry = fslot;
        for (uint32_t base = 0; base < total; base += BLOCK) {
          const uint32_t i = base + tid;
          bool active = i < total;
          const bool is_clos = i < nclos;
          uint32_t rmask = 0, j = 0;
          St y = x;
          uint32_t dep = 0;
          if (active) {
            if (is_clos) {
              rmask = i + 1u;
            } else {
              const uint32_t qq = i - nclos;
              const uint32_t leaf = qq / len;
              j = qq - leaf * len;
              rmask = kstar ? (uint32_t)s_leaf[leaf] : 0u;
            }
            const uint32_t ns = (uint32_t)__popc(rmask);
            if (is_clos && ns > kstar) active = false;
            // start the units of rmask: bit t of rmask is the t-th free unit
            uint32_t t = 0;
#pragma unroll
            for (int u = 0; u < kMaxCU; ++u) {
              if ((freem >> u) & 1u) {
                if ((rmask >> t) & 1u) y.rem[u] = r.d;
                ++t;
              }
            }
            y.pending -= ns;
            dep = fdep + ns;
            if (!is_clos) {
              if (lock) {
                const uint32_t e = end_at(r, idx0 + j);
                y.clock = x.clock + (e - e0);
#pragma unroll
                for (int u = 0; u < kMaxCU; ++u)
                  if (u < m && y.rem[u]) y.rem[u] = r.d - e;
              } else {
                advance_once(y, r, m);
              }
              dep += j + 1u;
              if (q.prune && y.clock > q.T) active = false;
            }
          }
          if (active && y.clock > q.max_clock) {
            set_error(q.ctrl, kDevErrOverflow);
            active = false;
          }
          uint32_t slot = kParentNone;
          bool fresh = false, term = false;
          if (active) {
            const Key<W> k = encode<W>(y, q.L);
            ++n_edges;
            const int res = table_insert<W, kScopeWG>(q.table, q.mask, k, slot, probes);
            if (res == kInsFail) {
              set_error(q.ctrl, kDevErrTableFull);
              s_stop = 1u;
              active = false;
              slot = kParentNone;
            } else if (res == kInsNew) {
              fresh = true;
              ++n_states;
              depth_max = dep > depth_max ? dep : depth_max;
              term = is_terminal(y, m);
              if (term) {
                ++n_terms;
                atomicMin(&q.tc[c], y.clock);
                if (q.prune) q.ctrl->violated = 1u;
              }
            } else {
              ++n_dups;
            }
            if (is_clos) s_mask_slot[rmask] = slot;
          }
          s_chunk_slot[tid] = slot;
          __syncthreads();
          if (fresh) {
            uint32_t par;
            if (is_clos) {
              const uint32_t pm = rmask & ~(1u << (31 - __clz(rmask)));
              par = pm ? s_mask_slot[pm] : fslot;
            } else if (j == 0u) {
              par = rmask ? s_mask_slot[rmask] : fslot;
            } else {
              par = tid ? s_chunk_slot[tid - 1] : s_carry;
            }
            *slot_parent<W>(q.table, slot) = par;
            if (!is_clos && j + 1u == len && !term) {
              const uint32_t pos = atomicAdd(&s_fcount[cur ^ 1], 1u);
              if (pos < (uint32_t)FCAP) {
                const Key<W> k = encode<W>(y, q.L);
#pragma unroll
                for (int w = 0; w < W; ++w) s_fkey[cur ^ 1][pos][w] = k.w[w];
                s_fslot[cur ^ 1][pos] = slot;
                s_fdep[cur ^ 1][pos] = dep;
              } else {
                set_error(q.ctrl, kDevErrOverflow);
              }
            }
          }
          __syncthreads();
          if (tid == BLOCK - 1) s_carry = s_chunk_slot[BLOCK - 1];
          __syncthreads();
        }
      }
      if (tid == 0) s_fcount[cur] = 0u;
      __syncthreads();
      cur ^= 1;
    }
  }
  flush_counters(q.ctrl, n_states, n_terms, n_edges, n_dups, probes, depth_max);
}

// ---- counterexample -----------------------------------------------------------------

template <int W>
__global__ void k_find(QueryArgs a, Key<W> k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) a.ctrl->target_slot = table_find<W>(a.table, a.mask, k);
}

// Follows parent slots from the target to the root, writing keys terminal-first.
template <int W>
__global__ void k_chase(QueryArgs a, unsigned long long* out, uint32_t cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t s = a.ctrl->target_slot;
  uint32_t n = 0;
  while (s != kParentRoot) {
    if (s == kParentNone || (unsigned long long)s > a.mask || n >= cap) {
      set_error(a.ctrl, kDevErrTrace);
      break;
    }
    const unsigned long long* p = slot_key<W>(a.table, s);
#pragma unroll
    for (int w = 0; w < W; ++w) out[(unsigned long long)n * W + w] = p[w];
    ++n;
    s = *slot_parent<W>(a.table, s);
  }
  a.ctrl->trace_len = n;
}

// ---- simulation mode ------------------------------------------------------------------
//
// One run from the root, choosing uniformly among the successors at every step with
// the choice of step t drawn from splitmix64(seed ^ splitmix64(t)); successors are
// ordered by configuration (SELECT) and by unit index (DISPATCH).  A lock-step ADVANCE
// run has one successor per step; it is taken in one jump that counts its steps.
__global__ void k_simulate(QueryArgs a, unsigned long long seed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = a.L.m;
  unsigned long long step = 0;
  const uint32_t c = (uint32_t)(splitmix64(seed ^ splitmix64(step)) % a.n_cfg);
  ++step;
  const CfgRec r = a.cfgs[c];
  St x{};
  x.cfg = c;
  x.pending = r.n;
  for (;;) {
    uint32_t freem = 0, busy = 0, brem = 0;
    bool same = true;
    for (int u = 0; u < m; ++u) {
      if (x.rem[u] == 0u) {
        freem |= 1u << u;
      } else {
        if (busy && x.rem[u] != brem) same = false;
        brem = x.rem[u];
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
            x.rem[u] = r.d;
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
      const uint32_t e0 = r.d - brem;
      step += r.b - ends_upto(r, e0);
      x.clock += brem;
      for (int u = 0; u < m; ++u) x.rem[u] = 0u;
    } else {
      advance_once(x, r, m);
      ++step;
    }
  }
  a.ctrl->sim_t = x.clock;
  a.ctrl->sim_cfg = c;
}

// ---- launch helpers (host) ------------------------------------------------------------

template <int W>
hipError_t launch_seed(hipStream_t st, const QueryArgs& q, Seed* seeds, void* front0) {
  hipLaunchKernelGGL((k_seed<W>), dim3(1), dim3(256), 0, st, q, seeds,
                     reinterpret_cast<Entry<W>*>(front0));
  return hipGetLastError();
}

template <int W>
hipError_t launch_level(hipStream_t st, uint32_t grid, const LevelArgs& la, const void* fin,
                        void* fout) {
  hipLaunchKernelGGL((k_level<W, kLevelBlock>), dim3(grid), dim3(kLevelBlock), 0, st, la,
                     reinterpret_cast<const Entry<W>*>(fin), reinterpret_cast<Entry<W>*>(fout));
  return hipGetLastError();
}

template <int W>
hipError_t launch_super(hipStream_t st, uint32_t grid, uint32_t block, const SuperArgs& sa) {
  switch (block) {
    case 256:
      hipLaunchKernelGGL((k_superstep<W, 256>), dim3(grid), dim3(256), 0, st, sa);
      break;
    case 512:
      hipLaunchKernelGGL((k_superstep<W, 512>), dim3(grid), dim3(512), 0, st, sa);
      break;
    default:
      hipLaunchKernelGGL((k_superstep<W, 1024>), dim3(grid), dim3(1024), 0, st, sa);
      break;
  }
  return hipGetLastError();
}

template <int W>
hipError_t launch_find(hipStream_t st, const QueryArgs& q, const unsigned long long* key) {
  Key<W> k;
  for (int w = 0; w < W; ++w) k.w[w] = key[w];
  hipLaunchKernelGGL((k_find<W>), dim3(1), dim3(64), 0, st, q, k);
  return hipGetLastError();
}

template <int W>
hipError_t launch_chase(hipStream_t st, const QueryArgs& q, unsigned long long* out, uint32_t cap) {
  hipLaunchKernelGGL((k_chase<W>), dim3(1), dim3(64), 0, st, q, out, cap);
  return hipGetLastError();
}

#define MC_INSTANTIATE(W)                                                                  \
  template hipError_t launch_seed<W>(hipStream_t, const QueryArgs&, Seed*, void*);         \
  template hipError_t launch_level<W>(hipStream_t, uint32_t, const LevelArgs&, const void*, \
                                      void*);                                              \
  template hipError_t launch_super<W>(hipStream_t, uint32_t, uint32_t, const SuperArgs&);  \
  template hipError_t launch_find<W>(hipStream_t, const QueryArgs&,                       \
                                     const unsigned long long*);                           \
  template hipError_t launch_chase<W>(hipStream_t, const QueryArgs&, unsigned long long*,  \
                                      uint32_t);
MC_INSTANTIATE(1)
MC_INSTANTIATE(2)
MC_INSTANTIATE(4)

hipError_t launch_clear(hipStream_t st, void* p, unsigned long long bytes) {
  const unsigned long long n16 = bytes / 16;
  unsigned long long grid = (n16 + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_clear, dim3((uint32_t)grid), dim3(256), 0, st, reinterpret_cast<uint4*>(p),
                     n16);
  return hipGetLastError();
}

hipError_t launch_reset(hipStream_t st, Ctrl* ctrl, uint32_t* tc, uint32_t n_cfg) {
  uint32_t grid = (n_cfg + 255) / 256;
  if (grid == 0) grid = 1;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, st, ctrl, tc, n_cfg);
  return hipGetLastError();
}

hipError_t launch_simulate(hipStream_t st, const QueryArgs& q, unsigned long long seed) {
  hipLaunchKernelGGL(k_simulate, dim3(1), dim3(64), 0, st, q, seed);
  return hipGetLastError();
}

}  // namespace mc
