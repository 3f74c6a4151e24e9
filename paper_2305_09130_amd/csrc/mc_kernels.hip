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
// The seeded walks (simulation and swarm search) are in mc_walks.hip; the counterexample
// and the count of a visited set up to a clock in mc_trace.hip.
#include <hip/hip_runtime.h>

#include "mc_launch.h"

// The file is compiled once per part, so that the many instances of the persistent
// kernel build in parallel: MC_PART 0 holds every kernel and launch helper except the
// k_superstep instances; MC_PART 1, 2 and 4 hold the k_superstep instances of that key
// width (launch_super_w).
#ifndef MC_PART
#define MC_PART 0
#endif

namespace mc {

#if MC_PART == 0
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
#endif  // MC_PART == 0


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
    const int res = table_insert<W, kScopeAgent>(a.table, a.mask, k, slot, probes, a.hkeep);
    if (res != kInsNew) set_error(a.ctrl, kDevErrTableFull);
    else set_links<W>(a.table, a.mask, slot, kParentRoot, kParentNone);
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
    const int res = table_insert<W, kScopeAgent>(a.table, a.mask, k, slot, probes, a.hkeep);
    if (res != kInsNew) {
      set_error(a.ctrl, kDevErrTableFull);
      slot = kParentNone;
    } else {
      set_links<W>(a.table, a.mask, slot, s_root, kParentNone);
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
  __shared__ uint32_t s_n_in;
  const QueryArgs& q = a.q;
  if (threadIdx.x == 0) {
    // one read of the frontier size and of the error and abort flags per workgroup: the
    // flags are set concurrently by other workgroups (or the host), and every wave must
    // run the same number of barrier-separated iterations below
    uint32_t n = __hip_atomic_load(&q.ctrl->fcount[a.in_idx], __ATOMIC_RELAXED, kScopeAgent);
    if (blockIdx.x == 0) {
      q.ctrl->fcount[a.clr_idx] = 0u;
      if (n) atomicAdd(&q.ctrl->levels, 1u);
    }
    if (__hip_atomic_load(&q.ctrl->error, __ATOMIC_RELAXED, kScopeAgent)) n = 0;  // stop
    if (n && a.abort && __hip_atomic_load(a.abort, __ATOMIC_RELAXED, kScopeSystem)) {
      set_error(q.ctrl, kDevErrAbort);
      n = 0;
    }
    if (n > a.fcap) n = a.fcap;  // appends beyond the capacity were dropped (error set)
    s_n_in = n;
  }
  __syncthreads();
  const uint32_t n_in = s_n_in;
  const int m = q.L.m;
  unsigned long long n_states = 0, n_terms = 0, n_edges = 0, n_dups = 0, depth_max = 0;
  uint32_t probes = 0, max_probe = 0;
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
      x = decode<W>(k, q.L, q.cfgs);
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
    if (advance) advance_once(adv, r, m, q.L.speed);
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j) {
      bool has = false;
      St y = x;
      if (dispatch && ((freem >> j) & 1u)) {
        y.rem[j] = unit_dur<true>(r, q.L.speed, j);
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
        const uint32_t p0 = probes;
        const int res = table_insert<W, kScopeAgent>(q.table, q.mask, k, slot, probes, q.hkeep);
        max_probe = probes - p0 > max_probe ? probes - p0 : max_probe;
        if (res == kInsFail) {
          set_error(q.ctrl, kDevErrTableFull);
        } else if (res == kInsNew) {
          fresh = true;
          set_links<W>(q.table, q.mask, slot, s_par[t], kParentNone);
          ++n_states;
          depth_max = dep > depth_max ? dep : depth_max;
          const St y = decode<W>(k, q.L, q.cfgs);
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
  const unsigned long long mp = wave_max(max_probe);
  if (lane_id() == 0 && mp) atomicMax(&q.ctrl->max_probe, (unsigned int)mp);
}

// ---- persistent super-step engine ------------------------------------------------------
//
// After SELECT the state graph is a disjoint union of one subgraph per configuration
// (the configuration index never changes), and the models of a batch are disjoint too.
// Each persistent workgroup takes a whole (model, configuration) subgraph from a queue
// (largest first) and explores it with workgroup-local synchronisation only.  A
// super-step expands one frontier state f:
//   * its DISPATCH closure: every set S of f's free units with |S| <= k* =
//     min(pending, #free) started (zero time; all dispatch orders reach the same set,
//     so the closure is enumerated as subsets; parent of S = S minus its highest unit);
//   * from every leaf (|S| = k*), the run of ADVANCE steps up to the next workgroup
//     completion.  When the busy units of the leaf are in lock step (same remaining
//     time) the j-th state of the run has operation end E[i0 + j] on every busy unit;
//     its key is built directly as base + rem * M (+ the clock field), M having one
//     bit at the low end of every busy unit's field.  Otherwise the leaf contributes
//     one ADVANCE step and the next super-step continues from it.
// A lock-step run from a single leaf ends in a state whose successors are again a
// closure and a run; up to kSegMax such segments are generated from one frontier
// state in the same batch, without waiting for the visited-set verdict on the run end.
// Every generated state is a successor of a generated state, so only reachable states
// are inserted, and the visited set alone decides which are new: a run end found to be
// a duplicate was expanded by whoever inserted it first, and its re-expansion only
// produces duplicates.  Run ends that are new and non-terminal form the next frontier.
//
// Blocks of rounds.  A full round (every unit idle, at least m workgroups pending)
// starts all m units at one clock; they stay in lock step and the round ends with every
// unit idle again, at clock + d with m fewer pending.  Every path of the configuration
// therefore passes through the state B_r reached after r full rounds, and a partition
// may cover rounds [r0, r1) only.  Such a block inserts B_r0 itself (it may find it
// already inserted by the block before), explores from it, and stops at B_r1: that
// state is inserted, given its parent and jump, and left to the next block.  B_r0 and
// B_r1 are the only states a block shares with another workgroup, and, the
// configuration, pending count and clock being in key word 0, the only word-0 values it
// shares; they are inserted with agent-scope ordering, every other key with
// workgroup-scope ordering as in a whole subgraph.  A block checks that its last run
// ends exactly on B_r1 with the depth r1 rounds give, so that the union of the blocks
// is the configuration's whole subgraph.
constexpr int kSegMax = 8;
constexpr int kSegMaxChain = 32;  // segments of a batch on units of unequal speed
constexpr uint32_t kNoItem = 0xFFFFFFFFu;
constexpr int kEMax = 4096;  // operation ends kept in LDS
constexpr int kFCap = 256;   // frontier states per super-step level (LDS)
constexpr int kMaxLeaves = 72;  // C(8, 4) = 70 leaves at most
constexpr int kChainCand = 1024;         // chain candidates: 1024 / m ends to go per unit
constexpr int kChainTimes = 1280;        // the batch's chain times, listed in E from here
static_assert(kChainTimes >= kChainCand + 1 && kChainTimes + kChainCand <= kEMax, "E use");
static_assert(kSegMax * 256 >= kChainCand + 1, "chain prefix sums fit in the closure slots");

struct SegDesc {
  unsigned long long fkey[4];  // frontier state of the segment
  unsigned long long base[4];  // run key with clock 0 and busy units' rem 0
  unsigned long long M[4];     // one bit at the low end of every busy unit's rem field
  uint32_t start, nclos, nleaf, len;
  uint32_t kstar, freem, lock, idx0;
  uint32_t e0, fclock, pend, fdep;
  uint32_t fslot, nfree, aux, pad;  // pad: 1 for a chain (states listed in gkey)
};

template <int BLOCK, int NI, int SEGS, int KW>  // KW: words of a key
struct SuperShared {
  uint32_t E[kEMax];
  uint32_t mslot[SEGS][256];
  uint8_t leaf[256];
  uint32_t chunk_slot[NI * BLOCK];
  SegDesc seg[SEGS];
  uint32_t segfslot[SEGS];
  unsigned long long fkey[2][kFCap][KW];
  uint32_t fslot[2][kFCap];
  uint32_t fdep[2][kFCap];
  uint32_t fcount[2];
  uint32_t part, carry, stop, nseg, total;
  uint32_t skip;        // the partition is not explored (an error, or an abort from the host)
  // a chain slice of units of unequal speed ends at clock `cut` (kNoClock: no cut);
  // `pr` = states past T are dropped (a check, branch and bound, or a cut)
  uint32_t cut, pr;
  uint32_t chain_more;  // another chain joined the batch: list it
  // end of a block of rounds: the state B_r1, its clock and depth, the batch item that
  // generates it, and whether it was reached
  unsigned long long stopkey[KW];
  uint32_t has_stop, stop_clock, stop_dep, stop_item, stop_slot, handed;
  uint32_t stop_capped;  // B_r1 ends a run cut short by run slices: no item generates it
  uint32_t T;   // prune threshold of this super-step (check(T), or the incumbent)
  ModelDev md;  // descriptor of the model being explored
  // successors of the leaves of a segment whose run is not in lock step (one ADVANCE
  // each), computed once per super-step outside the batch loop
  unsigned long long gkey[kMaxLeaves][KW];
  uint32_t gclk[kMaxLeaves];
  uint32_t gterm[kMaxLeaves];
};

struct Tally {
  unsigned long long states = 0, terms = 0, edges = 0, dups = 0, depth = 0, super = 0,
                     chunks = 0;
  uint32_t probes = 0, max_probe = 0;
};

// adds v to field f of a packed key (the field must not overflow into its neighbour)
template <int W>
__device__ __forceinline__ void field_add(unsigned long long* k, const Layout& L, int f,
                                          unsigned long long v) {
  if (L.width[f] == 0) return;  // a field the key does not store (an implied clock)
  const unsigned long long x = v << L.shift[f];
  const int wf = L.word[f];
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (wf == j) k[j] += x;
}

template <int W>
struct Item {
  unsigned long long key[W];
  uint32_t sgi, rmask, j, dep, clk;
  bool active, is_clos, term;
};

// State number i of the current batch: a closure state (a set of started units) or the
// j-th state of a run from a leaf, built directly from the segment's templates.
template <int W, int BLOCK, int NI, bool KEY, bool GEN, bool HET, int SEGS>
__device__ __forceinline__ void gen_item(uint32_t i, uint32_t total, uint32_t nseg,
                                         const SuperShared<BLOCK, NI, SEGS, W>& sh, const CfgRec& r,
                                         bool e_lds, const ModelDev& md, int m, Item<W>& it) {
  const Layout& L = md.L;
  it.active = i < total;
  it.sgi = 0;
  for (uint32_t k = 1; k < nseg; ++k)
    if (i >= sh.seg[k].start) it.sgi = k;
  const SegDesc& sg = sh.seg[it.sgi];
  const uint32_t loc = i - sg.start;
  it.is_clos = loc < sg.nclos;
  it.rmask = 0;
  it.j = 0;
  it.dep = 0;
  it.clk = sg.fclock;
  it.term = false;
#pragma unroll
  for (int w = 0; w < W; ++w) it.key[w] = 0ull;
  if (!it.active) return;
  if (it.is_clos) {
    it.rmask = loc + 1u;
    const uint32_t ns = (uint32_t)__popc(it.rmask);
    if (ns > sg.kstar) it.active = false;
    if (KEY) {
      if (L.shared_rem && sg.freem == (1u << m) - 1u) {
        // from an all-idle state (every dispatch on equal units): the dispatched units
        // are the mask's bits and all have time d
#pragma unroll
        for (int w = 0; w < W; ++w) it.key[w] = sg.fkey[w];
        field_add<W>(it.key, L, kFRem, it.rmask);
        field_add<W>(it.key, L, kFRem + 1, r.d);
        field_add<W>(it.key, L, kFPending, (unsigned long long)(-(long long)ns));
      } else if (L.shared_rem) {  // the dispatched units join the busy mask, all with time d
        Key<W> fk;
#pragma unroll
        for (int w = 0; w < W; ++w) fk.w[w] = sg.fkey[w];
        St y = decode<W>(fk, L, md.cfgs);
        uint32_t t = 0;
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u) {
          if ((sg.freem >> u) & 1u) {
            if ((it.rmask >> t) & 1u) y.rem[u] = r.d;
            ++t;
          }
        }
        y.pending -= ns;
        const Key<W> yk = encode<W>(y, L);
#pragma unroll
        for (int w = 0; w < W; ++w) it.key[w] = yk.w[w];
      } else {
#pragma unroll
        for (int w = 0; w < W; ++w) it.key[w] = sg.fkey[w];
        uint32_t t = 0;
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u) {
          if ((sg.freem >> u) & 1u) {
            if ((it.rmask >> t) & 1u) field_add<W>(it.key, L, kFRem + u, unit_dur<GEN>(r, L.speed, u));
            ++t;
          }
        }
        field_add<W>(it.key, L, kFPending, (unsigned long long)(-(long long)ns));
      }
    }
    it.dep = sg.fdep + ns;
    return;
  }
  const uint32_t qq = loc - sg.nclos;
  const uint32_t leaf = qq / sg.len;
  it.j = qq - leaf * sg.len;
  it.rmask = sg.kstar ? (sg.nleaf == 1u ? (1u << sg.nfree) - 1u : (uint32_t)sh.leaf[leaf]) : 0u;
  it.dep = sg.fdep + sg.kstar + it.j + 1u;
  if (sg.lock) {
    const uint32_t e = e_lds ? sh.E[sg.idx0 + it.j] : end_at_t<GEN>(r, sg.idx0 + it.j);
    it.clk = sg.fclock + (e - sg.e0);
    if (KEY) {
      const unsigned long long rem = r.d - e;
      unsigned long long Mv[W];
#pragma unroll
      for (int w = 0; w < W; ++w) Mv[w] = sg.M[w];
      // the run's busy units: the leaf's dispatched units, or the frontier's busy ones
      uint32_t um = sg.kstar ? sg.freem : (((1u << m) - 1u) & ~sg.freem);
      if (sg.kstar && sg.nleaf > 1u) {
        um = 0u;
        uint32_t t = 0;
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u) {
          if ((sg.freem >> u) & 1u) {
            if ((it.rmask >> t) & 1u) um |= 1u << u;
            ++t;
          }
        }
        if (!L.shared_rem) {
#pragma unroll
          for (int w = 0; w < W; ++w) Mv[w] = 0ull;
#pragma unroll
          for (int u = 0; u < kMaxCU; ++u)
            if ((um >> u) & 1u) field_add<W>(Mv, L, kFRem + u, 1ull);
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) it.key[w] = sg.base[w] + rem * Mv[w];
      // shared time left: the busy mask is set while the units are busy (rem > 0)
      if (L.shared_rem && rem) field_add<W>(it.key, L, kFRem, um);
      field_add<W>(it.key, L, kFClock, it.clk);
    }
    it.term = sg.pend == 0u && e == r.d;
  } else if (HET && sg.pad) {
    // state j of a chain: the frontier state advanced to the j-th listed time
    Key<W> fk;
#pragma unroll
    for (int w = 0; w < W; ++w) fk.w[w] = sg.fkey[w];
    St y = decode<W>(fk, L, md.cfgs);
    const uint32_t tau = sh.E[kChainTimes + sg.idx0 + it.j], dt = tau - y.clock;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u) y.rem[u] = y.rem[u] > dt ? y.rem[u] - dt : 0u;
    y.clock = tau;
    it.clk = tau;
    it.term = is_terminal(y, m);
    if (KEY) {
      const Key<W> yk = encode<W>(y, L);
#pragma unroll
      for (int w = 0; w < W; ++w) it.key[w] = yk.w[w];
    }
  } else {
    it.clk = sh.gclk[leaf];
    it.term = sh.gterm[leaf] != 0u;
    if (KEY) {
#pragma unroll
      for (int w = 0; w < W; ++w) it.key[w] = sh.gkey[leaf][w];
    }
  }
  if (sh.pr && it.clk > sh.T) it.active = false;
}

__device__ __forceinline__ void flush_tally(const ModelDev& md, const Tally& tl);

// A chain on units of unequal speed: from the frontier state x of the last segment (no
// DISPATCH enabled) the clock visits the union of the busy units' operation ends, up to
// the first workgroup end while work is pending (then a DISPATCH follows), or to the
// terminal.  Every lane writes one candidate end (unit u, its k-th end to go, k < p =
// 1024 / m) into the LDS table E (unused on such models: no run is in lock step), and the
// workgroup merges the units' lists, keeping the distinct times up to the smallest p-th
// candidate of any unit (below it no end of any unit is missing), in
// order, as the chain's states, from E[kChainTimes + idx0] (the batch's chains are
// listed one after another).  Their number is the segment's length.
template <int W, int BLOCK, int NI, int SEGS>
__device__ __noinline__ void build_chain(SuperShared<BLOCK, NI, SEGS, W>& sh, const CfgRec& r,
                                         const Layout& L, int m) {
  const uint32_t tid = threadIdx.x;
  SegDesc& sg = sh.seg[sh.nseg - 1];
  Key<W> fk;
#pragma unroll
  for (int w = 0; w < W; ++w) fk.w[w] = sg.fkey[w];
  const St x = decode<W>(fk, L, nullptr)  /* unequal units store the clock */;
  uint32_t H = 0xFFFFFFFFu;  // with work pending the chain stops at the first workgroup end
  if (x.pending)
    for (int u = 0; u < m; ++u)
      if (x.rem[u]) H = min(H, x.clock + x.rem[u]);
  uint32_t* ct = sh.E;
  if (tid == 0) ct[kChainCand] = 0xFFFFFFFFu;  // the smallest last-slot candidate
  __syncthreads();
  const uint32_t per = (uint32_t)kChainCand / (uint32_t)m;  // candidates per unit
  for (uint32_t i = tid; i < (uint32_t)kChainCand; i += BLOCK) {
    const int u = (int)(i / per);
    const uint32_t k = i - (uint32_t)u * per;
    uint32_t v = 0xFFFFFFFFu;
    if (u < m && x.rem[u]) {
      const uint32_t sp = L.speed[u];
      const uint32_t e = sp * r.d - x.rem[u];
      const uint32_t kk = ends_upto(r, e / sp) + k;
      if (kk < r.b) {
        const uint32_t tau = x.clock + sp * end_at(r, kk) - e;
        if (tau <= H) {
          v = tau;
          if (k + 1u == per) atomicMin(&ct[kChainCand], tau);
        }
      }
    }
    ct[i] = v;
  }
  __syncthreads();
  // Each unit's candidates ascend with k (then the unset ones), so a binary search in
  // unit j's list gives how many of its ends come before v and whether it ends at v.
  // An end counts once, on the lowest unit that has it ("first"); the chain's time of
  // rank q is the first end with q distinct ends before it: the first ends before it
  // are counted per unit from an exclusive prefix sum of the first flags.
  const uint32_t lim = ct[kChainCand];
  uint32_t* cg = &sh.mslot[0][0];  // free while chains are listed: closures fill it later
  constexpr int kPerThr = (kChainCand + BLOCK - 1) / BLOCK;
  uint32_t pos[kPerThr][kMaxCU];
  uint32_t val[kPerThr];
  bool fst[kPerThr];
#pragma unroll
  for (int q = 0; q < kPerThr; ++q) {
    const uint32_t i = tid + (uint32_t)q * BLOCK;
    fst[q] = false;
    val[q] = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j) pos[q][j] = 0u;
    if (i < (uint32_t)kChainCand) {
      const uint32_t u = i / per, k = i - u * per, v = ct[i];
      bool ok = u < (uint32_t)m && v <= lim && v != 0xFFFFFFFFu;
      if (ok) {
#pragma unroll
        for (int j = 0; j < kMaxCU; ++j) {
          if (j >= m) continue;
          if ((uint32_t)j == u) {
            pos[q][j] = k;
            continue;
          }
          const uint32_t* lj = ct + (uint32_t)j * per;
          uint32_t lo = 0, n = per;  // lower bound: the first entry >= v
          while (n) {
            const uint32_t half = n >> 1;
            if (lj[lo + half] < v) {
              lo += half + 1u;
              n -= half + 1u;
            } else {
              n = half;
            }
          }
          pos[q][j] = lo;
          if ((uint32_t)j < u && lo < per && lj[lo] == v) ok = false;
        }
      }
      fst[q] = ok;
      val[q] = v;
      cg[i] = ok ? 1u : 0u;
    }
  }
  __syncthreads();
  if (tid < 64) {  // exclusive prefix sum of the flags; cg[kChainCand] = their total
    constexpr int kPer = kChainCand / 64;
    uint32_t loc[kPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      loc[q] = cg[tid * kPer + q];
      sum += loc[q];
    }
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if ((int)tid >= off) incl += y;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      cg[tid * kPer + q] = run;
      run += loc[q];
    }
    if (tid == 63) {
      cg[kChainCand] = incl;
      sg.len = incl;
      sh.total = sg.start + incl;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPerThr; ++q) {
    if (!fst[q]) continue;
    uint32_t rank = 0;
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j)
      if (j < m) rank += cg[(uint32_t)j * per + pos[q][j]] - cg[(uint32_t)j * per];
    ct[kChainTimes + sg.idx0 + rank] = val[q];
  }
}

// After a chain is listed (thread 0): when its last state is neither terminal nor a
// choice among units (its dispatch has one leaf), what follows it is determined too, and
// joins the same batch: the dispatch closure (every idle unit takes a workgroup) and the
// chain from its leaf, or, after a chain cut by its candidate window, the chain that
// continues it.  sh.chain_more tells the workgroup to list the new chain.  Only a
// choice among units, a terminal, the prune threshold or the batch's room ends a batch.
template <int W, int BLOCK, int NI, int SEGS, bool GEN>
__device__ __noinline__ void extend_chain(SuperShared<BLOCK, NI, SEGS, W>& sh, const CfgRec& r,
                                          const ModelDev& md, int m, uint32_t batch_items) {
  const Layout& L = md.L;
  sh.chain_more = 0u;
  uint32_t nseg = sh.nseg;
  const SegDesc& sg = sh.seg[nseg - 1u];
  const uint32_t off = sg.idx0 + sg.len;  // the next chain's times start here
  if (sg.len == 0u || nseg + 2u > (uint32_t)SEGS || sh.total >= batch_items ||
      off + (uint32_t)kChainCand > (uint32_t)(kEMax - kChainTimes))
    return;
  const uint32_t tau = sh.E[kChainTimes + off - 1u];
  if ((sh.pr && tau > sh.T) || tau > md.max_clock) return;
  Key<W> fk;
#pragma unroll
  for (int w = 0; w < W; ++w) fk.w[w] = sg.fkey[w];
  St y = decode<W>(fk, L, md.cfgs);
  const uint32_t dt = tau - y.clock;
  uint32_t freem = 0;
#pragma unroll
  for (int u = 0; u < kMaxCU; ++u) {
    y.rem[u] = y.rem[u] > dt ? y.rem[u] - dt : 0u;
    if (u < m && y.rem[u] == 0u) freem |= 1u << u;
  }
  y.clock = tau;
  if (is_terminal(y, m)) return;
  const uint32_t nfree = (uint32_t)__popc(freem);
  const uint32_t kstar = y.pending < nfree ? y.pending : nfree;
  if (kstar && kstar < nfree) return;  // C(nfree, kstar) > 1 leaves: a choice
  const uint32_t dep = sg.fdep + sg.len;  // depth of the chain's last state
  uint32_t total = sh.total;
  if (kstar) {
    SegDesc& cs = sh.seg[nseg];
    const Key<W> yk = encode<W>(y, L);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      cs.fkey[w] = w < W ? yk.w[w] : 0ull;
      cs.base[w] = 0ull;
      cs.M[w] = 0ull;
    }
    cs.kstar = kstar;
    cs.freem = freem;
    cs.nfree = nfree;
    cs.nclos = (1u << nfree) - 1u;
    cs.nleaf = 1u;
    cs.lock = 0u;
    cs.aux = 0u;
    cs.pad = 0u;
    cs.len = 0u;
    cs.e0 = 0u;
    cs.idx0 = 0u;
    cs.pend = y.pending - kstar;
    cs.fclock = tau;
    cs.fdep = dep;
    cs.fslot = kParentNone;  // the chain's last state: its slot comes from that item
    cs.start = total;
    total += cs.nclos;
    ++nseg;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u)
      if ((freem >> u) & 1u) y.rem[u] = unit_dur<GEN>(r, L.speed, u);
    y.pending -= kstar;
  }
  SegDesc& nx = sh.seg[nseg];
  const Key<W> yk = encode<W>(y, L);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    nx.fkey[w] = w < W ? yk.w[w] : 0ull;
    nx.base[w] = 0ull;
    nx.M[w] = 0ull;
  }
  nx.kstar = 0u;
  nx.freem = 0u;
  nx.nfree = 0u;
  nx.nclos = 0u;
  nx.nleaf = 1u;
  nx.lock = 0u;
  nx.aux = 0u;
  nx.pad = 1u;
  nx.len = 0u;
  nx.e0 = 0u;
  nx.idx0 = off;
  nx.pend = y.pending;
  nx.fclock = tau;
  nx.fdep = dep + kstar;
  nx.fslot = kParentNone;
  nx.start = total;
  ++nseg;
  sh.nseg = nseg;
  sh.total = total;
  sh.chain_more = 1u;
}

// Prune threshold: the query's T, or under branch and bound the least terminal clock
// found so far when that is lower.  The incumbent only falls, so a stale value prunes
// less, never wrongly: every state on a path to an optimal terminal has a clock at most
// T_min, which never exceeds the incumbent.
__device__ __forceinline__ uint32_t prune_T(const ModelDev& md) {
  if (!md.bb) return md.T;
  const uint32_t b = __hip_atomic_load(&md.ctrl->bound, __ATOMIC_RELAXED, kScopeAgent);
  return b < md.T ? b : md.T;
}

template <int W, int BLOCK, int NI, bool GEN, bool HET, int SEGS>
__device__ void explore_partition(const ModelDev& md, const Part pt, uint32_t batch_items,
                                  uint32_t slice, const PartQueue& pq,
                                  SuperShared<BLOCK, NI, SEGS, W>& sh) {
  Tally tl;
  const Layout& L = md.L;
  const int m = L.m;
  const uint32_t tid = threadIdx.x;
  const uint32_t c = pt.cfg;
  const CfgRec r = md.cfgs[c];
  const bool e_lds = r.b <= (uint32_t)kEMax;
  if (e_lds)
    for (uint32_t k = tid; k < r.b; k += BLOCK) sh.E[k] = end_at_t<GEN>(r, k);
  const bool chain_slice = HET && pt.r0 == kChainSlice;
  if (tid == 0) {
    sh.has_stop = 0u;
    sh.handed = 0u;
    sh.stop_capped = 0u;
    sh.stop_item = kNoItem;
    sh.cut = chain_slice ? pt.r1 : kNoClock;
    sh.pr = (md.prune || sh.cut != kNoClock) ? 1u : 0u;
    sh.T = md.prune ? min(prune_T(md), sh.cut) : sh.cut;
    const Seed sd = md.seeds[c];
    const uint32_t round_dep = (uint32_t)m + r.b;  // m dispatches, b advances
    if (!chain_slice && pt.r1 != kRoundsToEnd) {
      unsigned long long k1[W];
#pragma unroll
      for (int w = 0; w < W; ++w) k1[w] = sd.k[w];
      field_add<W>(k1, L, kFClock, (unsigned long long)pt.r1 * r.d);
      field_add<W>(k1, L, kFPending, (unsigned long long)(-(long long)pt.r1 * m));
#pragma unroll
      for (int w = 0; w < W; ++w) sh.stopkey[w] = k1[w];
      sh.stop_clock = pt.r1 * r.d;
      sh.stop_dep = sd.depth + pt.r1 * round_dep;
      sh.has_stop = 1u;
    }
    if (md.pstate && md.pstate[pt.pidx].status == 1u) {  // resume a partition that yielded
      const PartState ps = md.pstate[pt.pidx];
#pragma unroll
      for (int w = 0; w < W; ++w) sh.fkey[0][0][w] = ps.k[w];
      sh.fslot[0][0] = ps.slot;
      sh.fdep[0][0] = ps.depth;
      sh.fcount[0] = 1u;
    } else {
      unsigned long long k0[W];
#pragma unroll
      for (int w = 0; w < W; ++w) k0[w] = sd.k[w];
      uint32_t slot0 = sd.slot, dep0 = sd.depth;
      sh.fcount[0] = sd.slot == kParentNone ? 0u : 1u;
      if (chain_slice && pt.j0 != 0u && sh.fcount[0]) {
        // a chain slice after the first starts at clock j0 of the configuration's
        // determined part, an instant at which no workgroup ends: every unit has run
        // workgroups back to back since clock 0, so unit u is in its floor(j0/(s_u d))-th
        // workgroup; the slice before ends on the same state
        St x{};
        x.cfg = c;
        x.clock = pt.j0;
        uint32_t started = 0;
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u) {
          if (u < m) {
            const uint32_t per = unit_dur<GEN>(r, L.speed, u), w = pt.j0 / per;
            x.rem[u] = (w + 1u) * per - pt.j0;
            started += w + 1u;
          }
        }
        x.pending = r.n - started;
        dep0 = pt.j1;
        if (sh.pr && pt.j0 > sh.T) {
          sh.fcount[0] = 0u;
        } else {
          const Key<W> k = encode<W>(x, L);
#pragma unroll
          for (int w = 0; w < W; ++w) k0[w] = k.w[w];
          const int res = table_insert<W, kScopeAgent>(md.table, md.mask, k, slot0, tl.probes, md.hkeep);
          if (res == kInsFail) {
            set_error(md.ctrl, kDevErrTableFull);
            sh.fcount[0] = 0u;
          } else if (res == kInsNew) {
            ++tl.states;
            tl.depth = dep0 > tl.depth ? dep0 : tl.depth;
          }
        }
      } else if (!chain_slice && pt.r0 != 0u && sh.fcount[0]) {
        // B_r0: r0 full rounds after the configuration's SELECT state
        field_add<W>(k0, L, kFClock, (unsigned long long)pt.r0 * r.d);
        field_add<W>(k0, L, kFPending, (unsigned long long)(-(long long)pt.r0 * m));
        dep0 = sd.depth + pt.r0 * round_dep;
        if (md.prune && (unsigned long long)pt.r0 * r.d > sh.T) {
          sh.fcount[0] = 0u;
        } else {
          Key<W> k;
#pragma unroll
          for (int w = 0; w < W; ++w) k.w[w] = k0[w];
          const int res = table_insert<W, kScopeAgent>(md.table, md.mask, k, slot0, tl.probes, md.hkeep);
          if (res == kInsFail) {
            set_error(md.ctrl, kDevErrTableFull);
            sh.fcount[0] = 0u;
          } else if (res == kInsNew) {
            ++tl.states;
            tl.depth = dep0 > tl.depth ? dep0 : tl.depth;
          }
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) sh.fkey[0][0][w] = k0[w];
      sh.fslot[0][0] = slot0;
      sh.fdep[0][0] = dep0;
    }
    sh.fcount[1] = 0u;
  }
  __syncthreads();
  int cur = 0;
  uint32_t levels = 0;
  bool yielded = false;
  while (sh.fcount[cur] > 0u && !sh.stop) {
    if (slice && md.pstate && levels >= slice && sh.fcount[cur] == 1u) {
      // out of budget for this launch: save the single frontier state and yield
      if (tid == 0) {
        PartState ps;
#pragma unroll
        for (int w = 0; w < 4; ++w) ps.k[w] = w < W ? sh.fkey[cur][0][w] : 0ull;
        ps.slot = sh.fslot[cur][0];
        ps.depth = sh.fdep[cur][0];
        ps.status = 1u;
        ps.pad = 0u;
        md.pstate[pt.pidx] = ps;
        const uint32_t pos = atomicAdd(pq.n_yielded, 1u);
        pq.yielded[pos] = pt;
      }
      yielded = true;
      break;
    }
    ++levels;
    const uint32_t nf = sh.fcount[cur] < (uint32_t)kFCap ? sh.fcount[cur] : (uint32_t)kFCap;
    for (uint32_t fi = 0; fi < nf; ++fi) {
      // ---- segments of this super-step (one thread builds them) ----
      if (tid == 0) {
        // the query's threshold (with branch and bound the incumbent), capped by a chain
        // slice's end; md.T means nothing when the query does not prune
        sh.T = md.prune ? min(prune_T(md), sh.cut) : sh.cut;
        Key<W> ck;
#pragma unroll
        for (int w = 0; w < W; ++w) ck.w[w] = sh.fkey[cur][fi][w];
        uint32_t fslot = sh.fslot[cur][fi], fdep = sh.fdep[cur][fi];
        uint32_t total = 0, nseg = 0;
        sh.stop_item = kNoItem;
        sh.stop_capped = 0u;
        bool decoded = false;  // sh.seg[nseg] already derived from the previous segment
        for (;;) {
          SegDesc& sg = sh.seg[nseg];
          if (!decoded) {
            const St x = decode<W>(ck, L, md.cfgs);
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
            if (kstar == 0u && busy == 0u) break;  // terminal
#pragma unroll
            for (int w = 0; w < W; ++w) sg.fkey[w] = ck.w[w];
            sg.kstar = kstar;
            sg.freem = freem;
            sg.nfree = nfree;
            sg.nclos = kstar ? (1u << nfree) - 1u : 0u;
            uint32_t nleaf = 1;  // C(nfree, kstar)
            for (uint32_t i = 1; i <= kstar; ++i) nleaf = nleaf * (nfree - kstar + i) / i;
            sg.nleaf = nleaf;
            // units of unequal speed leave lock step at once: one ADVANCE per leaf
            const bool lock = !(HET && L.hetero) && (kstar ? (busy == 0u) : bsame);
            sg.lock = lock ? 1u : 0u;
            sg.e0 = kstar ? 0u : r.d - brem;
            sg.idx0 = lock ? ends_upto_t<GEN>(r, sg.e0) : 0u;
            sg.len = lock ? r.b - sg.idx0 : 1u;
            // runs continued by run slices stop at the partition's cap
            if (lock && pt.j1 && sg.len > pt.j1) sg.len = pt.j1;
            sg.pend = x.pending - kstar;
            sg.fclock = x.clock;
            // run keys: every unit not busy in a lock-step run is idle
            St b{};
            b.cfg = x.cfg;
            b.pending = sg.pend;
            const Key<W> bk = encode<W>(b, L);
            unsigned long long Mv[W];
#pragma unroll
            for (int w = 0; w < W; ++w) Mv[w] = 0ull;
            const uint32_t busy_run = kstar ? freem : busy;  // single leaf: all free units start
            if (L.shared_rem) {
              field_add<W>(Mv, L, kFRem + 1, 1ull);  // one time left for every busy unit
            } else {
#pragma unroll
              for (int u = 0; u < kMaxCU; ++u)
                if (u < m && ((busy_run >> u) & 1u)) field_add<W>(Mv, L, kFRem + u, 1ull);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
              sg.base[w] = bk.w[w];
              sg.M[w] = Mv[w];
            }
            sg.aux = (kstar && busy == 0u && nleaf == 1u) ? 1u : 0u;  // a full round start
            sg.pad = 0u;
            // units of unequal speed, every idle unit takes work (one leaf): the segment
            // holds the dispatch closure only and the leaf's determined steps follow as
            // a chain segment in the same super-step
            if (HET && L.hetero && !lock && kstar && nleaf == 1u) sg.len = 0u;
            if (HET && L.hetero && !lock && kstar == 0u) {
              // units of unequal speed with nothing to dispatch: the ADVANCE steps up to
              // the next state with a dispatch (or the terminal) are determined; the
              // workgroup lists them below (a chain) and sets its length
              sg.len = 0u;
              sg.pad = 1u;
            }
          }
          sg.fdep = fdep;
          sg.fslot = fslot;
          sg.start = total;
          total += sg.nclos + sg.nleaf * sg.len;
          ++nseg;
          if (HET && L.hetero && !sg.lock && sg.kstar && sg.nleaf == 1u) {
            SegDesc& nx = sh.seg[nseg];
            Key<W> lk;
#pragma unroll
            for (int w = 0; w < W; ++w) lk.w[w] = sg.fkey[w];
            St y = decode<W>(lk, L, md.cfgs);
#pragma unroll
            for (int u = 0; u < kMaxCU; ++u)
              if ((sg.freem >> u) & 1u) y.rem[u] = unit_dur<GEN>(r, L.speed, u);
            y.pending -= sg.kstar;
            const Key<W> yk = encode<W>(y, L);
#pragma unroll
            for (int w = 0; w < W; ++w) nx.fkey[w] = yk.w[w];
            nx.kstar = 0u;
            nx.freem = 0u;
            nx.nfree = 0u;
            nx.nclos = 0u;
            nx.nleaf = 1u;
            nx.lock = 0u;
            nx.aux = 0u;
            nx.pad = 1u;  // a chain: build_chain lists it and sets its length
            nx.len = 0u;
            nx.e0 = 0u;
            nx.idx0 = 0u;
            nx.pend = y.pending;
            nx.fclock = y.clock;
            nx.fdep = fdep + sg.kstar;
            nx.fslot = kParentNone;  // the leaf: its slot comes from the closure's items
            nx.start = total;
            ++nseg;
            break;
          }
          // continue with the run end: a single lock-step run ending with work pending
          const uint32_t end_clock = sg.fclock + (r.d - sg.e0);
          if (sh.has_stop) {
            // inside a block every segment is a full round, and the block ends on B_r1
            if (!sg.aux || end_clock > sh.stop_clock) {
              set_error(md.ctrl, kDevErrSplit);
              sh.stop = 1u;
              break;
            }
            if (end_clock == sh.stop_clock) {
              // the run end is B_r1: generated by the same arithmetic as every run end,
              // it must be the state r1 full rounds give, at the depth they give
              // the last run state of this segment, unless run slices hold the run's end
              const bool capped = sg.len < r.b - sg.idx0;
              sh.stop_item = capped ? kNoItem : total - 1u;
              sh.stop_capped = capped ? 1u : 0u;
              sh.stop_slot = kParentNone;
              unsigned long long ek[W];
#pragma unroll
              for (int w = 0; w < W; ++w) ek[w] = sg.base[w];
              field_add<W>(ek, L, kFClock, end_clock);
              bool ok = fdep + sg.kstar + (r.b - sg.idx0) == sh.stop_dep;
              Key<W> k;
#pragma unroll
              for (int w = 0; w < W; ++w) {
                ok = ok && ek[w] == sh.stopkey[w];
                k.w[w] = ek[w];
              }
              if (!ok) {
                set_error(md.ctrl, kDevErrSplit);
                sh.stop = 1u;
              } else if (!(sh.pr && end_clock > sh.T)) {
                // shared with the next block: agent-scope ordering
                uint32_t slot = kParentNone;
                const int res = table_insert<W, kScopeAgent>(md.table, md.mask, k, slot, tl.probes, md.hkeep);
                ++tl.edges;
                if (res == kInsFail) {
                  set_error(md.ctrl, kDevErrTableFull);
                  sh.stop = 1u;
                } else {
                  if (res == kInsNew) {
                    ++tl.states;
                    tl.depth = sh.stop_dep > tl.depth ? sh.stop_dep : tl.depth;
                  } else {
                    ++tl.dups;
                  }
                  sh.stop_slot = slot;
                  sh.handed = 1u;
                }
              }
              break;
            }
          }
          const bool more = sg.lock && sg.nleaf == 1u && sg.pend > 0u &&
                            nseg < (uint32_t)SEGS && total < batch_items &&
                            !(sh.pr && end_clock > sh.T) && end_clock <= md.max_clock;
          if (!more) break;
          // the run end: every unit idle, `pend` workgroups pending
          unsigned long long ek[W];
#pragma unroll
          for (int w = 0; w < W; ++w) ek[w] = sg.base[w];
          field_add<W>(ek, L, kFClock, end_clock);
#pragma unroll
          for (int w = 0; w < W; ++w) ck.w[w] = ek[w];
          fslot = kParentNone;  // known once the run end is claimed
          fdep = fdep + sg.kstar + sg.len;
          // a full round from an idle start followed by at least one more full round has
          // the same shape: only the clock and the pending count move
          decoded = sg.aux && sg.pend >= sg.nfree;
          if (decoded) {
            SegDesc& nx = sh.seg[nseg];
            nx = sg;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              nx.fkey[w] = ek[w];
              nx.base[w] = sg.base[w];
            }
            field_add<W>(nx.base, L, kFPending, (unsigned long long)(-(long long)sg.kstar));
            nx.pend = sg.pend - sg.kstar;
            nx.fclock = end_clock;
          }
        }
        sh.nseg = nseg;
        sh.total = total;
        sh.carry = sh.fslot[cur][fi];
      }
      __syncthreads();
      if constexpr (HET) {
        if (sh.nseg && sh.seg[sh.nseg - 1].pad) {
          for (;;) {
            build_chain<W, BLOCK, NI>(sh, r, L, m);
            __syncthreads();
            if (tid == 0) extend_chain<W, BLOCK, NI, SEGS, GEN>(sh, r, md, m, batch_items);
            __syncthreads();
            if (!sh.chain_more) break;
          }
        }
      }
      const uint32_t nseg = sh.nseg;
      const uint32_t total = sh.total;
      const uint32_t stop_item = sh.stop_item;
      // B_r1, the end of a block, is left out of the batch and inserted below
      const uint32_t n_items = stop_item == kNoItem ? total : total - 1u;
      tl.super += nseg;
      // leaf list of a segment with several leaves (a partial round); only the last
      // segment of a batch can have several
      if (nseg && sh.seg[nseg - 1].nleaf > 1u) {
        const SegDesc& sg = sh.seg[nseg - 1];
        if (tid < 64) {
          uint32_t off = 0;
          for (uint32_t g0 = 1; g0 <= sg.nclos; g0 += 64) {
            const uint32_t mk = g0 + tid;
            const bool isleaf = mk <= sg.nclos && (uint32_t)__popc(mk) == sg.kstar;
            const unsigned long long bm = __ballot(isleaf);
            if (isleaf) sh.leaf[off + lanes_below(bm)] = (uint8_t)mk;
            off += (uint32_t)__popcll(bm);
          }
        }
        __syncthreads();
      }
      if (nseg && !sh.seg[nseg - 1].lock && !sh.seg[nseg - 1].pad) {
        // one ADVANCE from every leaf of a run that is not in lock step
        const SegDesc& sg = sh.seg[nseg - 1];
        if (tid < sg.nleaf && tid < (uint32_t)kMaxLeaves) {
          const uint32_t rmask =
              sg.kstar ? (sg.nleaf == 1u ? (1u << sg.nfree) - 1u : (uint32_t)sh.leaf[tid]) : 0u;
          Key<W> fk;
#pragma unroll
          for (int w = 0; w < W; ++w) fk.w[w] = sg.fkey[w];
          St y = decode<W>(fk, L, md.cfgs);
          uint32_t t = 0;
#pragma unroll
          for (int u = 0; u < kMaxCU; ++u) {
            if ((sg.freem >> u) & 1u) {
              if ((rmask >> t) & 1u) y.rem[u] = unit_dur<GEN>(r, L.speed, u);
              ++t;
            }
          }
          y.pending -= sg.kstar;
          advance_once<GEN>(y, r, m, L.speed);
          const Key<W> yk = encode<W>(y, L);
#pragma unroll
          for (int w = 0; w < W; ++w) sh.gkey[tid][w] = yk.w[w];
          sh.gclk[tid] = y.clock;
          sh.gterm[tid] = is_terminal(y, m) ? 1u : 0u;
        }
        __syncthreads();
      }
      for (uint32_t base = 0; base < n_items; base += NI * BLOCK) {
        ++tl.chunks;
        unsigned long long keys[NI][W];
        bool act[NI];
#pragma unroll
        for (int n = 0; n < NI; ++n) {
          Item<W> x;
          gen_item<W, BLOCK, NI, true, GEN, HET, SEGS>(base + (uint32_t)n * BLOCK + tid, n_items, nseg, sh, r,
                                       e_lds, md, m, x);
          if (x.active && x.clk > md.max_clock) {
            set_error(md.ctrl, kDevErrOverflow);
            x.active = false;
          }
          act[n] = x.active;
#pragma unroll
          for (int w = 0; w < W; ++w) keys[n][w] = x.key[w];
        }
        uint32_t slot[NI];
        int res[NI];
        const uint32_t p0 = tl.probes;
        // a chain slice shares its last state with the next slice's workgroup: its
        // inserts are at device scope
        if (chain_slice)
          table_insert_n<W, kScopeAgent, NI>(md.table, md.mask, keys, act, slot, res, tl.probes,
                                              md.hkeep);
        else
          table_insert_n<W, kScopeWG, NI>(md.table, md.mask, keys, act, slot, res, tl.probes,
                                           md.hkeep);
        tl.max_probe = (tl.probes - p0) > tl.max_probe ? (tl.probes - p0) : tl.max_probe;
        bool fresh[NI], cutlink[NI];
        Item<W> it[NI];  // bookkeeping of the batch's states, recomputed without the keys
#pragma unroll
        for (int n = 0; n < NI; ++n) {
          gen_item<W, BLOCK, NI, false, GEN, HET, SEGS>(base + (uint32_t)n * BLOCK + tid, n_items, nseg, sh, r,
                                        e_lds, md, m, it[n]);
          it[n].active = act[n];
          fresh[n] = false;
          // the state a chain slice ends on gets its parent from this slice even when
          // the next slice, which knows only its key, inserted it first
          cutlink[n] = chain_slice && act[n] && res[n] == kInsDup && it[n].clk == sh.cut;
          if (it[n].active) {
            ++tl.edges;
            if (res[n] == kInsFail) {
              set_error(md.ctrl, kDevErrTableFull);
              sh.stop = 1u;
              it[n].active = false;
              slot[n] = kParentNone;
            } else if (res[n] == kInsNew) {
              fresh[n] = true;
              ++tl.states;
              tl.depth = it[n].dep > tl.depth ? it[n].dep : tl.depth;
              if (it[n].term) {
                ++tl.terms;
                atomicMin(&md.tc[c], it[n].clk);
                if (md.prune) md.ctrl->violated = 1u;
                if (md.bb) atomicMin(&md.ctrl->bound, it[n].clk);
              }
            } else {
              ++tl.dups;
            }
            const SegDesc& sg = sh.seg[it[n].sgi];
            if (it[n].is_clos) {
              sh.mslot[it[n].sgi][it[n].rmask] = slot[n];
              // the full dispatch leaf starts the chain segment that follows
              if (HET && it[n].rmask == (1u << sg.nfree) - 1u && it[n].sgi + 1u < nseg &&
                  sh.seg[it[n].sgi + 1u].pad)
                sh.segfslot[it[n].sgi + 1u] = slot[n];
            }
            else if (it[n].j + 1u == sg.len && it[n].sgi + 1u < nseg)
              sh.segfslot[it[n].sgi + 1u] = slot[n];
          }
          sh.chunk_slot[n * BLOCK + tid] = it[n].active ? slot[n] : kParentNone;
        }
        __syncthreads();
#pragma unroll
        for (int n = 0; n < NI; ++n) {
          // a continued exploration expands a state it finds again below its floor (every
          // state there was inserted before), so its walk reaches the new states past it
          const bool again = !fresh[n] && it[n].active && res[n] == kInsDup &&
                             it[n].clk < md.refloor;
          if (!fresh[n] && !cutlink[n] && !again) continue;
          const Item<W>& x = it[n];
          const SegDesc& sg = sh.seg[x.sgi];
          const uint32_t segf = x.sgi ? sh.segfslot[x.sgi] : sg.fslot;
          uint32_t par, jmp = kParentNone;
          // the interior states of a lock-step run from a dispatch leaf store no links:
          // the trace derives the leaf from such a state's key (busy units back at d).
          // On units alike the inner states of a dispatch closure store none either, and
          // a leaf links to the closure's root: a counterexample passes through one chain
          // of the closure only, which the trace regenerates (the missing units started in
          // index order).  That is one link write per closure instead of 2^k - 1.
          const uint32_t ns = (uint32_t)__popc(x.rmask);
          const bool linkless = (!x.is_clos && sg.lock && sg.kstar && x.j + 1u < sg.len) ||
                                (!HET && x.is_clos && ns < sg.kstar);
          if (x.is_clos) {
            const uint32_t pm = x.rmask & ~(1u << (31 - __clz(x.rmask)));
            par = (pm && (HET || ns < sg.kstar)) ? sh.mslot[x.sgi][pm] : segf;
          } else {
            const uint32_t leaf_slot = x.rmask ? sh.mslot[x.sgi][x.rmask] : segf;
            const uint32_t li = (uint32_t)n * BLOCK + tid;  // local index of the item
            par = x.j == 0u ? leaf_slot : (li ? sh.chunk_slot[li - 1] : sh.carry);
            // a lock-step run, or a chain of units of unequal speed, jumps to the state it
            // starts from: the trace regenerates the steps in between
            if (sg.lock || (HET && sg.pad)) jmp = leaf_slot;
          }
          if (!linkless && (fresh[n] || cutlink[n])) {
            set_links<W>(md.table, md.mask, slot[n], par, jmp);
          }
          if (!fresh[n] && !again) continue;
          if (!x.is_clos && x.j + 1u == sg.len && !x.term && x.sgi + 1u == nseg &&
              !(sg.lock && sg.idx0 + sg.len < r.b)) {  // a capped run ends in the slices
            const uint32_t pos = atomicAdd(&sh.fcount[cur ^ 1], 1u);
            if (pos < (uint32_t)kFCap) {
#pragma unroll
              for (int w = 0; w < W; ++w) sh.fkey[cur ^ 1][pos][w] = keys[n][w];
              sh.fslot[cur ^ 1][pos] = slot[n];
              sh.fdep[cur ^ 1][pos] = x.dep;
            } else {
              set_error(md.ctrl, kDevErrOverflow);
            }
          }
        }
        __syncthreads();
        if (tid == BLOCK - 1) sh.carry = sh.chunk_slot[NI * BLOCK - 1];
        __syncthreads();
      }
      if (stop_item != kNoItem && tid == 0 && sh.stop_slot != kParentNone) {
        // B_r1 (claimed by the builder) gets its parent and jump from this block even if
        // the next block inserted it first: that block knows only its key.  Its parent
        // is the run's previous state, the last item of the batch's last chunk.
        const SegDesc& sg = sh.seg[nseg - 1u];
        const uint32_t leaf_slot = sh.mslot[nseg - 1u][(1u << sg.nfree) - 1u];
        const uint32_t par =
            sg.len > 1u ? sh.chunk_slot[(stop_item - 1u) % (NI * BLOCK)] : leaf_slot;
        set_links<W>(md.table, md.mask, sh.stop_slot, par, leaf_slot);
      } else if (sh.stop_capped && tid == 0 && sh.stop_slot != kParentNone) {
        // B_r1 after a run whose later states are in run slices: the run is regenerated
        // from its dispatch leaf, which is both links
        const SegDesc& sg = sh.seg[nseg - 1u];
        const uint32_t leaf_slot = sh.mslot[nseg - 1u][(1u << sg.nfree) - 1u];
        set_links<W>(md.table, md.mask, sh.stop_slot, leaf_slot, leaf_slot);
      }
    }
    if (tid == 0) sh.fcount[cur] = 0u;
    __syncthreads();
    cur ^= 1;
  }
  if (!yielded && tid == 0) {
    // a block that did not reach B_r1 (unless pruned away or stopped by an error) would
    // leave part of the subgraph unexplored
    if (sh.has_stop && !sh.handed && !sh.stop && !(md.prune && sh.stop_clock > prune_T(md)) &&
        __hip_atomic_load(&md.ctrl->error, __ATOMIC_RELAXED, kScopeAgent) == 0u)
      set_error(md.ctrl, kDevErrSplit);
    if (md.pstate) md.pstate[pt.pidx].status = 2u;
    atomicAdd(&md.ctrl->parts_done, 1u);
  }
  flush_tally(md, tl);
}

__device__ __forceinline__ void flush_tally(const ModelDev& md, const Tally& tl) {
  flush_counters(md.ctrl, tl.states, tl.terms, tl.edges, tl.dups, tl.probes, tl.depth);
  const unsigned long long mp = wave_max(tl.max_probe);
  if (lane_id() == 0 && mp) atomicMax(&md.ctrl->max_probe, (unsigned int)mp);
  if (threadIdx.x == 0) {
    if (tl.super) atomicAdd(&md.ctrl->supersteps, tl.super);
    if (tl.chunks) atomicAdd(&md.ctrl->chunks, tl.chunks);
  }
}

// A run slice (Part::r0 = kRunSlice, Part::r1 = the round r): states j0 <= j < j1 of
// every lock-step run of round r of a configuration.  At the start of the round every
// unit is idle (clock r*d, n - r*m pending) and k = min(m, n - r*m) workgroups start on
// one of the C(m, k) choices of units, so state j of the run of choice U is
// (c, r*d + E_j, n - r*m - k, d - E_j on U, 0 elsewhere): built from j alone, no
// frontier.  Items are ordered by choice, then j.  Interior states store no links (the
// trace derives their dispatch leaf from the key); a run ending at a terminal stores its
// predecessor, inserted by the same slice; a run ending at the next round's start is
// not in a slice (the round's block claims that state).  Inserts are agent-scope like a
// block's boundary states; no state of a slice has a (pending, clock) pair that another
// partition's states have.
template <int W, int BLOCK, int NI, bool GEN, int SEGS>
__device__ void explore_slice(const ModelDev& md, const Part pt, SuperShared<BLOCK, NI, SEGS, W>& sh) {
  Tally tl;
  const Layout& L = md.L;
  const int m = L.m;
  const uint32_t tid = threadIdx.x;
  const uint32_t c = pt.cfg;
  const CfgRec r = md.cfgs[c];
  const uint32_t rd = pt.r1;  // the round
  const uint32_t left = r.n - rd * (uint32_t)m;
  const uint32_t k = left < (uint32_t)m ? left : (uint32_t)m;
  const uint32_t pend = left - k;
  if (tid == 0) sh.T = prune_T(md);
  if (tid < 64) {  // the choices of k units out of m, in increasing mask order
    uint32_t off = 0;
    for (uint32_t g0 = 1; g0 < (1u << m); g0 += 64) {
      const uint32_t mk = g0 + tid;
      const bool isleaf = mk < (1u << m) && (uint32_t)__popc(mk) == k;
      const unsigned long long bm = __ballot(isleaf);
      if (isleaf) sh.leaf[off + lanes_below(bm)] = (uint8_t)mk;
      off += (uint32_t)__popcll(bm);
    }
    if (tid == 0) sh.nseg = off;  // number of choices
  }
  __syncthreads();
  const uint32_t nleaf = sh.nseg, len = pt.j1 - pt.j0, total = nleaf * len;
  // the dispatch leaf's depth: SELECT at 1, m dispatches and b advances per round, k more
  const uint32_t fdep = 1u + rd * ((uint32_t)m + r.b) + k;
  const uint32_t clock0 = rd * r.d;
  const uint32_t T = sh.T;
  for (uint32_t base = 0; base < total; base += NI * BLOCK) {
    ++tl.chunks;
    unsigned long long keys[NI][W];
    bool act[NI], term[NI];
    uint32_t clk[NI], dep[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const uint32_t i = base + (uint32_t)q * BLOCK + tid;
      act[q] = i < total;
      term[q] = false;
      clk[q] = 0u;
      dep[q] = 0u;
#pragma unroll
      for (int w = 0; w < W; ++w) keys[q][w] = 0ull;
      if (!act[q]) continue;
      const uint32_t leaf = i / len, j = pt.j0 + (i - leaf * len);
      const uint32_t e = end_at_t<GEN>(r, j);
      const uint32_t mask = sh.leaf[leaf];
      St y{};
      y.cfg = c;
      y.clock = clock0 + e;
      y.pending = pend;
#pragma unroll
      for (int u = 0; u < kMaxCU; ++u) y.rem[u] = ((mask >> u) & 1u) ? r.d - e : 0u;
      const Key<W> yk = encode<W>(y, L);
#pragma unroll
      for (int w = 0; w < W; ++w) keys[q][w] = yk.w[w];
      clk[q] = y.clock;
      dep[q] = fdep + j + 1u;
      term[q] = pend == 0u && j + 1u == r.b;
      if (md.prune && y.clock > T) act[q] = false;
    }
    uint32_t slot[NI];
    int res[NI];
    const uint32_t p0 = tl.probes;
    table_insert_n<W, kScopeAgent, NI>(md.table, md.mask, keys, act, slot, res, tl.probes,
                                              md.hkeep);
    tl.max_probe = (tl.probes - p0) > tl.max_probe ? (tl.probes - p0) : tl.max_probe;
    bool fresh[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      fresh[q] = false;
      if (act[q]) {
        ++tl.edges;
        if (res[q] == kInsFail) {
          set_error(md.ctrl, kDevErrTableFull);
          act[q] = false;
          slot[q] = kParentNone;
        } else if (res[q] == kInsNew) {
          fresh[q] = true;
          ++tl.states;
          tl.depth = dep[q] > tl.depth ? dep[q] : tl.depth;
          if (term[q]) {
            ++tl.terms;
            atomicMin(&md.tc[c], clk[q]);
            if (md.prune) md.ctrl->violated = 1u;
            if (md.bb) atomicMin(&md.ctrl->bound, clk[q]);
          }
        } else {
          ++tl.dups;
        }
      }
      sh.chunk_slot[q * BLOCK + tid] = act[q] ? slot[q] : kParentNone;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      if (!fresh[q] || !term[q]) continue;
      const uint32_t li = (uint32_t)q * BLOCK + tid;  // the run's previous state: item i-1
      set_links<W>(md.table, md.mask, slot[q], li ? sh.chunk_slot[li - 1] : sh.carry, kParentNone);
    }
    __syncthreads();
    if (tid == BLOCK - 1) sh.carry = sh.chunk_slot[NI * BLOCK - 1];
    __syncthreads();
  }
  if (tid == 0) {
    if (md.pstate) md.pstate[pt.pidx].status = 2u;
    atomicAdd(&md.ctrl->parts_done, 1u);
  }
  flush_tally(md, tl);
}

// The unequal-speed build at 512 threads asks for four waves per SIMD (at most 128 VGPRs):
// with its LDS under half a CU's, two workgroups then share a CU, and a partition's
// serial sections (listing a chain, the super-step's barriers) overlap another's.
template <int W, int BLOCK, int NI, bool GEN, bool HET>
__global__ __launch_bounds__(BLOCK, (HET && BLOCK == 512) ? 4 : 1) void k_superstep(PartQueue a) {
  __shared__ SuperShared<BLOCK, NI, HET ? kSegMaxChain : kSegMax, W> sh;
  const uint32_t tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      sh.part = atomicAdd(a.head, 1u);
      sh.stop = 0u;
    }
    __syncthreads();
    const uint32_t part = sh.part;
    if (part >= a.n_parts) break;
    const Part pc = a.parts[a.reverse ? a.n_parts - 1u - part : part];
    if (tid == 0) {
      sh.md = a.models[pc.model];
      // one read of the model's error flag for the whole workgroup: other workgroups set
      // it concurrently, and every wave must take the same branch around the barriers
      // of the exploration
      bool stop = __hip_atomic_load(&sh.md.ctrl->error, __ATOMIC_RELAXED, kScopeAgent) != 0u;
      if (!stop && a.abort && __hip_atomic_load(a.abort, __ATOMIC_RELAXED, kScopeSystem) != 0u) {
        set_error(sh.md.ctrl, kDevErrAbort);
        stop = true;
      }
      sh.skip = stop ? 1u : 0u;
    }
    __syncthreads();
    const ModelDev& md = sh.md;
    const bool skip = sh.skip != 0u;
    const unsigned long long t_part = __builtin_amdgcn_s_memrealtime();
    if (!skip && pc.r0 == kRunSlice) explore_slice<W, BLOCK, NI, GEN>(md, pc, sh);
    else if (!skip) explore_partition<W, BLOCK, NI, GEN, HET>(md, pc, a.batch_items, a.slice, a, sh);
    if (tid == 0) {
      const unsigned long long dt = __builtin_amdgcn_s_memrealtime() - t_part;
      const unsigned long long prev = atomicMax(&md.ctrl->crit_ticks, dt);
      if (dt > prev) md.ctrl->crit_part = pc.cfg;
    }
    __syncthreads();
  }
}

// k_superstep instances: built in the part of their key width only
template <int W, bool GEN, bool HET>
void launch_super_w(hipStream_t st, uint32_t grid, uint32_t block, uint32_t items,
                    const PartQueue& pq);

#if MC_PART != 0
template <int W, bool GEN, bool HET>
void launch_super_w(hipStream_t st, uint32_t grid, uint32_t block, uint32_t items,
                    const PartQueue& pq) {
#define MC_LAUNCH_SUPER(B, N) \
  hipLaunchKernelGGL((k_superstep<W, B, N, GEN, HET>), dim3(grid), dim3(B), 0, st, pq)
  if (block == 256) {
    if (items >= 2) MC_LAUNCH_SUPER(256, 2);
    else MC_LAUNCH_SUPER(256, 1);
  } else if (block == 1024) {
    if (items >= 2) MC_LAUNCH_SUPER(1024, 2);
    else MC_LAUNCH_SUPER(1024, 1);
  } else {
    if (items >= 2) MC_LAUNCH_SUPER(512, 2);
    else MC_LAUNCH_SUPER(512, 1);
  }
#undef MC_LAUNCH_SUPER
}
template void launch_super_w<MC_PART, false, false>(hipStream_t, uint32_t, uint32_t, uint32_t,
                                                    const PartQueue&);
template void launch_super_w<MC_PART, true, false>(hipStream_t, uint32_t, uint32_t, uint32_t,
                                                   const PartQueue&);
template void launch_super_w<MC_PART, true, true>(hipStream_t, uint32_t, uint32_t, uint32_t,
                                                  const PartQueue&);
#else
#define MC_EXTERN_SUPER(W)                                                                   \
  extern template void launch_super_w<W, false, false>(hipStream_t, uint32_t, uint32_t,     \
                                                       uint32_t, const PartQueue&);          \
  extern template void launch_super_w<W, true, false>(hipStream_t, uint32_t, uint32_t,      \
                                                      uint32_t, const PartQueue&);           \
  extern template void launch_super_w<W, true, true>(hipStream_t, uint32_t, uint32_t,       \
                                                     uint32_t, const PartQueue&);
MC_EXTERN_SUPER(1)
MC_EXTERN_SUPER(2)
MC_EXTERN_SUPER(4)
#undef MC_EXTERN_SUPER

// Root and SELECT successors of every model of a queue, one workgroup per model.
template <int W>
__device__ void seed_model(const ModelDev& md) {
  __shared__ uint32_t s_root;
  uint32_t probes = 0;
  if (threadIdx.x == 0) {
    St r{};
    r.cfg = md.n_cfg;
    const Key<W> k = encode<W>(r, md.L);
    uint32_t slot = kParentNone;
    const int res = table_insert<W, kScopeAgent>(md.table, md.mask, k, slot, probes, md.hkeep);
    if (res != kInsNew) set_error(md.ctrl, kDevErrTableFull);
    else set_links<W>(md.table, md.mask, slot, kParentRoot, kParentNone);
    s_root = slot;
    md.ctrl->root_slot = slot;
    md.ctrl->max_depth = 1;
    atomicAdd(&md.ctrl->states, 1ull + md.n_cfg);
    atomicAdd(&md.ctrl->edges, (unsigned long long)md.n_cfg);
  }
  __syncthreads();
  for (uint32_t c = threadIdx.x; c < md.n_cfg; c += blockDim.x) {
    St s{};
    s.cfg = c;
    s.pending = md.cfgs[c].n;
    const Key<W> k = encode<W>(s, md.L);
    uint32_t slot = kParentNone;
    const int res = table_insert<W, kScopeAgent>(md.table, md.mask, k, slot, probes, md.hkeep);
    if (res != kInsNew) {
      set_error(md.ctrl, kDevErrTableFull);
      slot = kParentNone;
    } else {
      set_links<W>(md.table, md.mask, slot, s_root, kParentNone);
    }
    Seed sd;
#pragma unroll
    for (int j = 0; j < 4; ++j) sd.k[j] = j < W ? k.w[j] : 0ull;
    sd.slot = slot;
    sd.depth = 1;
    sd.pad[0] = sd.pad[1] = 0;
    md.seeds[c] = sd;
  }
  const unsigned long long p = wave_sum(probes);
  if (lane_id() == 0 && p) atomicAdd(&md.ctrl->probes, p);
}

__global__ __launch_bounds__(256) void k_seed_models(const ModelDev* models) {
  const ModelDev md = models[blockIdx.x];
  switch (md.L.W) {
    case 1: seed_model<1>(md); break;
    case 2: seed_model<2>(md); break;
    default: seed_model<4>(md); break;
  }
}

// Per-model counters and clocks of every model of a queue, and the queue heads.
__global__ void k_reset_models(const ModelDev* models, unsigned int* head, uint32_t n_heads) {
  const ModelDev md = models[blockIdx.x];
  unsigned int* cw = reinterpret_cast<unsigned int*>(md.ctrl);
  constexpr uint32_t kBoundWord = offsetof(Ctrl, bound) / 4;
  for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x)
    cw[i] = i == kBoundWord ? md.T : 0u;
  for (uint32_t i = threadIdx.x; i < md.n_cfg; i += blockDim.x) md.tc[i] = kNoClock;
  if (md.pstate)
    for (uint32_t i = threadIdx.x; i < md.n_parts; i += blockDim.x) md.pstate[i].status = 0u;
  if (blockIdx.x == 0 && head)
    for (uint32_t i = threadIdx.x; i < n_heads; i += blockDim.x) head[i] = 0u;
}

// Prepares models whose exploration continues past an earlier threshold on the same
// visited set: counters and clocks are kept (states, terminals and least clocks
// accumulate across the explorations), the partition bookkeeping and the incumbent
// start again.
__global__ void k_resume_models(const ModelDev* models, unsigned int* head, uint32_t n_heads) {
  const ModelDev md = models[blockIdx.x];
  if (threadIdx.x == 0) {
    md.ctrl->parts_done = 0u;
    md.ctrl->bound = md.T;
    md.ctrl->violated = 0u;
    md.ctrl->queue_head = 0u;
  }
  if (md.pstate)
    for (uint32_t i = threadIdx.x; i < md.n_parts; i += blockDim.x) md.pstate[i].status = 0u;
  if (blockIdx.x == 0 && head)
    for (uint32_t i = threadIdx.x; i < n_heads; i += blockDim.x) head[i] = 0u;
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

hipError_t launch_super(hipStream_t st, uint32_t W, uint32_t grid, uint32_t block,
                        uint32_t items, const PartQueue& pq, bool general, bool hetero) {
  items = lane_items_for(items, W);
  if (hetero) {
    if (W == 1) launch_super_w<1, true, true>(st, grid, block, items, pq);
    else if (W == 2) launch_super_w<2, true, true>(st, grid, block, items, pq);
    else launch_super_w<4, true, true>(st, grid, block, items, pq);
  } else if (general) {
    if (W == 1) launch_super_w<1, true, false>(st, grid, block, items, pq);
    else if (W == 2) launch_super_w<2, true, false>(st, grid, block, items, pq);
    else launch_super_w<4, true, false>(st, grid, block, items, pq);
  } else {
    if (W == 1) launch_super_w<1, false, false>(st, grid, block, items, pq);
    else if (W == 2) launch_super_w<2, false, false>(st, grid, block, items, pq);
    else launch_super_w<4, false, false>(st, grid, block, items, pq);
  }
  return hipGetLastError();
}

hipError_t launch_super_fork(hipStream_t main, Fork& f, const PartQueue (&queue)[3],
                             const uint32_t (&grid)[3], uint32_t block, uint32_t items,
                             bool general, bool hetero) {
  static const uint32_t widths[3] = {1, 2, 4};
  int used = 0, last = -1;
  for (int w = 0; w < 3; ++w)
    if (queue[w].n_parts) {
      ++used;
      last = w;
    }
  if (used == 0) return hipSuccess;
  if (used == 1)  // no fork needed
    return launch_super(main, widths[last], grid[last], block, items, queue[last], general,
                        hetero);
  hipError_t e = hipEventRecord(f.fork, main);
  for (int w = 0; w < 3 && e == hipSuccess; ++w) {
    if (!queue[w].n_parts) continue;
    e = hipStreamWaitEvent(f.sub[w], f.fork, 0);
    if (e == hipSuccess)
      e = launch_super(f.sub[w], widths[w], grid[w], block, items, queue[w], general, hetero);
    if (e == hipSuccess) e = hipEventRecord(f.join[w], f.sub[w]);
    if (e == hipSuccess) e = hipStreamWaitEvent(main, f.join[w], 0);
  }
  return e;
}

hipError_t launch_seed_models(hipStream_t st, const ModelDev* models, uint32_t n) {
  hipLaunchKernelGGL(k_seed_models, dim3(n), dim3(256), 0, st, models);
  return hipGetLastError();
}

hipError_t launch_reset_models(hipStream_t st, const ModelDev* models, uint32_t n,
                               unsigned int* head, uint32_t n_heads) {
  hipLaunchKernelGGL(k_reset_models, dim3(n), dim3(256), 0, st, models, head, n_heads);
  return hipGetLastError();
}

hipError_t launch_resume_models(hipStream_t st, const ModelDev* models, uint32_t n,
                                unsigned int* head, uint32_t n_heads) {
  hipLaunchKernelGGL(k_resume_models, dim3(n), dim3(256), 0, st, models, head, n_heads);
  return hipGetLastError();
}

#define MC_INSTANTIATE(W)                                                                  \
  template hipError_t launch_seed<W>(hipStream_t, const QueryArgs&, Seed*, void*);         \
  template hipError_t launch_level<W>(hipStream_t, uint32_t, const LevelArgs&, const void*, \
                                      void*);
MC_INSTANTIATE(1)
MC_INSTANTIATE(2)
MC_INSTANTIATE(4)

hipError_t launch_clear(hipStream_t st, void* p, unsigned long long bytes) {
  // about two 16-byte stores per thread, at most 2^18 workgroups: a 4 GiB fill ran at
  // 6.3 TB/s with 2^18 workgroups against 5.2 TB/s with 2^13
  const unsigned long long n16 = bytes / 16;
  unsigned long long grid = (n16 + 511) / 512;
  if (grid > (1ull << 18)) grid = 1ull << 18;
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

#endif  // MC_PART == 0

}  // namespace mc
