// mc_trace.hip -- reading a visited set after an exploration.
//
//   k_find / k_chase   counterexample: locate the terminal, follow parent slots back to
//                      the root, regenerating the runs and closures that store no links
//   k_count_le         states of a visited set up to a clock (queries answered from it)
#include <hip/hip_runtime.h>

#include "mc_launch.h"

namespace mc {

// States of a visited set with clock <= T (the root included), summed into *out: the
// count of a check(T) answered from a set that holds every state up to a larger T
// (between the launches of an exploration that continues past that T: the states it
// adds all have larger clocks).
template <int W>
__global__ __launch_bounds__(256) void k_count_le(const unsigned char* __restrict__ table,
                                                  unsigned long long slots, Layout L,
                                                  const CfgRec* cfgs, uint32_t T,
                                                  unsigned long long* out) {
  unsigned long long n = 0;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long s = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
       s += stride) {
    const unsigned long long* w = reinterpret_cast<const unsigned long long*>(
        table + s * (8ull * W));
    Key<W> k;
    bool ready = true;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      k.w[j] = w[j];
      ready &= k.w[j] != ~0ull;
    }
    if (!ready) continue;  // an empty slot (or a key whose words are not all written)
    if (decode<W>(k, L, cfgs).clock <= T) ++n;
  }
  n = wave_sum(n);
  if (lane_id() == 0 && n) atomicAdd(out, n);
}

// ---- counterexample -----------------------------------------------------------------

template <int W>
__global__ void k_find(QueryArgs a, Key<W> k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) a.ctrl->target_slot = table_find<W>(a.table, a.mask, k, a.hkeep);
}

// Follows parent slots from the target to the root, writing keys terminal-first.  The
// end of a lock-step run carries a jump to the run's first predecessor (the leaf), and
// an interior state of a run from a dispatch leaf carries no link at all: its leaf is
// the same state with every busy unit back at d and the clock of the run's start, found
// by a lookup (on units alike every state inside a run is taken this way, told from its
// key).  The run's states are regenerated lane-parallel from the leaf (operation end
// E[i0+j] on every busy unit) instead of being chased one parent at a time.  On units
// alike a dispatch leaf links to its closure's root, the inner closure states storing no
// links: the states between the two are listed by starting the leaf's extra units one at
// a time in index order.
constexpr int kChaseCand = 1024;  // candidate ends of one chain the trace merges
constexpr uint32_t kChaseBlock = 256;  // threads of the trace kernel (four wavefronts)

// The states of a chain of units of unequal speed from f (excluded) to x (included): the
// distinct operation ends of f's busy units up to x's clock, each a state with the same
// pending count.  Merged block-wide like the exploration lists chains: thread i takes
// candidate end i (unit u's k-th end after f), which counts where no unit of lower index
// ends at the same time; its rank among the distinct times is the sum over units of the
// counted ends before it, from an exclusive prefix sum of the counted flags.  Operation
// ends come from the configuration record (end_at, ends_upto), as in the exploration.  The
// states go out terminal-first at out[n..n+cnt).  Returns cnt, or 0 when the chain has
// more candidate ends than S holds flags for (the caller follows the parent links
// instead); sets bad when the merge does not end on x or passes cap.
template <int W>
__device__ __forceinline__ uint32_t chase_chain(const St& f, const St& x, const Key<W>& xk,
                                                const CfgRec& r, const Layout& L, int m,
                                                uint32_t* S, unsigned long long* out, uint32_t n,
                                                uint32_t cap, bool& bad) {
  const uint32_t lane = threadIdx.x;
  uint32_t base[kMaxCU], sp[kMaxCU], k0[kMaxCU], nu[kMaxCU], O[kMaxCU + 1];
  uint32_t C = 0;
#pragma unroll
  for (int u = 0; u < kMaxCU; ++u) {
    base[u] = 0u;
    sp[u] = 1u;
    k0[u] = 0u;
    nu[u] = 0u;
    O[u] = C;
    if (u < m && f.rem[u]) {
      sp[u] = L.speed[u];
      // elapsed e < sp*d; the ends after f are sp*E[k] > e, i.e. E[k] > floor(e / sp)
      // (E: the configuration's operation ends)
      const uint32_t e = sp[u] * r.d - f.rem[u];
      base[u] = f.clock - e;  // the workgroup's start on unit u
      k0[u] = ends_upto(r, e / sp[u]);
      const uint32_t hi = ends_upto(r, (x.clock - base[u]) / sp[u]);
      nu[u] = hi > k0[u] ? hi - k0[u] : 0u;
    }
    C += nu[u];
  }
  O[kMaxCU] = C;
  if (C == 0u || C > (uint32_t)kChaseCand) return 0u;
  // candidate i: its unit u (the last whose first candidate index is at most i) and its
  // time; every per-unit array is read at compile-time indices, so it stays in registers
#define MC_CHASE_CAND(i, u, tau)                                  \
  do {                                                            \
    u = 0;                                                        \
    uint32_t bu_ = base[0], su_ = sp[0], ku_ = k0[0], ou_ = O[0]; \
    _Pragma("unroll") for (int j_ = 1; j_ < kMaxCU; ++j_) {       \
      if ((i) >= O[j_]) {                                         \
        u = j_;                                                   \
        bu_ = base[j_];                                           \
        su_ = sp[j_];                                             \
        ku_ = k0[j_];                                             \
        ou_ = O[j_];                                              \
      }                                                           \
    }                                                             \
    tau = bu_ + su_ * end_at(r, ku_ + ((i) - ou_));               \
  } while (0)
  // counted flags: a time counts on the lowest unit that ends at it
  for (uint32_t i = lane; i < C; i += kChaseBlock) {
    int u;
    uint32_t tau;
    MC_CHASE_CAND(i, u, tau);
    bool first = true;
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j) {
      if (j >= u || !nu[j] || tau < base[j] || (tau - base[j]) % sp[j]) continue;
      const uint32_t xj = (tau - base[j]) / sp[j];
      const uint32_t idx = ends_upto(r, xj);
      if (idx > k0[j] && end_at(r, idx - 1u) == xj) first = false;
    }
    S[i] = first ? 1u : 0u;
  }
  __syncthreads();
  __shared__ uint32_t on_x;  // some thread listed x as the chain's last state
  {  // exclusive prefix sum of the flags in place, by the first wavefront; S[C] = their total
    const bool scan = lane < 64u;
    const uint32_t per = (C + 63u) / 64u, lo = scan ? lane * per : 0u;
    const uint32_t hi = scan ? (lo + per < C ? lo + per : C) : 0u;
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i) sum += S[i];
    uint32_t incl = sum;
    if (scan) {
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if ((int)lane >= off) incl += y;
      }
    }
    __syncthreads();
    uint32_t run = incl - sum;
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t v = S[i];
      S[i] = run;
      run += v;
    }
    if (lane == 63u) S[C] = incl;
    if (lane == 0u) on_x = 0u;
  }
  __syncthreads();
  const uint32_t cnt = S[C];
  if (cnt == 0u || n + cnt > cap) {
    bad = true;
    return 0u;
  }
  for (uint32_t i = lane; i < C; i += kChaseBlock) {
    if (S[i + 1u] == S[i]) continue;  // not counted
    int u;
    uint32_t tau;
    MC_CHASE_CAND(i, u, tau);
    uint32_t rank = 0;
#pragma unroll
    for (int j = 0; j < kMaxCU; ++j) {
      if (!nu[j]) continue;
      // unit j's ends before tau: E[k] <= floor((tau - 1 - base_j) / sp_j)
      const uint32_t lt = ends_upto(r, (tau - 1u - base[j]) / sp[j]);
      uint32_t c = lt > k0[j] ? lt - k0[j] : 0u;
      c = c < nu[j] ? c : nu[j];
      rank += S[O[j] + c] - S[O[j]];
    }
    St y = f;
    y.clock = tau;
#pragma unroll
    for (int v = 0; v < kMaxCU; ++v) {
      if (v >= m) continue;
      const uint32_t wend = f.rem[v] ? base[v] + sp[v] * r.d : 0u;
      y.rem[v] = wend > tau ? wend - tau : 0u;
    }
    const Key<W> yk = encode<W>(y, L);
#pragma unroll
    for (int w = 0; w < W; ++w) out[(unsigned long long)(n + cnt - 1u - rank) * W + w] = yk.w[w];
    if (rank + 1u == cnt) {
      bool same = true;
#pragma unroll
      for (int w = 0; w < W; ++w) same = same && yk.w[w] == xk.w[w];
      if (same) on_x = 1u;
    }
  }
  __syncthreads();
  if (!on_x) bad = true;
  __syncthreads();  // S and on_x are the next chain's
  return cnt;
#undef MC_CHASE_CAND
}

template <int W>
__global__ __launch_bounds__(kChaseBlock) void k_chase(QueryArgs a, unsigned long long* out,
                                                     uint32_t cap) {
  if (blockIdx.x != 0) return;
  const uint32_t lane = threadIdx.x;
  const Layout& L = a.L;
  const int m = L.m;
  __shared__ uint32_t sS[kChaseCand + 1];  // a chain's counted flags and their prefix sums
  uint32_t s = a.ctrl->target_slot;
  uint32_t n = 0;
  bool bad = false;
  while (s != kParentRoot) {
    if (s == kParentNone || (unsigned long long)s > a.mask || n >= cap) {
      bad = true;
      break;
    }
    const unsigned long long* p = slot_key<W>(a.table, s);
    Key<W> k;
#pragma unroll
    for (int w = 0; w < W; ++w) k.w[w] = p[w];
    // on units alike a state with busy units short of d is inside a lock-step run: its
    // links, if it stored any, are not read (the link region is not cleared there)
    // (and one whose busy units are all at d may be a dispatch leaf linked to the root of
    // its closure)
    bool inside_run = false, leaf_like = false;
    if (L.shared_rem) {
      const St xs = decode<W>(k, L, a.cfgs);
      uint32_t rem = 0;
#pragma unroll
      for (int u = 0; u < kMaxCU; ++u) rem = (u < m && xs.rem[u]) ? xs.rem[u] : rem;
      const uint32_t d = (rem != 0u && xs.cfg < a.n_cfg) ? a.cfgs[xs.cfg].d : 0u;
      inside_run = rem != 0u && rem < d;
      leaf_like = rem != 0u && rem == d;
    }
    const uint32_t par = inside_run ? kParentNone : *slot_parent<W>(a.table, a.mask, s);
    uint32_t jmp = inside_run ? kParentNone : *slot_jump<W>(a.table, a.mask, s);
    if (par == kParentNone && jmp == kParentNone) {
      // an interior state of a lock-step run from a dispatch leaf (it stores no links):
      // the leaf has the same busy units, each at d, and the clock of the run's start
      const St x = decode<W>(k, L, a.cfgs);
      const CfgRec r = a.cfgs[x.cfg];
      St leaf = x;
      uint32_t rem = 0;
#pragma unroll
      for (int u = 0; u < kMaxCU; ++u)
        if (u < m && x.rem[u]) {
          rem = x.rem[u];
          leaf.rem[u] = r.d;
        }
      leaf.clock = x.clock - (r.d - rem);
      jmp = rem ? table_find<W>(a.table, a.mask, encode<W>(leaf, L), a.hkeep) : kParentNone;
      if (jmp == kParentNone) {
        bad = true;
        break;
      }
    }
    if (jmp == kParentNone || (unsigned long long)jmp > a.mask) {
      if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) out[(unsigned long long)n * W + w] = k.w[w];
      }
      ++n;
      if (leaf_like && par != kParentRoot && par != kParentNone &&
          (unsigned long long)par <= a.mask) {
        // a dispatch leaf linked to its closure's root (the closure's inner states store
        // no links): the states between them start the missing units one at a time, in
        // index order, at the root's clock
        const unsigned long long* pp = slot_key<W>(a.table, par);
        Key<W> pk;
#pragma unroll
        for (int w = 0; w < W; ++w) pk.w[w] = pp[w];
        const St root = decode<W>(pk, L, a.cfgs);
        const St x = decode<W>(k, L, a.cfgs);
        if (root.cfg == x.cfg && root.clock == x.clock && root.pending > x.pending + 1u) {
          const uint32_t gap = root.pending - x.pending - 1u;  // inner states to list
          if (n + gap > cap) {
            bad = true;
            break;
          }
          uint32_t dmask = 0;  // units the closure started
#pragma unroll
          for (int u = 0; u < kMaxCU; ++u)
            if (u < m && root.rem[u] == 0u && x.rem[u] != 0u) dmask |= 1u << u;
          if ((uint32_t)__popc(dmask) != gap + 1u) {
            bad = true;
            break;
          }
          // terminal-first: lane l lists the state with the first gap - l units started
          // (gap < m <= 8 states, one per lane)
          if (lane < gap) {
            const uint32_t i = gap - lane;
            St y = root;
            uint32_t left = i;
#pragma unroll
            for (int u = 0; u < kMaxCU; ++u)
              if (u < m && left && ((dmask >> u) & 1u)) {
                y.rem[u] = x.rem[u];
                --left;
              }
            y.pending = root.pending - i;
            const Key<W> yk = encode<W>(y, L);
#pragma unroll
            for (int w = 0; w < W; ++w) out[(unsigned long long)(n + lane) * W + w] = yk.w[w];
          }
          n += gap;
        }
      }
      s = par;
      continue;
    }
    if (!L.shared_rem) {
      // a chain of units of unequal speed: regenerated from the state it starts from
      const unsigned long long* fp = slot_key<W>(a.table, jmp);
      Key<W> fk;
#pragma unroll
      for (int w = 0; w < W; ++w) fk.w[w] = fp[w];
      const St f = decode<W>(fk, L, a.cfgs);
      const St x = decode<W>(k, L, a.cfgs);
      if (f.cfg != x.cfg || f.cfg >= a.n_cfg || f.pending != x.pending || f.clock >= x.clock) {
        bad = true;
        break;
      }
      const CfgRec r = a.cfgs[f.cfg];
      const uint32_t cnt = chase_chain<W>(f, x, k, r, L, m, sS, out, n, cap, bad);
      if (bad) break;
      if (cnt == 0u) {  // more candidates than flags: the parent link instead
        if (lane == 0) {
#pragma unroll
          for (int w = 0; w < W; ++w) out[(unsigned long long)n * W + w] = k.w[w];
        }
        ++n;
        s = par;
        continue;
      }
      n += cnt;
      s = jmp;
      continue;
    }
    // regenerate the run leaf -> s
    const unsigned long long* lp = slot_key<W>(a.table, jmp);
    Key<W> lk;
#pragma unroll
    for (int w = 0; w < W; ++w) lk.w[w] = lp[w];
    const St leaf = decode<W>(lk, L, a.cfgs);
    const St x = decode<W>(k, L, a.cfgs);
    const CfgRec r = a.cfgs[leaf.cfg];
    uint32_t busy = 0, lrem = 0;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u)
      if (u < m && leaf.rem[u]) {
        busy |= 1u << u;
        lrem = leaf.rem[u];
      }
    uint32_t xrem = 0;
#pragma unroll
    for (int u = 0; u < kMaxCU; ++u)
      if ((busy >> u) & 1u) xrem = x.rem[u];
    const uint32_t e0 = r.d - lrem, ex = r.d - xrem;
    const uint32_t idx0 = ends_upto(r, e0);
    const uint32_t cnt = ends_upto(r, ex) - idx0;  // run states from the leaf's successor to x
    if (n + cnt > cap || cnt == 0u) {
      bad = true;
      break;
    }
    for (uint32_t t0 = 0; t0 < cnt; t0 += kChaseBlock) {
      const uint32_t t = t0 + lane;
      if (t < cnt) {
        const uint32_t pos = cnt - 1u - t;  // terminal-first order
        const uint32_t e = end_at(r, idx0 + pos);
        St y = leaf;
        y.clock = leaf.clock + (e - e0);
#pragma unroll
        for (int u = 0; u < kMaxCU; ++u)
          if ((busy >> u) & 1u) y.rem[u] = r.d - e;
        const Key<W> yk = encode<W>(y, L);
#pragma unroll
        for (int w = 0; w < W; ++w) out[(unsigned long long)(n + t) * W + w] = yk.w[w];
      }
    }
    n += cnt;
    s = jmp;
  }
  if (lane == 0) {
    if (bad) set_error(a.ctrl, kDevErrTrace);
    a.ctrl->trace_len = n;
  }
}

// ---- launch helpers (host) ------------------------------------------------------------

template <int W>
hipError_t launch_find(hipStream_t st, const QueryArgs& q, const unsigned long long* key) {
  Key<W> k;
  for (int w = 0; w < W; ++w) k.w[w] = key[w];
  hipLaunchKernelGGL((k_find<W>), dim3(1), dim3(64), 0, st, q, k);
  return hipGetLastError();
}

template <int W>
hipError_t launch_chase(hipStream_t st, const QueryArgs& q, unsigned long long* out, uint32_t cap) {
  hipLaunchKernelGGL((k_chase<W>), dim3(1), dim3(kChaseBlock), 0, st, q, out, cap);
  return hipGetLastError();
}

template <int W>
hipError_t launch_count_le(hipStream_t st, const unsigned char* table, unsigned long long slots,
                           const Layout& L, const CfgRec* cfgs, uint32_t T,
                           unsigned long long* out) {
  unsigned long long grid = (slots + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL((k_count_le<W>), dim3((uint32_t)grid), dim3(256), 0, st, table, slots, L,
                     cfgs, T, out);
  return hipGetLastError();
}

#define MC_INSTANTIATE(W)                                                                  \
  template hipError_t launch_count_le<W>(hipStream_t, const unsigned char*,                \
                                         unsigned long long, const Layout&, const CfgRec*,  \
                                         uint32_t, unsigned long long*);                    \
  template hipError_t launch_find<W>(hipStream_t, const QueryArgs&,                       \
                                     const unsigned long long*);                           \
  template hipError_t launch_chase<W>(hipStream_t, const QueryArgs&, unsigned long long*,  \
                                      uint32_t);
MC_INSTANTIATE(1)
MC_INSTANTIATE(2)
MC_INSTANTIATE(4)
#undef MC_INSTANTIATE

}  // namespace mc
