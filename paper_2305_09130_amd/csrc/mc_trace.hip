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
template <int W>
__global__ __launch_bounds__(64) void k_chase(QueryArgs a, unsigned long long* out, uint32_t cap) {
  if (blockIdx.x != 0) return;
  const uint32_t lane = threadIdx.x;
  const Layout& L = a.L;
  const int m = L.m;
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
      for (int u = 0; u < m; ++u) rem = xs.rem[u] ? xs.rem[u] : rem;
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
      for (int u = 0; u < m; ++u)
        if (x.rem[u]) {
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
          for (int u = 0; u < m; ++u)
            if (root.rem[u] == 0u && x.rem[u] != 0u) dmask |= 1u << u;
          if ((uint32_t)__popc(dmask) != gap + 1u) {
            bad = true;
            break;
          }
          if (lane == 0) {
            // terminal-first: the state with the first gap units started comes first
            for (uint32_t i = gap; i >= 1u; --i) {
              St y = root;
              uint32_t left = i;
              for (int u = 0; u < m && left; ++u)
                if ((dmask >> u) & 1u) {
                  y.rem[u] = x.rem[u];
                  --left;
                }
              y.pending = root.pending - i;
              const Key<W> yk = encode<W>(y, L);
#pragma unroll
              for (int w = 0; w < W; ++w) out[(unsigned long long)(n + gap - i) * W + w] = yk.w[w];
            }
          }
          n += gap;
        }
      }
      s = par;
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
    for (int u = 0; u < m; ++u)
      if (leaf.rem[u]) {
        busy |= 1u << u;
        lrem = leaf.rem[u];
      }
    uint32_t xrem = 0;
    for (int u = 0; u < m; ++u)
      if ((busy >> u) & 1u) xrem = x.rem[u];
    const uint32_t e0 = r.d - lrem, ex = r.d - xrem;
    const uint32_t idx0 = ends_upto(r, e0);
    const uint32_t cnt = ends_upto(r, ex) - idx0;  // run states from the leaf's successor to x
    if (n + cnt > cap || cnt == 0u) {
      bad = true;
      break;
    }
    for (uint32_t t0 = 0; t0 < cnt; t0 += 64) {
      const uint32_t t = t0 + lane;
      if (t < cnt) {
        const uint32_t pos = cnt - 1u - t;  // terminal-first order
        const uint32_t e = end_at(r, idx0 + pos);
        St y = leaf;
        y.clock = leaf.clock + (e - e0);
        for (int u = 0; u < m; ++u)
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
  hipLaunchKernelGGL((k_chase<W>), dim3(1), dim3(64), 0, st, q, out, cap);
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
