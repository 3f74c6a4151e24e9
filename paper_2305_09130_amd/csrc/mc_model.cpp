// mc_model.cpp -- descriptor validation, per-configuration tables, key layout and the
// exact state counts used to size the device workspace.
//
// Counts.  Workgroups of one configuration all last d and dispatch is eager (no time
// passes while a free unit could take pending work), so every run proceeds in rounds:
// all units idle, min(pending, m) of them started in any order, a lock-step run
// through the b operation ends, all idle again.  With q = n div m full rounds and
// p = n mod m left over, one configuration's subgraph has
//     1 + q(2^m - 1 + b) + [p > 0](sum_{j=1..p} C(m, j) + C(m, p)(b - 1) + 1)
// states, its terminals all have clock ceil(n/m) d, and every path to its terminal has
// 1 + n + ceil(n/m) b edges.  These sizes bound the visited set, the frontiers and the
// trace buffer; the exploration itself does not use them.
#include "mc_model.h"

#include <algorithm>
#include <cstring>

namespace mc {

uint64_t binom(uint32_t n, uint32_t k) {
  if (k > n) return 0;
  uint64_t r = 1;
  for (uint32_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

uint32_t bit_length(uint64_t x) {
  uint32_t b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

static bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

static int fail(std::string* err, const std::string& msg) {
  if (err) *err = msg;
  return MC_E_INVAL;
}

// Operation phases of configuration c: (count, latency) in execution order.
static int phases(const mc_desc* d, const uint32_t* p, uint64_t* n, uint64_t cnt[4],
                  uint64_t lat[4], std::string* err) {
  if (d->kind == MC_KIND_REDUCTION) {
    const uint64_t G = d->size[0], WG = p[0], TS = p[1];
    if (!pow2(G) || !pow2(WG) || !pow2(TS)) return fail(err, "reduction sizes must be powers of two");
    if (WG > G) return fail(err, "WG larger than G");
    *n = G / WG;
    cnt[0] = (G + WG * TS - 1) / (WG * TS); lat[0] = d->lat_global;
    cnt[1] = bit_length(WG) - 1;            lat[1] = d->lat_local;
    cnt[2] = 1;                             lat[2] = d->lat_barrier;
    cnt[3] = TS;                            lat[3] = d->lat_compute;
    return MC_OK;
  }
  if (d->kind == MC_KIND_MATMUL) {
    const uint64_t M = d->size[0], N = d->size[1], K = d->size[2];
    const uint64_t X = p[0], Y = p[1], TS = p[2], VW = p[3] ? p[3] : 1;
    if (!pow2(M) || !pow2(N) || !pow2(K) || !pow2(X) || !pow2(Y) || !pow2(TS) || !pow2(VW))
      return fail(err, "matmul sizes must be powers of two");
    if (X > M || Y * VW > N || TS > K) return fail(err, "matmul tile larger than the matrix");
    *n = (M / X) * (N / (Y * VW));
    cnt[0] = 2 * K;          lat[0] = d->lat_global;
    cnt[1] = K * (1 + VW);   lat[1] = d->lat_local;
    cnt[2] = 2 * (K / TS);   lat[2] = d->lat_barrier;
    cnt[3] = K * VW;         lat[3] = d->lat_compute;
    return MC_OK;
  }
  return fail(err, "unknown model kind");
}

int build_model(const mc_desc* d, ModelHost* h, std::string* err) {
  if (!d || !h) return fail(err, "null descriptor");
  if (d->n_cu < 1 || d->n_cu > (uint32_t)kMaxCU) return fail(err, "n_cu out of range 1..8");
  if (d->n_cfg < 1 || d->n_cfg > (1u << 20)) return fail(err, "n_cfg out of range");
  if (!d->params) return fail(err, "params is null");
  if (d->lat_global < 1 || d->lat_local < 1 || d->lat_compute < 1)
    return fail(err, "latencies Lg, Ll, Lc must be >= 1");
  if (d->lat_global > (1u << 20) || d->lat_local > (1u << 20) || d->lat_compute > (1u << 20) ||
      d->lat_barrier > (1u << 20))
    return fail(err, "latency too large");
  h->desc = *d;
  h->m = d->n_cu;
  h->n_cfg = d->n_cfg;
  h->params.assign(d->params, d->params + 4ull * d->n_cfg);
  h->desc.params = h->params.data();
  h->cfgs.assign(d->n_cfg, CfgRec{});
  h->cfg_states.assign(d->n_cfg, 0);
  const uint32_t m = h->m;
  uint64_t total = 1, depth = 0, fb = d->n_cfg;
  uint64_t widest_sum = 0;
  uint32_t max_clock = 0, max_n = 0, max_d = 0;
  for (uint32_t c = 0; c < d->n_cfg; ++c) {
    uint64_t n, cnt[4], lat[4];
    int rc = phases(d, &h->params[4ull * c], &n, cnt, lat, err);
    if (rc) return rc;
    if (n == 0 || n >= (1ull << 31)) return fail(err, "workgroup count out of range");
    CfgRec& r = h->cfgs[c];
    std::memset(&r, 0, sizeof(r));
    uint64_t t = 0, b = 0;
    for (int j = 0; j < 4; ++j) {
      if (cnt[j] == 0 || lat[j] == 0) continue;
      if (cnt[j] >= (1ull << 31)) return fail(err, "operation count out of range");
      r.cnt[r.nph] = (uint32_t)cnt[j];
      r.lat[r.nph] = (uint32_t)lat[j];
      r.t0[r.nph] = (uint32_t)t;
      r.i0[r.nph] = (uint32_t)b;
      ++r.nph;
      t += cnt[j] * lat[j];
      b += cnt[j];
      if (t >= (1ull << 31)) return fail(err, "workgroup duration exceeds 2^31");
    }
    if (b == 0) return fail(err, "workgroup without timed operations");
    const uint64_t rounds = (n + m - 1) / m;
    const uint64_t tc = rounds * t;
    if (tc >= 0xFFFFFFFFull) return fail(err, "terminal clock exceeds 32 bits");
    r.n = (uint32_t)n;
    r.d = (uint32_t)t;
    r.b = (uint32_t)b;
    r.tc = (uint32_t)tc;
    const uint64_t q = n / m, p = n % m;
    uint64_t cs = 1 + q * (((1ull << m) - 1) + b);
    if (p) {
      uint64_t s = 0;
      for (uint32_t j = 1; j <= p; ++j) s += binom(m, j);
      cs += s + binom(m, (uint32_t)p) * (b - 1) + 1;
    }
    h->cfg_states[c] = cs;
    total += cs;
    depth = std::max<uint64_t>(depth, 1 + n + rounds * b);
    max_clock = std::max<uint32_t>(max_clock, (uint32_t)tc);
    max_n = std::max<uint32_t>(max_n, (uint32_t)n);
    max_d = std::max<uint32_t>(max_d, (uint32_t)t);
    // widest level of this subgraph: dispatch levels C(m, j), partial-round runs C(m, p)
    uint64_t w = 1;
    const uint32_t jmax = (uint32_t)std::min<uint64_t>(n, m);
    for (uint32_t j = 0; j <= jmax; ++j) w = std::max<uint64_t>(w, binom(m, j));
    widest_sum += w;
  }
  fb = std::max<uint64_t>(fb, widest_sum);
  h->states = total;
  h->max_depth = depth;
  h->max_clock = max_clock;
  h->max_n = max_n;
  h->max_d = max_d;
  h->frontier_bound = fb;

  // key layout: cfg | pending | clock | rem_0 .. rem_{m-1}
  uint32_t widths[kFields] = {0};
  widths[kFCfg] = std::max<uint32_t>(1, bit_length((uint64_t)d->n_cfg + 1));
  widths[kFPending] = std::max<uint32_t>(1, bit_length(max_n));
  widths[kFClock] = std::max<uint32_t>(1, bit_length(max_clock));
  for (uint32_t i = 0; i < m; ++i) widths[kFRem + i] = std::max<uint32_t>(1, bit_length(max_d));
  Layout L;
  std::memset(&L, 0, sizeof(L));
  // every word after the first keeps its top bit clear, so that no valid key has a word
  // equal to the all-ones of a cleared slot (word 0 cannot be: its configuration field
  // is never all-ones); a reader of a wide key can then tell a word not yet written
  uint32_t word = 0, off = 0, used = 0;
  for (uint32_t f = 0; f < 3 + m; ++f) {
    if (off + widths[f] > (word == 0 ? 64u : 63u)) {
      ++word;
      off = 0;
    }
    L.word[f] = (uint8_t)word;
    L.shift[f] = (uint8_t)off;
    L.width[f] = (uint8_t)widths[f];
    off += widths[f];
    used += widths[f];
  }
  uint32_t words = word + 1;
  if (words > 4) return fail(err, "packed state wider than 256 bits");
  L.W = (uint8_t)(words == 1 ? 1 : words == 2 ? 2 : 4);
  L.m = (uint8_t)m;
  L.used_bits = (uint8_t)used;
  h->layout = L;
  h->W = L.W;
  return MC_OK;
}

void plan_parts(const ModelHost& h, uint64_t target, std::vector<PartPlan>* out) {
  const Layout& L = h.layout;
  const bool cuttable = target > 0 && L.word[kFPending] == 0 && L.word[kFClock] == 0;
  for (uint32_t c = 0; c < h.n_cfg; ++c) {
    const CfgRec& r = h.cfgs[c];
    const uint64_t q = r.n / h.m;
    const uint64_t per_round = ((1ull << h.m) - 1) + r.b;
    uint64_t R = cuttable ? std::max<uint64_t>(kMinBlockRounds, target / per_round) : q;
    const uint64_t K = R ? (q + R - 1) / R : 1;
    if (!cuttable || K < 2) {
      out->push_back(PartPlan{c, 0u, kRoundsToEnd, h.cfg_states[c]});
      continue;
    }
    for (uint64_t k = 0; k + 1 < K; ++k)
      out->push_back(PartPlan{c, (uint32_t)(k * R), (uint32_t)((k + 1) * R), R * per_round});
    const uint64_t r0 = (K - 1) * R;
    out->push_back(PartPlan{c, (uint32_t)r0, kRoundsToEnd, h.cfg_states[c] - r0 * per_round});
  }
}

uint64_t auto_part_states(uint64_t states) {
  // about 256 partitions for small models (down to blocks of kMinBlockRounds rounds),
  // blocks of at most 2^14 states for large ones
  return std::min<uint64_t>(1ull << 14, std::max<uint64_t>(1, states / 256));
}

// operation ends of one workgroup at or before time x
static uint64_t ends_le(const CfgRec& r, uint64_t x) {
  uint64_t c = 0;
  for (uint32_t j = 0; j < r.nph; ++j)
    if (x >= (uint64_t)r.t0[j] + r.lat[j])
      c += std::min<uint64_t>(r.cnt[j], (x - r.t0[j]) / r.lat[j]);
  return c;
}

uint64_t count_le_bound(const ModelHost& h, uint64_t T) {
  const uint32_t m = h.m;
  const uint64_t closure = (1ull << m) - 1;
  uint64_t total = 1;  // the root
  for (uint32_t c = 0; c < h.n_cfg; ++c) {
    const CfgRec& r = h.cfgs[c];
    if (T >= r.tc) {
      total += h.cfg_states[c];
      continue;
    }
    const uint64_t q = r.n / m, p = r.n % m;
    const uint64_t full = std::min<uint64_t>(q, T / r.d);  // rounds ended by T
    uint64_t cnt = 1 + full * (closure + r.b);             // SELECT state, whole rounds
    const uint64_t x = T - full * r.d;                     // time into the next round
    if (full < q) {
      cnt += closure + ends_le(r, x);
    } else if (p) {
      for (uint32_t j = 1; j <= p; ++j) cnt += binom(m, j);
      cnt += binom(m, (uint32_t)p) * ends_le(r, x);
    }
    total += std::min<uint64_t>(cnt, h.cfg_states[c]);
  }
  return total;
}

}  // namespace mc
