// Sanitizer driver of the library's host-side model code (csrc/mc_model.cpp): descriptor
// validation, operation lists, key layouts, the closed-form sizes, the multithreaded walk
// of units of unequal speed, partition plans (blocks, run slices, chain slices, resumed
// explorations) and the host key codec, over a spread of valid and invalid descriptors.
// Built with AddressSanitizer + UndefinedBehaviorSanitizer, and separately with
// ThreadSanitizer, by tests/test_sanitizers.py; test infrastructure only.
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2305_09130_amd/csrc/mc_model.h"

using namespace mc;

static int failures = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

static void exercise(const mc_desc& d, bool valid) {
  ModelHost h;
  std::string err;
  const int rc = build_model(&d, &h, &err);
  expect((rc == MC_OK) == valid, valid ? "valid descriptor rejected" : "invalid accepted");
  if (rc != MC_OK) return;
  for (uint64_t target : {0ull, 1ull, 32ull, 500ull, 1ull << 14}) {
    std::vector<PartPlan> parts;
    plan_parts(h, target, &parts);
    expect(!parts.empty(), "no partitions");
    for (const PartPlan& p : parts) expect(p.cfg < h.n_cfg, "partition configuration");
    // bounded by a clock: the same plan without the parts of rounds starting after it
    if (!h.hetero)
      for (uint64_t cmax : {0ull, 7ull, 300ull, 5000ull}) {
        std::vector<PartPlan> bounded, want;
        plan_parts(h, target, &bounded, cmax);
        for (const PartPlan& p : parts) {
          const uint64_t round = p.r0 == kRunSlice ? p.r1 : p.r0;
          if (round * h.cfgs[p.cfg].d <= cmax) want.push_back(p);
        }
        bool same = bounded.size() == want.size();
        for (size_t i = 0; same && i < want.size(); ++i)
          same = bounded[i].cfg == want[i].cfg && bounded[i].r0 == want[i].r0 &&
                 bounded[i].r1 == want[i].r1 && bounded[i].j0 == want[i].j0 &&
                 bounded[i].j1 == want[i].j1;
        expect(same, "bounded plan");
      }
  }
  uint64_t last = 0;
  for (uint64_t T : {0ull, 1ull, 50ull, 500ull, 5000ull, 1ull << 31}) {
    const uint64_t n = count_le_bound(h, T);
    expect(n >= last && n <= h.states, "count_le_bound monotone and bounded");
    last = n;
    if (resumable(h)) {
      for (uint64_t target : {0ull, 64ull, 4096ull}) {
        std::vector<PartPlan> fresh, rp;
        plan_parts(h, target, &fresh);
        plan_resume(h, T, fresh, &rp);
        expect(rp.size() <= std::max<size_t>(fresh.size(), h.n_cfg), "resume plan size");
        if (h.hetero) {
          // chain slices ending past T, or whole configurations from SELECT; nothing of a
          // configuration whose terminals all lie at or below T
          for (const PartPlan& p : rp) {
            expect(p.cfg < h.n_cfg && h.cfgs[p.cfg].tc > T, "unequal units: finished resumed");
            if (p.r0 == kChainSlice)
              expect(p.r1 == kNoClock || p.r1 > T, "unequal units: slice ends past T");
            else
              expect(p.r0 == 0 && p.r1 == kRoundsToEnd, "unequal units: whole from SELECT");
          }
          for (uint32_t c = 0; c < h.n_cfg; ++c) {
            if (h.cfgs[c].tc <= T) continue;
            bool last = false;  // the part that runs through the tails is always kept
            for (const PartPlan& p : rp)
              last |= p.cfg == c && (p.r0 != kChainSlice || p.r1 == kNoClock);
            expect(last, "unequal units: configuration's end resumed");
          }
          continue;
        }
        // per configuration: the resumed rounds are [floor(T/d), rounds), disjoint, covered
        for (uint32_t c = 0; c < h.n_cfg; ++c) {
          const CfgRec& r = h.cfgs[c];
          const uint64_t rounds = (r.n + h.m - 1) / h.m;
          std::vector<std::pair<uint64_t, uint64_t>> iv;
          for (const PartPlan& p : rp)
            if (p.cfg == c) iv.push_back({p.r0, p.r1 == kRoundsToEnd ? rounds : p.r1});
          if (rounds * r.d <= T) {
            expect(iv.empty(), "finished configuration resumed");
            continue;
          }
          std::sort(iv.begin(), iv.end());
          uint64_t at = std::min<uint64_t>(T / r.d, rounds - 1);
          for (const auto& x : iv) {
            expect(x.first == at && x.second > x.first, "resumed rounds contiguous");
            at = x.second;
          }
          expect(at == rounds, "resumed rounds reach the end");
        }
      }
    }
  }
  if (h.hetero) {
    for (uint32_t c = 0; c < h.n_cfg; ++c) {
      std::vector<ChainCut> cuts;
      chain_cuts(h.cut_cands[h.cut_of[c]], 64, &cuts);
      expect(h.cut_cands[h.cut_of[c]].size() <= kMaxCuts, "cut points bounded");
      expect(h.cut_of[c] <= c && h.cut_of[h.cut_of[c]] == h.cut_of[c], "cut points shared");
      for (size_t k = 1; k < cuts.size(); ++k)
        expect(cuts[k].t > cuts[k - 1].t && cuts[k].depth > cuts[k - 1].depth &&
                   cuts[k].states >= cuts[k - 1].states + 64,
               "cut order");
      for (const ChainCut& k : cuts) expect(k.states < h.cfg_states[c], "cut inside");
    }
  }
  // the host key codec round trip on the SELECT states and a dispatched state
  for (uint32_t c = 0; c < h.n_cfg; ++c) {
    uint32_t f[kFields] = {0}, g[kFields] = {0};
    f[kFCfg] = c;
    f[kFPending] = h.cfgs[c].n;
    uint64_t w[4];
    encode_key_host(h.layout, f, w);
    decode_key_host(h.layout, w, g, h.cfgs.data());
    expect(std::memcmp(f, g, sizeof(uint32_t) * (3 + h.m)) == 0, "codec SELECT");
    if (h.cfgs[c].n >= 1) {
      f[kFPending] = h.cfgs[c].n - 1;
      f[kFRem] = h.hetero ? h.speed[0] * h.cfgs[c].d : h.cfgs[c].d;
      encode_key_host(h.layout, f, w);
      decode_key_host(h.layout, w, g, h.cfgs.data());
      expect(std::memcmp(f, g, sizeof(uint32_t) * (3 + h.m)) == 0, "codec dispatch");
    }
  }
}

int main() {
  std::vector<uint32_t> red, mat, unit;
  for (uint32_t wg = 1; wg <= 32; wg *= 2)
    for (uint32_t ts = 1; ts <= 4; ts *= 2) red.insert(red.end(), {wg, ts, 0, 0});
  for (uint32_t x = 1; x <= 4; x *= 2)
    for (uint32_t y = 1; y <= 4; y *= 2)
      for (uint32_t ts = 1; ts <= 4; ts *= 2)
        for (uint32_t vw = 1; vw <= 2; vw *= 2) mat.insert(mat.end(), {x, y, ts, vw});
  for (uint32_t wg = 2; wg <= 16; wg *= 2)
    for (uint32_t ts = 1; ts <= 8; ts *= 2) unit.insert(unit.end(), {wg, ts, 0, 0});
  const uint32_t speeds[8] = {1, 2, 3, 1, 5, 2, 7, 1};
  for (uint32_t m = 1; m <= 8; ++m) {
    for (int het = 0; het < 2; ++het) {
      mc_desc d;
      std::memset(&d, 0, sizeof(d));
      d.kind = MC_KIND_REDUCTION;
      d.n_cu = m;
      d.size[0] = 256;
      d.lat_global = 20 + m;
      d.lat_local = 3;
      d.lat_compute = 1;
      d.lat_barrier = m & 1;
      d.n_cfg = (uint32_t)(red.size() / 4);
      d.params = red.data();
      d.unit_speed = het ? speeds : nullptr;
      exercise(d, true);
      d.kind = MC_KIND_MATMUL;
      d.size[0] = d.size[1] = d.size[2] = 16;
      d.n_cfg = (uint32_t)(mat.size() / 4);
      d.params = mat.data();
      exercise(d, true);
      for (uint32_t kind : {MC_KIND_ABSTRACT, MC_KIND_MINIMUM}) {
        d.kind = kind;
        d.size[0] = 64;
        d.size[1] = 4;
        d.size[2] = 0;
        d.n_cfg = (uint32_t)(unit.size() / 4);
        d.params = unit.data();
        exercise(d, true);
      }
    }
  }
  {
    // a model whose host walk runs its configurations on several threads
    mc_desc d;
    std::memset(&d, 0, sizeof(d));
    d.kind = MC_KIND_REDUCTION;
    d.n_cu = 4;
    d.size[0] = 1u << 12;
    d.lat_global = 29;
    d.lat_local = 3;
    d.lat_compute = 1;
    d.n_cfg = (uint32_t)(red.size() / 4);
    d.params = red.data();
    d.unit_speed = speeds;
    ModelHost h;
    std::string err;
    expect(build_model(&d, &h, &err) == MC_OK && h.hetero, "threaded walk");
  }
  // invalid descriptors
  mc_desc bad;
  std::memset(&bad, 0, sizeof(bad));
  bad.kind = MC_KIND_REDUCTION;
  bad.n_cu = 2;
  bad.size[0] = 96;  // not a power of two
  bad.lat_global = bad.lat_local = bad.lat_compute = 1;
  bad.n_cfg = (uint32_t)(red.size() / 4);
  bad.params = red.data();
  exercise(bad, false);
  bad.size[0] = 256;
  bad.n_cu = 9;  // too many units
  exercise(bad, false);
  bad.n_cu = 2;
  bad.params = nullptr;
  exercise(bad, false);
  bad.params = red.data();
  bad.kind = 7;
  exercise(bad, false);
  std::printf("host driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
