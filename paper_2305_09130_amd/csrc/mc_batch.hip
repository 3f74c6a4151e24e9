// mc_batch.hip -- many models explored in one persistent launch: arena layout, the
// (model, configuration) partition queue, the autotuner and hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mctune.h"
#include "mc_launch.h"
#include "mc_model.h"

using namespace mc;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}
// visited-set bytes per slot: the key words, then the parent and jump words
uint32_t slot_bytes_for(uint32_t W) { return 8u * W + 8u; }
constexpr size_t kCtrlStride = 256;

struct BatchPlan {
  size_t ctrl = 0, tc = 0, cfgs = 0, seeds = 0, md = 0, parts = 0, head = 0, ranges = 0;
  size_t tables = 0, tables_bytes = 0, total = 0;
  std::vector<size_t> tc_off, cfg_off, seed_off, table_off;
  std::vector<uint64_t> slots;
  uint64_t n_parts = 0;
};

// The part of each model's visited set a query clears, as (first, count) of 16-byte units
// from the tables' start: the key region on units alike (their links are read only where
// written), the whole set on units of unequal speed.  One workgroup row per model.
__global__ void k_clear_ranges(uint4* base, const ulonglong2* ranges, uint32_t n) {
  const uint4 v = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  for (uint32_t r = blockIdx.y; r < n; r += gridDim.y) {
    const ulonglong2 rg = ranges[r];
    uint4* p = base + rg.x;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         i < rg.y; i += stride)
      p[i] = v;
  }
}

mc_batch_opts default_bopts(const mc_batch_opts* o) {
  mc_batch_opts r;
  std::memset(&r, 0, sizeof(r));
  if (o) r = *o;
  if (r.block != 256 && r.block != 512 && r.block != 1024) r.block = 512;
  if (!(r.load_factor > 0.f && r.load_factor < 1.f)) r.load_factor = 0.5f;
  if (r.lane_items > 2) r.lane_items = 0;
  return r;
}

// Partitions of a batch: every model's configurations, cut into blocks of whole rounds,
// grouped by key width (one launch each) and largest first within a group.
struct BPart {
  uint64_t size;
  uint32_t model, cfg, r0, r1, j0, j1;
};

int width_group(uint32_t W) { return W == 1 ? 0 : W == 2 ? 1 : 2; }

std::vector<BPart> batch_parts(const std::vector<ModelHost>& ms, const mc_batch_opts& o) {
  uint64_t total = 0;
  for (const auto& m : ms) total += m.states;
  const uint64_t target = o.part_states == 0xFFFFFFFFu ? 0u
                          : o.part_states              ? o.part_states
                                                       : auto_part_states(total);
  std::vector<BPart> ps;
  std::vector<PartPlan> plan;
  for (uint32_t i = 0; i < (uint32_t)ms.size(); ++i) {
    plan.clear();
    plan_parts(ms[i], target, &plan);
    for (const auto& q : plan) ps.push_back({q.states, i, q.cfg, q.r0, q.r1, q.j0, q.j1});
  }
  std::stable_sort(ps.begin(), ps.end(), [&](const BPart& a, const BPart& c) {
    const int ga = width_group(ms[a.model].W), gc = width_group(ms[c.model].W);
    return ga != gc ? ga < gc : a.size > c.size;
  });
  return ps;
}

int plan_batch(const std::vector<ModelHost>& ms, const mc_batch_opts& o, uint64_t n_parts,
               BatchPlan* p) {
  const size_t n = ms.size();
  size_t off = 0;
  p->ctrl = off;
  off = align_up(off + kCtrlStride * n);
  p->tc = off;
  p->tc_off.resize(n);
  for (size_t i = 0; i < n; ++i) {
    p->tc_off[i] = off;
    off += 4ull * ms[i].n_cfg;
  }
  off = align_up(off);
  p->cfg_off.resize(n);
  p->cfgs = off;
  for (size_t i = 0; i < n; ++i) {
    p->cfg_off[i] = off;
    off += sizeof(CfgRec) * ms[i].n_cfg;
  }
  off = align_up(off);
  p->seed_off.resize(n);
  p->seeds = off;
  for (size_t i = 0; i < n; ++i) {
    p->seed_off[i] = off;
    off += sizeof(Seed) * ms[i].n_cfg;
  }
  off = align_up(off);
  p->md = off;
  off = align_up(off + sizeof(ModelDev) * n);
  p->ranges = off;
  off = align_up(off + sizeof(unsigned long long) * 2 * n);
  p->n_parts = n_parts;
  p->parts = off;
  off = align_up(off + sizeof(Part) * p->n_parts);
  p->head = off;
  off = align_up(off + 16);
  p->tables = off;
  p->table_off.resize(n);
  p->slots.resize(n);
  for (size_t i = 0; i < n; ++i) {
    uint64_t slots = next_pow2((uint64_t)((double)ms[i].states / o.load_factor) + 1);
    slots = std::max<uint64_t>(slots, 1024);
    if (slots > (1ull << 31)) return MC_E_INVAL;
    p->slots[i] = slots;
    p->table_off[i] = off;
    off = align_up(off + slots * slot_bytes_for(ms[i].W));
  }
  p->tables_bytes = off - p->tables;
  p->total = off;
  return MC_OK;
}

int build_models(const mc_desc* models, uint32_t n, std::vector<ModelHost>* ms) {
  if (!models || n == 0) return MC_E_INVAL;
  ms->resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    std::string err;
    const int rc = build_model(&models[i], &(*ms)[i], &err);
    if (rc) return rc;
  }
  return MC_OK;
}

#define HIPCHK(x)              \
  do {                         \
    hipError_t e_ = (x);       \
    if (e_ != hipSuccess) {    \
      (void)hipGetLastError(); \
      return MC_E_DEVICE;      \
    }                          \
  } while (0)

}  // namespace

struct mc_batch {
  std::vector<ModelHost> ms;
  mc_batch_opts opts{};
  BatchPlan plan;
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  ModelDev* dmd = nullptr;
  Part* parts = nullptr;
  unsigned int* head = nullptr;
  unsigned char* hctrl = nullptr;  // pinned: n * kCtrlStride
  uint32_t* htc = nullptr;         // pinned: all clocks
  size_t tc_words = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ran = false;
  uint64_t max_range16 = 0;  // the largest range of the clear, in 16-byte units
  uint32_t grid[3] = {0, 0, 0};
  uint32_t group_off[3] = {0, 0, 0}, group_n[3] = {0, 0, 0};  // partitions per key width
  Fork fork;
};

namespace {

int enqueue_query(mc_batch* b) {
  hipStream_t s = b->stream;
  const uint32_t n = (uint32_t)b->ms.size();
  {
    // about two 16-byte stores per thread of the largest range, at most 65535 model rows
    const unsigned long long x = std::min<unsigned long long>(
        std::max<unsigned long long>(1, (b->max_range16 + 511) / 512), 1024);
    const uint32_t y = std::min<uint32_t>(n, 65535u);
    hipLaunchKernelGGL(k_clear_ranges, dim3((uint32_t)x, y), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(b->ws + b->plan.tables),
                       reinterpret_cast<const ulonglong2*>(b->ws + b->plan.ranges), n);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(launch_reset_models(s, b->dmd, n, b->head, 3));
  HIPCHK(launch_seed_models(s, b->dmd, n));
  const uint32_t li = b->opts.lane_items;  // 0: per key width
  PartQueue pq[3];
  for (int w = 0; w < 3; ++w) {
    pq[w].models = b->dmd;
    pq[w].parts = b->parts + b->group_off[w];
    pq[w].n_parts = b->group_n[w];
    pq[w].batch_items =
        b->opts.chunk ? b->opts.chunk : 2u * lane_items_for(li, 1u << w) * b->opts.block;
    pq[w].head = b->head + w;
    pq[w].slice = 0u;
    pq[w].reverse = 0u;
    pq[w].yielded = nullptr;
    pq[w].n_yielded = nullptr;
    pq[w].abort = nullptr;
  }
  bool general = false, hetero = false;
  for (const ModelHost& mh : b->ms) {
    general |= mh.general;
    hetero |= mh.hetero;
  }
  HIPCHK(launch_super_fork(s, b->fork, pq, b->grid, b->opts.block, li, general, hetero));
  HIPCHK(hipMemcpyAsync(b->hctrl, b->ws + b->plan.ctrl, kCtrlStride * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(b->htc, b->ws + b->plan.tc, 4ull * b->tc_words, hipMemcpyDeviceToHost, s));
  return MC_OK;
}

void free_batch(mc_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->hctrl) (void)hipHostFree(b->hctrl);
  if (b->htc) (void)hipHostFree(b->htc);
  b->fork.destroy();
  delete b;
}

// autotuner cache: batch signature -> chosen options
std::mutex g_tune_mu;
std::map<std::string, mc_batch_opts> g_tune_cache;

std::string signature(const std::vector<ModelHost>& ms) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  for (const auto& m : ms) {
    mix(m.desc.kind);
    mix(m.m);
    mix(m.n_cfg);
    mix(m.states);
    mix(m.desc.lat_global);
    mix(m.desc.lat_local);
  }
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "?";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  (void)hipGetLastError();
  return arch + ":" + std::to_string(ms.size()) + ":" + std::to_string(h);
}

}  // namespace

extern "C" {

int mc_batch_workspace_bytes(const mc_desc* models, uint32_t n, const mc_batch_opts* o,
                             size_t* bytes) {
  if (!bytes) return MC_E_INVAL;
  try {
    std::vector<ModelHost> ms;
    int rc = build_models(models, n, &ms);
    if (rc) return rc;
    BatchPlan p;
    const mc_batch_opts oo = default_bopts(o);
    rc = plan_batch(ms, oo, batch_parts(ms, oo).size(), &p);
    if (rc) return rc;
    *bytes = p.total;
    return MC_OK;
  } catch (...) {
    return MC_E_INVAL;
  }
}

int mc_batch_create(const mc_desc* models, uint32_t n, const mc_batch_opts* o, void* dev_ws,
                    size_t ws_bytes, void* stream, mc_batch** out) {
  if (!out || !dev_ws) return MC_E_INVAL;
  *out = nullptr;
  mc_batch* b = nullptr;
  try {
    b = new mc_batch();
    int rc = build_models(models, n, &b->ms);
    if (rc) {
      delete b;
      return rc;
    }
    b->opts = default_bopts(o);
    const std::vector<BPart> ps = batch_parts(b->ms, b->opts);
    rc = plan_batch(b->ms, b->opts, ps.size(), &b->plan);
    if (rc) {
      delete b;
      return rc;
    }
    if (ws_bytes < b->plan.total) {
      delete b;
      return MC_E_NOMEM;
    }
    b->stream = reinterpret_cast<hipStream_t>(stream);
    b->ws = reinterpret_cast<unsigned char*>(dev_ws);
    b->dmd = reinterpret_cast<ModelDev*>(b->ws + b->plan.md);
    b->parts = reinterpret_cast<Part*>(b->ws + b->plan.parts);
    b->head = reinterpret_cast<unsigned int*>(b->ws + b->plan.head);
    for (const auto& m : b->ms) b->tc_words += m.n_cfg;
    if (hipHostMalloc(reinterpret_cast<void**>(&b->hctrl), kCtrlStride * n, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&b->htc), 4ull * b->tc_words,
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&b->ev[0]) != hipSuccess || hipEventCreate(&b->ev[1]) != hipSuccess ||
        b->fork.create() != hipSuccess) {
      (void)hipGetLastError();
      free_batch(b);
      return MC_E_DEVICE;
    }
    // descriptors, configuration tables and the partition queue (largest first)
    std::vector<ModelDev> md(n);
    for (uint32_t i = 0; i < n; ++i) {
      const ModelHost& m = b->ms[i];
      ModelDev& d = md[i];
      std::memset(&d, 0, sizeof(d));
      d.ctrl = reinterpret_cast<Ctrl*>(b->ws + b->plan.ctrl + kCtrlStride * i);
      d.tc = reinterpret_cast<uint32_t*>(b->ws + b->plan.tc_off[i]);
      d.cfgs = reinterpret_cast<const CfgRec*>(b->ws + b->plan.cfg_off[i]);
      d.seeds = reinterpret_cast<Seed*>(b->ws + b->plan.seed_off[i]);
      d.table = b->ws + b->plan.table_off[i];
      d.mask = b->plan.slots[i] - 1;
      d.L = m.layout;
      d.n_cfg = m.n_cfg;
      d.max_clock = m.max_clock;
    }
    for (const BPart& q : ps) ++md[q.model].n_parts;
    std::vector<Part> parts(ps.size());
    std::vector<uint32_t> pidx(n, 0u);  // partitions of each model so far
    for (size_t k = 0; k < ps.size(); ++k) {
      parts[k] = Part{ps[k].model, ps[k].cfg, ps[k].r0, ps[k].r1, pidx[ps[k].model]++, ps[k].j0,
                      ps[k].j1, 0u};
      ++b->group_n[width_group(b->ms[ps[k].model].W)];
    }
    b->group_off[0] = 0;
    b->group_off[1] = b->group_n[0];
    b->group_off[2] = b->group_n[0] + b->group_n[1];
    hipStream_t s = b->stream;
    for (uint32_t i = 0; i < n; ++i)
      if (hipMemcpyAsync(b->ws + b->plan.cfg_off[i], b->ms[i].cfgs.data(),
                         sizeof(CfgRec) * b->ms[i].n_cfg, hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        free_batch(b);
        return MC_E_DEVICE;
      }
    // the part of each visited set a query clears (16-byte units from the tables' start)
    std::vector<unsigned long long> ranges(2ull * n);
    for (uint32_t i = 0; i < n; ++i) {
      const ModelHost& m = b->ms[i];
      const uint64_t bytes = b->plan.slots[i] * (m.hetero ? slot_bytes_for(m.W) : 8ull * m.W);
      ranges[2 * i] = (b->plan.table_off[i] - b->plan.tables) / 16;
      ranges[2 * i + 1] = bytes / 16;
      b->max_range16 = std::max<uint64_t>(b->max_range16, bytes / 16);
    }
    if (hipMemcpyAsync(b->ws + b->plan.ranges, ranges.data(), sizeof(unsigned long long) * 2 * n,
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->dmd, md.data(), sizeof(ModelDev) * n, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(b->parts, parts.data(), sizeof(Part) * parts.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      free_batch(b);
      return MC_E_DEVICE;
    }
    for (int w = 0; w < 3; ++w)
      b->grid[w] = b->opts.grid ? b->opts.grid
                                : std::min<uint32_t>(std::max<uint32_t>(b->group_n[w], 1u),
                                                     b->opts.block >= 1024 ? 512u : 1024u);
    if (b->opts.use_graph) {
      if (s == nullptr) {  // the null stream cannot be captured
        free_batch(b);
        return MC_E_INVAL;
      }
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        free_batch(b);
        return MC_E_DEVICE;
      }
      const int erc = enqueue_query(b);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(s, &g);
      if (erc != MC_OK || e2 != hipSuccess || !g ||
          hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        free_batch(b);
        return MC_E_DEVICE;
      }
      b->graph = g;
    }
    *out = b;
    return MC_OK;
  } catch (const std::bad_alloc&) {
    if (b) free_batch(b);
    return MC_E_NOMEM;
  } catch (...) {
    if (b) free_batch(b);
    return MC_E_INVAL;
  }
}

int mc_batch_min_time(mc_batch* b, uint32_t* t_min, uint64_t* states, mc_stats* st) {
  if (!b) return MC_E_INVAL;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = b->stream;
  HIPCHK(hipEventRecord(b->ev[0], s));
  if (b->exec) {
    HIPCHK(hipGraphLaunch(b->exec, s));
  } else {
    const int rc = enqueue_query(b);
    if (rc) return rc;
  }
  HIPCHK(hipEventRecord(b->ev[1], s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
  const uint32_t n = (uint32_t)b->ms.size();
  mc_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  size_t tcpos = 0;
  int rc = MC_OK;
  for (uint32_t i = 0; i < n; ++i) {
    const Ctrl* c = reinterpret_cast<const Ctrl*>(b->hctrl + kCtrlStride * i);
    if (c->error && rc == MC_OK)
      rc = dev_error_code(c->error);
    uint32_t best = kNoClock;
    for (uint32_t k = 0; k < b->ms[i].n_cfg; ++k) best = std::min(best, b->htc[tcpos + k]);
    tcpos += b->ms[i].n_cfg;
    if (t_min) t_min[i] = best;
    if (states) states[i] = c->states;
    acc.states += c->states;
    acc.terminals += c->terminals;
    acc.edges += c->edges;
    acc.dups += c->dups;
    acc.probes += c->probes;
    acc.cas_fail += c->probes > c->states + c->dups ? c->probes - c->states - c->dups : 0u;
    acc.levels = std::max<uint64_t>(acc.levels, c->max_depth + 1);
    acc.supersteps += c->supersteps;
    acc.batches += c->chunks;
    acc.max_probe = std::max<uint64_t>(acc.max_probe, c->max_probe);
    if (c->crit_ticks * 10ull > acc.critical_ns) {
      acc.critical_ns = c->crit_ticks * 10ull;
      acc.critical_cfg = c->crit_part;
    }
  }
  acc.parts = b->plan.n_parts;
  acc.launches = b->exec ? 1 : 4;
  acc.explore_ns = (uint64_t)(ms * 1e6);
  acc.engine_ns = acc.explore_ns;
  acc.total_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now() - t0)
                     .count();
  if (st) *st = acc;
  b->ran = rc == MC_OK;
  return rc;
}

int mc_batch_terminal_clocks(const mc_batch* b, uint32_t model, uint32_t* tc, size_t cap) {
  if (!b || !tc || model >= b->ms.size()) return MC_E_INVAL;
  if (!b->ran) return MC_E_STATE;
  if (cap < b->ms[model].n_cfg) return MC_E_BUFFER;
  size_t pos = 0;
  for (uint32_t i = 0; i < model; ++i) pos += b->ms[i].n_cfg;
  std::memcpy(tc, b->htc + pos, 4ull * b->ms[model].n_cfg);
  return MC_OK;
}

int mc_batch_free(mc_batch* b) {
  if (!b) return MC_E_INVAL;
  free_batch(b);
  return MC_OK;
}

// Autotuner: runs the batch once per candidate (block, load factor, batch items) in the
// caller's workspace (sized for the smallest load factor tried) and keeps the fastest;
// results are cached per batch signature and device architecture.
int mc_batch_autotune(const mc_desc* models, uint32_t n, void* dev_ws, size_t ws_bytes,
                      void* stream, mc_batch_opts* best, float* best_ms) {
  if (!best) return MC_E_INVAL;
  try {
    std::vector<ModelHost> ms;
    int rc = build_models(models, n, &ms);
    if (rc) return rc;
    const std::string sig = signature(ms);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(sig);
      if (it != g_tune_cache.end()) {
        *best = it->second;
        if (best_ms) *best_ms = -1.f;
        return MC_OK;
      }
    }
    const uint32_t blocks[] = {256, 512, 1024};
    const float lfs[] = {0.25f, 0.5f, 0.7f};
    const uint32_t lane_items[] = {1, 2};
    const uint32_t items_mult[] = {1, 2};
    float best_t = 1e30f;
    mc_batch_opts bo;
    std::memset(&bo, 0, sizeof(bo));
    bool any = false;
    for (float lf : lfs) {
      for (uint32_t bl : blocks) {
        for (uint32_t li : lane_items) {
        for (uint32_t im : items_mult) {
          mc_batch_opts o;
          std::memset(&o, 0, sizeof(o));
          o.block = bl;
          o.load_factor = lf;
          o.lane_items = li;
          o.chunk = im * bl * li;
          size_t need = 0;
          rc = mc_batch_workspace_bytes(models, n, &o, &need);
          if (rc || need > ws_bytes) continue;
          mc_batch* b = nullptr;
          rc = mc_batch_create(models, n, &o, dev_ws, ws_bytes, stream, &b);
          if (rc) continue;
          mc_stats st;
          float t = 1e30f;
          for (int rep = 0; rep < 2; ++rep) {  // first run warms the code object
            if (mc_batch_min_time(b, nullptr, nullptr, &st) == MC_OK)
              t = std::min(t, (float)(st.explore_ns * 1e-6));
          }
          mc_batch_free(b);
          if (t < best_t) {
            best_t = t;
            bo = o;
            any = true;
          }
        }
        }
      }
    }
    if (!any) return MC_E_NOMEM;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[sig] = bo;
    }
    *best = bo;
    if (best_ms) *best_ms = best_t;
    return MC_OK;
  } catch (...) {
    return MC_E_INVAL;
  }
}

}  // extern "C"
