// mc_engine.hip -- continuous-batching query server over the persistent engine.
//
// Queries (min_time or check(T) of a model) are submitted at any time.  Every engine
// step (1) retires queries whose partitions are all explored, freeing their memory and
// model slot, (2) admits waiting queries in arrival order while their footprint (visited
// set, tables, saved frontiers) fits the arena and a model slot is free, and (3) runs one
// persistent launch over the unfinished partitions of every active query; a partition
// explores at most `slice` super-step levels per launch, saves its frontier and yields,
// so queries admitted later overlap with queries already on the device instead of
// waiting for them.  Each query owns its visited set, so its result is the same alone and
// in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <unordered_map>
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
uint32_t slot_bytes_for(uint32_t W) { return W == 1 ? 16u : W == 2 ? 32u : 64u; }
constexpr size_t kCtrlStride = 256;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
    size_ = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

struct Query {
  uint64_t ticket = 0;
  uint32_t kind = 0, T = 0;
  ModelHost mh;
  size_t off = 0, bytes = 0;  // arena region
  size_t cfg_off = 0, seed_off = 0, pstate_off = 0, table_off = 0;
  uint64_t slots = 0;
  std::vector<PartPlan> parts;  // configurations cut into blocks of whole rounds
  int slot_idx = -1;  // model slot
  uint64_t submit_ns = 0, admit_ns = 0, done_ns = 0;
  uint32_t steps = 0;
  mc_query_result res{};
};

// Arena bytes of a query: tables, one PartState per partition and a visited set sized for
// the states it can insert (all of them for min_time, those with clock <= T for check).
// a query's configurations are cut into at most this many more partitions
constexpr size_t kExtraParts = 256;

size_t footprint(const ModelHost& mh, uint64_t states, size_t n_parts, float lf, uint64_t* slots,
                 size_t* cfg_off, size_t* seed_off, size_t* pstate_off, size_t* table_off) {
  uint64_t s = next_pow2((uint64_t)((double)states / lf) + 1);
  s = std::max<uint64_t>(s, 1024);
  size_t off = 0;
  *cfg_off = off;
  off = align_up(off + sizeof(CfgRec) * mh.n_cfg);
  *seed_off = off;
  off = align_up(off + sizeof(Seed) * mh.n_cfg);
  *pstate_off = off;
  off = align_up(off + sizeof(PartState) * n_parts);
  *table_off = off;
  off = align_up(off + s * slot_bytes_for(mh.W));
  *slots = s;
  return off;
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

struct mc_engine {
  mc_engine_opts opts{};
  hipStream_t stream = nullptr;
  unsigned char* base = nullptr;  // caller's device buffer
  size_t bytes = 0;
  // fixed regions at the start of the buffer
  size_t ctrl_off = 0, tc_off = 0, md_off = 0, stage_off = 0, parts_off[2] = {0, 0},
         nyield_off = 0, head_off = 0, arena_off = 0;
  Arena arena;
  uint64_t next_ticket = 1;
  std::deque<Query*> waiting;
  std::vector<Query*> slots;  // model slot -> active query
  std::unordered_map<uint64_t, Query*> all;
  std::vector<Part> pending_parts;  // partitions of the next launch (host side)
  uint32_t n_cur = 0;                // partitions in parts buffer `cur`
  int cur = 0;
  unsigned char* hctrl = nullptr;  // pinned
  uint32_t* htc = nullptr;         // pinned
  unsigned int* hny = nullptr;     // pinned
  ModelDev* hmd = nullptr;         // pinned staging of new descriptors
  uint64_t launches = 0;
  Fork fork;
};

namespace {

ModelDev make_dev(mc_engine* e, Query* q) {
  ModelDev d;
  std::memset(&d, 0, sizeof(d));
  unsigned char* r = e->base + e->arena_off + q->off;
  d.ctrl = reinterpret_cast<Ctrl*>(e->base + e->ctrl_off + kCtrlStride * q->slot_idx);
  d.tc = reinterpret_cast<uint32_t*>(e->base + e->tc_off + 4ull * e->opts.max_cfg * q->slot_idx);
  d.cfgs = reinterpret_cast<const CfgRec*>(r + q->cfg_off);
  d.seeds = reinterpret_cast<Seed*>(r + q->seed_off);
  d.table = r + q->table_off;
  d.mask = q->slots - 1;
  d.L = q->mh.layout;
  d.n_cfg = q->mh.n_cfg;
  d.prune = q->kind == MC_QUERY_CHECK ? 1u : 0u;
  d.T = q->T;
  d.max_clock = q->mh.max_clock;
  d.n_parts = (uint32_t)q->parts.size();
  d.pstate = reinterpret_cast<PartState*>(r + q->pstate_off);
  return d;
}

void finish(mc_engine* e, Query* q) {
  e->arena.release(q->off, q->bytes);
  e->slots[q->slot_idx] = nullptr;
  q->slot_idx = -1;
  q->done_ns = now_ns();
  q->res.submit_ns = q->submit_ns;
  q->res.admit_ns = q->admit_ns;
  q->res.done_ns = q->done_ns;
  q->res.steps = q->steps;
  q->res.done = 1;
}

}  // namespace

extern "C" {

int mc_engine_bytes(const mc_engine_opts* o, size_t arena_bytes, size_t* bytes) {
  if (!o || !bytes || o->max_active == 0 || o->max_cfg == 0) return MC_E_INVAL;
  size_t off = 0;
  off = align_up(off + kCtrlStride * o->max_active);
  off = align_up(off + 4ull * o->max_cfg * o->max_active);
  off = align_up(off + sizeof(ModelDev) * o->max_active);
  off = align_up(off + sizeof(ModelDev) * o->max_active);
  const size_t maxparts = ((size_t)o->max_cfg + kExtraParts) * o->max_active;
  off = align_up(off + sizeof(Part) * maxparts);
  off = align_up(off + sizeof(Part) * maxparts);
  off = align_up(off + 4);
  off = align_up(off + 16);
  *bytes = off + align_up(arena_bytes);
  return MC_OK;
}

int mc_engine_create(const mc_engine_opts* o, void* dev_buf, size_t buf_bytes, void* stream,
                     mc_engine** out) {
  if (!o || !dev_buf || !out) return MC_E_INVAL;
  *out = nullptr;
  if (o->max_active == 0 || o->max_cfg == 0) return MC_E_INVAL;
  mc_engine* e = nullptr;
  try {
    e = new mc_engine();
    e->opts = *o;
    if (e->opts.block != 256 && e->opts.block != 512 && e->opts.block != 1024) e->opts.block = 512;
    if (e->opts.lane_items > 2) e->opts.lane_items = 0;
    if (!(e->opts.load_factor > 0.f && e->opts.load_factor < 1.f)) e->opts.load_factor = 0.5f;
    e->stream = reinterpret_cast<hipStream_t>(stream);
    e->base = reinterpret_cast<unsigned char*>(dev_buf);
    e->bytes = buf_bytes;
    const uint32_t A = e->opts.max_active;
    const size_t maxparts = ((size_t)e->opts.max_cfg + kExtraParts) * A;
    size_t off = 0;
    e->ctrl_off = off;
    off = align_up(off + kCtrlStride * A);
    e->tc_off = off;
    off = align_up(off + 4ull * e->opts.max_cfg * A);
    e->md_off = off;
    off = align_up(off + sizeof(ModelDev) * A);
    e->stage_off = off;
    off = align_up(off + sizeof(ModelDev) * A);
    e->parts_off[0] = off;
    off = align_up(off + sizeof(Part) * maxparts);
    e->parts_off[1] = off;
    off = align_up(off + sizeof(Part) * maxparts);
    e->nyield_off = off;
    off = align_up(off + 4);
    e->head_off = off;
    off = align_up(off + 16);
    e->arena_off = off;
    if (buf_bytes <= off + (1u << 20)) {
      delete e;
      return MC_E_NOMEM;
    }
    e->arena.init(buf_bytes - off);
    e->slots.assign(A, nullptr);
    if (hipHostMalloc(reinterpret_cast<void**>(&e->hctrl), kCtrlStride * A, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->htc), 4ull * e->opts.max_cfg * A,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->hny), 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->hmd), sizeof(ModelDev) * A,
                      hipHostMallocDefault) != hipSuccess ||
        e->fork.create() != hipSuccess) {
      (void)hipGetLastError();
      mc_engine_destroy(e);
      return MC_E_DEVICE;
    }
    *out = e;
    return MC_OK;
  } catch (...) {
    if (e) mc_engine_destroy(e);
    return MC_E_NOMEM;
  }
}

int mc_engine_destroy(mc_engine* e) {
  if (!e) return MC_E_INVAL;
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  for (auto& kv : e->all) delete kv.second;
  if (e->hctrl) (void)hipHostFree(e->hctrl);
  if (e->htc) (void)hipHostFree(e->htc);
  if (e->hny) (void)hipHostFree(e->hny);
  if (e->hmd) (void)hipHostFree(e->hmd);
  e->fork.destroy();
  delete e;
  return MC_OK;
}

int mc_engine_submit(mc_engine* e, const mc_desc* model, uint32_t kind, uint32_t T,
                     uint64_t* ticket) {
  if (!e || !model || !ticket || (kind != MC_QUERY_MIN_TIME && kind != MC_QUERY_CHECK))
    return MC_E_INVAL;
  try {
    Query* q = new Query();
    std::string err;
    const int rc = build_model(model, &q->mh, &err);
    if (rc) {
      delete q;
      return rc;
    }
    q->kind = kind;
    q->T = T;
    // blocks of about states/256, with larger blocks while the plan has more than
    // kExtraParts partitions beyond one per configuration (whole configurations last)
    const uint32_t ps = e->opts.part_states;
    uint64_t target =
        ps == 0xFFFFFFFFu ? 0u : ps ? ps : std::max<uint64_t>(1, q->mh.states / kExtraParts);
    plan_parts(q->mh, target, &q->parts);
    while (target && q->parts.size() > (size_t)q->mh.n_cfg + kExtraParts) {
      target = target >= (1ull << 40) ? 0u : target * 4;
      q->parts.clear();
      plan_parts(q->mh, target, &q->parts);
    }
    std::stable_sort(q->parts.begin(), q->parts.end(),
                     [](const PartPlan& a, const PartPlan& b) { return a.states > b.states; });
    const uint64_t need = kind == MC_QUERY_CHECK ? count_le_bound(q->mh, T) : q->mh.states;
    q->bytes = footprint(q->mh, need, q->parts.size(), e->opts.load_factor, &q->slots,
                         &q->cfg_off, &q->seed_off, &q->pstate_off, &q->table_off);
    q->ticket = e->next_ticket++;
    q->submit_ns = now_ns();
    q->res.kind = kind;
    q->res.T = T;
    q->res.t_min = kNoClock;
    if (q->bytes > e->arena.size() || q->mh.n_cfg > e->opts.max_cfg) {
      q->res.status = MC_E_ADMIT;  // can never fit
      q->res.done = 1;
      q->done_ns = q->submit_ns;
      q->res.submit_ns = q->res.admit_ns = q->res.done_ns = q->submit_ns;
    } else {
      e->waiting.push_back(q);
    }
    e->all[q->ticket] = q;
    *ticket = q->ticket;
    return MC_OK;
  } catch (...) {
    return MC_E_NOMEM;
  }
}

int mc_engine_step(mc_engine* e, uint32_t* n_active, uint32_t* n_waiting) {
  if (!e) return MC_E_INVAL;
  hipStream_t s = e->stream;
  // ---- admission (arrival order; a query that does not fit blocks the queue) ----
  std::vector<Query*> admitted;
  while (!e->waiting.empty()) {
    Query* q = e->waiting.front();
    int slot = -1;
    for (size_t i = 0; i < e->slots.size(); ++i)
      if (!e->slots[i]) {
        slot = (int)i;
        break;
      }
    if (slot < 0) break;
    size_t off = 0;
    if (!e->arena.alloc(q->bytes, &off)) break;
    e->waiting.pop_front();
    q->off = off;
    q->slot_idx = slot;
    e->slots[slot] = q;
    q->admit_ns = now_ns();
    admitted.push_back(q);
  }
  if (!admitted.empty()) {
    std::vector<ModelDev> fresh(admitted.size());
    for (size_t i = 0; i < admitted.size(); ++i) {
      Query* q = admitted[i];
      fresh[i] = make_dev(e, q);
      unsigned char* r = e->base + e->arena_off + q->off;
      HIPCHK(hipMemcpyAsync(r + q->cfg_off, q->mh.cfgs.data(), sizeof(CfgRec) * q->mh.n_cfg,
                            hipMemcpyHostToDevice, s));
      HIPCHK(launch_clear(s, r + q->table_off, q->slots * slot_bytes_for(q->mh.W)));
      e->hmd[i] = fresh[i];
    }
    const size_t nb = sizeof(ModelDev) * admitted.size();
    HIPCHK(hipMemcpyAsync(e->base + e->stage_off, e->hmd, nb, hipMemcpyHostToDevice, s));
    for (size_t i = 0; i < admitted.size(); ++i)
      HIPCHK(hipMemcpyAsync(e->base + e->md_off + sizeof(ModelDev) * admitted[i]->slot_idx,
                            e->base + e->stage_off + sizeof(ModelDev) * i, sizeof(ModelDev),
                            hipMemcpyDeviceToDevice, s));
    const ModelDev* stage = reinterpret_cast<const ModelDev*>(e->base + e->stage_off);
    HIPCHK(launch_reset_models(s, stage, (uint32_t)admitted.size(), nullptr, 0));
    HIPCHK(launch_seed_models(s, stage, (uint32_t)admitted.size()));
    // new partitions, largest first within each query
    for (Query* q : admitted)
      for (size_t k = 0; k < q->parts.size(); ++k) {
        const PartPlan& pp = q->parts[k];
        e->pending_parts.push_back(
            Part{(uint32_t)q->slot_idx, pp.cfg, pp.r0, pp.r1, (uint32_t)k, pp.j0, pp.j1, 0u});
      }
    // the host must not overwrite the pinned staging before the copy ran
    HIPCHK(hipStreamSynchronize(s));
  }
  // ---- one persistent launch over every unfinished partition ----
  bool any_active = false;
  uint32_t hi = 0;  // one past the highest slot in use
  for (size_t i = 0; i < e->slots.size(); ++i)
    if (e->slots[i]) {
      any_active = true;
      hi = (uint32_t)i + 1u;
    }
  // partitions are cut into slices only while queries wait for admission: otherwise the
  // launch runs everything admitted to the end, with no host round trip per slice
  const uint32_t slice = e->waiting.empty() ? 0u : e->opts.slice;
  if (any_active && !e->pending_parts.empty()) {
    const int cur = e->cur;
    Part* parts = reinterpret_cast<Part*>(e->base + e->parts_off[cur]);
    Part* next = reinterpret_cast<Part*>(e->base + e->parts_off[cur ^ 1]);
    // one launch per key width: group the partitions, keeping their order within a group
    std::vector<Part> grouped;
    grouped.reserve(e->pending_parts.size());
    uint32_t gn[3] = {0, 0, 0};
    bool general = false, hetero = false;
    for (const Part& p : e->pending_parts) {
      general |= e->slots[p.model]->mh.general;
      hetero |= e->slots[p.model]->mh.hetero;
    }
    for (int g = 0; g < 3; ++g)
      for (const Part& p : e->pending_parts) {
        const uint32_t W = e->slots[p.model]->mh.W;
        if ((W == 1 ? 0 : W == 2 ? 1 : 2) == g) {
          grouped.push_back(p);
          ++gn[g];
        }
      }
    HIPCHK(hipMemcpyAsync(parts, grouped.data(), sizeof(Part) * grouped.size(),
                          hipMemcpyHostToDevice, s));
    unsigned int* head = reinterpret_cast<unsigned int*>(e->base + e->head_off);
    unsigned int* ny = reinterpret_cast<unsigned int*>(e->base + e->nyield_off);
    HIPCHK(hipMemsetAsync(head, 0, 16, s));
    HIPCHK(hipMemsetAsync(ny, 0, 4, s));
    const uint32_t li = e->opts.lane_items;  // 0: per key width
    PartQueue pq[3];
    uint32_t grid[3];
    uint32_t off = 0;
    for (int g = 0; g < 3; ++g) {
      pq[g].models = reinterpret_cast<const ModelDev*>(e->base + e->md_off);
      pq[g].parts = parts + off;
      pq[g].n_parts = gn[g];
      pq[g].batch_items =
          e->opts.chunk ? e->opts.chunk : 2u * lane_items_for(li, 1u << g) * e->opts.block;
      pq[g].head = head + g;
      pq[g].slice = slice;
      pq[g].reverse = 0u;
      pq[g].yielded = next;
      pq[g].n_yielded = ny;
      pq[g].abort = nullptr;
      grid[g] = std::max<uint32_t>(1u, std::min<uint32_t>(gn[g], e->opts.grid ? e->opts.grid : 1024u));
      off += gn[g];
    }
    HIPCHK(launch_super_fork(s, e->fork, pq, grid, e->opts.block, li, general, hetero));
    ++e->launches;
    HIPCHK(hipMemcpyAsync(e->hny, ny, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(e->hctrl, e->base + e->ctrl_off, kCtrlStride * hi, hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipMemcpyAsync(e->htc, e->base + e->tc_off, 4ull * e->opts.max_cfg * hi,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (Query* q : e->slots)
      if (q) ++q->steps;
    // partitions that yielded continue in the next launch
    const uint32_t nyield = *e->hny;
    e->pending_parts.resize(nyield);
    if (nyield)
      HIPCHK(hipMemcpy(e->pending_parts.data(), next, sizeof(Part) * nyield,
                       hipMemcpyDeviceToHost));
    // ---- retire finished queries ----
    for (size_t i = 0; i < e->slots.size(); ++i) {
      Query* q = e->slots[i];
      if (!q) continue;
      const Ctrl* c = reinterpret_cast<const Ctrl*>(e->hctrl + kCtrlStride * i);
      const bool failed = c->error != 0u;
      if (c->parts_done < q->parts.size() && !failed) continue;
      const uint32_t* tc = e->htc + (size_t)e->opts.max_cfg * i;
      mc_query_result& r = q->res;
      r.status = dev_error_code(c->error);
      r.states = c->states;
      r.levels = c->max_depth + 1;
      uint32_t best = kNoClock, first = kNoClock, n = 0;
      for (uint32_t k = 0; k < q->mh.n_cfg; ++k) best = std::min(best, tc[k]);
      for (uint32_t k = 0; k < q->mh.n_cfg; ++k)
        if (tc[k] == best && best != kNoClock) {
          if (first == kNoClock) first = k;
          ++n;
        }
      r.t_min = best;
      r.argmin_first = first;
      r.n_argmin = n;
      r.violated = c->violated ? 1 : 0;
      finish(e, q);
      // drop any partition of a failed query still queued
      if (failed) {
        std::vector<Part> keep;
        for (const Part& p : e->pending_parts)
          if (p.model != (uint32_t)i) keep.push_back(p);
        e->pending_parts.swap(keep);
      }
    }
  }
  uint32_t na = 0;
  for (Query* q : e->slots) na += q != nullptr;
  if (n_active) *n_active = na;
  if (n_waiting) *n_waiting = (uint32_t)e->waiting.size();
  return MC_OK;
}

int mc_engine_poll(mc_engine* e, uint64_t ticket, mc_query_result* out) {
  if (!e || !out) return MC_E_INVAL;
  auto it = e->all.find(ticket);
  if (it == e->all.end()) return MC_E_NOTFOUND;
  *out = it->second->res;
  return it->second->res.done ? MC_OK : MC_E_STATE;
}

int mc_engine_release(mc_engine* e, uint64_t ticket) {
  if (!e) return MC_E_INVAL;
  auto it = e->all.find(ticket);
  if (it == e->all.end()) return MC_E_NOTFOUND;
  if (!it->second->res.done) return MC_E_STATE;
  delete it->second;
  e->all.erase(it);
  return MC_OK;
}

}  // extern "C"
