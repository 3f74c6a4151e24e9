// mc_engine.hip -- continuous-batching query server over the persistent engine.
//
// Queries (min_time or check(T) of a model) are submitted at any time.  A model's
// explored state stays on the device between its queries (a Resident): its visited set,
// sized for all of its states, its per-configuration least clocks and the threshold
// T_done up to which every state is in the set.  Every engine step (1) admits waiting
// queries in arrival order -- answering those the resident state covers (a count scan
// for check), continuing the exploration of those above T_done, and placing new models
// in the arena (evicting idle ones, least recently used first) -- (2) runs one
// persistent launch over the unfinished partitions of every active query; a partition
// explores at most `slice` super-step levels per launch while queries wait, saves its
// frontier and yields, so queries admitted later overlap with queries already on the
// device -- and (3) retires the queries whose partitions are all explored.  Each model
// has its own visited set, so a query's result is the same alone and in the mix.
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
// visited-set bytes per slot: the key words, then the parent and jump words
uint32_t slot_bytes_for(uint32_t W) { return 8u * W + 8u; }
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
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

// How a query is served.
enum Mode { kFresh = 0, kResume = 1, kCount = 2, kKnown = 3 };

struct Query;

// A model's explored state on the device.
struct Resident {
  uint64_t id = 0;
  std::string key;  // the descriptor, canonically
  ModelHost mh;
  std::vector<PartPlan> parts;  // partitions of an exploration from scratch
  size_t off = 0, bytes = 0;    // arena region
  size_t cfg_off = 0, seed_off = 0, pstate_off = 0, table_off = 0;
  uint64_t slots = 0;
  int slot_idx = -1;  // model slot: counters, clocks, descriptor
  bool explored = false;   // the set holds every state with clock <= T_done
  bool complete = false;   // ... every reachable state
  uint32_t T_done = 0;
  std::vector<uint32_t> tc;  // least terminal clocks after the last exploration
  uint64_t states = 0, levels = 0;
  Query* busy = nullptr;  // the query exploring the model now
  Query* counting = nullptr;  // a query answered from the set in the current step
  uint64_t last_used = 0;
};

struct Query {
  uint64_t ticket = 0;
  uint32_t kind = 0, T = 0;
  std::string key;
  ModelHost mh;              // until its Resident is created
  uint64_t resident = 0;     // the Resident's id
  int mode = kFresh;
  uint32_t n_parts = 0;      // partitions of its exploration
  uint64_t submit_ns = 0, admit_ns = 0, done_ns = 0;
  uint32_t steps = 0;
  mc_query_result res{};
  std::vector<uint32_t> argmin;
  bool has_target = false;   // trace target: (argmin[0], t_min)
};

// a query's configurations are cut into at most this many more partitions
constexpr size_t kExtraParts = 256;

// Arena bytes of a model: configuration records, seeds, one PartState per partition and
// a visited set for `states` states at load factor lf.
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

std::string model_key(const mc_desc* d) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
  put(&d->kind, 4);
  put(&d->n_cu, 4);
  put(d->size, 12);
  put(&d->lat_global, 16);
  put(&d->n_cfg, 4);
  put(d->params, 16ull * d->n_cfg);
  const uint32_t one = 1;
  for (uint32_t i = 0; i < d->n_cu; ++i) put(d->unit_speed ? &d->unit_speed[i] : &one, 4);
  return k;
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
         nyield_off = 0, head_off = 0, count_off = 0, arena_off = 0;
  Arena arena;
  uint64_t next_ticket = 1, next_resident = 1, clock = 0;
  std::deque<Query*> waiting;
  std::vector<Resident*> slots;  // model slot -> resident model
  std::unordered_map<std::string, Resident*> by_key;
  std::unordered_map<uint64_t, Resident*> by_id;
  std::unordered_map<uint64_t, Query*> all;
  std::vector<Part> pending_parts;  // partitions of the next launch (host side)
  int cur = 0;
  unsigned char* hctrl = nullptr;           // pinned
  uint32_t* htc = nullptr;                  // pinned
  unsigned int* hny = nullptr;              // pinned
  ModelDev* hmd = nullptr;                  // pinned staging of descriptors
  unsigned long long* hcount = nullptr;     // pinned
  uint64_t launches = 0;
  Fork fork;
};

namespace {

ModelDev make_dev(mc_engine* e, const Resident* r, const Query* q, uint32_t n_parts) {
  ModelDev d;
  std::memset(&d, 0, sizeof(d));
  unsigned char* g = e->base + e->arena_off + r->off;
  d.ctrl = reinterpret_cast<Ctrl*>(e->base + e->ctrl_off + kCtrlStride * r->slot_idx);
  d.tc = reinterpret_cast<uint32_t*>(e->base + e->tc_off + 4ull * e->opts.max_cfg * r->slot_idx);
  d.cfgs = reinterpret_cast<const CfgRec*>(g + r->cfg_off);
  d.seeds = reinterpret_cast<Seed*>(g + r->seed_off);
  d.table = g + r->table_off;
  d.mask = r->slots - 1;
  d.L = r->mh.layout;
  d.n_cfg = r->mh.n_cfg;
  d.prune = q->kind == MC_QUERY_CHECK ? 1u : 0u;
  d.T = q->T;
  d.max_clock = r->mh.max_clock;
  d.n_parts = n_parts;
  d.pstate = reinterpret_cast<PartState*>(g + r->pstate_off);
  // a continued exploration expands the states it finds again below T_done
  d.refloor = q->mode == kResume ? r->T_done + 1u : 0u;
  return d;
}

void drop_resident(mc_engine* e, Resident* r) {
  e->arena.release(r->off, r->bytes);
  if (r->slot_idx >= 0) e->slots[r->slot_idx] = nullptr;
  e->by_key.erase(r->key);
  e->by_id.erase(r->id);
  delete r;
}

int free_slot(const mc_engine* e) {
  for (size_t i = 0; i < e->slots.size(); ++i)
    if (!e->slots[i]) return (int)i;
  return -1;
}

// Places a new model: a slot and an arena region, evicting idle models (least recently
// used first) until both are free.  False if the busy models leave no room.
bool place(mc_engine* e, Resident* r) {
  for (;;) {
    int slot = free_slot(e);
    size_t off = 0;
    if (slot >= 0 && e->arena.alloc(r->bytes, &off)) {
      r->off = off;
      r->slot_idx = slot;
      e->slots[slot] = r;
      return true;
    }
    Resident* victim = nullptr;
    for (Resident* x : e->slots)
      if (x && !x->busy && !x->counting && (!victim || x->last_used < victim->last_used))
        victim = x;
    if (!victim) return false;
    drop_resident(e, victim);
  }
}

// The query's result from the model's least clocks (terminals within T for check).
void fill_result(Query* q, const std::vector<uint32_t>& tc) {
  const uint32_t lim = q->kind == MC_QUERY_CHECK ? q->T : kNoClock - 1u;
  uint32_t best = kNoClock;
  for (uint32_t c : tc)
    if (c <= lim) best = std::min(best, c);
  q->argmin.clear();
  if (best != kNoClock)
    for (uint32_t k = 0; k < (uint32_t)tc.size(); ++k)
      if (tc[k] == best) q->argmin.push_back(k);
  mc_query_result& res = q->res;
  res.t_min = best;
  res.n_argmin = (uint32_t)q->argmin.size();
  res.argmin_first = q->argmin.empty() ? kNoClock : q->argmin[0];
  res.violated = q->kind == MC_QUERY_CHECK && best != kNoClock ? 1 : 0;
  q->has_target = best != kNoClock;
}

void finish(mc_engine* e, Query* q) {
  q->done_ns = now_ns();
  q->res.submit_ns = q->submit_ns;
  q->res.admit_ns = q->admit_ns;
  q->res.done_ns = q->done_ns;
  q->res.steps = q->steps;
  q->res.reuse = q->mode == kFresh ? MC_REUSE_NONE
                 : q->mode == kResume ? MC_REUSE_RESUMED
                                      : MC_REUSE_ANSWERED;
  q->res.done = 1;
  (void)e;
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
  off = align_up(off + 8ull * o->max_active);
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
    e->count_off = off;
    off = align_up(off + 8ull * A);
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
        hipHostMalloc(reinterpret_cast<void**>(&e->hcount), 8ull * A, hipHostMallocDefault) !=
            hipSuccess ||
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
  for (auto& kv : e->by_id) delete kv.second;
  if (e->hctrl) (void)hipHostFree(e->hctrl);
  if (e->htc) (void)hipHostFree(e->htc);
  if (e->hny) (void)hipHostFree(e->hny);
  if (e->hmd) (void)hipHostFree(e->hmd);
  if (e->hcount) (void)hipHostFree(e->hcount);
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
    q->key = model_key(model);
    q->ticket = e->next_ticket++;
    q->submit_ns = now_ns();
    q->res.kind = kind;
    q->res.T = T;
    q->res.t_min = kNoClock;
    q->res.argmin_first = kNoClock;
    // a model needs room for all its states (any later query can reuse them), or with
    // no_reuse for the states this query inserts
    const uint64_t need = !e->opts.no_reuse || kind == MC_QUERY_MIN_TIME
                              ? q->mh.states
                              : count_le_bound(q->mh, T);
    uint64_t slots;
    size_t a, b, c, d;
    const size_t bytes = footprint(q->mh, need, q->mh.n_cfg + kExtraParts, e->opts.load_factor,
                                   &slots, &a, &b, &c, &d);
    if (bytes > e->arena.size() || q->mh.n_cfg > e->opts.max_cfg) {
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
  // ---- admission (arrival order) ----
  struct Start {
    Query* q;
    Resident* r;
    std::vector<PartPlan> plan;  // fresh or resumed exploration
  };
  std::vector<Start> starts;
  std::vector<Query*> counts;  // check queries answered by a scan of the set
  std::deque<Query*> still;
  bool blocked = false;  // a query needing new memory did not fit: later ones wait too
  bool wait_memory = false;  // some query waits for arena room or a model slot
  try {
    while (!e->waiting.empty()) {
      Query* q = e->waiting.front();
      e->waiting.pop_front();
      auto it = e->by_key.find(q->key);
      Resident* r = it == e->by_key.end() ? nullptr : it->second;
      if (r && (r->busy || r->counting)) {
        // a query the set already covers is answered while the model's previous query
        // continues the exploration past T_done: that exploration only adds states with
        // larger clocks (and a scan skips a slot whose key is still being written)
        const bool covered = r->explored && (r->complete || (q->kind == MC_QUERY_CHECK &&
                                                             q->T <= r->T_done));
        const bool resuming = !r->busy || r->busy->mode == kResume;
        if (covered && resuming && !r->counting) {
          q->resident = r->id;
          q->admit_ns = now_ns();
          r->last_used = ++e->clock;
          if (q->kind == MC_QUERY_MIN_TIME) {
            q->mode = kKnown;
            fill_result(q, r->tc);
            q->res.status = MC_OK;
            q->res.states = r->states;
            q->res.levels = r->levels;
            finish(e, q);
          } else {
            q->mode = kCount;
            r->counting = q;
            counts.push_back(q);
          }
          continue;
        }
        still.push_back(q);  // the model's previous query still runs
        continue;
      }
      if (!r) {
        if (blocked) {
          wait_memory = true;
          still.push_back(q);
          continue;
        }
        r = new Resident();
        r->id = e->next_resident++;
        r->key = q->key;
        r->mh = std::move(q->mh);
        // blocks of about states/256, with larger blocks while the plan has more than
        // kExtraParts partitions beyond one per configuration (whole configurations last)
        const uint32_t ps = e->opts.part_states;
        uint64_t target = ps == 0xFFFFFFFFu ? 0u
                          : ps              ? ps
                                            : std::max<uint64_t>(1, r->mh.states / kExtraParts);
        plan_parts(r->mh, target, &r->parts);
        while (target && r->parts.size() > (size_t)r->mh.n_cfg + kExtraParts) {
          target = target >= (1ull << 40) ? 0u : target * 4;
          r->parts.clear();
          plan_parts(r->mh, target, &r->parts);
        }
        std::stable_sort(r->parts.begin(), r->parts.end(),
                         [](const PartPlan& a, const PartPlan& b) { return a.states > b.states; });
        const uint64_t need = !e->opts.no_reuse || q->kind == MC_QUERY_MIN_TIME
                                  ? r->mh.states
                                  : count_le_bound(r->mh, q->T);
        r->bytes = footprint(r->mh, need, std::max<size_t>(r->parts.size(), r->mh.n_cfg),
                             e->opts.load_factor, &r->slots, &r->cfg_off, &r->seed_off,
                             &r->pstate_off, &r->table_off);
        if (!place(e, r)) {
          q->mh = std::move(r->mh);
          delete r;
          blocked = wait_memory = true;
          still.push_back(q);
          continue;
        }
        e->by_key[r->key] = r;
        e->by_id[r->id] = r;
        HIPCHK(hipMemcpyAsync(e->base + e->arena_off + r->off + r->cfg_off, r->mh.cfgs.data(),
                              sizeof(CfgRec) * r->mh.n_cfg, hipMemcpyHostToDevice, s));
      }
      q->resident = r->id;
      q->admit_ns = now_ns();
      r->last_used = ++e->clock;
      const bool covered = r->explored && (r->complete || (q->kind == MC_QUERY_CHECK &&
                                                           q->T <= r->T_done));
      if (covered && q->kind == MC_QUERY_MIN_TIME) {
        q->mode = kKnown;
        fill_result(q, r->tc);
        q->res.status = MC_OK;
        q->res.states = r->states;
        q->res.levels = r->levels;
        finish(e, q);
        continue;
      }
      if (covered) {
        q->mode = kCount;
        r->counting = q;
        counts.push_back(q);
        continue;
      }
      r->busy = q;
      if (r->explored && resumable(r->mh)) {
        q->mode = kResume;
        Start st{q, r, {}};
        plan_resume(r->mh, r->T_done, r->parts, &st.plan);
        starts.push_back(std::move(st));
      } else {
        q->mode = kFresh;
        starts.push_back(Start{q, r, r->parts});
      }
    }
  } catch (const std::bad_alloc&) {
    for (Query* q : still) e->waiting.push_back(q);
    return MC_E_NOMEM;
  }
  e->waiting.swap(still);
  // ---- device work of the admitted queries ----
  if (!starts.empty()) {
    std::vector<ModelDev> fresh_md, resume_md;
    std::vector<int> fresh_slot, resume_slot;
    for (Start& st : starts) {
      Query* q = st.q;
      Resident* r = st.r;
      q->n_parts = (uint32_t)st.plan.size();
      const ModelDev md = make_dev(e, r, q, q->n_parts);
      if (q->mode == kFresh) {
        // units alike clear the keys only (their links are read only where written)
        HIPCHK(launch_clear(s, e->base + e->arena_off + r->off + r->table_off,
                            r->slots * (r->mh.hetero ? slot_bytes_for(r->mh.W) : 8ull * r->mh.W)));
        fresh_md.push_back(md);
        fresh_slot.push_back(r->slot_idx);
      } else {
        resume_md.push_back(md);
        resume_slot.push_back(r->slot_idx);
      }
      for (size_t k = 0; k < st.plan.size(); ++k) {
        const PartPlan& pp = st.plan[k];
        e->pending_parts.push_back(
            Part{(uint32_t)r->slot_idx, pp.cfg, pp.r0, pp.r1, (uint32_t)k, pp.j0, pp.j1, 0u});
      }
    }
    // descriptors: staged through pinned memory, then copied to their model slots
    const auto upload = [&](const std::vector<ModelDev>& mds, const std::vector<int>& sl) -> int {
      if (mds.empty()) return MC_OK;
      std::memcpy(e->hmd, mds.data(), sizeof(ModelDev) * mds.size());
      HIPCHK(hipMemcpyAsync(e->base + e->stage_off, e->hmd, sizeof(ModelDev) * mds.size(),
                            hipMemcpyHostToDevice, s));
      for (size_t i = 0; i < mds.size(); ++i)
        HIPCHK(hipMemcpyAsync(e->base + e->md_off + sizeof(ModelDev) * sl[i],
                              e->base + e->stage_off + sizeof(ModelDev) * i, sizeof(ModelDev),
                              hipMemcpyDeviceToDevice, s));
      return MC_OK;
    };
    const ModelDev* stage = reinterpret_cast<const ModelDev*>(e->base + e->stage_off);
    int rc = upload(fresh_md, fresh_slot);
    if (rc) return rc;
    if (!fresh_md.empty()) {
      HIPCHK(launch_reset_models(s, stage, (uint32_t)fresh_md.size(), nullptr, 0));
      HIPCHK(launch_seed_models(s, stage, (uint32_t)fresh_md.size()));
    }
    // the pinned staging is reused: the copies above must have run
    HIPCHK(hipStreamSynchronize(s));
    rc = upload(resume_md, resume_slot);
    if (rc) return rc;
    if (!resume_md.empty())
      HIPCHK(launch_resume_models(s, stage, (uint32_t)resume_md.size(), nullptr, 0));
    HIPCHK(hipStreamSynchronize(s));
  }
  // counts of check queries answered from a resident set: states with clock <= T
  for (Query* q : counts) {
    Resident* r = e->by_id[q->resident];
    unsigned long long* out =
        reinterpret_cast<unsigned long long*>(e->base + e->count_off) + r->slot_idx;
    HIPCHK(hipMemsetAsync(out, 0, 8, s));
    const unsigned char* table = e->base + e->arena_off + r->off + r->table_off;
    const CfgRec* cfgs = reinterpret_cast<const CfgRec*>(e->base + e->arena_off + r->off +
                                                         r->cfg_off);
    hipError_t he;
    switch (r->mh.W) {
      case 1: he = launch_count_le<1>(s, table, r->slots, r->mh.layout, cfgs, q->T, out); break;
      case 2: he = launch_count_le<2>(s, table, r->slots, r->mh.layout, cfgs, q->T, out); break;
      default: he = launch_count_le<4>(s, table, r->slots, r->mh.layout, cfgs, q->T, out); break;
    }
    HIPCHK(he);
  }
  // ---- one persistent launch over every unfinished partition ----
  bool any_active = false;
  uint32_t hi = 0;  // one past the highest slot in use
  for (size_t i = 0; i < e->slots.size(); ++i) {
    if (e->slots[i] && e->slots[i]->busy) any_active = true;
    if (e->slots[i] && (e->slots[i]->busy || e->slots[i]->counting)) hi = (uint32_t)i + 1u;
  }
  // partitions are cut into slices only while queries wait for memory to be admitted:
  // otherwise the launch runs everything admitted to the end, with no host round trip
  // per slice (a query waiting for its model's running query gains nothing from slices)
  const uint32_t slice = wait_memory ? e->opts.slice : 0u;
  const bool launch = any_active && !e->pending_parts.empty();
  if (launch) {
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
  }
  if (hi) {
    HIPCHK(hipMemcpyAsync(e->hctrl, e->base + e->ctrl_off, kCtrlStride * hi, hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipMemcpyAsync(e->htc, e->base + e->tc_off, 4ull * e->opts.max_cfg * hi,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(e->hcount, e->base + e->count_off, 8ull * hi, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (Resident* r : e->slots)
    if (r && r->busy) ++r->busy->steps;
  if (launch) {
    // partitions that yielded continue in the next launch
    const uint32_t nyield = *e->hny;
    e->pending_parts.resize(nyield);
    if (nyield)
      HIPCHK(hipMemcpy(e->pending_parts.data(),
                       e->base + e->parts_off[e->cur ^ 1], sizeof(Part) * nyield,
                       hipMemcpyDeviceToHost));
  }
  // ---- retire finished queries ----
  for (size_t i = 0; i < e->slots.size(); ++i) {
    Resident* r = e->slots[i];
    if (!r || !r->counting) continue;
    Query* q = r->counting;
    fill_result(q, r->tc);  // terminals within T <= T_done: those of the resident clocks
    q->res.status = MC_OK;
    q->res.states = e->hcount[i];
    q->res.levels = 0;  // not known without exploring
    finish(e, q);
    r->counting = nullptr;
  }
  for (size_t i = 0; i < e->slots.size(); ++i) {
    Resident* r = e->slots[i];
    if (!r || !r->busy) continue;
    Query* q = r->busy;
    const Ctrl* c = reinterpret_cast<const Ctrl*>(e->hctrl + kCtrlStride * i);
    const uint32_t* tc = e->htc + (size_t)e->opts.max_cfg * i;
    mc_query_result& res = q->res;
    const bool failed = c->error != 0u;
    if (c->parts_done < q->n_parts && !failed) continue;
    res.status = dev_error_code(c->error);
    res.states = c->states;
    res.levels = c->max_depth + 1;
    r->tc.assign(tc, tc + r->mh.n_cfg);
    fill_result(q, r->tc);
    finish(e, q);
    r->busy = nullptr;
    if (failed || e->opts.no_reuse) {
      // drop any partition of the model still queued; its set is not kept
      std::vector<Part> keep;
      for (const Part& p : e->pending_parts)
        if (p.model != (uint32_t)i) keep.push_back(p);
      e->pending_parts.swap(keep);
      drop_resident(e, r);
      continue;
    }
    r->explored = true;
    r->states = c->states;
    r->levels = c->max_depth + 1;
    if (q->kind == MC_QUERY_MIN_TIME) {
      r->complete = true;
    } else {
      r->T_done = std::max(r->T_done, q->T);
      // every terminal within T_done: nothing is left to explore
      uint32_t last = 0;
      for (uint32_t k = 0; k < r->mh.n_cfg; ++k) last = std::max(last, r->mh.cfgs[k].tc);
      r->complete = !r->mh.hetero && last <= r->T_done;
    }
  }
  uint32_t na = 0;
  for (Resident* r : e->slots) na += r && r->busy;
  if (e->opts.no_reuse)  // nothing is kept: every idle model is dropped
    for (Resident* r : e->slots)
      if (r && !r->busy && !r->counting) drop_resident(e, r);
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

int mc_engine_argmin(mc_engine* e, uint64_t ticket, uint32_t* argmin, size_t cap, size_t* n) {
  if (!e || !n || (cap && !argmin)) return MC_E_INVAL;
  auto it = e->all.find(ticket);
  if (it == e->all.end()) return MC_E_NOTFOUND;
  const Query* q = it->second;
  if (!q->res.done) return MC_E_STATE;
  *n = q->argmin.size();
  const size_t k = std::min(cap, q->argmin.size());
  if (k) std::memcpy(argmin, q->argmin.data(), 4 * k);
  return cap < q->argmin.size() && argmin ? MC_E_BUFFER : MC_OK;
}

}  // extern "C"

namespace {

template <int W>
int engine_trace_w(mc_engine* e, Resident* r, uint32_t cfg, uint32_t clock,
                   std::vector<uint32_t>* rows) {
  hipStream_t s = e->stream;
  const size_t cap = r->mh.max_depth + 2;
  size_t off = 0;
  if (!e->arena.alloc(8ull * W * cap, &off)) return MC_E_NOMEM;
  unsigned long long* buf = reinterpret_cast<unsigned long long*>(e->base + e->arena_off + off);
  unsigned char* g = e->base + e->arena_off + r->off;
  QueryArgs q;
  std::memset(&q, 0, sizeof(q));
  q.ctrl = reinterpret_cast<Ctrl*>(e->base + e->ctrl_off + kCtrlStride * r->slot_idx);
  q.tc = reinterpret_cast<uint32_t*>(e->base + e->tc_off + 4ull * e->opts.max_cfg * r->slot_idx);
  q.cfgs = reinterpret_cast<const CfgRec*>(g + r->cfg_off);
  q.table = g + r->table_off;
  q.mask = r->slots - 1;
  q.L = r->mh.layout;
  q.n_cfg = r->mh.n_cfg;
  q.max_clock = r->mh.max_clock;
  uint32_t fields[kFields] = {0};
  fields[kFCfg] = cfg;
  fields[kFClock] = clock;
  uint64_t words[4];
  encode_key_host(r->mh.layout, fields, words);
  int rc = MC_OK;
  Ctrl* hc = reinterpret_cast<Ctrl*>(e->hctrl);
  std::vector<uint64_t> keys;
  if (launch_find<W>(s, q, reinterpret_cast<const unsigned long long*>(words)) != hipSuccess ||
      launch_chase<W>(s, q, buf, (uint32_t)cap) != hipSuccess ||
      hipMemcpyAsync(hc, q.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    rc = MC_E_DEVICE;
  } else if (hc->target_slot == kParentNone) {
    rc = MC_E_STATE;
  } else if (hc->error == kDevErrTrace) {
    rc = MC_E_DEVICE;
  } else {
    const uint32_t n = hc->trace_len;
    keys.resize((size_t)n * W);
    if (n && (hipMemcpy(keys.data(), buf, 8ull * W * n, hipMemcpyDeviceToHost) != hipSuccess)) {
      (void)hipGetLastError();
      rc = MC_E_DEVICE;
    }
    const uint32_t m = r->mh.m, S = 3 + m;
    rows->assign((size_t)n * S, 0);
    for (uint32_t i = 0; rc == MC_OK && i < n; ++i) {
      uint64_t w[4] = {0, 0, 0, 0};
      for (int j = 0; j < W; ++j) w[j] = keys[(size_t)(n - 1 - i) * W + j];
      uint32_t f[kFields];
      decode_key_host(r->mh.layout, w, f, r->mh.cfgs.data());
      uint32_t* row = &(*rows)[(size_t)i * S];
      row[0] = f[kFCfg] == r->mh.n_cfg ? 0xFFFFFFFFu : f[kFCfg];
      row[1] = f[kFClock];
      row[2] = f[kFPending];
      for (uint32_t u = 0; u < m; ++u) row[3 + u] = f[kFRem + u];
    }
  }
  e->arena.release(off, 8ull * W * cap);
  return rc;
}

}  // namespace

extern "C" {

int mc_engine_trace(mc_engine* e, uint64_t ticket, uint32_t* rows, size_t cap, size_t* len) {
  if (!e || !len || (cap && !rows)) return MC_E_INVAL;
  auto it = e->all.find(ticket);
  if (it == e->all.end()) return MC_E_NOTFOUND;
  const Query* q = it->second;
  if (!q->res.done || q->res.status != MC_OK || !q->has_target) return MC_E_STATE;
  auto rt = e->by_id.find(q->resident);
  if (rt == e->by_id.end() || rt->second->busy || rt->second->counting) return MC_E_STATE;
  Resident* r = rt->second;
  std::vector<uint32_t> out;
  int rc;
  try {
    switch (r->mh.W) {
      case 1: rc = engine_trace_w<1>(e, r, q->argmin[0], q->res.t_min, &out); break;
      case 2: rc = engine_trace_w<2>(e, r, q->argmin[0], q->res.t_min, &out); break;
      default: rc = engine_trace_w<4>(e, r, q->argmin[0], q->res.t_min, &out); break;
    }
  } catch (...) {
    return MC_E_NOMEM;
  }
  if (rc) return rc;
  const size_t S = 3 + r->mh.m, n = out.size() / S;
  *len = n;
  if (cap < n) return rows ? MC_E_BUFFER : MC_OK;
  if (n) std::memcpy(rows, out.data(), 4 * out.size());
  return MC_OK;
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
