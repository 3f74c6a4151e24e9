// mc_api.hip -- the C ABI: workspace planning, model load, query drivers (min_time,
// check(T), bisection), counterexample decoding and simulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mctune.h"
#include "mc_host_pool.h"
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

struct WsPlan {
  size_t ctrl = 0, tc = 0, cfgs = 0, order = 0, seeds = 0, front0 = 0, front1 = 0, trace = 0,
         table = 0, total = 0, md = 0, head = 0;
  uint64_t slots = 0;
  uint32_t slot_bytes = 0;
  uint64_t fcap = 0;
  uint64_t trace_cap = 0;
  size_t table_bytes = 0;
  uint64_t n_parts = 0;
};

// visited-set bytes per slot: the key words, then the parent and jump words
uint32_t slot_bytes_for(uint32_t W) { return 8u * W + 8u; }

// Slots for `states` keys at the given load factor, rounded up to a power of two.  The
// automatic target (load_factor 0) is 3/8: a large single query is bound by the rate of
// random compare-and-swaps, and keeping the final load under 3/8 (rather than 1/2) cuts
// the probes per insert by more than the larger table costs to clear (58M states: 1.38 ->
// 1.14 probes per state, min_time launch 4.88 -> 4.27 ms, clear 0.46 -> 0.79 ms); it
// falls back to 1/2 where 3/8 would pass the 2^31-slot limit of the 32-bit slot links.
uint64_t table_slots(uint64_t states, float load_factor) {
  if (load_factor > 0.f && load_factor < 1.f)
    return next_pow2((uint64_t)((double)states / load_factor) + 1);
  const uint64_t s = next_pow2((uint64_t)((double)states / 0.375) + 1);
  return s <= (1ull << 31) ? s : next_pow2(2 * states + 1);
}

// Failed claims of an exploration: every insert ends on one deciding probe (a claim or
// its own key found), the others met a slot holding another state.
uint64_t cas_fails(uint64_t probes, uint64_t states, uint64_t dups) {
  return probes > states + dups ? probes - states - dups : 0u;
}

int plan_ws(const ModelHost& mh, const mc_opts& o, uint64_t n_parts, WsPlan* p) {
  if (o.test_hash_bits > 24u) return MC_E_INVAL;
  uint64_t slots;
  if (o.log2_slots) {
    if (o.log2_slots < 4 || o.log2_slots > 31) return MC_E_INVAL;
    slots = 1ull << o.log2_slots;
  } else {
    slots = std::max<uint64_t>(table_slots(mh.states, o.load_factor), 1024);
    if (slots > (1ull << 31)) return MC_E_INVAL;
  }
  const uint32_t W = mh.W;
  const size_t entry = 8ull * W + 8ull;
  // the visited set first: it starts at the same place for every model, so a handle that
  // loads another model knows which of its bytes are still cleared
  p->slots = slots;
  p->slot_bytes = slot_bytes_for(W);
  p->table = 0;
  p->table_bytes = (size_t)slots * p->slot_bytes;
  size_t off = align_up(p->table_bytes);
  p->ctrl = off;   off = align_up(off + sizeof(Ctrl));
  p->tc = off;     off = align_up(off + 4ull * mh.n_cfg);
  p->cfgs = off;   off = align_up(off + sizeof(CfgRec) * mh.n_cfg);
  p->n_parts = n_parts;
  p->order = off;  off = align_up(off + sizeof(Part) * n_parts);
  p->md = off;     off = align_up(off + sizeof(ModelDev));
  p->head = off;   off = align_up(off + 4);
  p->seeds = off;  off = align_up(off + sizeof(Seed) * mh.n_cfg);
  p->fcap = mh.frontier_bound + 64;
  p->front0 = off; off = align_up(off + entry * p->fcap);
  p->front1 = off; off = align_up(off + entry * p->fcap);
  p->trace_cap = mh.max_depth + 2;
  p->trace = off;  off = align_up(off + 8ull * W * p->trace_cap);
  p->total = off;
  return MC_OK;
}

constexpr uint32_t kWideParts = 256;
// With thousands of partitions in flight a lane inserts one key per round trip: on
// matmul128_vw_cu8 (3,828 partitions) two keys per lane took 8.4 ms against 6.5 ms with
// one; on matmul64_cu4 (376 partitions) two keys per lane stay ahead (0.48 vs 0.50 ms).
constexpr uint32_t kManyParts = 2048;

mc_opts default_opts(const mc_opts* o) {
  mc_opts r;
  std::memset(&r, 0, sizeof(r));
  if (o) r = *o;
  if (r.block != 256 && r.block != 512 && r.block != 1024) r.block = 0;  // chosen at load
  if (r.engine > MC_ENGINE_LEVEL) r.engine = MC_ENGINE_SUPERSTEP;
  if (r.lane_items > 2) r.lane_items = 0;
  return r;
}

// Partitions of a single-model query, largest expected block first.
std::vector<Part> model_parts(const ModelHost& mh, const mc_opts& o) {
  const uint64_t target = o.part_states == 0xFFFFFFFFu ? 0u
                          : o.part_states              ? o.part_states
                                                       : auto_part_states(mh.states, mh.m);
  std::vector<PartPlan> plan;
  plan_parts(mh, target, &plan);
  std::stable_sort(plan.begin(), plan.end(),
                   [](const PartPlan& a, const PartPlan& b) { return a.states > b.states; });
  std::vector<Part> parts(plan.size());
  for (size_t i = 0; i < plan.size(); ++i)
    parts[i] = Part{0u, plan[i].cfg, plan[i].r0, plan[i].r1, (uint32_t)i, plan[i].j0, plan[i].j1, 0u};
  return parts;
}

#define HIPCHK(x)                      \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) {            \
      (void)hipGetLastError();         \
      return MC_E_DEVICE;              \
    }                                  \
  } while (0)

// Timing events are optional: a handle bound to the static scratch has none (it creates
// no runtime objects), and its stats then carry host wall-clock times only.
hipError_t ev_record(hipEvent_t e, hipStream_t s) { return e ? hipEventRecord(e, s) : hipSuccess; }
hipError_t ev_ms(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = 0.f;
  return a && b ? hipEventElapsedTime(ms, a, b) : hipSuccess;
}

}  // namespace

enum { kQueryNone = 0, kQueryMin = 1, kQueryCheck = 2 };

struct mc_model {
  ModelHost mh;
  mc_opts opts{};
  WsPlan plan;
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  Ctrl* ctrl = nullptr;
  uint32_t* tc = nullptr;
  CfgRec* cfgs = nullptr;
  Part* parts = nullptr;
  uint32_t n_parts = 0;  // partitions of the load's plan (the capacity of `parts`)
  uint32_t q_parts = 0;  // partitions of the last query's launch
  ModelDev* dmd = nullptr;
  unsigned int* head = nullptr;
  unsigned char* pin = nullptr;  // pooled pinned block: hctrl, hpoll, hmd, tc_host, uploads
  size_t pin_bytes = 0;
  ModelDev* hmd = nullptr;  // pinned host staging of the device descriptor
  Seed* seeds = nullptr;
  unsigned char* front[2] = {nullptr, nullptr};
  unsigned long long* trace_buf = nullptr;
  unsigned char* table = nullptr;
  Ctrl* hctrl = nullptr;  // pinned host copy
  uint32_t* hpoll = nullptr;
  // stop request of mc_abort: a pinned host word the kernels read at system scope; the
  // query that returns MC_E_ABORTED clears it
  unsigned int* habort = nullptr;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // Clearing the visited set.  Bytes [0, dirty_in) of the table may hold an earlier
  // query's data; the rest of [0, max_need) is cleared (empty slots) once the side
  // stream's clear, if one is pending, has ended.  max_need: the most a query of this model
  // needs cleared (every key; with units of unequal speed every slot).  A query clears what
  // it needs of the dirty prefix on the handle's stream, and once its results are on their
  // way hands the dirty bytes past those it touched to the side stream (pooled handles),
  // which clears them while the host reads the results and loads the next query.
  uint64_t dirty_in = 0, max_need = 0;
  uint64_t behind_lo = 0, behind_hi = 0;  // the current query's bytes to clear behind it
  uint64_t side_hi = 0;                    // end of the side stream's pending clear
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_side = nullptr;
  bool side_pending = false;
  mc_opts opts_in{};  // the options given at load: a reload derives its own from them
  size_t ws_bytes = 0;
  int last = kQueryNone;
  uint32_t last_T = 0;
  int last_violated = 0;
  uint32_t* tc_host = nullptr;  // pinned, n_cfg entries
  // last swarm: member records in the visited-set region, the best trail's walk
  uint32_t swarm_members = 0, swarm_bits_log2 = 10;
  bool swarm_best = false;
  unsigned long long swarm_best_seed = 0, swarm_best_start = 0;
  uint64_t q_slots = 0;          // visited-set slots of the last query (a prefix of the table)
  bool trace_ready = false;
  std::vector<uint32_t> trace_rows;
  // the visited set holds every state with clock <= resident_T (an incremental
  // bisection's pruned exploration), which run_resume continues
  bool resident = false;
  uint32_t resident_T = 0;
  std::vector<Part> parts_host;  // the load's partition plan (run_resume overwrites parts)
  bool parts_resumed = false;
  // unpooled binding (the static scratch): host staging in ordinary memory, no events
  bool pooled = true;
  std::vector<unsigned char> host_stage;
};

namespace {

QueryArgs make_args(mc_model* h, bool prune, uint32_t T) {
  QueryArgs q;
  q.ctrl = h->ctrl;
  q.tc = h->tc;
  q.cfgs = h->cfgs;
  q.table = h->table;
  q.mask = h->q_slots - 1;
  q.L = h->mh.layout;
  q.n_cfg = h->mh.n_cfg;
  q.prune = prune ? 1u : 0u;
  q.T = T;
  q.max_clock = h->mh.max_clock;
  q.hkeep = h->opts.test_hash_bits;
  return q;
}

// Bytes of the table a query with q slots needs cleared (its keys; with units of unequal
// speed its links too), and the bytes it may write (keys and links), within max_need.
uint64_t need_bytes(const mc_model* h, uint64_t q) {
  return q * (h->mh.hetero ? (uint64_t)h->plan.slot_bytes : 8ull * h->mh.W);
}
uint64_t touched_bytes(const mc_model* h, uint64_t q) {
  return std::min<uint64_t>(q * h->plan.slot_bytes, h->max_need);
}

// Orders the handle's stream after the side stream's clear, if one is in flight: every
// use that may touch the table or the regions after it (a query, a swarm, a reload's
// uploads) calls this first.
hipError_t join_side(mc_model* h) {
  if (!h->side_pending) return hipSuccess;
  h->side_pending = false;
  return hipStreamWaitEvent(h->stream, h->ev_side, 0);
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // unknown: keep to the one stream
  }
  return st != hipStreamCaptureStatusNone;
}

// Before a query whose visited set has q slots: clears the dirty part of what it needs on
// the handle's stream (between events ev[0] and ev[1]; *cleared says whether it did), and
// notes the dirty bytes past what it touches, which finish_query hands to the side stream.
int prepare_table(mc_model* h, uint64_t q, bool* cleared) {
  hipStream_t s = h->stream;
  HIPCHK(join_side(h));
  const uint64_t need = need_bytes(h, q), touched = touched_bytes(h, q);
  const uint64_t now = std::min<uint64_t>(need, h->dirty_in);
  h->behind_lo = h->behind_hi = 0;
  if (h->dirty_in > touched && h->side && !capturing(s)) {
    h->behind_lo = touched;
    h->behind_hi = h->dirty_in;
  }
  *cleared = now > 0;
  if (now) {
    HIPCHK(ev_record(h->ev[0], s));
    HIPCHK(launch_clear(s, h->table, now));
    HIPCHK(ev_record(h->ev[1], s));
  }
  h->dirty_in = std::max<uint64_t>(h->dirty_in, touched);  // what the query will write
  return MC_OK;
}

// After a query's launches and the copies of its results: clears the dirty bytes past the
// ones it touched on the side stream.  Started there rather than beside the query, the
// clear's workgroups do not hold back the query's own (a latency-bound launch) or its
// result copies; it runs while the host reads the results and prepares the next query.
int clear_behind(mc_model* h) {
  if (h->behind_hi <= h->behind_lo) return MC_OK;
  const uint64_t lo = h->behind_lo, hi = h->behind_hi;
  h->behind_lo = h->behind_hi = 0;
  HIPCHK(hipEventRecord(h->ev_fork, h->stream));
  HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  HIPCHK(launch_clear(h->side, h->table + lo, hi - lo));
  HIPCHK(hipEventRecord(h->ev_side, h->side));
  h->side_pending = true;
  h->side_hi = hi;
  h->dirty_in = lo;  // [lo, hi) is the side stream's; past hi it was cleared already
  return MC_OK;
}

template <int W>
int level_loop(mc_model* h, const QueryArgs& q, uint64_t* launches);

template <int W>
int explore_w(mc_model* h, const QueryArgs& q, uint64_t* launches) {
  hipStream_t s = h->stream;
  HIPCHK(launch_seed<W>(s, q, h->seeds, h->front[0]));
  *launches = 1;
  HIPCHK(ev_record(h->ev[4], s));
  const int rc = level_loop<W>(h, q, launches);
  HIPCHK(ev_record(h->ev[5], s));
  return rc;
}

template <int W>
int level_loop(mc_model* h, const QueryArgs& q, uint64_t* launches) {
  hipStream_t s = h->stream;
  // plain level-synchronous BFS: one launch per level; the frontier size lives on the
  // device, the host polls it once per batch of launches
  const uint64_t fcap = h->plan.fcap;
  uint32_t grid = (uint32_t)std::min<uint64_t>((fcap + kLevelBlock - 1) / kLevelBlock, 256);
  grid = std::max<uint32_t>(grid, 1);
  LevelArgs la;
  la.q = q;
  la.fcap = (uint32_t)fcap;
  la.abort = h->habort;
  const uint64_t limit = h->mh.max_depth + 64;
  const uint32_t batch = 64;
  uint64_t L = 0;
  for (;;) {
    for (uint32_t b = 0; b < batch; ++b, ++L) {
      la.in_idx = (uint32_t)(L % 3);
      la.out_idx = (uint32_t)((L + 1) % 3);
      la.clr_idx = (uint32_t)((L + 2) % 3);
      HIPCHK(launch_level<W>(s, grid, la, h->front[L % 2], h->front[(L + 1) % 2]));
    }
    *launches += batch;
    HIPCHK(hipMemcpyAsync(h->hpoll, &h->ctrl->fcount[L % 3], 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h->hpoll + 1, &h->ctrl->error, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->hpoll[0] == 0 || h->hpoll[1] != 0) break;
    if (L > limit) return MC_E_OVERFLOW;
  }
  return MC_OK;
}

int finish_query(mc_model* h, std::chrono::steady_clock::time_point t0, bool cleared,
                 uint64_t launches, mc_stats* st);

// prune: drop states with clock > T.  bb (super-step engine): branch and bound, the
// threshold falls to the least terminal clock found so far and partitions are taken
// smallest first.
int run_query(mc_model* h, bool prune, uint32_t T, mc_stats* st, bool bb = false,
              uint32_t T_size = 0) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = h->stream;
  h->trace_ready = false;
  h->last = kQueryNone;
  h->swarm_members = 0;  // the visited set overwrites a swarm's records
  // a check(T) inserts only the states with clock <= T: its visited set is the prefix of
  // the table sized for their number at the same load factor
  uint64_t q_slots = h->plan.slots;
  if (prune && !h->opts.log2_slots) {
    const uint64_t need = count_le_bound(h->mh, std::max(T, T_size));
    q_slots = std::min<uint64_t>(h->plan.slots,
                                 std::max<uint64_t>(1024, table_slots(need, h->opts.load_factor)));
  }
  h->q_slots = q_slots;
  h->resident = false;
  // A check(T) explores only the states with clock <= T.  The load's plan cuts
  // configurations into blocks sized for the whole exploration, so one block can hold most
  // of what a check explores and decide its time alone; on models cut into round blocks a
  // check gets its own plan, sized for the states up to T, without the blocks that start
  // past T.
  uint32_t n_parts = h->n_parts;
  bool own_plan = false;
  if (prune && !bb && h->opts.engine == MC_ENGINE_SUPERSTEP && h->opts.part_states == 0 &&
      !h->mh.hetero && word0_orders_rounds(h->mh)) {
    std::vector<PartPlan> keep;
    plan_parts(h->mh, auto_part_states(count_le_bound(h->mh, T), h->mh.m), &keep, T);
    if (keep.size() <= h->n_parts) {
      std::stable_sort(keep.begin(), keep.end(), [](const PartPlan& a, const PartPlan& b) {
        return a.states > b.states;
      });
      std::vector<Part> parts(keep.size());
      for (size_t i = 0; i < keep.size(); ++i)
        parts[i] = Part{0u, keep[i].cfg, keep[i].r0, keep[i].r1, (uint32_t)i, keep[i].j0,
                        keep[i].j1, 0u};
      if (!parts.empty())
        HIPCHK(hipMemcpyAsync(h->parts, parts.data(), sizeof(Part) * parts.size(),
                              hipMemcpyHostToDevice, s));
      n_parts = (uint32_t)parts.size();
      own_plan = true;
      h->parts_resumed = true;  // the load's plan goes back before the next other query
    }
  }
  if (!own_plan && h->parts_resumed) {
    HIPCHK(hipMemcpyAsync(h->parts, h->parts_host.data(), sizeof(Part) * h->parts_host.size(),
                          hipMemcpyHostToDevice, s));
    h->parts_resumed = false;
  }
  h->q_parts = n_parts;
  // units alike need their keys cleared only (their links are read only where written)
  bool cleared = false;
  if (const int prc = prepare_table(h, h->q_slots, &cleared)) return prc;
  const QueryArgs q = make_args(h, prune, T);
  uint64_t launches = 0;
  int rc = MC_OK;
  if (h->opts.engine == MC_ENGINE_SUPERSTEP) {
    ModelDev& md = *h->hmd;
    md.ctrl = h->ctrl;
    md.tc = h->tc;
    md.cfgs = h->cfgs;
    md.seeds = h->seeds;
    md.table = h->table;
    md.mask = h->q_slots - 1;
    md.L = h->mh.layout;
    md.n_cfg = h->mh.n_cfg;
    md.prune = prune ? 1u : 0u;
    md.T = T;
    md.max_clock = h->mh.max_clock;
    md.n_parts = n_parts;
    md.bb = bb ? 1u : 0u;
    md.pstate = nullptr;
    md.hkeep = h->opts.test_hash_bits;
    md.refloor = 0u;
    HIPCHK(hipMemcpyAsync(h->dmd, h->hmd, sizeof(ModelDev), hipMemcpyHostToDevice, s));
    HIPCHK(launch_reset_models(s, h->dmd, 1, h->head, 1));
    HIPCHK(ev_record(h->ev[2], s));
    HIPCHK(launch_seed_models(s, h->dmd, 1));
    HIPCHK(ev_record(h->ev[4], s));
    PartQueue pq;
    pq.models = h->dmd;
    pq.parts = h->parts;
    pq.n_parts = n_parts;
    const uint32_t li = h->opts.lane_items || n_parts < kManyParts
                            ? lane_items_for(h->opts.lane_items, h->mh.W)
                            : 1u;
    pq.batch_items = h->opts.batch_items ? h->opts.batch_items : 2u * li * h->opts.block;
    pq.head = h->head;
    pq.slice = 0u;
    pq.reverse = bb ? 1u : 0u;
    pq.yielded = nullptr;
    pq.n_yielded = nullptr;
    pq.abort = h->habort;
    const uint32_t grid =
        h->opts.grid ? h->opts.grid : std::max<uint32_t>(1u, std::min<uint32_t>(n_parts, 4096u));
    HIPCHK(launch_super(s, h->mh.W, grid, h->opts.block, li, pq, h->mh.general, h->mh.hetero));
    HIPCHK(ev_record(h->ev[5], s));
    launches = 2;
  } else {
    HIPCHK(launch_reset(s, h->ctrl, h->tc, h->mh.n_cfg));
    HIPCHK(ev_record(h->ev[2], s));
    switch (h->mh.W) {
      case 1: rc = explore_w<1>(h, q, &launches); break;
      case 2: rc = explore_w<2>(h, q, &launches); break;
      default: rc = explore_w<4>(h, q, &launches); break;
    }
  }
  if (rc != MC_OK) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  return finish_query(h, t0, cleared, launches, st);
}

// Waits for a query's launches and reads its counters and clocks back.
int finish_query(mc_model* h, std::chrono::steady_clock::time_point t0, bool cleared,
                 uint64_t launches, mc_stats* st) {
  hipStream_t s = h->stream;
  HIPCHK(ev_record(h->ev[3], s));
  HIPCHK(hipMemcpyAsync(h->hctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(h->tc_host, h->tc, 4ull * h->mh.n_cfg, hipMemcpyDeviceToHost, s));
  if (const int crc = clear_behind(h)) return crc;
  HIPCHK(hipStreamSynchronize(s));
  const int derr = dev_error_code(h->hctrl->error);
  if (derr == MC_E_ABORTED && h->habort) __atomic_store_n(h->habort, 0u, __ATOMIC_RELEASE);
  if (derr != MC_OK) return derr;
  float ms_explore = 0.f, ms_clear = 0.f, ms_engine = 0.f;
  HIPCHK(ev_ms(&ms_explore, h->ev[2], h->ev[3]));
  HIPCHK(ev_ms(&ms_engine, h->ev[4], h->ev[5]));
  if (cleared) HIPCHK(ev_ms(&ms_clear, h->ev[0], h->ev[1]));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->states = h->hctrl->states;
    st->levels = h->hctrl->max_depth + 1;
    st->terminals = h->hctrl->terminals;
    st->edges = h->hctrl->edges;
    st->dups = h->hctrl->dups;
    st->probes = h->hctrl->probes;
    st->launches = launches;
    st->explore_ns = (uint64_t)(ms_explore * 1e6);
    st->clear_ns = (uint64_t)(ms_clear * 1e6);
    st->engine_ns = (uint64_t)(ms_engine * 1e6);
    st->supersteps = h->hctrl->supersteps;
    st->batches = h->hctrl->chunks;
    st->max_probe = h->hctrl->max_probe;
    st->critical_ns = h->hctrl->crit_ticks * 10ull;  // 100 MHz device clock
    st->critical_cfg = h->hctrl->crit_part;
    st->parts = h->opts.engine == MC_ENGINE_SUPERSTEP ? h->q_parts : 0u;
    st->cas_fail = cas_fails(st->probes, st->states, st->dups);
    st->total_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                       std::chrono::steady_clock::now() - t0)
                       .count();
  }
  return MC_OK;
}

// Continues the last pruned exploration (every state with clock <= h->resident_T is in
// the visited set) up to T > resident_T on the same set: no clear, no seeding; each
// configuration not yet at its terminals is re-explored from the start of the round
// holding resident_T.  Counters and clocks accumulate, so the result is that of
// check(T).  Super-step engine and resumable models only (the caller checks).
int run_resume(mc_model* h, uint32_t T, mc_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = h->stream;
  h->trace_ready = false;
  h->last = kQueryNone;
  HIPCHK(join_side(h));
  h->behind_lo = h->behind_hi = 0;  // a continued exploration clears nothing behind it
  h->dirty_in = std::max<uint64_t>(h->dirty_in, touched_bytes(h, h->q_slots));
  std::vector<PartPlan> fresh(h->parts_host.size()), plan;
  for (size_t i = 0; i < fresh.size(); ++i) {
    const Part& p = h->parts_host[i];
    fresh[i] = PartPlan{p.cfg, p.r0, p.r1, 0u};
    fresh[i].j0 = p.j0;
    fresh[i].j1 = p.j1;
  }
  plan_resume(h->mh, h->resident_T, fresh, &plan);
  std::vector<Part> parts(plan.size());
  for (size_t i = 0; i < plan.size(); ++i)
    parts[i] = Part{0u, plan[i].cfg, plan[i].r0, plan[i].r1, (uint32_t)i, plan[i].j0,
                    plan[i].j1, 0u};
  h->parts_resumed = true;
  if (!parts.empty())
    HIPCHK(hipMemcpyAsync(h->parts, parts.data(), sizeof(Part) * parts.size(),
                          hipMemcpyHostToDevice, s));
  ModelDev& md = *h->hmd;
  md.prune = 1u;
  md.T = T;
  md.bb = 0u;
  md.refloor = h->resident_T + 1u;  // resident_T < T <= the largest clock
  md.n_parts = (uint32_t)parts.size();
  h->q_parts = md.n_parts;
  HIPCHK(hipMemcpyAsync(h->dmd, h->hmd, sizeof(ModelDev), hipMemcpyHostToDevice, s));
  HIPCHK(launch_resume_models(s, h->dmd, 1, h->head, 1));
  HIPCHK(ev_record(h->ev[2], s));
  HIPCHK(ev_record(h->ev[4], s));
  uint64_t launches = 1;
  if (!parts.empty()) {
    PartQueue pq;
    pq.models = h->dmd;
    pq.parts = h->parts;
    pq.n_parts = (uint32_t)parts.size();
    const uint32_t li = lane_items_for(h->opts.lane_items, h->mh.W);
    pq.batch_items = h->opts.batch_items ? h->opts.batch_items : 2u * li * h->opts.block;
    pq.head = h->head;
    pq.slice = 0u;
    pq.reverse = 0u;
    pq.yielded = nullptr;
    pq.n_yielded = nullptr;
    pq.abort = h->habort;
    const uint32_t grid = h->opts.grid ? h->opts.grid : std::min<uint32_t>(pq.n_parts, 4096u);
    HIPCHK(launch_super(s, h->mh.W, grid, h->opts.block, li, pq, h->mh.general, h->mh.hetero));
    ++launches;
  }
  HIPCHK(ev_record(h->ev[5], s));
  const int rc = finish_query(h, t0, false, launches, st);
  if (rc == MC_OK) h->resident_T = T;
  else h->resident = false;
  return rc;
}

template <int W>
int trace_w(mc_model* h, uint32_t cfg, uint32_t clock) {
  hipStream_t s = h->stream;
  uint32_t fields[kFields] = {0};
  fields[kFCfg] = cfg;
  fields[kFClock] = clock;
  uint64_t words[4];
  encode_key_host(h->mh.layout, fields, words);
  const QueryArgs q = make_args(h, false, 0);
  HIPCHK(launch_find<W>(s, q, reinterpret_cast<const unsigned long long*>(words)));
  HIPCHK(launch_chase<W>(s, q, h->trace_buf, (uint32_t)h->plan.trace_cap));
  HIPCHK(hipMemcpyAsync(h->hctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h->hctrl->target_slot == kParentNone) return MC_E_STATE;
  if (h->hctrl->error == kDevErrTrace) return MC_E_DEVICE;
  const uint32_t n = h->hctrl->trace_len;
  std::vector<uint64_t> keys((size_t)n * W);
  if (n)
    HIPCHK(hipMemcpyAsync(keys.data(), h->trace_buf, 8ull * W * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint32_t m = h->mh.m, S = 3 + m;
  h->trace_rows.assign((size_t)n * S, 0);
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t w[4] = {0, 0, 0, 0};
    for (int j = 0; j < W; ++j) w[j] = keys[(size_t)(n - 1 - i) * W + j];
    uint32_t f[kFields];
    decode_key_host(h->mh.layout, w, f, h->mh.cfgs.data());
    uint32_t* row = &h->trace_rows[(size_t)i * S];
    row[0] = f[kFCfg] == h->mh.n_cfg ? 0xFFFFFFFFu : f[kFCfg];
    row[1] = f[kFClock];
    row[2] = f[kFPending];
    for (uint32_t u = 0; u < m; ++u) row[3 + u] = f[kFRem + u];
  }
  h->trace_ready = true;
  return MC_OK;
}

}  // namespace

extern "C" {

const char* mc_strerror(int code) {
  switch (code) {
    case MC_OK: return "ok";
    case MC_E_INVAL: return "invalid descriptor, option or argument";
    case MC_E_NOMEM: return "workspace too small";
    case MC_E_DEVICE: return "HIP runtime error";
    case MC_E_TABLE_FULL: return "visited-set capacity exceeded";
    case MC_E_BUFFER: return "output buffer too small";
    case MC_E_STATE: return "no query result for this request";
    case MC_E_OVERFLOW: return "frontier or packed field overflow";
    case MC_E_ADMIT: return "query cannot fit the memory budget";
    case MC_E_NOTFOUND: return "not found";
    case MC_E_INTERNAL: return "internal consistency check failed";
    case MC_E_ABORTED: return "query stopped by an abort request";
    default: return "unknown error";
  }
}

int mc_describe(const mc_desc* d, uint64_t* states, uint64_t* max_depth, uint32_t* key_words) {
  try {
    ModelHost mh;
    std::string err;
    const int rc = build_model(d, &mh, &err);
    if (rc) return rc;
    if (states) *states = mh.states;
    if (max_depth) *max_depth = mh.max_depth;
    if (key_words) *key_words = mh.W;
    return MC_OK;
  } catch (...) {
    return MC_E_INVAL;
  }
}

int mc_config_ends(const mc_desc* d, uint32_t cfg, uint32_t* n, uint32_t* b, uint32_t* dur,
                   uint32_t* ends, uint64_t cap) {
  if (!n || !b || !dur || (cap && !ends)) return MC_E_INVAL;
  try {
    ModelHost mh;
    std::string err;
    const int rc = build_model(d, &mh, &err);
    if (rc) return rc;
    if (cfg >= mh.n_cfg) return MC_E_INVAL;
    const CfgRec& r = mh.cfgs[cfg];
    *n = r.n;
    *b = r.b;
    *dur = r.d;
    if (cap < r.b) return MC_E_BUFFER;
    for (uint32_t k = 0; k < r.b; ++k) ends[k] = (uint32_t)end_at_host(r, k);
    return MC_OK;
  } catch (...) {
    return MC_E_INVAL;
  }
}

int mc_workspace_bytes(const mc_desc* d, const mc_opts* o, size_t* bytes) {
  if (!bytes) return MC_E_INVAL;
  try {
    ModelHost mh;
    std::string err;
    int rc = build_model(d, &mh, &err);
    if (rc) return rc;
    WsPlan p;
    const mc_opts oo = default_opts(o);
    rc = plan_ws(mh, oo, model_parts(mh, oo).size(), &p);
    if (rc) return rc;
    *bytes = p.total;
    return MC_OK;
  } catch (...) {
    return MC_E_INVAL;
  }
}

int mc_model_free(mc_model* h) {
  if (!h) return MC_E_INVAL;
  if (h->pooled) {
    // the side stream may still be clearing bytes of the caller's workspace
    if (h->side) (void)hipStreamSynchronize(h->side);
    for (auto& e : h->ev)
      if (e) event_put(e);
    if (h->ev_fork) event_put(h->ev_fork);
    if (h->ev_side) event_put(h->ev_side);
    if (h->side) stream_put(h->side);
    if (h->pin) pinned_put(h->pin, h->pin_bytes);
  }
  delete h;
  return MC_OK;
}

}  // extern "C"

namespace {

// The host side of a load: the model, its options, its partitions and its workspace plan.
struct Loaded {
  ModelHost mh;
  mc_opts opts{};
  WsPlan plan;
  std::vector<Part> parts;
};

int prepare_load(const mc_desc* d, const mc_opts& opts_in, size_t ws_bytes, Loaded* L) {
  std::string err;
  int rc = build_model(d, &L->mh, &err);
  if (rc) return rc;
  L->opts = opts_in;
  L->parts = model_parts(L->mh, L->opts);
  rc = plan_ws(L->mh, L->opts, L->parts.size(), &L->plan);
  if (rc) return rc;
  if (ws_bytes < L->plan.total) return MC_E_NOMEM;
  // automatic workgroup size: with fewer partitions than a wide launch has workgroups,
  // each runs nearly alone on its compute unit and its chain of insert round trips is
  // the launch time, which 512 threads shorten; with many, 256 keeps more of them
  // resident
  // units of unequal speed: 512 (their chain listing is block-wide; on the 1.4M-state
  // workload the launch took 0.70 ms against 0.95 with 256 and 0.83 with 1024)
  if (!L->opts.block)
    L->opts.block = (L->mh.hetero || L->parts.size() < kWideParts) ? 512u : 256u;
  return MC_OK;
}

// Bytes of the table that a query of the model may need cleared (see mc_model::max_need).
uint64_t max_need_of(const Loaded& L) {
  return L.plan.slots * (L.mh.hetero ? (uint64_t)L.plan.slot_bytes : 8ull * L.mh.W);
}

// Puts a prepared model into a handle whose stream, workspace and pooled objects are set:
// its regions, its staging and the upload of its tables.  The per-query state starts over.
int install(mc_model* h, Loaded& L) {
  h->mh = std::move(L.mh);
  h->opts = L.opts;
  h->plan = L.plan;
  h->parts_host = std::move(L.parts);
  h->ctrl = reinterpret_cast<Ctrl*>(h->ws + h->plan.ctrl);
  h->tc = reinterpret_cast<uint32_t*>(h->ws + h->plan.tc);
  h->cfgs = reinterpret_cast<CfgRec*>(h->ws + h->plan.cfgs);
  h->parts = reinterpret_cast<Part*>(h->ws + h->plan.order);
  h->dmd = reinterpret_cast<ModelDev*>(h->ws + h->plan.md);
  h->head = reinterpret_cast<unsigned int*>(h->ws + h->plan.head);
  h->seeds = reinterpret_cast<Seed*>(h->ws + h->plan.seeds);
  h->front[0] = h->ws + h->plan.front0;
  h->front[1] = h->ws + h->plan.front1;
  h->trace_buf = reinterpret_cast<unsigned long long*>(h->ws + h->plan.trace);
  h->table = h->ws + h->plan.table;
  h->q_slots = h->plan.slots;
  h->q_parts = 0;
  const std::vector<Part>& parts = h->parts_host;
  h->n_parts = (uint32_t)parts.size();
  h->trace_ready = false;
  h->trace_rows.clear();
  h->last = kQueryNone;
  h->last_T = 0;
  h->last_violated = 0;
  h->swarm_members = 0;
  h->swarm_best = false;
  h->resident = false;
  h->resident_T = 0;
  h->parts_resumed = false;
  // one staging block: counters, poll words, descriptor, clocks and, when small, the
  // staging of the uploads below
  static_assert(sizeof(Ctrl) <= 256 && sizeof(ModelDev) <= 256, "staging block layout");
  const size_t tc_off = 768, up_off = align_up(tc_off + 4ull * h->mh.n_cfg);
  const size_t cfg_bytes = sizeof(CfgRec) * h->mh.n_cfg, part_bytes = sizeof(Part) * parts.size();
  const bool stage = cfg_bytes + part_bytes <= (4u << 20);
  const size_t pin_bytes = stage ? up_off + cfg_bytes + part_bytes : up_off;
  unsigned char* blk = nullptr;
  if (h->pooled) {
    if (!h->pin || pin_bytes > h->pin_bytes) {
      unsigned char* nb = static_cast<unsigned char*>(pinned_get(pin_bytes));
      if (!nb) return MC_E_DEVICE;
      if (h->pin) pinned_put(h->pin, h->pin_bytes);
      h->pin = nb;
      h->pin_bytes = pin_bytes;
    }
    blk = h->pin;
  } else {
    h->host_stage.assign(pin_bytes, 0);
    blk = h->host_stage.data();
  }
  h->hctrl = reinterpret_cast<Ctrl*>(blk);
  h->hpoll = reinterpret_cast<uint32_t*>(blk + 256);
  // the stop request is a word the kernels read at system scope: pinned memory only
  h->habort = h->pooled ? reinterpret_cast<unsigned int*>(blk + 256 + 128) : nullptr;
  if (h->habort) __atomic_store_n(h->habort, 0u, __ATOMIC_RELEASE);
  h->hmd = reinterpret_cast<ModelDev*>(blk + 512);
  h->tc_host = reinterpret_cast<uint32_t*>(blk + tc_off);
  for (uint32_t c = 0; c < h->mh.n_cfg; ++c) h->tc_host[c] = kNoClock;
  const void* up_cfg = h->mh.cfgs.data();
  const void* up_part = parts.data();
  if (stage) {
    std::memcpy(blk + up_off, up_cfg, cfg_bytes);
    std::memcpy(blk + up_off + cfg_bytes, up_part, part_bytes);
    up_cfg = blk + up_off;
    up_part = blk + up_off + cfg_bytes;
  }
  hipStream_t s = h->stream;
  if (hipMemcpyAsync(h->cfgs, up_cfg, cfg_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->parts, up_part, part_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return MC_E_DEVICE;
  }
  return MC_OK;
}

// Builds a handle over a caller's workspace.  pooled: counters, descriptor and clocks
// are staged in a pooled pinned block, the query is timed with pooled events and dead
// bytes of the visited set are cleared on a pooled side stream (the ordinary handle);
// otherwise they are staged in ordinary host memory and no runtime object is created
// (the handle over the static scratch).
int bind_model(const mc_desc* d, const mc_opts* o, void* dev_ws, size_t ws_bytes, void* stream,
               bool pooled, mc_model** out) {
  if (!out || !dev_ws) return MC_E_INVAL;
  *out = nullptr;
  mc_model* h = nullptr;
  try {
    Loaded L;
    const mc_opts opts_in = default_opts(o);
    int rc = prepare_load(d, opts_in, ws_bytes, &L);
    if (rc) return rc;
    h = new mc_model();
    h->pooled = pooled;
    h->opts_in = opts_in;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->ws = reinterpret_cast<unsigned char*>(dev_ws);
    h->ws_bytes = ws_bytes;
    h->max_need = max_need_of(L);
    h->dirty_in = h->max_need;  // a workspace of unknown content
    if (pooled) {
      bool ok = true;
      for (auto& e : h->ev) {
        e = event_get();
        ok = ok && e != nullptr;
      }
      h->ev_fork = event_get();
      h->ev_side = event_get();
      h->side = stream_get();
      ok = ok && h->ev_fork && h->ev_side && h->side;
      if (!ok) {
        mc_model_free(h);
        return MC_E_DEVICE;
      }
    }
    rc = install(h, L);
    if (rc) {
      mc_model_free(h);
      return rc;
    }
    *out = h;
    return MC_OK;
  } catch (const std::bad_alloc&) {
    if (h) mc_model_free(h);
    return MC_E_NOMEM;
  } catch (...) {
    if (h) mc_model_free(h);
    return MC_E_INVAL;
  }
}

}  // namespace

namespace mc {

int min_time_in_place(const mc_desc* d, const mc_opts* o, void* dev_ws, size_t ws_bytes,
                      void* stream, uint32_t* t_min, uint32_t* argmin, size_t cap,
                      size_t* n_argmin, mc_stats* st) {
  if (!t_min || !n_argmin) return MC_E_INVAL;
  mc_model* h = nullptr;
  int rc = bind_model(d, o, dev_ws, ws_bytes, stream, false, &h);
  if (rc) return rc;
  rc = mc_min_time(h, t_min, argmin, cap, n_argmin, st);
  mc_model_free(h);
  return rc;
}

}  // namespace mc

extern "C" {

int mc_model_load(const mc_desc* d, const mc_opts* o, void* dev_ws, size_t ws_bytes, void* stream,
                  mc_model** out) {
  return bind_model(d, o, dev_ws, ws_bytes, stream, true, out);
}

int mc_model_reload(mc_model* h, const mc_desc* d) {
  if (!h || !d) return MC_E_INVAL;
  try {
    Loaded L;
    const int rc = prepare_load(d, h->opts_in, h->ws_bytes, &L);
    if (rc) return rc;  // the handle keeps its model
    // the new model's tables go past its visited set: where the side stream is still
    // clearing bytes there, the uploads wait for it (its own queries wait anyway)
    if (h->side_pending && h->side_hi > L.plan.table + L.plan.table_bytes &&
        join_side(h) != hipSuccess) {
      (void)hipGetLastError();
      return MC_E_DEVICE;
    }
    // the table's cleared bytes carry over as far as the new model's need reaches into the
    // old one's; past that lay the old model's links and tables: dirty
    const uint64_t need = max_need_of(L);
    h->dirty_in = need <= h->max_need ? std::min<uint64_t>(h->dirty_in, need) : need;
    h->max_need = need;
    return install(h, L);
  } catch (const std::bad_alloc&) {
    return MC_E_NOMEM;
  } catch (...) {
    return MC_E_INVAL;
  }
}


int mc_model_info_get(const mc_model* h, mc_model_info* info) {
  if (!h || !info) return MC_E_INVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_cu = h->mh.m;
  info->n_cfg = h->mh.n_cfg;
  info->key_words = h->mh.W;
  info->key_bits = h->mh.layout.used_bits;
  info->slots = h->plan.slots;
  info->slot_bytes = h->plan.slot_bytes;
  info->bound_states = h->mh.states;
  info->max_depth = h->mh.max_depth;
  return MC_OK;
}

int mc_abort(mc_model* h) {
  if (!h || !h->habort) return MC_E_INVAL;
  __atomic_store_n(h->habort, 1u, __ATOMIC_RELEASE);
  return MC_OK;
}

int mc_set_engine(mc_model* h, uint32_t engine) {
  if (!h || engine > MC_ENGINE_LEVEL) return MC_E_INVAL;
  h->opts.engine = engine;
  return MC_OK;
}

int mc_min_time(mc_model* h, uint32_t* t_min, uint32_t* argmin, size_t cap, size_t* n_argmin,
                mc_stats* st) {
  if (!h || !t_min || !n_argmin) return MC_E_INVAL;
  try {
    const int rc = run_query(h, false, 0, st);
    if (rc) return rc;
    uint32_t best = kNoClock;
    for (uint32_t c = 0; c < h->mh.n_cfg; ++c) best = std::min(best, h->tc_host[c]);
    if (best == kNoClock) return MC_E_STATE;
    size_t n = 0;
    for (uint32_t c = 0; c < h->mh.n_cfg; ++c) {
      if (h->tc_host[c] != best) continue;
      if (argmin && n < cap) argmin[n] = c;
      ++n;
    }
    *t_min = best;
    *n_argmin = n;
    h->last = kQueryMin;
    h->last_T = best;
    return n > cap && argmin ? MC_E_BUFFER : MC_OK;
  } catch (...) {
    return MC_E_DEVICE;
  }
}

int mc_min_time_bb(mc_model* h, uint32_t T_init, uint32_t* t_min, uint32_t* argmin, size_t cap,
                   size_t* n_argmin, mc_stats* st) {
  if (!h || !t_min || !n_argmin) return MC_E_INVAL;
  try {
    const uint32_t T = T_init ? T_init : kNoClock - 1u;
    const int rc = run_query(h, true, T, st, h->opts.engine == MC_ENGINE_SUPERSTEP);
    if (rc) return rc;
    uint32_t best = kNoClock;
    for (uint32_t c = 0; c < h->mh.n_cfg; ++c) best = std::min(best, h->tc_host[c]);
    h->last = kQueryCheck;  // what the table holds: the states of a pruned search
    h->last_T = T;
    h->last_violated = 0;
    if (best == kNoClock) return MC_E_STATE;  // no terminal within T_init
    // configurations whose terminal was found before the incumbent fell below it may
    // carry a larger clock: only those at the least clock are the optimum
    size_t n = 0;
    for (uint32_t c = 0; c < h->mh.n_cfg; ++c) {
      if (h->tc_host[c] != best) continue;
      if (argmin && n < cap) argmin[n] = c;
      ++n;
    }
    *t_min = best;
    *n_argmin = n;
    h->last = kQueryMin;
    h->last_T = best;
    return n > cap && argmin ? MC_E_BUFFER : MC_OK;
  } catch (...) {
    return MC_E_DEVICE;
  }
}

int mc_check(mc_model* h, uint32_t T, int* violated, mc_stats* st) {
  if (!h || !violated) return MC_E_INVAL;
  try {
    const int rc = run_query(h, true, T, st);
    if (rc) return rc;
    *violated = h->hctrl->violated ? 1 : 0;
    h->last = kQueryCheck;
    h->last_T = T;
    h->last_violated = *violated;
    return MC_OK;
  } catch (...) {
    return MC_E_DEVICE;
  }
}

int mc_terminal_clocks(const mc_model* h, uint32_t* tc, size_t cap) {
  if (!h || !tc) return MC_E_INVAL;
  if (h->last == kQueryNone) return MC_E_STATE;
  if (cap < h->mh.n_cfg) return MC_E_BUFFER;
  std::memcpy(tc, h->tc_host, 4ull * h->mh.n_cfg);
  return MC_OK;
}

int mc_trace(mc_model* h, uint32_t* rows, size_t cap, size_t* len) {
  if (!h || !len) return MC_E_INVAL;
  try {
    if (!h->trace_ready) {
      if (h->last == kQueryNone) return MC_E_STATE;
      if (h->last == kQueryCheck && !h->last_violated) return MC_E_STATE;
      uint32_t cfg = kNoClock;
      for (uint32_t c = 0; c < h->mh.n_cfg; ++c) {
        if (h->tc_host[c] == kNoClock) continue;
        if (h->last == kQueryMin && h->tc_host[c] != h->last_T) continue;
        if (h->last == kQueryCheck && h->tc_host[c] > h->last_T) continue;
        cfg = c;
        break;
      }
      if (cfg == kNoClock) return MC_E_STATE;
      int rc;
      switch (h->mh.W) {
        case 1: rc = trace_w<1>(h, cfg, h->tc_host[cfg]); break;
        case 2: rc = trace_w<2>(h, cfg, h->tc_host[cfg]); break;
        default: rc = trace_w<4>(h, cfg, h->tc_host[cfg]); break;
      }
      if (rc) return rc;
    }
    const size_t S = 3 + h->mh.m;
    const size_t n = h->trace_rows.size() / S;
    *len = n;
    if (!rows) return cap ? MC_E_INVAL : MC_OK;
    if (cap < n) return MC_E_BUFFER;
    std::memcpy(rows, h->trace_rows.data(), 4ull * h->trace_rows.size());
    return MC_OK;
  } catch (...) {
    return MC_E_DEVICE;
  }
}

int mc_simulate(mc_model* h, uint64_t seed, uint32_t* t_end, uint32_t* cfg) {
  if (!h || !t_end || !cfg) return MC_E_INVAL;
  hipStream_t s = h->stream;
  const QueryArgs q = make_args(h, false, 0);
  HIPCHK(launch_simulate(s, q, seed));
  HIPCHK(hipMemcpyAsync(h->hpoll, &h->ctrl->sim_t, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *t_end = h->hpoll[0];
  *cfg = h->hpoll[1];
  return MC_OK;
}

}  // extern "C"

namespace {

uint64_t splitmix64_host(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Layout of a swarm in the visited-set region: member records, replay rows, bit arrays.
struct SwarmPlan {
  size_t rec = 0, rows = 0, bits = 0, total = 0;
};
SwarmPlan swarm_plan(const mc_model* h, uint32_t members, uint32_t bits_log2) {
  SwarmPlan p;
  size_t off = 0;
  p.rec = off;
  off = align_up(off + sizeof(SwarmMember) * members);
  p.rows = off;
  off = align_up(off + 4ull * (3 + h->mh.m) * h->plan.trace_cap);
  p.bits = off;
  off = align_up(off + (size_t)members * ((1ull << bits_log2) / 8));
  p.total = off;
  return p;
}

SwarmArgs swarm_args(mc_model* h, const mc_swarm_opts& o, const SwarmPlan& p) {
  SwarmArgs a;
  a.cfgs = h->cfgs;
  a.n_cfg = h->mh.n_cfg;
  a.m = h->mh.m;
  a.seed = o.seed;
  a.budget = o.budget;
  a.members = o.members;
  a.bits_log2 = o.bits_log2;
  a.prune = o.prune ? 1u : 0u;
  a.T = o.T;
  a.bits = reinterpret_cast<uint32_t*>(h->table + p.bits);
  a.out = reinterpret_cast<SwarmMember*>(h->table + p.rec);
  for (int u = 0; u < kMaxCU; ++u) a.speed[u] = h->mh.layout.speed[u];
  return a;
}

}  // namespace

extern "C" {

int mc_swarm(mc_model* h, const mc_swarm_opts* o, mc_swarm_result* r) {
  if (!h || !o || !r || o->members == 0 || o->bits_log2 < 10 || o->bits_log2 > 30)
    return MC_E_INVAL;
  const SwarmPlan p = swarm_plan(h, o->members, o->bits_log2);
  if (p.total > h->plan.table_bytes) return MC_E_NOMEM;
  hipStream_t s = h->stream;
  // the region is no longer a visited set
  HIPCHK(join_side(h));
  h->dirty_in = std::max<uint64_t>(h->dirty_in, std::min<uint64_t>(p.total, h->max_need));
  h->trace_ready = false;
  h->last = kQueryNone;
  h->swarm_members = 0;
  h->swarm_best = false;
  const SwarmArgs a = swarm_args(h, *o, p);
  HIPCHK(hipMemsetAsync(a.bits, 0, p.total - p.bits, s));
  HIPCHK(ev_record(h->ev[4], s));
  HIPCHK(launch_swarm(s, a));
  HIPCHK(ev_record(h->ev[5], s));
  std::vector<SwarmMember> rec(o->members);
  HIPCHK(hipMemcpyAsync(rec.data(), a.out, sizeof(SwarmMember) * o->members,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(ev_ms(&ms, h->ev[4], h->ev[5]));
  std::memset(r, 0, sizeof(*r));
  r->best_clock = r->first_clock = kNoClock;
  r->best_cfg = r->first_cfg = r->best_member = kParentNone;
  unsigned long long start = ~0ull, first = ~0ull;
  for (uint32_t i = 0; i < o->members; ++i) {
    const SwarmMember& x = rec[i];
    r->trails += x.trails;
    r->walks += x.walks;
    r->steps += x.steps;
    start = std::min(start, x.start_ticks);
    if (x.trails && x.best_clock < r->best_clock) {
      r->best_clock = x.best_clock;
      r->best_cfg = x.best_cfg;
      r->best_member = i;
    }
    if (x.trails && x.first_ticks < first) {
      first = x.first_ticks;
      r->first_clock = x.first_clock;
      r->first_cfg = x.first_cfg;
    }
  }
  r->first_trail_ns = first != ~0ull ? (first - start) * 10ull : 0ull;  // 100 MHz clock
  r->swarm_ns = (uint64_t)(ms * 1e6);
  h->swarm_members = o->members;
  h->swarm_bits_log2 = o->bits_log2;
  if (r->trails) {
    h->swarm_best = true;
    h->swarm_best_seed = splitmix64_host(o->seed + r->best_member);
    h->swarm_best_start = rec[r->best_member].best_walk_start;
  }
  return MC_OK;
}

int mc_swarm_members(const mc_model* h, mc_swarm_member* out, size_t cap) {
  if (!h || !out) return MC_E_INVAL;
  if (!h->swarm_members) return MC_E_STATE;
  if (cap < h->swarm_members) return MC_E_BUFFER;
  static_assert(sizeof(mc_swarm_member) == sizeof(SwarmMember), "swarm member record");
  const SwarmPlan p = swarm_plan(h, h->swarm_members, 10);
  HIPCHK(hipMemcpy(out, h->table + p.rec, sizeof(SwarmMember) * h->swarm_members,
                   hipMemcpyDeviceToHost));
  return MC_OK;
}

int mc_swarm_tune(mc_model* h, const mc_swarm_opts* o, uint32_t* t_found, uint32_t* rounds,
                  mc_swarm_result* best) {
  if (!h || !o || !t_found || !rounds) return MC_E_INVAL;
  mc_swarm_opts q = *o;
  q.prune = 0u;
  mc_swarm_result r;
  int rc = mc_swarm(h, &q, &r);
  if (rc) return rc;
  *rounds = 1;
  if (!r.trails) return MC_E_STATE;
  mc_swarm_result found = r;
  unsigned long long bseed = h->swarm_best_seed, bstart = h->swarm_best_start;
  while (found.best_clock > 0u) {
    q.prune = 1u;
    q.T = found.best_clock - 1u;
    q.seed = o->seed + *rounds;
    rc = mc_swarm(h, &q, &r);
    if (rc) return rc;
    ++*rounds;
    if (!r.trails) break;  // nothing below T within the same budget: stop
    found = r;
    bseed = h->swarm_best_seed;
    bstart = h->swarm_best_start;
  }
  // the best trail of the search stays available to mc_swarm_trace
  h->swarm_best = true;
  h->swarm_best_seed = bseed;
  h->swarm_best_start = bstart;
  *t_found = found.best_clock;
  if (best) *best = found;
  return MC_OK;
}

int mc_swarm_trace(mc_model* h, uint32_t* rows, size_t cap, size_t* len) {
  if (!h || !len) return MC_E_INVAL;
  if (!h->swarm_best) return MC_E_STATE;
  hipStream_t s = h->stream;
  // the rows go after the last swarm's member records, over its bit arrays
  mc_swarm_opts o{};
  o.members = h->swarm_members;
  o.bits_log2 = h->swarm_bits_log2;
  const SwarmPlan p = swarm_plan(h, o.members, o.bits_log2);
  const SwarmArgs a = swarm_args(h, o, p);
  uint32_t* drows = reinterpret_cast<uint32_t*>(h->table + p.rows);
  HIPCHK(join_side(h));  // the rows overwrite the visited-set region
  const uint64_t rows_end = p.rows + 4ull * (3 + h->mh.m) * h->plan.trace_cap;
  h->dirty_in = std::max<uint64_t>(h->dirty_in, std::min<uint64_t>(rows_end, h->max_need));
  h->trace_ready = false;
  h->last = kQueryNone;
  HIPCHK(hipMemsetAsync(&h->ctrl->error, 0, 4, s));
  HIPCHK(launch_swarm_replay(s, a, h->ctrl, h->swarm_best_seed, h->swarm_best_start, drows,
                             (uint32_t)h->plan.trace_cap));
  HIPCHK(hipMemcpyAsync(h->hctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h->hctrl->error == kDevErrTrace) return MC_E_DEVICE;
  const uint32_t n = h->hctrl->trace_len;
  *len = n;
  if (!rows) return cap ? MC_E_INVAL : MC_OK;
  if (cap < n) return MC_E_BUFFER;
  HIPCHK(hipMemcpy(rows, drows, 4ull * (3 + h->mh.m) * n, hipMemcpyDeviceToHost));
  return MC_OK;
}

}  // extern "C"

namespace {

// check(T) inside an incremental bisection: the visited set is kept from check to check
// and holds every state with clock <= h->resident_T.  A check at or below that is
// answered from the per-configuration least clocks (a terminal with clock <= T is one of
// them); a check above it continues the exploration (run_resume).  The first check sizes
// the set for T_size, the largest threshold the bisection can reach.
int inc_check(mc_model* h, uint32_t T, uint32_t T_size, int* violated, mc_stats* st) {
  if (st) std::memset(st, 0, sizeof(*st));
  int rc = MC_OK;
  if (!h->resident) {
    rc = run_query(h, true, T, st, false, T_size);
    if (rc) return rc;
    h->resident = true;
    h->resident_T = T;
  } else if (T > h->resident_T) {
    rc = run_resume(h, T, st);
    if (rc) return rc;
  }
  uint32_t best = kNoClock;
  for (uint32_t c = 0; c < h->mh.n_cfg; ++c) best = std::min(best, h->tc_host[c]);
  *violated = best <= T ? 1 : 0;
  h->last = kQueryCheck;
  h->last_T = T;
  h->last_violated = *violated;
  return MC_OK;
}

}  // namespace

extern "C" {

int mc_tune_bisect(mc_model* h, uint64_t seed, uint32_t* t_min, uint32_t* n_checks, mc_stats* st) {
  if (!h || !t_min || !n_checks) return MC_E_INVAL;
  uint32_t t_ini = 0, c0 = 0;
  int rc = mc_simulate(h, seed, &t_ini, &c0);
  if (rc) return rc;
  mc_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  mc_stats one;
  // one visited set for the whole bisection where the exploration can be continued
  const bool inc = h->opts.engine == MC_ENGINE_SUPERSTEP && resumable(h->mh);
  h->resident = false;
  // check(lo) holds (clock >= 1 at every terminal), check(hi) fails (the simulated run)
  uint32_t lo = 0, hi = t_ini, n = 0;
  int last_violated = -1;
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    int v = 0;
    rc = inc ? inc_check(h, mid, t_ini, &v, &one) : mc_check(h, mid, &v, &one);
    if (rc) return rc;
    ++n;
    acc.explore_ns += one.explore_ns;
    acc.clear_ns += one.clear_ns;
    acc.engine_ns += one.engine_ns;
    acc.launches += one.launches;
    // an incremental bisection's counters run on: its states are the last total
    if (inc) acc.states = std::max<uint64_t>(acc.states, one.states);
    else acc.states += one.states;
    if (v) hi = mid;
    else lo = mid;
    last_violated = v;
  }
  if (last_violated != 1) {  // leave the counterexample of check(T_min) behind
    int v = 0;
    rc = inc ? inc_check(h, hi, t_ini, &v, &one) : mc_check(h, hi, &v, &one);
    if (rc) return rc;
    acc.explore_ns += one.explore_ns;
    acc.clear_ns += one.clear_ns;
    acc.launches += one.launches;
    if (inc) acc.states = std::max<uint64_t>(acc.states, one.states);
    if (!v) return MC_E_STATE;
  }
  *t_min = hi;
  *n_checks = n;
  if (st) *st = acc;
  return MC_OK;
}

int mc_config(const mc_model* h, uint32_t cfg, uint32_t* params4) {
  if (!h || !params4 || cfg >= h->mh.n_cfg) return MC_E_INVAL;
  std::memcpy(params4, &h->mh.params[4ull * cfg], 16);
  return MC_OK;
}

}  // extern "C"
