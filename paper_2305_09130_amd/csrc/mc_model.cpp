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
#include <map>
#include <array>
#include <numeric>
#include <atomic>
#include <cstring>
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>

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

// One wave of a configuration's workgroup: its timed phases (zero-latency operations
// dropped), how many waves make a workgroup and how many workgroups there are.
struct WaveSpec {
  uint64_t n = 0, waves = 1, t = 0;  // t: wave duration so far
  uint32_t nph = 0;
  uint64_t cnt[kMaxPhases] = {}, lat[kMaxPhases] = {}, la[kMaxPhases] = {}, t0[kMaxPhases] = {};
  // cnt operations of latency lat, back to back from the current end
  void seq(uint64_t c, uint64_t l) {
    if (!c || !l) return;
    grid(t, c, l, 0);
  }
  // cnt ends on the grid t0 + k*l (+ a for two-operation periods)
  void grid(uint64_t start, uint64_t c, uint64_t l, uint64_t a) {
    cnt[nph] = c; lat[nph] = l; la[nph] = a; t0[nph] = start;
    ++nph;
    t = start + (a ? c / 2 : c) * l;
  }
};

static int phases(const mc_desc* d, const uint32_t* p, WaveSpec* w, std::string* err) {
  if (d->kind == MC_KIND_REDUCTION) {
    const uint64_t G = d->size[0], WG = p[0], TS = p[1];
    if (!pow2(G) || !pow2(WG) || !pow2(TS)) return fail(err, "reduction sizes must be powers of two");
    if (WG > G) return fail(err, "WG larger than G");
    w->n = G / WG;
    w->seq((G + WG * TS - 1) / (WG * TS), d->lat_global);
    w->seq(bit_length(WG) - 1, d->lat_local);
    w->seq(1, d->lat_barrier);
    w->seq(TS, d->lat_compute);
    return MC_OK;
  }
  if (d->kind == MC_KIND_MATMUL) {
    const uint64_t M = d->size[0], N = d->size[1], K = d->size[2];
    const uint64_t X = p[0], Y = p[1], TS = p[2], VW = p[3] ? p[3] : 1;
    if (!pow2(M) || !pow2(N) || !pow2(K) || !pow2(X) || !pow2(Y) || !pow2(TS) || !pow2(VW))
      return fail(err, "matmul sizes must be powers of two");
    if (X > M || Y * VW > N || TS > K) return fail(err, "matmul tile larger than the matrix");
    w->n = (M / X) * (N / (Y * VW));
    w->seq(2 * K, d->lat_global);
    w->seq(K * (1 + VW), d->lat_local);
    w->seq(2 * (K / TS), d->lat_barrier);
    w->seq(K * VW, d->lat_compute);
    return MC_OK;
  }
  if (d->kind == MC_KIND_ABSTRACT || d->kind == MC_KIND_MINIMUM) {
    const uint64_t S = d->size[0], NP = d->size[1], WG = p[0], TS = p[1];
    const uint64_t Lg = d->lat_global, Ll = d->lat_local;
    if (!pow2(S) || !pow2(NP) || !pow2(WG) || !pow2(TS))
      return fail(err, "size, NP, WG and TS must be powers of two");
    if (WG > S || TS > S) return fail(err, "WG or TS larger than the data size");
    w->n = std::max<uint64_t>(1, S / (WG * TS));  // one workgroup where WG*TS > S
    const uint64_t waves = WG > NP ? WG / NP : 1;  // NP elements run WG items in waves
    if (d->kind == MC_KIND_MINIMUM) {
      w->seq(waves * TS, Lg);                       // MAP: TS global accesses per item
      w->seq(std::min(WG, NP) - 1, Ll);             // REDUCE local by element 0
      w->seq(1, Lg);                                // the workgroup's minimum to global
      return MC_OK;
    }
    // abstract pex: long_work(gt, tz) ends one tick after start_time + gt*tz; start_time
    // is reset before each local step but not before the next tile's global load
    const uint64_t s = S / TS, bb = Ll * TS + 1, g = Lg > Ll ? (Lg - Ll) * TS : 0;
    w->waves = waves;
    if (g) {
      // tile k: global load ends at k(g+bb), local step at k(g+bb)+bb: a grid from bb
      w->grid(bb, 2 * s, g + bb, g);
    } else {
      w->seq(1, Lg * TS + 1);  // first tile's load; later loads end at once
      w->seq(s, bb);
    }
    w->seq(1, Lg + 1);  // the work item's result to global memory
    return MC_OK;
  }
  return fail(err, "unknown model kind");
}

// Units of unequal speed.  Dispatch is eager: while a workgroup is pending no unit
// stays idle, so as long as at least as many workgroups are pending as units fall idle
// together every run of a configuration is the same one (only the order of the
// zero-time dispatches differs, giving the subsets of the idle units as states).  At
// the first instant with p pending < f idle, every choice of p units starts a tail in
// which nothing is dispatched any more.  This walks that determined part and every
// tail.  Tails are counted separately even where they meet (once only some units are
// still busy two tails can agree), so `states` bounds the reachable count from above;
// `depth` (edges from the SELECT state) and `max_clock` are exact maxima.  Only states
// with clock <= T are counted.
namespace {

// One unit's workgroup in progress: when it started and its next operation end.
struct UnitRun {
  uint64_t start = 0, next = 0;
  uint32_t k = 0;  // index of that end in E
};

// Moves the clock to the next operation end of any busy unit; units whose workgroup
// ends there fall idle.
uint64_t advance_units(const CfgRec& r, const uint32_t* sp, uint32_t m, UnitRun* ur,
                       uint32_t* busy) {
  uint64_t t = ~0ull;
  for (uint32_t u = 0; u < m; ++u)
    if ((*busy >> u) & 1u) t = std::min(t, ur[u].next);
  for (uint32_t u = 0; u < m; ++u) {
    if (!((*busy >> u) & 1u) || ur[u].next != t) continue;
    if (++ur[u].k == r.b) *busy &= ~(1u << u);
    else ur[u].next = ur[u].start + (uint64_t)sp[u] * end_at_host(r, ur[u].k);
  }
  return t;
}

void start_unit(const CfgRec& r, const uint32_t* sp, UnitRun* ur, uint32_t u, uint64_t t) {
  ur[u].start = t;
  ur[u].k = 0;
  ur[u].next = t + (uint64_t)sp[u] * end_at_host(r, 0);
}

void tail_walk(const CfgRec& r, const uint32_t* sp, uint32_t m, uint64_t T, uint64_t t,
               UnitRun* ur, uint32_t busy, uint64_t dep, ChainCount* out) {
  while (busy) {
    t = advance_units(r, sp, m, ur, &busy);
    ++dep;
    if (t <= T) ++out->states;
  }
  out->depth = std::max(out->depth, dep);
  out->max_clock = std::max(out->max_clock, t);
}

}  // namespace

ChainCount walk_unequal(const CfgRec& r, const uint32_t* sp, uint32_t m, uint64_t T,
                        std::vector<ChainCut>* cuts) {
  ChainCount out;
  uint64_t t = 0, p = r.n, dep = 0;
  UnitRun ur[kMaxCU];
  uint32_t busy = 0;
  const uint32_t all = (1u << m) - 1u;
  uint64_t spacing = kCutSpacing, last = 0;
  out.states = 1;  // the SELECT state, clock 0
  const auto record = [&](const ChainCut& c) {
    if (c.states - last < spacing) return;
    if (cuts->size() == kMaxCuts) {  // keep every other candidate, twice as far apart
      size_t k = 0;
      for (size_t i = 1; i < cuts->size(); i += 2) (*cuts)[k++] = (*cuts)[i];
      cuts->resize(k);
      spacing *= 2;
    }
    cuts->push_back(c);
    last = c.states;
  };
  // While work is pending every unit restarts at each of its workgroup ends, so unit u
  // runs workgroups back to back from clock 0 and all units end together at the period
  // P = lcm(sp) * d, where every unit is idle again with Wp = sum(lcm / sp[u]) fewer
  // workgroups pending.  Each later period that finds at least Wp pending repeats the
  // first one shifted by P in clock, and by its states and edges: it is not walked.
  uint64_t lcm = 1;
  for (uint32_t u = 0; u < m && lcm <= kMaxPeriodLcm; ++u)
    lcm = lcm / std::gcd<uint64_t>(lcm, sp[u]) * sp[u];
  uint64_t Wp = 0;
  for (uint32_t u = 0; u < m; ++u) Wp += lcm / sp[u];
  const bool jump = T == ~0ull && lcm <= kMaxPeriodLcm && (uint64_t)r.n >= 2 * Wp;
  const uint64_t P = lcm * r.d;
  bool jumped = false;
  std::vector<ChainCut> period;  // cut points of the first period
  for (;;) {
    const uint32_t freem = all & ~busy;
    const uint32_t f = (uint32_t)__builtin_popcount(freem);
    if (p > 0 && f > 0) {
      if (p >= f) {
        if (t <= T) out.states += (1ull << f) - 1;
        dep += f;
        p -= f;
        for (uint32_t u = 0; u < m; ++u)
          if ((freem >> u) & 1u) start_unit(r, sp, ur, u, t);
        busy |= freem;
      } else {
        if (t <= T)
          for (uint32_t j = 1; j <= p; ++j) out.states += binom(f, j);
        // one tail per choice of p idle units
        for (uint32_t sub = freem;; sub = (sub - 1) & freem) {
          if ((uint32_t)__builtin_popcount(sub) == p) {
            UnitRun tu[kMaxCU];
            for (uint32_t u = 0; u < m; ++u) tu[u] = ur[u];
            for (uint32_t u = 0; u < m; ++u)
              if ((sub >> u) & 1u) start_unit(r, sp, tu, u, t);
            tail_walk(r, sp, m, T, t, tu, busy | sub, dep + p, &out);
          }
          if (sub == 0) break;
        }
        return out;
      }
    }
    if (!busy) {  // every workgroup done: the terminal (counted as the last advance)
      out.depth = std::max(out.depth, dep);
      out.max_clock = std::max(out.max_clock, t);
      return out;
    }
    if (p == 0) {  // nothing left to dispatch: one tail
      tail_walk(r, sp, m, T, t, ur, busy, dep, &out);
      return out;
    }
    t = advance_units(r, sp, m, ur, &busy);
    ++dep;
    if (t <= T) ++out.states;
    // every unit still busy after the advance (no workgroup ended at t) and work pending:
    // the state at t lies on every run of the configuration
    if (cuts && busy == all) {
      if (jump && !jumped) period.push_back(ChainCut{t, dep + 1, out.states});
      record(ChainCut{t, dep + 1, out.states});  // depth from the root
    }
    if (jump && !jumped && t == P) {  // the first period ends: every unit is idle
      jumped = true;
      const uint64_t J = p / Wp, dS = out.states - 1, dD = dep;
      if (cuts)
        for (uint64_t j = 1; j <= J; ++j) {
          // record() takes a candidate at least `spacing` states past the last one
          // taken, and the period's states ascend: search for the next such candidate
          // instead of offering it every one
          auto it = period.begin();
          for (;;) {
            const uint64_t want = last + spacing;  // in states, after the shift by j periods
            const uint64_t lo = want > j * dS ? want - j * dS : 0;
            it = std::lower_bound(it, period.end(), lo, [](const ChainCut& c, uint64_t v) {
              return c.states < v;
            });
            if (it == period.end()) break;
            record(ChainCut{it->t + j * P, it->depth + j * dD, it->states + j * dS});
            ++it;
          }
        }
      out.states += J * dS;
      dep += J * dD;
      t += J * P;
      p -= J * Wp;
    }
  }
}

void chain_cuts(const std::vector<ChainCut>& cands, uint64_t target,
                std::vector<ChainCut>* out) {
  uint64_t last = 0;
  for (const ChainCut& c : cands)
    if (c.states - last >= target) {
      out->push_back(c);
      last = c.states;
    }
}

namespace {

// Process-wide workers for the walks of a load: starting and joining threads per load
// cost about 0.2 ms for seven of them.  Workers are started as first needed (at most
// 15, detached: they wait for work until the process ends); one job runs at a time and
// the caller takes part in it.  A worker joins a job only while the caller still admits
// helpers, and the caller returns once every helper that joined has finished; the first
// exception of any item ends the job and is rethrown to the caller.
class WalkPool {
 public:
  static WalkPool& get() {
    static WalkPool* p = new WalkPool();  // never destroyed: its workers never stop
    return *p;
  }

  // fn(i) for every i < n, on up to `threads` threads (the caller's included)
  void run(uint32_t n, uint32_t threads, const std::function<void(uint32_t)>& fn) {
    std::lock_guard<std::mutex> job(job_mu_);
    const uint32_t helpers = threads > 1 ? start(threads - 1) : 0u;
    {
      std::lock_guard<std::mutex> g(mu_);
      fn_ = &fn;
      n_ = n;
      next_.store(0);
      want_ = helpers;
      taken_ = 0;
      ++gen_;
    }
    if (helpers) cv_.notify_all();
    work(fn, n);
    std::unique_lock<std::mutex> g(mu_);
    want_ = 0;  // no helper joins from here on
    done_.wait(g, [&] { return active_ == 0u; });
    fn_ = nullptr;
    std::exception_ptr e = error_;
    error_ = nullptr;
    g.unlock();
    if (e) std::rethrow_exception(e);  // after every helper has left the job
  }

 private:
  // workers up to k (fewer if the system refuses threads); returns how many there are
  uint32_t start(uint32_t k) {
    k = std::min<uint32_t>(k, 15u);
    while (workers_ < k) {
      try {
        std::thread([this] { loop(); }).detach();
      } catch (...) {
        break;
      }
      ++workers_;
    }
    return workers_ < k ? workers_ : k;
  }

  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> g(mu_);
    for (;;) {
      cv_.wait(g, [&] { return gen_ != seen; });
      seen = gen_;
      if (taken_ >= want_) continue;  // enough helpers, or the job is over
      ++taken_;
      ++active_;
      const std::function<void(uint32_t)>* fn = fn_;
      const uint32_t n = n_;
      g.unlock();
      work(*fn, n);
      g.lock();
      if (--active_ == 0u) done_.notify_all();
    }
  }

  // the job's items until none is left; the first exception stops the job and is kept
  void work(const std::function<void(uint32_t)>& fn, uint32_t n) {
    try {
      for (uint32_t i; (i = next_.fetch_add(1)) < n;) fn(i);
    } catch (...) {
      next_.store(n);  // no further items
      std::lock_guard<std::mutex> g(err_mu_);
      if (!error_) error_ = std::current_exception();
    }
  }

  std::mutex job_mu_, mu_, err_mu_;
  std::condition_variable cv_, done_;
  std::exception_ptr error_;  // the job's first exception (read once every helper left)
  const std::function<void(uint32_t)>* fn_ = nullptr;
  std::atomic<uint32_t> next_{0};
  uint32_t n_ = 0, want_ = 0, taken_ = 0, active_ = 0, workers_ = 0;
  uint64_t gen_ = 0;
};

}  // namespace

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
  h->hetero = false;
  for (int i = 0; i < kMaxCU; ++i) h->speed[i] = 1;
  if (d->unit_speed) {
    for (uint32_t i = 0; i < d->n_cu; ++i) {
      if (d->unit_speed[i] < 1 || d->unit_speed[i] > MC_MAX_SPEED)
        return fail(err, "unit speed out of range 1..64");
      h->speed[i] = d->unit_speed[i];
      if (h->speed[i] != h->speed[0]) h->hetero = true;
    }
    if (!h->hetero && h->speed[0] != 1) h->hetero = true;  // one common factor: still scaled
  }
  h->desc = *d;
  h->desc.unit_speed = nullptr;  // the speeds live in h->speed
  h->m = d->n_cu;
  h->n_cfg = d->n_cfg;
  h->params.assign(d->params, d->params + 4ull * d->n_cfg);
  h->desc.params = h->params.data();
  h->cfgs.assign(d->n_cfg, CfgRec{});
  h->general = false;
  h->cfg_states.assign(d->n_cfg, 0);
  h->cut_cands.clear();
  h->cut_of.clear();
  const uint32_t m = h->m;
  uint64_t total = 1, depth = 0, fb = d->n_cfg;
  uint64_t widest_sum = 0;
  uint32_t max_clock = 0, max_n = 0, max_d = 0;
  // per configuration: latest terminal clock, state count (bound), longest path
  std::vector<uint64_t> c_tc(d->n_cfg), c_depth(d->n_cfg);
  uint64_t walk_work = 0;  // operation ends the walks of units of unequal speed visit
  for (uint32_t c = 0; c < d->n_cfg; ++c) {
    WaveSpec ws;
    int rc = phases(d, &h->params[4ull * c], &ws, err);
    if (rc) return rc;
    const uint64_t n = ws.n;
    if (n == 0 || n >= (1ull << 31)) return fail(err, "workgroup count out of range");
    CfgRec& r = h->cfgs[c];
    std::memset(&r, 0, sizeof(r));
    uint64_t bw = 0;
    for (uint32_t j = 0; j < ws.nph; ++j) {
      if (ws.cnt[j] >= (1ull << 31)) return fail(err, "operation count out of range");
      r.cnt[j] = (uint32_t)ws.cnt[j];
      r.lat[j] = (uint32_t)ws.lat[j];
      r.la[j] = (uint32_t)ws.la[j];
      r.t0[j] = (uint32_t)ws.t0[j];
      r.i0[j] = (uint32_t)bw;
      bw += ws.cnt[j];
    }
    r.nph = ws.nph;
    if (ws.t >= (1ull << 31) || ws.waves >= (1ull << 31)) return fail(err, "workgroup duration exceeds 2^31");
    const uint64_t t = ws.waves * ws.t, b = ws.waves * bw;
    if (t >= (1ull << 31)) return fail(err, "workgroup duration exceeds 2^31");
    if (b >= (1ull << 31)) return fail(err, "operation count out of range");
    r.waves = (uint32_t)ws.waves;
    r.dw = (uint32_t)ws.t;
    r.bw = (uint32_t)bw;
    for (uint32_t j = 0; j < ws.nph; ++j)
      if (r.la[j] || r.t0[j] != (j ? r.t0[j - 1] + r.cnt[j - 1] * r.lat[j - 1] : 0u)) h->general = true;
    if (r.waves > 1) h->general = true;
    if (b == 0) return fail(err, "workgroup without timed operations");
    const uint64_t rounds = (n + m - 1) / m;
    uint64_t tc = rounds * t;
    r.n = (uint32_t)n;
    r.d = (uint32_t)t;
    r.b = (uint32_t)b;
    uint64_t cs = 0, cdepth = 0;
    if (h->hetero) {
      h->general = true;
      uint32_t smax = 1;
      for (uint32_t i = 0; i < m; ++i) smax = std::max(smax, h->speed[i]);
      if ((uint64_t)smax * t >= (1ull << 31)) return fail(err, "workgroup duration exceeds 2^31");
      if (rounds * b * m > (1ull << 26)) return fail(err, "model too long for units of unequal speed");
      walk_work += rounds * b * m;  // walked below, every configuration on its own
    } else {
      const uint64_t q = n / m, p = n % m;
      cs = 1 + q * (((1ull << m) - 1) + b);
      if (p) {
        uint64_t s = 0;
        for (uint32_t j = 1; j <= p; ++j) s += binom(m, j);
        cs += s + binom(m, (uint32_t)p) * (b - 1) + 1;
      }
      cdepth = 1 + n + rounds * b;
    }
    c_tc[c] = tc;
    h->cfg_states[c] = cs;
    c_depth[c] = cdepth;
    max_n = std::max<uint32_t>(max_n, (uint32_t)n);
    max_d = std::max<uint32_t>(max_d, (uint32_t)t);
    // widest level of this subgraph: dispatch levels C(m, j), partial-round runs C(m, p)
    uint64_t w = 1;
    const uint32_t jmax = (uint32_t)std::min<uint64_t>(n, m);
    for (uint32_t j = 0; j <= jmax; ++j) w = std::max<uint64_t>(w, binom(m, j));
    widest_sum += w;
  }
  if (h->hetero) {
    h->cut_cands.assign(d->n_cfg, {});
    h->cut_of.assign(d->n_cfg, 0u);
    // configurations whose workgroups have the same count and operation ends (the same
    // record but for its terminal clock) walk alike: each distinct one is walked once, and
    // the others take its sizes and share its cut points
    std::vector<uint32_t> walked;
    {
      std::map<std::array<uint32_t, sizeof(CfgRec) / 4>, uint32_t> first;
      for (uint32_t c = 0; c < d->n_cfg; ++c) {
        CfgRec k = h->cfgs[c];
        k.tc = 0;
        std::array<uint32_t, sizeof(CfgRec) / 4> key;
        std::memcpy(key.data(), &k, sizeof(CfgRec));
        const auto ins = first.emplace(key, c);
        h->cut_of[c] = ins.first->second;
        if (ins.second) walked.push_back(c);
      }
    }
    // the walks are independent: long ones share the host's cores
    const auto walk = [&](uint32_t i) {
      const uint32_t c = walked[i];
      const ChainCount cc = walk_unequal(h->cfgs[c], h->speed, m, ~0ull, &h->cut_cands[c]);
      c_tc[c] = cc.max_clock;  // the latest terminal clock of this configuration
      h->cfg_states[c] = cc.states;
      c_depth[c] = 1 + cc.depth;
    };
    const uint32_t nw = (uint32_t)walked.size();
    const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
    const uint32_t nt = walk_work < (1ull << 17) ? 1u : std::min<uint32_t>({hw, 16u, nw});
    WalkPool::get().run(nw, nt, walk);
    for (uint32_t c = 0; c < d->n_cfg; ++c) {
      const uint32_t w = h->cut_of[c];
      c_tc[c] = c_tc[w];
      h->cfg_states[c] = h->cfg_states[w];
      c_depth[c] = c_depth[w];
    }
  }
  for (uint32_t c = 0; c < d->n_cfg; ++c) {
    if (c_tc[c] >= 0xFFFFFFFFull) return fail(err, "terminal clock exceeds 32 bits");
    h->cfgs[c].tc = (uint32_t)c_tc[c];
    total += h->cfg_states[c];
    depth = std::max<uint64_t>(depth, c_depth[c]);
    max_clock = std::max<uint32_t>(max_clock, (uint32_t)c_tc[c]);
  }
  fb = std::max<uint64_t>(fb, widest_sum);
  h->states = total;
  h->max_depth = depth;
  h->max_clock = max_clock;
  h->max_n = max_n;
  h->max_d = max_d;
  h->frontier_bound = fb;

  // key layout: cfg | pending | clock | rem_0 .. rem_{m-1}
  // equal units start their workgroups together (every dispatch is from an all-idle
  // state), so every busy unit has the same time left: a mask and one field hold them;
  // and the rounds are in lock step, so the clock follows from the other fields and is
  // not stored (Layout::clock_implied)
  const bool shared = !h->hetero;
  uint32_t widths[kFields] = {0};
  widths[kFCfg] = std::max<uint32_t>(1, bit_length((uint64_t)d->n_cfg + 1));
  widths[kFPending] = std::max<uint32_t>(1, bit_length(max_n));
  widths[kFClock] = shared ? 0u : std::max<uint32_t>(1, bit_length(max_clock));
  if (shared) {
    widths[kFRem] = m;
    widths[kFRem + 1] = std::max<uint32_t>(1, bit_length(max_d));
  } else {
    for (uint32_t i = 0; i < m; ++i)
      widths[kFRem + i] = std::max<uint32_t>(1, bit_length((uint64_t)h->speed[i] * max_d));
  }
  const uint32_t nfields = shared ? 5u : 3u + m;
  Layout L;
  std::memset(&L, 0, sizeof(L));
  // every word after the first keeps its top bit clear, so that no valid key has a word
  // equal to the all-ones of a cleared slot (word 0 cannot be: its configuration field
  // is never all-ones); a reader of a wide key can then tell a word not yet written
  uint32_t word = 0, off = 0, used = 0;
  for (uint32_t f = 0; f < nfields; ++f) {
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
  L.hetero = h->hetero ? 1 : 0;
  L.shared_rem = shared ? 1 : 0;
  L.clock_implied = shared ? 1 : 0;
  L.n_cfg = d->n_cfg;
  for (int i = 0; i < kMaxCU; ++i) L.speed[i] = (uint8_t)h->speed[i];
  L.used_bits = (uint8_t)used;
  h->layout = L;
  h->W = L.W;
  return MC_OK;
}

void plan_parts(const ModelHost& h, uint64_t target, std::vector<PartPlan>* out,
                uint64_t clock_max) {
  // units of unequal speed pass through no common idle state after whole rounds
  const bool cuttable = target > 0 && word0_orders_rounds(h);
  // ... but their determined part is cut into chain slices, which share no word-0 value
  // but their boundary states when the clock is in word 0
  const Layout& L = h.layout;
  const bool chains = target > 0 && h.hetero && L.word[kFClock] == 0 && L.word[kFPending] == 0;
  const uint64_t chain_target = std::max<uint64_t>(32, target);
  for (uint32_t c = 0; c < h.n_cfg; ++c) {
    const CfgRec& r = h.cfgs[c];
    if (chains) {
      std::vector<ChainCut> cuts;
      if (h.cfg_states[c] >= 2 * chain_target)
        chain_cuts(h.cut_cands[h.cut_of[c]], chain_target, &cuts);
      if (cuts.empty()) {
        out->push_back(PartPlan{c, 0u, kRoundsToEnd, h.cfg_states[c]});
        continue;
      }
      uint64_t prev_t = 0, prev_dep = 0, prev_states = 0;
      for (size_t k = 0; k <= cuts.size(); ++k) {
        const bool last = k == cuts.size();
        const uint64_t upto = last ? h.cfg_states[c] : cuts[k].states;
        PartPlan pp{c, kChainSlice, last ? kNoClock : (uint32_t)cuts[k].t,
                    upto > prev_states ? upto - prev_states : 1};
        pp.j0 = (uint32_t)prev_t;
        pp.j1 = (uint32_t)prev_dep;
        out->push_back(pp);
        if (!last) {
          prev_t = cuts[k].t;
          prev_dep = cuts[k].depth;
          prev_states = cuts[k].states;
        }
      }
      continue;
    }
    const uint64_t q = r.n / h.m;
    const uint64_t per_round = ((1ull << h.m) - 1) + r.b;
    // blocks of at least kMinBlockRounds rounds, or of fewer when the rounds are long
    const uint64_t min_rounds = std::min<uint64_t>(
        kMinBlockRounds, std::max<uint64_t>(1, (kMinBlockStates + per_round - 1) / per_round));
    uint64_t R = cuttable ? std::max<uint64_t>(min_rounds, target / per_round) : q;
    const uint64_t K = R ? (q + R - 1) / R : 1;
    const uint64_t p = r.n % h.m;
    // a slice spans every run of its round (one per choice of units), about `target`
    // states in all
    const auto slice_of = [&](uint64_t choices) {
      return std::max<uint64_t>(
          kMinSlice,
          std::min<uint64_t>(kMaxSlice, std::max<uint64_t>(kMinSlice, target)) / choices);
    };
    // run slices of round rd: states [sl, b) of its runs when they end at a terminal (the
    // last slice keeps at least two states, so a run's end and the state before it are
    // inserted together), else [sl, b - 1) (the next round's start is the block's)
    const auto add_slices = [&](uint64_t rd, uint64_t choices, uint64_t sl, bool terminal) {
      const uint64_t end = terminal ? r.b : r.b - 1;
      for (uint64_t j0 = sl; j0 < end;) {
        uint64_t j1 = std::min<uint64_t>(j0 + sl, end);
        if (terminal && end - j1 < 2) j1 = end;
        PartPlan sp{c, kRunSlice, (uint32_t)rd, choices * (j1 - j0)};
        sp.j0 = (uint32_t)j0;
        sp.j1 = (uint32_t)j1;
        out->push_back(sp);
        j0 = j1;
      }
    };
    if (cuttable && r.n <= h.m) {
      // one round: the SELECT closure and the first `slice` states of every run, then
      // slices of the runs
      const uint64_t choices = binom(h.m, r.n), sl = slice_of(choices);
      if (r.b > sl + 1) {
        PartPlan a{c, 0u, kRoundsToEnd, h.cfg_states[c] - choices * (r.b - sl)};
        a.j1 = (uint32_t)sl;
        out->push_back(a);
        add_slices(0, choices, sl, true);
        continue;
      }
    }
    const uint64_t sl1 = slice_of(1);
    if (cuttable && R == 1 && q >= 1 && r.n > h.m && r.b > sl1 + 1) {
      // long rounds: one block per round that explores the round's closure and the first
      // `sl1` states of its run and claims the next round's start; slices hold the rest
      const uint64_t full_blocks = p ? q : q - 1;  // rounds whose block ends at a cut
      for (uint64_t k = 0; k < full_blocks; ++k) {
        if (k * r.d > clock_max) break;  // the round starts past every state asked for
        PartPlan b{c, (uint32_t)k, (uint32_t)(k + 1), per_round - (r.b - 1 - sl1)};
        b.j1 = (uint32_t)sl1;
        out->push_back(b);
        add_slices(k, 1, sl1, false);
      }
      if ((p ? q : q - 1) * r.d > clock_max) continue;
      if (p) {  // the partial round, to the terminals
        const uint64_t choices = binom(h.m, (uint32_t)p), slp = slice_of(choices);
        const bool cut = r.b > slp + 1;
        PartPlan b{c, (uint32_t)q, kRoundsToEnd,
                   h.cfg_states[c] - q * per_round - (cut ? choices * (r.b - slp) : 0)};
        b.j1 = cut ? (uint32_t)slp : 0u;
        out->push_back(b);
        if (cut) add_slices(q, choices, slp, true);
      } else {  // the last full round, to the terminal
        PartPlan b{c, (uint32_t)(q - 1), kRoundsToEnd, (uint64_t)h.cfg_states[c] -
                                                      (q - 1) * per_round - (r.b - sl1)};
        b.j1 = (uint32_t)sl1;
        out->push_back(b);
        add_slices(q - 1, 1, sl1, true);
      }
      continue;
    }
    if (!cuttable || K < 2) {
      out->push_back(PartPlan{c, 0u, kRoundsToEnd, h.cfg_states[c]});
      continue;
    }
    for (uint64_t k = 0; k + 1 < K && k * R * r.d <= clock_max; ++k)
      out->push_back(PartPlan{c, (uint32_t)(k * R), (uint32_t)((k + 1) * R), R * per_round});
    const uint64_t r0 = (K - 1) * R;
    if (r0 * r.d <= clock_max)
      out->push_back(PartPlan{c, (uint32_t)r0, kRoundsToEnd, h.cfg_states[c] - r0 * per_round});
  }
}

bool word0_orders_rounds(const ModelHost& h) {
  const Layout& L = h.layout;
  if (h.hetero || L.word[kFPending] != 0) return false;
  // with the clock stored, pending and clock in word 0 tell rounds and run positions
  // apart; with the clock implied, the mask and the time left must be there too
  return L.clock_implied ? L.word[kFRem] == 0 && L.word[kFRem + 1] == 0 : L.word[kFClock] == 0;
}

bool resumable(const ModelHost& h) { return h.hetero || word0_orders_rounds(h); }

void plan_resume(const ModelHost& h, uint64_t T_done, const std::vector<PartPlan>& fresh,
                 std::vector<PartPlan>* out) {
  if (h.hetero) {
    // units of unequal speed: a configuration whose latest terminal clock is at most
    // T_done is done; otherwise its chain slices that end past T_done are kept (each
    // starts on a cut of the determined part, whose state is in the set when the cut's
    // clock is at most T_done, and the last one runs through the tails), and a
    // configuration the fresh plan does not cut continues from its SELECT state
    std::vector<uint8_t> seen(h.n_cfg, 0);
    for (const PartPlan& p : fresh) {
      if (p.cfg >= h.n_cfg) continue;
      const uint32_t c = p.cfg;
      seen[c] = 1;
      if (h.cfgs[c].tc <= T_done) continue;
      if (p.r0 == kChainSlice) {
        if (p.r1 != kNoClock && p.r1 <= T_done) continue;
        out->push_back(p);
      } else {
        out->push_back(PartPlan{c, 0u, kRoundsToEnd, h.cfg_states[c]});
      }
    }
    for (uint32_t c = 0; c < h.n_cfg; ++c)
      if (!seen[c] && h.cfgs[c].tc > T_done)
        out->push_back(PartPlan{c, 0u, kRoundsToEnd, h.cfg_states[c]});
    return;
  }
  // configurations that the fresh plan cuts into round blocks only keep those blocks past
  // T_done; every other one resumes as one partition
  std::vector<uint32_t> nparts(h.n_cfg, 0);
  std::vector<uint8_t> blocks(h.n_cfg, 1), done(h.n_cfg, 0);
  for (const PartPlan& p : fresh) {
    if (p.cfg >= h.n_cfg) continue;
    ++nparts[p.cfg];
    if (p.r0 == kRunSlice || p.r0 == kChainSlice || p.j1 != 0) blocks[p.cfg] = 0;
  }
  const auto whole = [&](uint32_t c) {
    const CfgRec& r = h.cfgs[c];
    const uint64_t rounds = (r.n + h.m - 1) / h.m;
    if (rounds * r.d <= T_done) return;  // its terminals are in already
    // round r0 starts at clock r0*d <= T_done: its start state was inserted, the states
    // of the round past T_done were not
    const uint64_t r0 = std::min<uint64_t>(T_done / r.d, rounds - 1);
    const uint64_t left = h.cfg_states[c] * (rounds - r0) / rounds + 1;
    out->push_back(PartPlan{c, (uint32_t)r0, kRoundsToEnd, left});
  };
  for (const PartPlan& p : fresh) {  // in the fresh plan's order (largest first)
    const uint32_t c = p.cfg;
    if (c >= h.n_cfg) continue;
    if (!blocks[c] || nparts[c] < 2) {
      if (!done[c]) whole(c);
      done[c] = 1;
      continue;
    }
    const CfgRec& r = h.cfgs[c];
    const uint64_t rounds = (r.n + h.m - 1) / h.m;
    if (rounds * r.d <= T_done) continue;
    const uint64_t rs = std::min<uint64_t>(T_done / r.d, rounds - 1);
    const uint64_t b = p.r1 == kRoundsToEnd ? rounds : p.r1;
    if (b <= rs) continue;  // every state of the block has clock <= b*d <= T_done
    const uint64_t a = std::max<uint64_t>(p.r0, rs);
    const uint64_t left = p.states * (b - a) / std::max<uint64_t>(1, b - p.r0) + 1;
    out->push_back(PartPlan{c, (uint32_t)a, p.r1, left});
  }
  for (uint32_t c = 0; c < h.n_cfg; ++c)  // configurations absent from the fresh plan
    if (!nparts[c]) whole(c);
}

uint64_t auto_part_states(uint64_t states, uint32_t m) {
  // about 640 partitions for small models (256 on one unit), down to blocks of
  // kMinBlockRounds rounds; blocks of at most 2^14 states for large ones.  With one-word
  // keys more partitions in flight pay: matmul64_cu4 0.48 -> 0.45 ms (376 -> 692 blocks),
  // abstract_s1024_np4_cu4 0.31 -> 0.26, minimum_s1024_np4_cu4 0.135 -> 0.125; on one
  // unit (abstract_s1024_np4_cu1) 0.27 -> 0.31 ms, so it keeps 256.
  const uint64_t parts = m == 1u ? 256u : 640u;
  return std::min<uint64_t>(1ull << 14, std::max<uint64_t>(1, states / parts));
}

// operation ends of one workgroup at or before time x
uint64_t ends_le(const CfgRec& r, uint64_t x) {
  if (x >= r.d) return r.b;
  const uint64_t w = x / r.dw;
  x -= w * r.dw;
  uint64_t c = 0;
  for (uint32_t j = 0; j < r.nph; ++j) {
    if (x < r.t0[j]) break;
    const uint64_t rel = x - r.t0[j], reps = rel / r.lat[j];
    const uint64_t k = r.la[j] ? 2 * reps + (rel - reps * r.lat[j] >= r.la[j] ? 1 : 0) : reps;
    c = r.i0[j] + std::min<uint64_t>(k, r.cnt[j]);
  }
  return w * r.bw + c;
}

uint64_t end_at_host(const CfgRec& r, uint64_t k) {
  const uint64_t w = k / r.bw;
  k -= w * r.bw;
  for (uint32_t j = 0; j < r.nph; ++j) {
    if (k >= (uint64_t)r.i0[j] + r.cnt[j]) continue;
    const uint64_t q = k - r.i0[j];
    const uint64_t t = r.la[j] ? r.t0[j] + (q / 2) * r.lat[j] + (q % 2 ? r.lat[j] : r.la[j])
                               : r.t0[j] + (q + 1) * r.lat[j];
    return w * r.dw + t;
  }
  return (w + 1) * r.dw;
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
    if (h.hetero) {  // no closed form: the configuration's whole bound
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

// fields: cfg, pending, clock, then the time left on every unit (packed as a busy mask
// and one shared time when the layout says so)
void encode_key_host(const Layout& L, const uint32_t* fields, uint64_t* words) {
  for (int j = 0; j < 4; ++j) words[j] = 0;
  uint32_t packed[kFields];
  for (int f = 0; f < 3 + L.m; ++f) packed[f] = fields[f];
  int nf = 3 + L.m;
  if (L.shared_rem) {
    uint32_t mask = 0, rem = 0;
    for (int u = 0; u < L.m; ++u)
      if (fields[kFRem + u]) {
        mask |= 1u << u;
        rem = fields[kFRem + u];
      }
    packed[kFRem] = mask;
    packed[kFRem + 1] = rem;
    nf = 5;
  }
  if (L.clock_implied) packed[kFClock] = 0;  // not stored
  for (int f = 0; f < nf; ++f) words[L.word[f]] |= (uint64_t)packed[f] << L.shift[f];
}

// cfgs: the configuration records, from which an implied clock is derived (as the
// device's implied_clock does)
void decode_key_host(const Layout& L, const uint64_t* words, uint32_t* fields, const CfgRec* cfgs) {
  const int nf = L.shared_rem ? 5 : 3 + L.m;
  for (int f = 0; f < nf; ++f)
    fields[f] = (uint32_t)((words[L.word[f]] >> L.shift[f]) & ((1ull << L.width[f]) - 1ull));
  if (L.shared_rem) {
    const uint32_t mask = fields[kFRem], rem = fields[kFRem + 1];
    for (int u = 0; u < L.m; ++u) fields[kFRem + u] = ((mask >> u) & 1u) ? rem : 0u;
    if (L.clock_implied) {
      const uint32_t c = fields[kFCfg];
      if (c >= L.n_cfg) {
        fields[kFClock] = 0;
      } else {
        const uint32_t done = cfgs[c].n - fields[kFPending] - (uint32_t)__builtin_popcount(mask);
        fields[kFClock] = (done + L.m - 1u) / L.m * cfgs[c].d + (mask ? cfgs[c].d - rem : 0u);
      }
    }
  }
}

}  // namespace mc
