"""Benchmark: explicit-state exploration throughput of one tuning query on one GPU.

One step = the whole query path on one model: load the model (validation, tables,
upload), min_time (root/SELECT seed, exploration, terminal-clock reduction, argmin),
the counterexample trace, and check(T_min - 1) (pruned exploration proving T_min is
minimal).  Inputs are synthetic (seeded latencies, the parameter domains of the
workload); the workspace stays resident in HBM across steps.

value = unique states explored (min_time + check) per second of step wall time.
The same step on the plain level-synchronous BFS engine and the CPU oracle are
reported beside it.  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LINE_BYTES = 64          # HBM access granule assumed per random visited-set touch


def graph_edges(mc, model) -> int | None:
    """Edges of the model's reachable state graph (root included), from its round
    structure, for models whose units all work alike: every configuration runs
    floor(n/m) full rounds (a closure over all 2^m unit subsets, m*2^(m-1) dispatch
    edges, then b ADVANCE edges) and, when n mod m = p > 0, one partial round (subsets
    of at most p units, then one b-step run from each of its C(m, p) leaves).  None for
    units of unequal speed, which have no such structure."""
    from math import comb
    if model.get("speed") is not None and len(set(model["speed"])) > 1:
        return None
    m = model["m"]
    edges = len(model["params"])  # SELECT
    for c in range(len(model["params"])):
        e = mc.mc_config_ends(model, c)
        n, b = e["n"], e["b"]
        q, p = divmod(n, m)
        edges += q * (m * (1 << (m - 1)) + b)
        if p:
            edges += sum(j * comb(m, j) for j in range(1, p + 1)) + comb(m, p) * b
    return edges


def bytes_per_state(key_bytes: int, r_dup: float) -> float:
    """Algorithmic HBM bytes per new state of a breadth-first exploration with an
    open-addressing visited set: one random line read-modify-write for the claim (key
    and parent in one line), the frontier write and read of the key, and one random
    line read per duplicate edge: 2L + 2S + r_dup * L."""
    return 2 * LINE_BYTES + 2 * key_bytes + r_dup * LINE_BYTES


def algo_bytes_per_state(mc, model, step) -> float:
    """bytes_per_state for the model's key width, with r_dup = duplicate edges of the
    state graph per reachable state (graph_edges), or, on units of unequal speed, the
    duplicate inserts the run counted."""
    key_bytes = 8 * mc.mc_describe(model)["key_words"]
    n = step["min_states"]
    edges = graph_edges(mc, model)
    dup = edges - (n - 1) if edges is not None else step["min_dups"]
    return bytes_per_state(key_bytes, dup / n)


def _progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mc_kernels.hip", "mc_device.h", "mc_launch.h"):
        with open(os.path.join(ROOT, "paper_2305_09130_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, kernel: str, src_hash: str, slots: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source with a visited set of the same size."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != src_hash or d.get("table_slots") != slots:
        return None
    return d.get("hbm_bytes_per_launch")


def run_step(mc, model, engine, workspace, block, load_factor=0.0, handle=None):
    """One tuning query: load the model (into `handle`, the query's handle kept across
    steps, when given; else into a new one, freed at the end), min_time, its trace and
    check(T_min - 1)."""
    t0 = time.perf_counter()
    if handle is not None:
        handle.mc_model_reload(model)
        g = handle
    else:
        g = mc.Model(model, engine=engine, block=block, workspace=workspace,
                     load_factor=load_factor)
    t1 = time.perf_counter()
    t_min, argmin = g.mc_min_time()
    st_min = dict(g.last_stats)
    t2 = time.perf_counter()
    trace = g.mc_trace()
    t3 = time.perf_counter()
    holds = not g.mc_check(t_min - 1)
    st_chk = dict(g.last_stats)
    slots = g.mc_model_info_get()["slots"]
    if handle is None:
        g.close()
    t4 = time.perf_counter()
    return {"t_min": t_min, "argmin": argmin, "trace_len": len(trace), "minimal": holds,
            "states": st_min["states"] + st_chk["states"], "min_states": st_min["states"],
            "min_dups": st_min["dups"],
            "engine_ns": st_min["engine_ns"] + st_chk["engine_ns"],
            "engine_ns_min": st_min["engine_ns"], "seconds": t4 - t0, "levels": st_min["levels"],
            "min_stats": {k: st_min[k] for k in ("probes", "max_probe", "dups", "edges",
                                                 "supersteps", "batches", "critical_ns",
                                                 "critical_cfg", "parts")},
            "parts": st_min["parts"], "slots": slots,
            "check_stats": {k: st_chk[k] for k in ("states", "probes", "max_probe", "supersteps",
                                                   "critical_ns", "critical_cfg", "parts")},
            "breakdown_ms": {"load": 1e3 * (t1 - t0), "min_time": 1e3 * (t2 - t1),
                             "min_time_engine": st_min["engine_ns"] / 1e6,
                             "min_time_clear": st_min["clear_ns"] / 1e6,
                             "trace": 1e3 * (t3 - t2), "check": 1e3 * (t4 - t3),
                             "check_engine": st_chk["engine_ns"] / 1e6,
                             "check_clear": st_chk["clear_ns"] / 1e6}}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(model, t_min=None, sample_every: int = 1):
    """The oracle as it stands, single-threaded and pinned to one host core (the
    process's affinity is narrowed for the call and restored), on the same query step:
    min_time then check(T_min - 1).  With sample_every = k only every k-th
    configuration is explored (a bounded sample of the same workload); t_min is then
    the sample's own.  Exploration time is measured inside the oracle."""
    import oracle
    oracle.build(force=False)
    sub = dict(model, params=model["params"][::sample_every]) if sample_every > 1 else model
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        r = oracle.explore(sub, trace=True)
        c = oracle.explore(sub, T=r["t_min"] - 1, trace=False)
        wall = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, before)
    states = r["reachable"] + c["reachable"]
    what = ("the whole workload" if sample_every == 1 else
            f"every {sample_every}th configuration ({len(sub['params'])} of "
            f"{len(model['params'])})")
    return {"value": states / (r["seconds"] + c["seconds"]), "unit": "states/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{what}: min_time ({r['reachable']} states) + check(T_min-1) "
                      f"({c['reachable']} states); exploration {r['seconds'] + c['seconds']:.2f} s, "
                      f"wall {wall:.2f} s",
            "pinned_core": core, "nproc": os.cpu_count(), "affinity_cores": len(before),
            "cpu_model": _cpu_model(),
            "agrees": (t_min is None or sample_every > 1 or r["t_min"] == t_min)}


BATCH_BUDGET = 1 << 20


def named_workload(workloads, name: str) -> dict:
    """A single-query workload by name: the three plain ones, the paper's unit models,
    or the models on units of unequal speed."""
    if name in workloads.WORKLOADS:
        return workloads.WORKLOADS[name]()
    if name in workloads.UNIT_WORKLOADS:
        return workloads.UNIT_WORKLOADS[name]()
    return workloads.hetero_workloads()[name]


def batched_leg(mc, torch, workloads, n_inst: int, reps: int, sample_alone: int):
    """The seeded mix of uneven instances explored in one persistent launch (hipGraph
    replay, autotuned options), against the same instances explored one at a time."""
    models, rejected = workloads.draw_batch(
        3, n_inst, lambda x: (mc.state_count(x) or BATCH_BUDGET + 1) <= BATCH_BUDGET)
    need = mc.mc_batch_workspace_bytes(models, mc.make_batch_opts(load_factor=0.25))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    t0 = time.perf_counter()
    _progress(f"autotuning the batch of {n_inst} ({len(models)} drawn, {rejected} redrawn)")
    best, best_ms = mc.mc_batch_autotune(models, ws)
    tune_s = time.perf_counter() - t0
    best.use_graph = 1
    b = mc.Batch(models, best, workspace=ws)
    b.mc_batch_min_time()  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        t_min, states = b.mc_batch_min_time()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    gpu_ms = b.last_stats["explore_ns"] / 1e6
    total = sum(states)
    b.close()
    del ws
    torch.cuda.empty_cache()
    # one at a time on a sample: each instance loaded into one handle over a preallocated
    # workspace (mc_model_reload), with the library's automatic launch options and with the
    # batch's autotuned ones; the faster of the two is the baseline
    idx = list(range(0, n_inst, max(1, n_inst // sample_alone)))[:sample_alone]
    variants = {
        "automatic": {},
        "autotuned": {"block": int(best.block), "load_factor": float(best.load_factor),
                      "lane_items": int(best.lane_items), "part_states": int(best.part_states)},
    }
    alone = {}
    for name, opts in variants.items():
        mo = mc.make_opts(**opts)
        ws1 = torch.empty(max(mc.mc_workspace_bytes(models[i], mo) for i in idx),
                          dtype=torch.uint8, device="cuda:0")
        g = mc.Model(models[idx[0]], workspace=ws1, **opts)  # warm; kept for every instance
        g.mc_min_time()
        torch.cuda.synchronize()
        t_alone, s_alone = 0.0, 0
        for i in idx:
            t1 = time.perf_counter()
            g.mc_model_reload(models[i])
            tm, _ = g.mc_min_time()
            s_alone += g.last_stats["states"]
            t_alone += time.perf_counter() - t1
            assert tm == t_min[i]
        g.close()
        del ws1
        torch.cuda.empty_cache()
        alone[name] = {"value": s_alone / t_alone, "queries_per_s": len(idx) / t_alone}
    base = max(alone, key=lambda k: alone[k]["value"])
    return {"instances": n_inst, "rejected_draws": rejected,
            "draw_filter": f"instances above {BATCH_BUDGET} states redrawn "
                           f"({rejected} of {rejected + n_inst} draws)",
            "states": total,
            "value": total / el, "unit": "states/s", "queries_per_s": n_inst / el,
            "ms_per_batch": 1e3 * el, "gpu_ms": gpu_ms,
            "autotuned": best.as_dict(), "autotune_s": tune_s,
            "one_at_a_time": {"sample": len(idx), "value": alone[base]["value"],
                              "queries_per_s": alone[base]["queries_per_s"],
                              "options": base, "variants": alone,
                              "how": "one handle over a preallocated workspace, each "
                                     "instance reloaded into it; the faster of the automatic "
                                     "and the batch's autotuned launch options"},
            "speedup_vs_one_at_a_time": (total / el) / alone[base]["value"]}


def swarm_leg(mc, workloads, names, members: int = 16384, bits_log2: int = 16,
              budget: int = 20000):
    """The swarm search of Sec. 5 on each named workload: one swarm against G(!FIN)
    (time to its first trail, that trail's optimality T_min / T_first), then the search
    loop with the over-time property; against the exact min_time on the same GPU (best
    of three launches).  The first trail is the first on the device clock, so which
    member's trail it is, and its optimality, can change from run to run."""
    out = {}
    # the swarm's bit arrays and member records live in the visited-set region
    need = members * ((1 << bits_log2) // 8 + 128)
    for name in names:
        model = named_workload(workloads, name)
        g = mc.Model(model)
        if g.mc_model_info_get()["slots"] * g.mc_model_info_get()["slot_bytes"] < need:
            g.close()
            g = mc.Model(model, log2_slots=max(10, (need // 16 - 1).bit_length()))
        t_min, _ = g.mc_min_time()
        exact_ms = g.last_stats["engine_ns"] / 1e6
        for _ in range(2):  # the first call also pays the first launch of its instance
            g.mc_min_time()
            exact_ms = min(exact_ms, g.last_stats["engine_ns"] / 1e6)
        r = g.mc_swarm(members, bits_log2, budget, 1)
        t0 = time.perf_counter()
        t_found, rounds, best = g.mc_swarm_tune(members, bits_log2, budget, 1)
        tune_s = time.perf_counter() - t0
        g.close()
        out[name] = {"members": members, "bits_per_member": 1 << bits_log2,
                     "budget_steps": budget, "t_min_exact": t_min, "exact_min_time_ms": exact_ms,
                     "first_trail_us": r["first_trail_ns"] / 1e3,
                     "first_trail_optimality": t_min / r["first_clock"],
                     "swarm_ms": r["swarm_ns"] / 1e6, "trails": r["trails"],
                     "walks": r["walks"], "best_of_one_swarm": r["best_clock"],
                     "search_t_found": t_found, "search_swarms": rounds,
                     "search_optimality": t_min / t_found, "search_wall_ms": 1e3 * tune_s}
    return out


def units_leg(mc, torch, workloads, reps: int = 5, cpu: bool = True):
    """The paper's own unit models (abstract kernel, Minimum problem; NP elements per
    unit, WG/NP waves) at S = 1024: the same step as the timed one (load + min_time +
    trace + check(T_min - 1)) on the super-step engine built for general phases, with
    its roofline figure and, on the CPU, the oracle on the same step."""
    return model_leg(mc, torch, {k: f() for k, f in workloads.UNIT_WORKLOADS.items()},
                     reps, cpu)


def hetero_leg(mc, torch, workloads, reps: int = 5, cpu: bool = True):
    """Models on units of unequal speed (1, 1, 2, 3): the same step, the general-phase
    engine with determined ADVANCE chains, and the oracle on the same step."""
    return model_leg(mc, torch, workloads.hetero_workloads(), reps, cpu)


def model_leg(mc, torch, models: dict, reps: int, cpu: bool):
    out = {}
    for name, model in models.items():
        nbytes = mc.mc_workspace_bytes(model)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        g = mc.Model(model, workspace=ws)
        run_step(mc, model, mc.MC_ENGINE_SUPERSTEP, ws, 0, handle=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = [run_step(mc, model, mc.MC_ENGINE_SUPERSTEP, ws, 0, handle=g)
                 for _ in range(reps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        g.close()
        del ws
        states = sum(s["states"] for s in steps)
        eng_s = sum(s["engine_ns_min"] for s in steps) * 1e-9 / reps
        bps = algo_bytes_per_state(mc, model, steps[0])
        achieved = steps[0]["min_states"] * bps / eng_s / 1e9
        rec = {"kind": model["kind"], "cu": model["m"], "configurations": len(model["params"]),
               "Lg": model["Lg"], "Ll": model["Ll"],
               "reachable": steps[0]["min_states"], "levels": steps[0]["levels"],
               "t_min": steps[0]["t_min"], "argmin": steps[0]["argmin"],
               "ms_per_step": 1e3 * elapsed / reps, "states_per_s": states / elapsed,
               "min_time_engine_ms": eng_s * 1e3, "roofline_frac": achieved / HBM_PEAK_GBS,
               "algo_bytes_per_state": bps,
               "partitions": steps[0]["parts"],
               "step_breakdown_ms": {k: sum(s["breakdown_ms"][k] for s in steps) / reps
                                     for k in steps[0]["breakdown_ms"]}}
        for k in ("S", "NP", "G", "M", "N", "K", "speed"):
            if k in model:
                rec[k] = model[k]
        if cpu:
            c = cpu_baseline(model, steps[0]["t_min"])
            rec["cpu_oracle_states_per_s"] = c["value"]
            rec["cpu_oracle_agrees"] = c["agrees"]
            rec["gpu_over_cpu"] = rec["states_per_s"] / c["value"]
        out[name] = rec
        _progress(f"model leg: {name} {rec['ms_per_step']:.2f} ms/step")
    return out


def bb_leg(mc, torch, workloads, names, reps: int = 5):
    """Step 3 of the method three ways on one handle: exhaustive min_time; a simulated
    run's time T_ini followed by bisection over check(T) (the paper's loop); T_ini
    followed by one branch-and-bound search.  Wall time per query (host clock, queries
    synchronous) and the states each claimed."""
    out = {}
    for name in names:
        model = named_workload(workloads, name)
        g = mc.Model(model)
        g.mc_min_time()
        g.mc_min_time_bb(0)
        rec = {}

        def timed(fn):
            ts, res = [], None
            for _ in range(reps):
                t0 = time.perf_counter()
                res = fn()
                ts.append(time.perf_counter() - t0)
            return 1e3 * sorted(ts)[len(ts) // 2], res

        ms, (t_min, _) = timed(g.mc_min_time)
        rec["exhaustive"] = {"ms": ms, "states": g.last_stats["states"],
                             "engine_ms": g.last_stats["engine_ns"] / 1e6}

        def bisect():
            return g.mc_tune_bisect(7)
        ms, (t_b, n_checks) = timed(bisect)
        rec["bisection"] = {"ms": ms, "checks": n_checks, "states": g.last_stats["states"],
                            "engine_ms": g.last_stats["engine_ns"] / 1e6}

        def bb():
            t_ini, _ = g.mc_simulate(7)
            return g.mc_min_time_bb(t_ini)
        ms, (t_bb, _) = timed(bb)
        rec["branch_and_bound"] = {"ms": ms, "states": g.last_stats["states"],
                                   "engine_ms": g.last_stats["engine_ns"] / 1e6,
                                   "clear_ms": g.last_stats["clear_ns"] / 1e6}
        ms, (t_bb0, _) = timed(lambda: g.mc_min_time_bb(0))
        rec["branch_and_bound_no_init"] = {"ms": ms, "states": g.last_stats["states"],
                                           "engine_ms": g.last_stats["engine_ns"] / 1e6,
                                           "clear_ms": g.last_stats["clear_ns"] / 1e6}
        g.close()
        assert t_min == t_b == t_bb == t_bb0
        rec["t_min"] = t_min
        rec["bb_speedup_vs_exhaustive"] = rec["exhaustive"]["ms"] / rec["branch_and_bound"]["ms"]
        rec["bb_speedup_vs_bisection"] = rec["bisection"]["ms"] / rec["branch_and_bound"]["ms"]
        out[name] = rec
        _progress(f"bb leg: {name} exhaustive {rec['exhaustive']['ms']:.2f} ms, bisection "
                  f"{rec['bisection']['ms']:.2f} ms, bb {rec['branch_and_bound']['ms']:.2f} ms")
    return out


def served_leg(mc, torch, workloads, n_queries: int, qps_factors, pool_size: int = 32):
    """Poisson arrivals of check(T)/min_time queries over a pool of models: the
    continuous-batching engine against FIFO one-query-at-a-time service, both run in
    real time under the same arrival stream.  FIFO service loads each query's model into
    one handle over a preallocated workspace (mc_model_reload) with the library's
    automatic launch options."""
    pool, rejected = workloads.draw_batch(
        4, pool_size, lambda x: (mc.state_count(x) or BATCH_BUDGET + 1) <= BATCH_BUDGET)
    mix = workloads.query_mix(4, n_queries, pool_size)
    ws = torch.empty(max(mc.mc_workspace_bytes(m) for m in pool), dtype=torch.uint8,
                     device="cuda:0")
    tmins = []  # the threshold recipe needs each model's T_min: one untimed GPU query each
    for m in pool:
        g = mc.Model(m, workspace=ws)
        tmins.append(g.mc_min_time()[0])
        g.close()
    qs = [(i, kind, int(u * tmins[i])) for i, kind, u in mix]

    fifo = mc.Model(pool[0], workspace=ws)  # the FIFO server's one handle

    def serve_one(i, kind, T):
        fifo.mc_model_reload(pool[i])
        if kind == "min_time":
            fifo.mc_min_time()
        else:
            fifo.mc_check(T)

    # FIFO capacity: every query of the stream served back to back
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in qs:
        serve_one(*q)
    fifo_capacity = n_queries / (time.perf_counter() - t0)
    out = {"queries": n_queries, "pool": pool_size, "rejected_draws": rejected,
           "draw_filter": f"models above {BATCH_BUDGET} states redrawn",
           "fifo_capacity_qps": fifo_capacity, "runs": []}

    def pct(xs, p):
        xs = sorted(xs)
        return xs[min(len(xs) - 1, int(p * len(xs)))]

    def wait_until(t0, a):
        while True:
            d = a - (time.perf_counter() - t0)
            if d <= 0:
                return
            if d > 2e-3:
                time.sleep(d - 1e-3)

    for f in qps_factors:
        _progress(f"served run at {f}x the FIFO capacity")
        qps = f * fifo_capacity
        arr = workloads.poisson_arrivals(4, n_queries, qps)
        # FIFO one at a time, in real time
        lat_fifo = []
        t0 = time.perf_counter()
        for k, q in enumerate(qs):
            wait_until(t0, arr[k])
            serve_one(*q)
            lat_fifo.append(time.perf_counter() - t0 - arr[k])
        fifo_wall = time.perf_counter() - t0
        # continuous batching engine, driven in real time: with each model's state kept
        # resident between its queries, and (at 1x) with every query explored afresh
        run = {"qps_offered": qps, "factor": f,
               "fifo_p50_ms": 1e3 * pct(lat_fifo, 0.5), "fifo_p99_ms": 1e3 * pct(lat_fifo, 0.99),
               "fifo_queries_per_s": n_queries / fifo_wall}
        for no_reuse in ((False, True) if f == 1.0 else (False,)):
            r_ = serve_engine(mc, torch, pool, qs, arr, no_reuse)
            if no_reuse:
                run["no_reuse"] = r_
            else:
                run.update(r_)
        out["runs"].append(run)
    fifo.close()
    del ws
    torch.cuda.empty_cache()
    return out


def serve_engine(mc, torch, pool, qs, arr, no_reuse: bool) -> dict:
    """Drives the engine in real time under the arrival stream `arr`; latency from
    arrival to completion on the host's monotonic clock."""
    n_queries = len(qs)
    e = mc.Engine(arena_bytes=24 << 30, max_active=128, max_cfg=512, block=512, slice=16,
                  no_reuse=no_reuse)
    tickets = []
    # arrivals are offsets from t0; the library stamps completions on the same monotonic
    # clock (CLOCK_MONOTONIC) as time.monotonic_ns
    t0_ns = time.monotonic_ns()
    t0 = time.perf_counter()
    nxt = 0
    busy = True
    while nxt < n_queries or busy:
        now = time.perf_counter() - t0
        while nxt < n_queries and arr[nxt] <= now:
            i, kind, T = qs[nxt]
            tickets.append(e.mc_engine_submit(
                pool[i], mc.MC_QUERY_MIN_TIME if kind == "min_time" else mc.MC_QUERY_CHECK, T))
            nxt += 1
        a_, w_ = e.mc_engine_step()
        busy = a_ + w_ > 0
        if not busy and nxt < n_queries:
            time.sleep(max(0.0, min(arr[nxt] - (time.perf_counter() - t0), 0.001)))
    e.drain()
    wall = time.perf_counter() - t0
    lat = []
    reuse = [0, 0, 0]
    by_kind = {0: [], 1: [], 2: []}  # latency and admission wait per way of service
    for k, t in enumerate(tickets):
        r = e.mc_engine_poll(t)
        assert r is not None and r["status"] == 0
        reuse[r["reuse"]] += 1
        lat.append((r["done_ns"] - t0_ns) * 1e-9 - arr[k])
        by_kind[r["reuse"]].append((lat[-1], (r["admit_ns"] - r["submit_ns"]) * 1e-9, k))
    e.close()
    torch.cuda.empty_cache()
    first = [x for k, x in enumerate(lat) if k < 100]
    lat.sort()

    def q(xs, p):
        xs = sorted(xs)
        return 1e3 * xs[min(len(xs) - 1, int(p * len(xs)))] if xs else None

    names = {0: "explored_fresh", 1: "resumed", 2: "answered_from_resident"}
    return {"queries_per_s": n_queries / wall,
            "p50_ms": 1e3 * lat[min(len(lat) - 1, int(0.5 * len(lat)))],
            "p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            "explored_fresh": reuse[0], "resumed": reuse[1], "answered_from_resident": reuse[2],
            "hit_rate": (reuse[1] + reuse[2]) / n_queries,
            "first_100_p99_ms": q(first, 0.99),
            "by_service": {names[k]: {"n": len(v), "p50_ms": q([x[0] for x in v], 0.5),
                                      "p99_ms": q([x[0] for x in v], 0.99),
                                      "max_ms": q([x[0] for x in v], 1.0),
                                      "admit_wait_p99_ms": q([x[1] for x in v], 0.99),
                                      "mean_arrival_index":
                                          sum(x[2] for x in v) / len(v) if v else None}
                           for k, v in by_kind.items()}}


def peak_leg(buf_bytes: int) -> dict:
    """Random-access peaks of the device on a buffer of the visited set's size class."""
    from paper_2305_09130_amd import peak
    return peak.measure(buf_bytes=buf_bytes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="matmul128_vw_cu8")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = library default)")
    ap.add_argument("--load-factor", type=float, default=0.0)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-instances", type=int, default=512)
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--legs", default="peak,plain,cpu,batch,serve,swarm,units,bb,hetero",
                    help="extra legs beside the timed single-query step")
    ap.add_argument("--cpu-sample-states", type=int, default=16_000_000,
                    help="largest state count the CPU oracle explores: every k-th "
                         "configuration of the workload, k the least that fits")
    ap.add_argument("--peak-buffer-gib", type=int, default=8,
                    help="buffer of the random-access peak probes (GiB, a power of two)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the exploration "
              "shards by configuration subgraphs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2305_09130_amd as mc

    if args.copy_probe_mib:
        # a copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters give the factor
        # that turns those counters into bytes for the exploration kernel
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    model = named_workload(workloads, args.workload)
    nbytes = max(mc.mc_workspace_bytes(model, mc.make_opts(engine=e, block=args.block,
                                                          load_factor=args.load_factor))
                 for e in (0, 1))
    workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    # the input as a caller holds it: the parameter table as a uint32 array (the step still
    # validates, builds, plans and uploads the model)
    import numpy as np
    model_in = dict(model, params=np.ascontiguousarray(model["params"], dtype=np.uint32))
    # the query handle over the workspace, kept across steps: each step reloads its model
    handle = mc.Model(model_in, engine=mc.MC_ENGINE_SUPERSTEP, block=args.block,
                      workspace=workspace, load_factor=args.load_factor)
    for _ in range(args.warmup):
        run_step(mc, model_in, mc.MC_ENGINE_SUPERSTEP, workspace, args.block, args.load_factor,
                 handle=handle)
    torch.cuda.synchronize()
    steps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        steps.append(run_step(mc, model_in, mc.MC_ENGINE_SUPERSTEP, workspace, args.block,
                              args.load_factor, handle=handle))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    handle.close()  # before the workspace serves other handles
    states = sum(s["states"] for s in steps)
    assert all(s["minimal"] for s in steps)
    lat = sorted(s["seconds"] for s in steps)

    def pct(p):
        return lat[min(len(lat) - 1, int(p * len(lat)))]

    # roofline of the dominant kernel (the persistent super-step engine), per launch:
    # the min_time launch, timed with HIP events on the query's stream
    eng_s = sum(s["engine_ns_min"] for s in steps) * 1e-9 / len(steps)
    bps = algo_bytes_per_state(mc, model, steps[-1])
    algo_bytes = steps[-1]["min_states"] * bps
    achieved = algo_bytes / eng_s / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(args.workload, "k_superstep", src_hash, steps[-1]["slots"])

    legs = set(x for x in args.legs.split(",") if x)
    _progress(f"timed step done: {1e3 * elapsed / args.steps:.3f} ms/step")
    peak = None
    if "peak" in legs:
        peak = peak_leg(args.peak_buffer_gib << 30)
        _progress(f"peak leg: random CAS {peak['random_cas_per_s'] / 1e9:.2f} G/s, random 64-B "
                  f"reads {peak['random_read_GBps']:.0f} GB/s, copy {peak['copy_GBps']:.0f} GB/s")
    plain = None
    if args.plain_steps > 0 and "plain" in legs:
        ps = [run_step(mc, model, mc.MC_ENGINE_LEVEL, workspace, args.block, args.load_factor)
              for _ in range(args.plain_steps)]
        p_states = sum(s["states"] for s in ps)
        p_time = sum(s["seconds"] for s in ps)
        plain = {"engine": "level-synchronous BFS, one launch per level",
                 "value": p_states / p_time, "unit": "states/s",
                 "ms_per_step": 1e3 * p_time / len(ps), "steps": len(ps),
                 "levels": ps[0]["levels"],
                 "speedup": (states / elapsed) / (p_states / p_time)}
        assert all(s["t_min"] == steps[0]["t_min"] for s in ps)

    _progress("plain BFS leg done" if plain else "plain BFS leg skipped")
    cpu = None
    if not args.no_cpu and "cpu" in legs:
        k = 1
        while (mc.state_count(dict(model, params=model["params"][::k])) or 0) > \
                args.cpu_sample_states:
            k += 1
        cpu = cpu_baseline(model, steps[0]["t_min"], sample_every=k)
    batched = served = None
    if "batch" in legs:
        _progress("cpu leg done; batched leg")
        batched = batched_leg(mc, torch, workloads, args.batch_instances, 5, 16)
    if "serve" in legs:
        _progress("batched leg done; served leg")
        served = served_leg(mc, torch, workloads, args.serve_queries, (0.5, 1.0, 2.0))
    swarm = None
    if "swarm" in legs:
        _progress("swarm leg")
        swarm = swarm_leg(mc, workloads, ["reduction_g256_cu4_s1123", "matmul32_cu4_s1123",
                                          args.workload])
    bbr = None
    if "bb" in legs:
        _progress("branch-and-bound leg")
        bbr = bb_leg(mc, torch, workloads,
                     list(dict.fromkeys([args.workload, "reduction_g256_cu2", "matmul64_cu4",
                                         "matmul128_vw_cu8", "abstract_s1024_np4_cu4",
                                         "matmul32_cu4_s1123"])))
    hetero = None
    if "hetero" in legs:
        _progress("unequal-units leg")
        hetero = hetero_leg(mc, torch, workloads, cpu=not args.no_cpu and "cpu" in legs)
    units = None
    if "units" in legs:
        _progress("unit-model leg")
        units = units_leg(mc, torch, workloads, cpu=not args.no_cpu and "cpu" in legs)

    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_superstep", "launch": "min_time exploration",
                "algo_bytes_per_state": bps, "algo_bytes_per_launch": algo_bytes,
                "states_per_launch": steps[-1]["min_states"],
                "avg_launch_ms": eng_s * 1e3, "kernel_source_hash": src_hash,
                "table_slots": steps[-1]["slots"]}
    if peak:
        # the measured random-access ceiling: random 64-byte line reads (the granule of
        # every visited-set touch) and random 64-bit CAS (one per claim)
        roofline["peak_measured"] = peak["random_read_GBps"]
        roofline["frac_measured"] = achieved / peak["random_read_GBps"]
        roofline["states_per_s_launch"] = steps[-1]["min_states"] / eng_s
        roofline["cas_peak_per_s"] = peak["random_cas_per_s"]
        roofline["states_over_cas_peak"] = roofline["states_per_s_launch"] / peak["random_cas_per_s"]
        roofline["peak_probe"] = peak
    cfg = {"workload": args.workload, "kind": model["kind"], "cu": model["m"],
           "configurations": len(model["params"]),
           "Lg": model["Lg"], "Ll": model["Ll"], "Lc": model.get("Lc", 1), "Lb": model.get("Lb", 0),
           "states_per_step": steps[0]["states"], "reachable": steps[0]["min_states"],
           "t_min": steps[0]["t_min"], "argmin": steps[0]["argmin"],
           "trace_len": steps[0]["trace_len"], "block": args.block,
           "load_factor": args.load_factor or 0.5,
           "step": "load + min_time + trace + check(T_min-1)"}
    for k in ("G", "M", "N", "K", "S", "NP", "speed"):
        if k in model:
            cfg[k] = model[k]
    out = {
        "metric": "states/sec explored + tuning queries/sec, p50/p99 latency vs plain BFS",
        "value": states / elapsed,
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": cfg,
        "tuning_queries_per_s": args.steps / elapsed,
        "step_breakdown_ms": {k: sum(s["breakdown_ms"][k] for s in steps) / len(steps)
                              for k in steps[0]["breakdown_ms"]},
        "partitions": steps[0]["parts"],
        "min_time_stats": steps[-1]["min_stats"],
        "check_stats": steps[-1]["check_stats"],
        "latency_ms": {"p50": 1e3 * pct(0.5), "p99": 1e3 * pct(0.99)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_bfs": plain,
        "batched": batched,
        "served": served,
        "swarm": swarm,
        "unit_models": units,
        "branch_and_bound": bbr,
        "unequal_units": hetero,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
