"""GPU parity on units of unequal speed (the paper's assumption that every unit works
alike, dropped) against the CPU oracle, through the C ABI: T_min, the argmin set, the
per-configuration least clocks, the reachable count (count_T under pruning) and the
verdict bit-exact; traces replayed through the oracle; the seeded walk and the swarm
members equal the oracle's.  The graph is not graded here, so BFS levels are compared
for the level engine only.
"""
import sys

import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ENGINES = {"superstep": 0, "level": 1}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_09130_amd as mc
    return mc


def check_min_time(g, model, r, engine):
    t_min, argmin = g.mc_min_time()
    st = g.last_stats
    assert (t_min, argmin) == (r["t_min"], r["argmin"])
    assert st["states"] == r["reachable"]
    assert st["terminals"] == r["terminals"]
    if engine == ENGINES["level"]:
        assert st["levels"] == r["levels"]
    else:
        # the super-step engine reports each state's depth at its first claim: at least its
        # BFS depth, at most the longest path to it
        assert r["levels"] <= st["levels"] <= g.mc_model_info_get()["max_depth"] + 1
    assert st["probes"] >= st["states"] + st["dups"]
    assert st["cas_fail"] == st["probes"] - st["states"] - st["dups"]
    assert g.mc_terminal_clocks() == r["tc"]
    oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])


def check_threshold(mc, g, model, T):
    r = oracle.explore(model, T=T, trace=False)
    v = g.mc_check(T)
    assert v == r["violated"], T
    assert g.last_stats["states"] == r["reachable"], T
    assert g.mc_terminal_clocks() == r["tc"], T
    if v:
        oracle.check_trace(model, g.mc_trace(), max_clock=T)
    else:
        with pytest.raises(mc.McError):
            g.mc_trace()


@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_hetero_tiny_sweep(mc, engine):
    cases = workloads.tiny_hetero_models(601, 50, max_cu=8) + workloads.tiny_hetero_models(602, 20)
    for i, model in enumerate(cases):
        _say(f"hetero tiny[{i}] engine={engine} {workloads.describe(model)}")
        r = oracle.explore(model)
        g = mc.Model(model, engine=ENGINES[engine])
        check_min_time(g, model, r, ENGINES[engine])
        for T in (r["t_min"] - 1, r["t_min"], max(r["tc"]) - 1):
            check_threshold(mc, g, model, T)
        g.close()


@pytest.mark.parametrize("name", sorted(workloads.hetero_workloads()))
def test_hetero_workloads_full_size(mc, name):
    model = workloads.hetero_workloads()[name]
    _say(f"{name} min_time")
    r = oracle.explore(model)
    g = mc.Model(model)
    check_min_time(g, model, r, ENGINES["superstep"])
    for T in sorted({r["t_min"] - 1, r["t_min"], (r["t_min"] + max(r["tc"])) // 2}):
        _say(f"  check T={T}")
        check_threshold(mc, g, model, T)
    _say("  branch and bound")
    assert g.mc_min_time_bb(0) == (r["t_min"], r["argmin"])
    oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
    g.close()


def test_hetero_simulate_and_bisect(mc):
    for model in workloads.tiny_hetero_models(603, 20, max_cu=6):
        g = mc.Model(model)
        for seed in (1, 2, 3):
            assert g.mc_simulate(seed) == oracle.simulate(model, seed), workloads.describe(model)
        r = oracle.explore(model, trace=False)
        assert g.mc_tune_bisect(5)[0] == r["t_min"]
        g.close()


SWARM_KEYS = ("walks", "trails", "steps", "best_walk_start", "first_step", "best_clock",
              "best_cfg", "first_clock", "first_cfg")


def test_hetero_swarm_members_equal_oracle(mc):
    for model in (workloads.hetero_workloads()["reduction_g256_cu4_s1123"],
                  workloads.tiny_hetero_models(604, 1, max_cu=4)[0]):
        r = oracle.explore(model, trace=False)
        g = mc.Model(model, log2_slots=22)
        for T in (None, r["t_min"], r["t_min"] - 1):
            _say(f"hetero swarm T={T} {workloads.describe(model)}")
            res = g.mc_swarm(64, 12, 20000, 9, T)
            gpu = g.mc_swarm_members(64)
            ora = oracle.swarm(model, 9, 64, 20000, 12, T)
            for i, (a, b) in enumerate(zip(gpu, ora)):
                assert {k: a[k] for k in SWARM_KEYS} == {k: b[k] for k in SWARM_KEYS}, (T, i)
            if res["trails"]:
                oracle.check_trace(model, g.mc_swarm_trace(), target_clock=res["best_clock"],
                                   cfgs=[res["best_cfg"]])
        g.close()


def test_hetero_batch_and_served(mc):
    models = workloads.tiny_hetero_models(605, 20, max_cu=8) + workloads.tiny_models(606, 8)
    _say(f"batch of {len(models)} models, unequal and equal units")
    b = mc.Batch(models, mc.make_batch_opts(block=256))
    t_min, states = b.mc_batch_min_time()
    for i, m in enumerate(models):
        r = oracle.explore(m, trace=False)
        assert (t_min[i], states[i]) == (r["t_min"], r["reachable"]), workloads.describe(m)
        assert b.mc_batch_terminal_clocks(i) == r["tc"]
    b.close()
    pool = workloads.tiny_hetero_models(607, 6, max_cu=4)
    e = mc.Engine(arena_bytes=64 << 20, max_active=3, slice=2)
    qs = []
    for i, m in enumerate(pool):
        r = oracle.explore(m, trace=False)
        qs += [(i, "min_time", 0), (i, "check", r["t_min"] - 1), (i, "check", r["t_min"])]
    tickets = [e.mc_engine_submit(pool[i], mc.MC_QUERY_MIN_TIME if k == "min_time"
                                  else mc.MC_QUERY_CHECK, T) for i, k, T in qs]
    e.drain()
    traced = 0
    for (i, kind, T), t in zip(qs, tickets):
        res = e.mc_engine_poll(t)
        assert res["done"] == 1 and res["status"] == 0
        r = oracle.explore(pool[i], T=None if kind == "min_time" else T, trace=False)
        full = oracle.explore(pool[i], trace=False)
        assert res["states"] == r["reachable"], (i, kind, T)
        if kind == "min_time":
            assert res["t_min"] == r["t_min"]
        else:
            assert res["violated"] == int(r["violated"])
        if kind == "min_time" or r["violated"]:
            assert e.mc_engine_argmin(t) == full["argmin"], (i, kind, T)
            try:   # readable while the model's state is still resident
                rows = e.mc_engine_trace(t, pool[i]["m"])
            except mc.McError as err:
                assert err.code == mc.MC_E_STATE
                continue
            oracle.check_trace(pool[i], rows, target_clock=full["t_min"], cfgs=full["argmin"])
            traced += 1
    assert traced >= 3
    e.close()


def _chain_models():
    w = workloads
    return [w.with_speeds(w.reduction_model(G, m, w.pow2_range(0, 3), w.pow2_range(0, 1),
                                            *w.latencies(2)), sp)
            for G, m, sp in ((128, 3, [1, 2, 3]), (256, 2, [1, 3]), (64, 4, [1, 1, 2, 5]))]


@pytest.mark.parametrize("block,batch_items", [(256, 0), (512, 0), (1024, 0), (256, 64),
                                               (512, 600)])
def test_hetero_chains_across_dispatches(mc, block, batch_items):
    """Workgroups of up to 257 operations: a batch lists chain after chain, through the
    determined dispatches between them and past chains cut by their candidate window,
    until a choice among units, a terminal, the threshold or the batch's room ends it."""
    for model in _chain_models():
        _say(f"chains block={block} batch_items={batch_items} {workloads.describe(model)}")
        r = oracle.explore(model)
        g = mc.Model(model, block=block, batch_items=batch_items)
        check_min_time(g, model, r, ENGINES["superstep"])
        for T in sorted({r["t_min"] - 1, r["t_min"], max(r["tc"]) // 2}):
            check_threshold(mc, g, model, T)
        assert g.mc_min_time_bb(0) == (r["t_min"], r["argmin"])
        oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
        g.close()


def test_hetero_simulate_full_size(mc):
    """The seeded run on the full-size workloads, whose stretches between dispatches the
    wavefront crosses a window of operation ends at a time: the same terminal (clock and
    configuration) as the oracle's one-step-at-a-time walk, hence the same step count
    at every draw."""
    for model in list(workloads.hetero_workloads().values()) + _chain_models():
        g = mc.Model(model)
        for seed in range(1, 9):
            assert g.mc_simulate(seed) == oracle.simulate(model, seed), (
                workloads.describe(model), seed)
        g.close()


@pytest.mark.parametrize("part_states", [32, 100, 400])
def test_hetero_chain_slices(mc, part_states):
    """The determined part of each configuration cut into chain slices of about
    `part_states` states, explored by separate workgroups that share only their boundary
    states: counts, clocks, verdicts and traces stay the oracle's."""
    cases = (workloads.tiny_hetero_models(611, 24, max_cu=6)
             + [workloads.with_speeds(workloads.reduction_model(128, 3, [1, 2, 4], [1, 2], 9, 2),
                                      [1, 2, 3]),
                workloads.with_speeds(workloads.reduction_model(256, 4, [2, 4], [1, 4], 7, 3),
                                      [1, 1, 2, 3])])
    for model in cases:
        _say(f"chain slices {part_states}: {workloads.describe(model)}")
        r = oracle.explore(model, trace=False)
        g = mc.Model(model, part_states=part_states)
        check_min_time(g, model, r, ENGINES["superstep"])
        for T in sorted({r["t_min"] - 1, r["t_min"], (r["t_min"] + max(r["tc"])) // 2}):
            if T >= 0:
                check_threshold(mc, g, model, T)
        g.close()


def test_hetero_workloads_sliced_full_size(mc):
    """The two full-size workloads at the automatic cut (chain slices of about
    states/640): exact against the oracle, with traces."""
    for name, model in workloads.hetero_workloads().items():
        _say(f"full size {name}")
        r = oracle.explore(model, trace=False)
        g = mc.Model(model)
        assert g.last_stats == {} and g.mc_min_time() == (r["t_min"], r["argmin"])
        st = g.last_stats
        assert st["states"] == r["reachable"] and st["parts"] > len(model["params"])
        assert g.mc_terminal_clocks() == r["tc"]
        oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
        g.close()


def _long_chain_models():
    """One 16-item workgroup per dispatch with K / 16 * 80 operation ends (b): chains
    between dispatches and the tails after the last one run from a few hundred to many
    thousand states."""
    w = workloads
    return [(w.with_speeds(w.matmul_model(16, 16, K, m, [16], [1], [1], [1], 23, 3), sp), b)
            for K, m, sp, b in ((64, 2, [1, 2], 320), (128, 2, [1, 2], 640),
                                (256, 3, [1, 2, 3], 1280), (1024, 2, [2, 1], 5120))]


def test_hetero_long_chain_traces(mc):
    """Counterexamples through long chains of units of unequal speed, replayed through the
    oracle: the trace rebuilds a chain wavefront-wide from the state it starts from (several
    candidate ends per lane at b = 320), and follows parent links one state at a time where
    a chain has more than 1,024 candidate ends (the tails at b = 640 and 1280, the chains of
    b = 5120)."""
    for model, b in _long_chain_models():
        _say(f"long chains b={b}: {workloads.describe(model)}")
        assert len(mc.mc_config_ends(model, 0)["E"]) == b
        r = oracle.explore(model)
        g = mc.Model(model)
        check_min_time(g, model, r, ENGINES["superstep"])
        for T in (r["t_min"] - 1, r["t_min"]):
            check_threshold(mc, g, model, T)
        g.close()
