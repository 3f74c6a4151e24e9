"""GPU parity of the unit-model kinds (abstract kernel of Sec. 4, Minimum problem of
Sec. 7) through the C ABI, against the CPU oracle: bit-exact T_min, argmin, per-
configuration clocks, reachable counts (count_T under pruning) and BFS levels; traces
replayed through the oracle.  These models have operation lists with waves and
two-operation periods, so they run the super-step engine built for general phases.
"""
import sys

import pytest

import oracle
import workloads
from oracle import closed_form as cf

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


_REF = {}


def ref(name, model, T=None):
    key = (name, T)
    if key not in _REF:
        _REF[key] = oracle.explore(model, T=T)
    return _REF[key]


def check_min_time(g, model, r):
    t_min, argmin = g.mc_min_time()
    st = g.last_stats
    assert (t_min, argmin) == (r["t_min"], r["argmin"])
    assert st["states"] == r["reachable"]
    assert st["levels"] == r["levels"]
    assert st["terminals"] == r["terminals"]
    assert g.mc_terminal_clocks() == r["tc"]
    tr = g.mc_trace()
    assert len(tr) == len(r["trace"])
    oracle.check_trace(model, tr, target_clock=r["t_min"], cfgs=r["argmin"])


def check_threshold(mc, g, model, T, r):
    v = g.mc_check(T)
    assert v == r["violated"], (T, v)
    assert g.last_stats["states"] == r["reachable"], T
    assert g.mc_terminal_clocks() == r["tc"]
    if v:
        oracle.check_trace(model, g.mc_trace(), max_clock=T)
    else:
        with pytest.raises(mc.McError):
            g.mc_trace()


@pytest.mark.parametrize("name", sorted(workloads.UNIT_WORKLOADS))
def test_unit_workload_full_size(mc, name):
    model = workloads.UNIT_WORKLOADS[name]()
    _say(f"{name} min_time (super-step)")
    r = ref(name, model)
    g = mc.Model(model)
    check_min_time(g, model, r)
    for T in sorted({r["t_min"] - 1, r["t_min"], r["t_min"] // 2,
                     (r["t_min"] + max(r["tc"])) // 2}):
        _say(f"  check T={T}")
        check_threshold(mc, g, model, T, ref(name, model, T))
    g.close()


@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_unit_tiny_sweep(mc, engine):
    cases = workloads.tiny_unit_models(401, 40, max_cu=8) + workloads.tiny_unit_models(402, 20)
    for i, model in enumerate(cases):
        _say(f"unit tiny[{i}] engine={engine} {workloads.describe(model)}")
        r = oracle.explore(model)
        g = mc.Model(model, engine=ENGINES[engine])
        check_min_time(g, model, r)
        for T in (r["t_min"] - 1, r["t_min"]):
            check_threshold(mc, g, model, T, oracle.explore(model, T=T))
        g.close()


@pytest.mark.parametrize("part_states", [1, 4096, 0xFFFFFFFF])
def test_unit_round_blocks(mc, part_states):
    """Subgraphs cut into blocks of whole rounds (waves inside every round)."""
    name = "minimum_s1024_np4_cu4"
    model = workloads.UNIT_WORKLOADS[name]()
    _say(f"{name} part_states={part_states:#x}")
    g = mc.Model(model, part_states=part_states)
    check_min_time(g, model, ref(name, model))
    g.close()
    small = workloads.unit_model(workloads.KIND_ABSTRACT, 64, 2, 3, [1, 2, 4, 8], [1, 2], 3, 1)
    _say(f"abstract S=64 m=3 part_states={part_states:#x}")
    g = mc.Model(small, part_states=part_states)
    check_min_time(g, small, oracle.explore(small))
    g.close()


def test_unit_level_engine_paper_shape(mc):
    """The plain level-synchronous engine on the abstract kernel at S = 256."""
    model = workloads.abstract_paper(256, 4)
    _say("abstract S=256 m=4 level engine")
    g = mc.Model(model, engine=ENGINES["level"])
    check_min_time(g, model, oracle.explore(model))
    g.close()


def test_unit_simulate_and_bisect(mc):
    model = workloads.minimum_paper(256, 2)
    r = oracle.explore(model, trace=False)
    g = mc.Model(model)
    for seed in (1, 2, 3):
        assert g.mc_simulate(seed) == oracle.simulate(model, seed)
    t_min, _ = g.mc_tune_bisect(5)
    assert t_min == r["t_min"]
    g.close()


def test_unit_batch_mixed_kinds(mc):
    """One batch holding unit models next to reduction and matmul models: the launch
    runs the general-phase engine for all of them."""
    models = (workloads.tiny_unit_models(403, 24, max_cu=8) + workloads.tiny_models(404, 12)
              + [workloads.abstract_paper(256, 2), workloads.minimum_paper(256, 8)])
    _say(f"batch of {len(models)} mixed-kind models")
    b = mc.Batch(models, mc.make_batch_opts(block=256))
    t_min, states = b.mc_batch_min_time()
    for i, m in enumerate(models):
        r = oracle.explore(m, trace=False)
        assert t_min[i] == r["t_min"], (i, workloads.describe(m))
        assert states[i] == r["reachable"], (i, workloads.describe(m))
        assert b.mc_batch_terminal_clocks(i) == r["tc"]
    b.close()


def test_unit_served_queries(mc):
    pool = workloads.tiny_unit_models(405, 8, max_cu=4) + [workloads.minimum_paper(256, 4)]
    e = mc.Engine(arena_bytes=128 << 20, max_active=4, slice=2)
    qs = []
    for i, m in enumerate(pool):
        t_min = cf.summary(m, with_E=False)["t_min"]
        qs += [(i, "min_time", 0), (i, "check", t_min - 1), (i, "check", t_min)]
    tickets = [e.mc_engine_submit(pool[i], mc.MC_QUERY_MIN_TIME if k == "min_time"
                                  else mc.MC_QUERY_CHECK, T) for i, k, T in qs]
    e.drain()
    for (i, kind, T), t in zip(qs, tickets):
        res = e.mc_engine_poll(t)
        assert res["done"] == 1 and res["status"] == 0
        r = oracle.explore(pool[i], T=None if kind == "min_time" else T, trace=False)
        assert res["states"] == r["reachable"], (i, kind, T)
        if kind == "min_time":
            assert (res["t_min"], res["n_argmin"]) == (r["t_min"], len(r["argmin"]))
        else:
            assert res["violated"] == int(r["violated"])
    e.close()


SWARM_KEYS = ("walks", "trails", "steps", "best_walk_start", "first_step", "best_clock",
              "best_cfg", "first_clock", "first_cfg")


def test_unit_swarm_members_equal_oracle(mc):
    model = workloads.unit_model(workloads.KIND_ABSTRACT, 32, 2, 3, [1, 2, 4, 8], [1, 2, 4], 3, 1)
    s = cf.summary(model, with_E=False)
    g = mc.Model(model, log2_slots=22)
    for T in (None, s["t_min"], s["t_min"] - 1):
        _say(f"unit swarm T={T}")
        r = g.mc_swarm(64, 12, 20000, 9, T)
        gpu = g.mc_swarm_members(64)
        ora = oracle.swarm(model, 9, 64, 20000, 12, T)
        for i, (a, b) in enumerate(zip(gpu, ora)):
            assert {k: a[k] for k in SWARM_KEYS} == {k: b[k] for k in SWARM_KEYS}, (T, i)
        if r["trails"]:
            oracle.check_trace(model, g.mc_swarm_trace(), target_clock=r["best_clock"],
                               cfgs=[r["best_cfg"]])
    g.close()


def test_table1_rows_on_the_gpu(mc):
    """Table 1 rows 1-5 (tests/golden/table1_abstract.txt): the printed model time is
    T_min of the printed configuration on one unit of four elements with GMT = 4, now
    computed by the HIP path."""
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "table1_abstract.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    for n, size, t_printed, ts, wg in rows[:5]:
        model = workloads.unit_model(workloads.KIND_ABSTRACT, size, workloads.PAPER_NP, 1,
                                     [wg], [ts], workloads.PAPER_GMT, workloads.PAPER_LOCAL)
        g = mc.Model(model)
        assert g.mc_min_time()[0] == t_printed, (n, size)
        g.close()


@pytest.mark.parametrize("m", [1, 2, 3])
def test_long_rounds_cut_into_round_blocks_and_run_slices(mc, m):
    """Workgroups of 2056 operation ends (8 waves of 257): with small partitions every
    round is a block of its own and its run beyond 64 states goes to run slices (m = 3:
    16 workgroups leave a partial round with 3 choices of units)."""
    model = workloads.unit_model(workloads.KIND_ABSTRACT, 256, 1, m, [8, 4], [2], 3, 1)
    _say(f"long rounds m={m}")
    r = oracle.explore(model)
    for ps in (1, 0):
        g = mc.Model(model, part_states=ps)
        check_min_time(g, model, r)
        for T in (r["t_min"] - 1, r["t_min"], max(r["tc"]) // 2):
            check_threshold(mc, g, model, T, oracle.explore(model, T=T))
        assert g.mc_min_time_bb(0) == (r["t_min"], r["argmin"])
        g.close()
