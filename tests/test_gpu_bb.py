"""GPU parity of the branch-and-bound min_time (one pruned search instead of the
bisection of Sec. 4 Step 3) against the CPU oracle: T_min and the argmin set bit-exact,
the counterexample replayed through the oracle, and the number of claimed states
between the count of states with clock <= T_min and the count with clock <= T_init
(both from the oracle-pinned round structure).
"""
import sys

import pytest

import oracle
import workloads
from oracle import closed_form as cf

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_09130_amd as mc
    return mc


def check_bb(mc, g, model, s, T_init):
    """s: closed-form summary (T_min, argmin, reachable)."""
    t_min, argmin = g.mc_min_time_bb(T_init)
    st = g.last_stats
    assert (t_min, argmin) == (s["t_min"], s["argmin"]), T_init
    lo = cf.count_le(model, s["t_min"])
    hi = s["reachable"] if T_init == 0 else cf.count_le(model, T_init)
    assert lo <= st["states"] <= hi, (T_init, lo, st["states"], hi)
    tc = g.mc_terminal_clocks()
    for c in argmin:
        assert tc[c] == t_min
    for c, t in enumerate(tc):
        assert t is None or t >= s["tc"][c]     # a found clock is a real terminal clock
    tr = g.mc_trace()
    oracle.check_trace(model, tr, target_clock=t_min, cfgs=argmin)
    return st["states"]


@pytest.mark.parametrize("name", ["reduction_g256_cu2", "matmul64_cu4"])
def test_bb_workloads(mc, name):
    model = workloads.WORKLOADS[name]()
    s = cf.summary(model)
    g = mc.Model(model)
    t_sim, _ = g.mc_simulate(3)
    for T_init in (0, t_sim, s["t_min"], s["t_min"] + 1):
        _say(f"{name} bb T_init={T_init}")
        n = check_bb(mc, g, model, s, T_init)
        _say(f"  claimed {n} of {s['reachable']}")
    with pytest.raises(mc.McError) as e:
        g.mc_min_time_bb(s["t_min"] - 1)
    assert e.value.code == mc.MC_E_STATE
    # the handle still answers the exhaustive query with its own counts
    t_min, argmin = g.mc_min_time()
    assert (t_min, argmin, g.last_stats["states"]) == (s["t_min"], s["argmin"], s["reachable"])
    g.close()


def test_bb_matmul128_full_size(mc):
    model = workloads.matmul_128_vw()
    s = cf.summary(model, with_E=True)
    g = mc.Model(model)
    _say("matmul128_vw_cu8 bb")
    n = check_bb(mc, g, model, s, 0)
    assert n < s["reachable"] // 4
    g.close()


@pytest.mark.parametrize("name", sorted(workloads.UNIT_WORKLOADS))
def test_bb_unit_workloads(mc, name):
    model = workloads.UNIT_WORKLOADS[name]()
    s = cf.summary(model)
    g = mc.Model(model)
    _say(f"{name} bb")
    check_bb(mc, g, model, s, 0)
    check_bb(mc, g, model, s, g.mc_simulate(1)[0])
    g.close()


@pytest.mark.parametrize("engine", [0, 1])
def test_bb_tiny_sweep(mc, engine):
    cases = (workloads.tiny_models(501, 30, max_cu=8) + workloads.tiny_unit_models(502, 20)
             + workloads.tiny_models(503, 10, max_cu=3))
    for i, model in enumerate(cases):
        _say(f"bb tiny[{i}] engine={engine} {workloads.describe(model)}")
        s = cf.summary(model)
        g = mc.Model(model, engine=engine)
        for T_init in (0, max(s["tc"]), s["t_min"]):
            check_bb(mc, g, model, s, T_init)
        g.close()


@pytest.mark.parametrize("part_states", [1, 0xFFFFFFFF])
def test_bb_round_blocks(mc, part_states):
    """Blocks of rounds whose cut state lies beyond the incumbent are skipped or end
    early without tripping the check that a block ends on its predicted state."""
    model = workloads.matmul_64()
    s = cf.summary(model)
    g = mc.Model(model, part_states=part_states)
    _say(f"matmul64 bb part_states={part_states:#x}")
    check_bb(mc, g, model, s, 0)
    g.close()
