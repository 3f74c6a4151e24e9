"""GPU parity of the swarm search (Sec. 5) against the oracle's swarm.

Every member of a swarm is deterministic given its seed (its bit array is its own), so
the GPU members must equal the oracle's member by member: walks, trails, steps, the
clock, configuration and walk start of the best trail, the step and trail of the first.
The best trail is replayed through the oracle's successor function, and the swarm
search (mc_swarm_tune) must run the same rounds as the oracle's swarms with the same
seeds."""
import sys

import pytest

import oracle
import workloads
from oracle import closed_form as cf

pytestmark = pytest.mark.gpu
KEYS = ("walks", "trails", "steps", "best_walk_start", "first_step", "best_clock", "best_cfg",
        "first_clock", "first_cfg")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available()
    import paper_2305_09130_amd as mc
    return mc


CASES = [
    ("reduction_g256", workloads.reduction_g256),
    ("reduction_m3", lambda: workloads.reduction_model(64, 3, [1, 2, 4], [1, 2], 4, 3)),
    ("matmul8_lb1", lambda: workloads.matmul_model(8, 8, 8, 4, [1, 2], [1, 2], [1, 2], [1], 3, 2, Lb=1)),
    ("matmul16_m8", lambda: workloads.matmul_model(16, 16, 8, 8, [1, 2], [1], [1, 2], [1, 2], 2, 1)),
]


def _members_equal(gpu, ora, ctx):
    for i, (g, o) in enumerate(zip(gpu, ora)):
        assert {k: g[k] for k in KEYS} == {k: o[k] for k in KEYS}, (ctx, i, g, o)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("bits_log2", [10, 20])
def test_swarm_members_equal_oracle(mc, case, bits_log2):
    name, make = CASES[case]
    model = make()
    s = cf.summary(model, with_E=False)
    g = mc.Model(model, log2_slots=22)   # room for the members' bit arrays
    for T in (None, s["t_min"], s["t_min"] - 1, (s["t_min"] + max(s["tc"])) // 2):
        _say(f"swarm {name} bits 2^{bits_log2} T={T}")
        members, budget, seed = 96, 20000, 17
        r = g.mc_swarm(members, bits_log2, budget, seed, T)
        gpu = g.mc_swarm_members(members)
        ora = oracle.swarm(model, seed, members, budget, bits_log2, T)
        _members_equal(gpu, ora, (name, T))
        assert r["trails"] == sum(o["trails"] for o in ora)
        assert r["steps"] == sum(o["steps"] for o in ora)
        best = min((o["best_clock"] for o in ora if o["trails"]), default=oracle.NONE)
        assert r["best_clock"] == best
        if r["trails"]:
            tr = g.mc_swarm_trace()
            oracle.check_trace(model, tr, target_clock=r["best_clock"], cfgs=[r["best_cfg"]])
        else:
            with pytest.raises(mc.McError):
                g.mc_swarm_trace()
    g.close()


def _tune_oracle(model, members, bits_log2, budget, seed):
    rounds, T = 1, None
    ora = oracle.swarm(model, seed, members, budget, bits_log2)
    best = min(o["best_clock"] for o in ora if o["trails"])
    while best > 0:
        ora = oracle.swarm(model, seed + rounds, members, budget, bits_log2, best - 1)
        rounds += 1
        if not any(o["trails"] for o in ora):
            break
        best = min(o["best_clock"] for o in ora if o["trails"])
    return best, rounds


@pytest.mark.parametrize("case", range(len(CASES)))
def test_swarm_tune_matches_oracle_rounds(mc, case):
    name, make = CASES[case]
    model = make()
    s = cf.summary(model, with_E=False)
    g = mc.Model(model, log2_slots=22)
    _say(f"swarm tune {name}")
    t, rounds, r = g.mc_swarm_tune(64, 16, 5000, 3)
    assert (t, rounds) == _tune_oracle(model, 64, 16, 5000, 3)
    assert t >= s["t_min"] and t in s["tc"]
    tr = g.mc_swarm_trace()
    oracle.check_trace(model, tr, target_clock=t)
    g.close()


def test_swarm_matmul64_sample(mc):
    """The 5.15M-state workload: a sample of members against the oracle, the swarm
    search's time against the exact T_min."""
    model = workloads.matmul_64()
    s = cf.summary(model, with_E=False)
    g = mc.Model(model)
    _say("swarm matmul64")
    g.mc_swarm(48, 16, 30000, 5)
    _members_equal(g.mc_swarm_members(48), oracle.swarm(model, 5, 48, 30000, 16), "matmul64")
    t, rounds, r = g.mc_swarm_tune(4096, 16, 20000, 1)
    assert t >= s["t_min"] and t in s["tc"]
    g.close()


def test_swarm_memory_bound(mc):
    g = mc.Model(workloads.reduction_g256())
    with pytest.raises(mc.McError) as e:
        g.mc_swarm(1 << 16, 30, 10, 1)
    assert e.value.code == mc.MC_E_NOMEM
    g.close()
