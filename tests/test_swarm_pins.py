"""Pins of the oracle's swarm search (Sec. 5), against facts other than its own code.

* A member's first walk starts with empty bits at member step 0 with the member's seed,
  so (with bit arrays large enough for no collision) it is the seeded simulation run
  of the oracle: same terminal clock and configuration.
* Every trail is a terminal, so its clock is the closed-form clock of its
  configuration; under a threshold T no trail exceeds T, and none exists below T_min.
* A model with a single run (one configuration, one unit) has a single terminal: the
  first walk is a trail, every later walk meets the visited terminal.
* A member counts at most one trail per terminal state, i.e. per configuration.
* The budget: a member stops starting walks at the first walk start at or past it.
"""
import pytest

import oracle
import workloads
from oracle import closed_form as cf

M64 = (1 << 64) - 1


def _splitmix64(z):
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


MODELS = [workloads.reduction_g256(), workloads.reduction_model(64, 3, [1, 2, 4], [1, 2], 4, 3),
          workloads.matmul_model(8, 8, 8, 4, [1, 2], [1, 2], [1, 2], [1], 3, 2, Lb=1)]


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_first_walk_is_the_seeded_simulation(k):
    model = MODELS[k]
    members = oracle.swarm(model, 11, 16, 1, 26)   # budget 1: exactly one walk each
    for i, r in enumerate(members):
        assert r["walks"] == 1
        t, c = oracle.simulate(model, _splitmix64(11 + i))
        assert r["trails"] == 1 and (r["first_clock"], r["first_cfg"]) == (t, c)
        assert (r["best_clock"], r["best_cfg"]) == (t, c) and r["best_walk_start"] == 0


@pytest.mark.parametrize("k", range(len(MODELS)))
@pytest.mark.parametrize("T", [None, "tmin", "tmin-1", "mid"])
def test_trail_clocks_are_terminal_clocks(k, T):
    model = MODELS[k]
    s = cf.summary(model, with_E=False)
    thr = {None: None, "tmin": s["t_min"], "tmin-1": s["t_min"] - 1,
           "mid": (s["t_min"] + max(s["tc"])) // 2}[T]
    members = oracle.swarm(model, 5, 12, 30000, 12, thr)
    for r in members:
        assert r["trails"] <= len(model["params"])
        if r["trails"] == 0:
            assert r["best_clock"] == oracle.NONE and r["first_step"] == M64
            continue
        for clock, cfg in ((r["best_clock"], r["best_cfg"]), (r["first_clock"], r["first_cfg"])):
            assert clock == s["tc"][cfg]
            assert clock >= s["t_min"]
            if thr is not None:
                assert clock <= thr
        assert r["best_clock"] <= r["first_clock"]
        assert r["best_walk_start"] < r["steps"] and r["first_step"] <= r["steps"]
    if thr is not None and thr < s["t_min"]:
        assert all(r["trails"] == 0 for r in members)


def test_single_run_model_gives_one_trail():
    model = workloads.reduction_model(16, 1, [2], [2], 5, 2)
    s = cf.summary(model)
    path = s["trace_len"] - 1   # transitions of the only run
    for budget in (1, path, path + 1, 10 * path):
        for r in oracle.swarm(model, 3, 4, budget, 10):
            assert r["trails"] == 1 and r["best_clock"] == s["t_min"]
            assert r["walks"] == -(-budget // path) and r["steps"] == r["walks"] * path


def test_budget_semantics():
    model = MODELS[0]
    depth = cf.summary(model, with_E=False)["levels"]
    for budget in (1, 500, 5000):
        for r in oracle.swarm(model, 9, 6, budget, 14):
            assert r["steps"] >= budget
            assert r["steps"] < budget + depth   # only the walk in progress overshoots


def test_deterministic():
    a = oracle.swarm(MODELS[1], 21, 10, 2000, 11, 700)
    b = oracle.swarm(MODELS[1], 21, 10, 2000, 11, 700)
    assert a == b
