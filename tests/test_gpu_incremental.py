"""Incremental bisection on the GPU: the checks of mc_tune_bisect share one visited set
(checks below the largest threshold explored so far are answered from the least clocks,
checks above it continue that exploration).  Its T_min and number of checks equal the
oracle's bisection, its trace replays, and it explores exactly the states with clock up
to the largest threshold it checked (each once)."""
import sys

import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available()
    import paper_2305_09130_amd as mc
    return mc


def _thresholds(t_ini, t_min):
    """The thresholds the bisection checks (violated exactly when T >= T_min) and how
    many of them the loop makes (the last one may be a closing check of hi that leaves
    the counterexample behind)."""
    lo, hi, out = 0, t_ini, []
    while hi - lo > 1:
        mid = (lo + hi) // 2
        out.append(mid)
        if mid >= t_min:
            hi = mid
        else:
            lo = mid
    n = len(out)
    if not out or out[-1] < t_min:
        out.append(hi)
    return out, n


def _models():
    return ([workloads.reduction_g256(), workloads.matmul_64()]
            + workloads.tiny_models(71, 24, max_cu=6)
            + workloads.tiny_unit_models(72, 12))


@pytest.mark.parametrize("k", range(38))
def test_incremental_bisection(mc, k):
    models = _models()
    if k >= len(models):
        pytest.skip("fewer models")
    model = models[k]
    _say(f"incremental bisection on {workloads.describe(model)}")
    r = oracle.explore(model, trace=False)
    g = mc.Model(model)
    for seed in (3, 11):
        t_min, n = g.mc_tune_bisect(seed)
        t_ini, _ = oracle.simulate(model, seed)
        checks, n_loop = _thresholds(t_ini, r["t_min"])
        assert (t_min, n) == (r["t_min"], n_loop)
        if r["reachable"] < 200_000:
            assert (t_min, n) == oracle.bisect_t_min(model, t_ini)
        top = max(checks)
        assert g.last_stats["states"] == oracle.explore(model, T=top, trace=False)["reachable"]
        oracle.check_trace(model, g.mc_trace(), max_clock=t_min)
    # a fresh query after the bisection starts over on a cleared set
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    g.close()


def _hetero_models():
    return ([workloads.with_speeds(workloads.reduction_model(64, 3, [1, 2, 4], [1, 2], 6, 2),
                                   [1, 2, 3])]
            + list(workloads.hetero_workloads().values())
            + workloads.tiny_hetero_models(73, 16, max_cu=4, max_speed=3))


@pytest.mark.parametrize("k", range(19))
def test_unequal_units_bisect_incremental(mc, k):
    """Units of unequal speed continue a check from the cuts of their chain slices (or
    from SELECT): the bisection equals the oracle's and explores each state up to the
    largest threshold it checked once, also with every configuration uncut."""
    models = _hetero_models()
    if k >= len(models):
        pytest.skip("fewer models")
    model = models[k]
    _say(f"incremental bisection, unequal units: {workloads.describe(model)}")
    r = oracle.explore(model, trace=False)
    for part_states in (0, 32, mc.NEVER_CUT):
        g = mc.Model(model, part_states=part_states)
        for seed in (5, 11):
            t_min, n = g.mc_tune_bisect(seed)
            t_ini, _ = oracle.simulate(model, seed)
            checks, n_loop = _thresholds(t_ini, r["t_min"])
            assert (t_min, n) == (r["t_min"], n_loop)
            if r["reachable"] < 200_000:
                assert (t_min, n) == oracle.bisect_t_min(model, t_ini)
            top = max(checks)
            assert g.last_stats["states"] == oracle.explore(model, T=top,
                                                            trace=False)["reachable"]
            oracle.check_trace(model, g.mc_trace(), max_clock=t_min)
        assert g.mc_min_time() == (r["t_min"], r["argmin"])
        assert g.last_stats["states"] == r["reachable"]
        g.close()
