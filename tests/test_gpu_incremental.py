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


def test_unequal_units_bisect_fresh_checks(mc):
    """Units of unequal speed have no common state after whole rounds: every check is a
    fresh exploration, and the result is the oracle's."""
    model = workloads.with_speeds(workloads.reduction_model(64, 3, [1, 2, 4], [1, 2], 6, 2),
                                  [1, 2, 3])
    g = mc.Model(model)
    t_min, n = g.mc_tune_bisect(5)
    t_ini, _ = oracle.simulate(model, 5)
    assert (t_min, n) == oracle.bisect_t_min(model, t_ini)
    g.close()
