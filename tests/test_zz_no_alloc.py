"""The allocation-free entry point (mc_min_time_static) against mc_min_time on the same
models: two calls in a row on one device, the second on a smaller model, each result
bit-exact with the allocating entry point's (and with the oracle's)."""
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


def _alloc(mc, model):
    g = mc.Model(model)
    t, a = g.mc_min_time()
    st = dict(g.last_stats)
    g.close()
    return t, a, st


def test_static_matches_allocating_entry_point_twice(mc):
    big = workloads.reduction_model(256, 4, [1, 2, 4, 8, 16], [1, 2, 4], 23, 3, Lb=1)
    small = workloads.reduction_g256()
    for model in (big, small):
        _say(f"static min_time on {workloads.describe(model)}")
        t, a, st = mc.mc_min_time_static(model)
        t0, a0, st0 = _alloc(mc, model)
        ref = oracle.explore(model, trace=False)
        assert (t, a) == (t0, a0) == (ref["t_min"], ref["argmin"])
        for k in ("states", "levels", "terminals"):
            assert st[k] == st0[k], k
        assert st["states"] == ref["reachable"]


def test_static_both_engines_and_unequal_units(mc):
    models = [workloads.matmul_model(16, 16, 16, 4, [1, 2, 4], [1, 2], [1, 2], [1, 2], 5, 2),
              workloads.with_speeds(workloads.reduction_model(64, 3, [1, 2, 4], [1, 2], 6, 2),
                                    [1, 2, 3])]
    for model in models:
        for engine in (mc.MC_ENGINE_SUPERSTEP, mc.MC_ENGINE_LEVEL):
            _say(f"static min_time engine {engine} on {workloads.describe(model)}")
            t, a, st = mc.mc_min_time_static(model, mc.make_opts(engine=engine))
            ref = oracle.explore(model, trace=False)
            assert (t, a) == (ref["t_min"], ref["argmin"])
            assert st["states"] == ref["reachable"]


def test_static_rejects_models_beyond_the_scratch(mc):
    model = workloads.matmul_64()   # 5.15M states: a visited set of 256 MiB
    assert mc.mc_workspace_bytes(model) > mc.MC_STATIC_SCRATCH_BYTES
    with pytest.raises(mc.McError) as e:
        mc.mc_min_time_static(model)
    assert e.value.code == mc.MC_E_NOMEM
    # and the scratch still answers afterwards
    small = workloads.reduction_g256()
    t, a, _ = mc.mc_min_time_static(small)
    ref = oracle.explore(small, trace=False)
    assert (t, a) == (ref["t_min"], ref["argmin"])
