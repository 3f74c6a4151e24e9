"""One handle, model after model (mc_model_reload), with the visited set's dead bytes
cleared behind the queries on the handle's side stream: every count, clock, verdict and
trace against the oracle, in orders that make a query rely on bytes an earlier one left
cleared (a check, then the larger min_time), reuse a smaller model's table for a larger one
and the other way round, and put a swarm's bit arrays into the table.  The workspace starts
filled with bytes that are no empty slot, so a byte taken for cleared that is not fails a
count."""
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


def _models():
    w = workloads
    return {
        "mm32": w.matmul_model(32, 32, 32, 4, [1, 2, 4, 8], [1, 2, 4, 8], [1, 2, 4], [1], 23, 3),
        "red256": w.reduction_g256(),
        "het": w.with_speeds(w.reduction_model(128, 3, [1, 2, 4], [1, 2], 9, 2), [1, 2, 3]),
        "w4": w.with_speeds(w.reduction_model(64, 8, [1, 2, 4], [1, 2], 37, 3),
                            [1, 2, 3, 4, 5, 6, 7, 8]),
        "mm16_8cu": w.matmul_model(16, 16, 16, 8, [1, 2, 4], [1, 2, 4], [1, 2], [1, 2], 11, 2),
    }


def _workspace(mc, models):
    import torch
    need = max(mc.mc_workspace_bytes(m, mc.make_opts()) for m in models)
    return torch.full((need,), 0xA5, dtype=torch.uint8, device="cuda:0")


def _check_first(mc, g, model, r):
    """check(T_min - 1), check(T_min), then min_time and its trace: the checks leave the
    bytes past their prefix to the side stream, which the min_time then needs cleared."""
    q = oracle.explore(model, T=r["t_min"] - 1, trace=False)
    assert g.mc_check(r["t_min"] - 1) is False
    assert g.last_stats["states"] == q["reachable"]
    assert g.mc_check(r["t_min"]) is True
    assert g.last_stats["states"] == oracle.explore(model, T=r["t_min"], trace=False)["reachable"]
    oracle.check_trace(model, g.mc_trace(), max_clock=r["t_min"])
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    assert g.mc_terminal_clocks() == r["tc"]
    oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])


def _min_time_first(mc, g, model, r):
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
    q = oracle.explore(model, T=r["t_min"] - 1, trace=False)
    assert g.mc_check(r["t_min"] - 1) is False
    assert g.last_stats["states"] == q["reachable"]
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]


@pytest.mark.parametrize("order", ["grow", "shrink", "mixed"])
def test_reload_sequence(mc, order):
    ms = _models()
    names = {"grow": ["w4", "het", "red256", "mm16_8cu", "mm32"],
             "shrink": ["mm32", "mm16_8cu", "red256", "het", "w4"],
             "mixed": ["red256", "mm32", "w4", "mm32", "het", "mm16_8cu", "red256"]}[order]
    ws = _workspace(mc, ms.values())
    g = None
    for i, name in enumerate(names):
        model = ms[name]
        _say(f"{order}[{i}] {name}: {workloads.describe(model)}")
        r = oracle.explore(model)
        if g is None:
            g = mc.Model(model, workspace=ws)
        else:
            g.mc_model_reload(model)
        (_check_first if i % 2 == 0 else _min_time_first)(mc, g, model, r)
    g.close()


def test_reload_keeps_model_when_too_big(mc):
    ms = _models()
    import torch
    small = ms["red256"]
    ws = torch.full((mc.mc_workspace_bytes(small, mc.make_opts()),), 0x5A, dtype=torch.uint8,
                    device="cuda:0")
    g = mc.Model(small, workspace=ws)
    r = oracle.explore(small)
    assert g.mc_check(r["t_min"] - 1) is False
    with pytest.raises(mc.McError) as e:
        g.mc_model_reload(ms["mm32"])
    assert e.value.code == mc.MC_E_NOMEM
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    g.close()


def test_swarm_then_queries(mc):
    """A swarm writes its bit arrays over the visited set; the queries after it, and after a
    reload, clear what they need of them."""
    ms = _models()
    ws = _workspace(mc, ms.values())
    model = ms["mm32"]
    r = oracle.explore(model)
    g = mc.Model(model, workspace=ws)
    q = oracle.explore(model, T=r["t_min"] - 1, trace=False)
    assert g.mc_check(r["t_min"] - 1) is False
    g.mc_swarm(256, 12, 2000, 3, None)
    assert g.mc_check(r["t_min"] - 1) is False
    assert g.last_stats["states"] == q["reachable"]
    g.mc_swarm(256, 12, 2000, 4, None)
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    other = ms["mm16_8cu"]
    g.mc_model_reload(other)
    ro = oracle.explore(other)
    _check_first(mc, g, other, ro)
    g.close()


def test_bench_pattern(mc):
    """The bench's step on one handle: reload the same model, min_time, trace,
    check(T_min - 1), several times over."""
    model = _models()["mm32"]
    r = oracle.explore(model)
    q = oracle.explore(model, T=r["t_min"] - 1, trace=False)
    ws = _workspace(mc, [model])
    g = mc.Model(model, workspace=ws)
    for step in range(4):
        if step:
            g.mc_model_reload(model)
        assert g.mc_min_time() == (r["t_min"], r["argmin"])
        assert g.last_stats["states"] == r["reachable"]
        oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
        assert g.mc_check(r["t_min"] - 1) is False
        assert g.last_stats["states"] == q["reachable"]
    g.close()
