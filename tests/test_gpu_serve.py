"""GPU tests of the continuous-batching server.

Every query's result must equal the same query alone and the oracle's answer (closed
forms pinned to the oracle for min_time; verdict and count of states with clock <= T for
check; the whole argmin set, ascending), whatever the admission pressure, slice length,
submission order and reuse of a model's resident state (answered from it, continued
from it, or explored from scratch).  Counterexamples read back from the server replay
through the oracle's successor function.
"""
import random
import sys

import pytest

import oracle
import workloads
from oracle import closed_form as cf

pytestmark = pytest.mark.gpu
BUDGET = 1 << 20


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available()
    import paper_2305_09130_amd as mc
    return mc


def _pool(mc, n=8, seed=4):
    ms, _ = workloads.draw_batch(seed, n, lambda x: (mc.state_count(x) or BUDGET + 1) <= BUDGET)
    return ms


def _queries(pool, n, seed):
    qs = []
    for i, kind, u in workloads.query_mix(seed, n, len(pool)):
        t_min = cf.summary(pool[i], with_E=False)["t_min"]
        qs.append((i, kind, int(u * t_min)))
    return qs


NO_CLOCK = 0xFFFFFFFF


def _expected(pool, q):
    i, kind, T = q
    s = cf.summary(pool[i], with_E=False)
    if kind == "min_time":
        return {"t_min": s["t_min"], "states": s["reachable"], "n_argmin": len(s["argmin"]),
                "argmin_first": s["argmin"][0], "argmin": s["argmin"]}
    hit = T >= s["t_min"]
    return {"violated": int(hit), "states": cf.count_le(pool[i], T),
            "t_min": s["t_min"] if hit else NO_CLOCK, "argmin": s["argmin"] if hit else []}


def _run(mc, pool, qs, order=None, traces=False, **eng):
    e = mc.Engine(**eng)
    order = order if order is not None else list(range(len(qs)))
    tickets = {}
    for k in order:
        i, kind, T = qs[k]
        tickets[k] = e.mc_engine_submit(pool[i], mc.MC_QUERY_MIN_TIME if kind == "min_time"
                                        else mc.MC_QUERY_CHECK, T)
    e.drain()
    out = {}
    for k, t in tickets.items():
        r = e.mc_engine_poll(t)
        assert r is not None and r["done"] == 1 and r["status"] == 0, r
        r["argmin"] = e.mc_engine_argmin(t)
        if traces and r["t_min"] != NO_CLOCK:
            try:   # readable while the model's state is still resident
                r["trace"] = e.mc_engine_trace(t, pool[qs[k][0]]["m"])
            except mc.McError as err:
                assert err.code == mc.MC_E_STATE
        out[k] = r
    if traces:
        assert sum("trace" in r for r in out.values()) >= 3
    e.close()
    return out


def _check(pool, qs, res):
    for k, q in enumerate(qs):
        exp = _expected(pool, q)
        got = {key: res[k][key] for key in exp}
        assert got == exp, (k, q, workloads.describe(pool[q[0]]), got, exp)
        if "trace" in res[k]:
            oracle.check_trace(pool[q[0]], res[k]["trace"], target_clock=res[k]["t_min"],
                               cfgs=exp["argmin"])


@pytest.mark.parametrize("part_states", [0, 0xFFFFFFFF])
def test_serve_results_equal_oracle_under_pressure(mc, part_states):
    """Queries wait for admission, so partitions are cut into 2-level slices that yield
    and resume; with configurations cut into blocks of rounds (automatic) or whole."""
    pool = _pool(mc)
    qs = _queries(pool, 40, seed=1)
    _say(f"40 queries, small arena, slice 2, part_states {part_states:#x}")
    res = _run(mc, pool, qs, arena_bytes=256 << 20, max_active=6, slice=2,
               part_states=part_states)
    _check(pool, qs, res)
    assert max(r["steps"] for r in res.values()) > 1   # partitions really yielded


def test_serve_alone_equals_mix(mc):
    pool = _pool(mc)
    qs = _queries(pool, 24, seed=2)
    _say("mix vs alone")
    mix = _run(mc, pool, qs, traces=True, arena_bytes=1 << 30, max_active=32, slice=8)
    alone = _run(mc, pool, qs, arena_bytes=1 << 30, max_active=1, slice=0)
    fresh = _run(mc, pool, qs, arena_bytes=1 << 30, max_active=32, slice=8, no_reuse=True)
    keys = ("violated", "t_min", "n_argmin", "argmin_first", "states", "argmin")
    for k in range(len(qs)):
        assert {x: mix[k][x] for x in keys} == {x: alone[k][x] for x in keys}, k
        assert {x: mix[k][x] for x in keys} == {x: fresh[k][x] for x in keys}, k
        assert fresh[k]["reuse"] == mc.MC_REUSE_NONE
        # levels are reported whenever the query explored
        if mix[k]["reuse"] != mc.MC_REUSE_ANSWERED and fresh[k]["reuse"] == mc.MC_REUSE_NONE:
            if qs[k][1] == "min_time":
                assert mix[k]["levels"] == fresh[k]["levels"], k
    _check(pool, qs, mix)
    # a pool of 8 models and 24 queries: most queries find their model resident
    assert sum(r["reuse"] != mc.MC_REUSE_NONE for r in mix.values()) >= 8


def test_serve_submission_order_does_not_matter(mc):
    pool = _pool(mc)
    qs = _queries(pool, 20, seed=3)
    a = _run(mc, pool, qs, arena_bytes=512 << 20, max_active=8, slice=2)
    order = list(range(len(qs)))
    random.Random(7).shuffle(order)
    b = _run(mc, pool, qs, order=order, arena_bytes=512 << 20, max_active=8, slice=2)
    for k in range(len(qs)):
        assert (a[k]["states"], a[k]["t_min"], a[k]["violated"]) == \
            (b[k]["states"], b[k]["t_min"], b[k]["violated"])


def test_serve_small_models_against_oracle(mc):
    pool = workloads.tiny_models(77, 10, max_cu=8)
    qs = []
    for i, m in enumerate(pool):
        r = oracle.explore(m, trace=False)
        qs += [(i, "min_time", 0), (i, "check", r["t_min"] - 1), (i, "check", r["t_min"])]
    res = _run(mc, pool, qs, traces=True, arena_bytes=64 << 20, max_active=5, slice=1)
    for k, (i, kind, T) in enumerate(qs):
        r = oracle.explore(pool[i], T=None if kind == "min_time" else T, trace=False)
        assert res[k]["states"] == r["reachable"]
        if kind == "min_time":
            assert (res[k]["t_min"], res[k]["argmin"]) == (r["t_min"], r["argmin"])
            if res[k]["reuse"] != mc.MC_REUSE_ANSWERED or res[k]["levels"]:
                assert res[k]["levels"] == r["levels"]
        else:
            assert res[k]["violated"] == int(r["violated"])
            if r["violated"]:
                full = oracle.explore(pool[i], trace=False)
                assert res[k]["argmin"] == full["argmin"]
        if "trace" in res[k]:
            oracle.check_trace(pool[i], res[k]["trace"], target_clock=res[k]["t_min"],
                               cfgs=res[k]["argmin"])


def test_resident_state_is_reused_exactly(mc):
    """One model through a sequence of queries: check(T1) explores, check(T2 < T1) is
    answered from the resident set (a count scan), check(T3 > T1) continues the
    exploration, min_time continues it to the end, then every query is answered; each
    count is the oracle's count_T and each verdict and argmin set the oracle's."""
    for model in (workloads.reduction_g256(),
                  workloads.matmul_model(16, 16, 16, 4, [1, 2, 4], [1, 2], [1, 2, 4], [1, 2],
                                         5, 2),
                  workloads.unit_model(workloads.KIND_MINIMUM, 64, 4, 3, [2, 4, 8], [1, 4], 4,
                                       1),
                  # units of unequal speed continue from the cuts of their chain slices
                  workloads.with_speeds(workloads.reduction_model(64, 4, [1, 2, 4], [1, 2], 37,
                                                                  3), [1, 2, 3, 4]),
                  workloads.hetero_workloads()["reduction_g256_cu4_s1123"]):
        full = oracle.explore(model, trace=False)
        t = full["t_min"]
        seq = [("check", t // 2), ("check", t // 4), ("check", t - 1), ("check", t),
               ("min_time", 0), ("check", t + 3), ("check", t // 3), ("min_time", 0)]
        want_reuse = [mc.MC_REUSE_NONE, mc.MC_REUSE_ANSWERED, mc.MC_REUSE_RESUMED,
                      mc.MC_REUSE_RESUMED, mc.MC_REUSE_RESUMED, mc.MC_REUSE_ANSWERED,
                      mc.MC_REUSE_ANSWERED, mc.MC_REUSE_ANSWERED]
        _say(f"resident reuse on {workloads.describe(model)}")
        e = mc.Engine(arena_bytes=256 << 20, max_active=4, slice=0)
        for (kind, T), reuse in zip(seq, want_reuse):
            tk = e.mc_engine_submit(model, mc.MC_QUERY_MIN_TIME if kind == "min_time"
                                    else mc.MC_QUERY_CHECK, T)
            e.drain()
            r = e.mc_engine_poll(tk)
            assert r["status"] == 0 and r["reuse"] == reuse, (kind, T, r)
            ref = oracle.explore(model, T=None if kind == "min_time" else T, trace=False)
            assert r["states"] == ref["reachable"], (kind, T)
            if kind == "check":
                assert r["violated"] == int(ref["violated"])
            if kind == "min_time" or ref["violated"]:
                assert e.mc_engine_argmin(tk) == full["argmin"]
                oracle.check_trace(model, e.mc_engine_trace(tk, model["m"]),
                                   target_clock=t, cfgs=full["argmin"])
        e.close()


def test_serve_admission_reject(mc):
    big = workloads.matmul_64()
    e = mc.Engine(arena_bytes=64 << 20, max_active=4)
    t = e.mc_engine_submit(big, mc.MC_QUERY_MIN_TIME)
    r = e.mc_engine_poll(t)
    assert r is not None and r["status"] == mc.MC_E_ADMIT
    e.close()
