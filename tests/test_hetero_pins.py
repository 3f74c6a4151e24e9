"""Pins of the oracle on units of unequal speed (CPU only).

The paper assumes that every unit works alike (Sec. 4); dropping that, unit i runs every
operation s_i times as long, so the choice of units for the last workgroups changes the
makespan.  The oracle is trusted after it matches:
  * two models enumerated by hand below;
  * brute force (every configuration x dispatch order, one cycle at a time, each unit
    running its operations s_i cycles each) on tiny models;
  * equal speeds s = the homogeneous model with every time multiplied by s;
  * check(T) = the reachable states with clock <= T (clocks never fall along a path);
and planted mistakes in the speed handling of a copy of the oracle fail these.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import workloads
from oracle import brute
from oracle import closed_form as cf


def _minimum(S, WG, TS, m, speeds, NP=1, gmt=1, loc=1):
    base = workloads.unit_model(workloads.KIND_MINIMUM, S, NP, m, [WG], [TS], gmt, loc)
    return workloads.with_speeds(base, speeds)


def test_hand_worked_two_workgroups():
    """Minimum kind, S=8, WG=1, TS=4, NP=1, GMT=1: n = 2 workgroups of 5 accesses of 1
    (4 map + 1 write; no local step), E = 1..5, d = 5.  Units of speed (1, 2).
      root; SELECT (p=2); dispatch closure {u0}, {u1}, {u0,u1}: 3 states;
      both busy from 0: unit 0 ends ops at 1..5, unit 1 at 2,4,..,10, so the clock stops
      at 1,2,3,4,5 (unit 0 done, nothing pending) and then 6,8,10: 8 states;
      13 states, the terminal at 10; the deepest state (the terminal) at depth 11."""
    model = _minimum(8, 1, 4, 2, [1, 2])
    r = oracle.explore(model)
    assert r["reachable"] == 13
    assert r["tc"] == [10] and r["t_min"] == 10
    assert r["levels"] == 12
    homo = oracle.explore(_minimum(8, 1, 4, 2, [1, 1]))
    assert homo["reachable"] == 10 and homo["t_min"] == 5


def test_hand_worked_choice():
    """Same operations, one workgroup (S=4), units of speed (1, 3): the SELECT state has
    one pending workgroup and two idle units, so there are two runs: on unit 0 the clock
    stops at 1..5, on unit 1 at 3,6,..,15.  root + SELECT + 2 dispatch states + 5 + 5 =
    14 states; two terminals (clocks 5 and 15); T_c = 5 (the fast unit)."""
    model = _minimum(4, 1, 4, 2, [1, 3])
    r = oracle.explore(model)
    assert r["reachable"] == 14
    assert r["terminals"] == 2
    assert r["tc"] == [5]
    q = oracle.explore(model, T=14)
    assert q["violated"] and q["reachable"] == 1 + 1 + 2 + 5 + 4


def _brute_cases(max_paths=4000):
    cases = []
    for m in workloads.tiny_hetero_models(41, 60, max_cu=4):
        try:
            cases.append((m, brute.summary(m, max_paths=max_paths)))
        except RuntimeError:  # too many dispatch orders for brute force
            continue
    return cases


_CASES = None


def brute_cases():
    global _CASES
    if _CASES is None:
        _CASES = _brute_cases()
    return _CASES


def test_brute_force_unequal_units(oracle_lib):
    cases = brute_cases()
    assert len(cases) >= 30
    several = 0
    for model, b in cases:
        d = workloads.describe(model)
        r = oracle.explore(model)
        assert oracle.reach(model) == b["states"], d
        assert r["tc"] == b["tc"], d
        assert r["argmin"] == b["argmin"], d
        several += any(len(set(v)) > 1 for v in b["terminal_clocks"].values())
    # the point of unequal units: runs of one configuration end at different clocks
    assert several >= len(cases) // 3


def test_equal_speeds_scale_the_homogeneous_model(oracle_lib):
    for model in workloads.tiny_models(43, 40, max_cu=4) + workloads.tiny_unit_models(44, 20):
        for s in (2, 3):
            scaled = workloads.with_speeds(model, [s] * model["m"])
            a = oracle.explore(model, trace=False)
            b = oracle.explore(scaled, trace=False)
            d = workloads.describe(model)
            assert b["reachable"] == a["reachable"], d
            assert b["levels"] == a["levels"], d
            assert b["tc"] == [s * t for t in a["tc"]], d
            assert b["argmin"] == a["argmin"], d


def test_one_unit(oracle_lib):
    """One unit of speed s runs the n workgroups back to back: T_c = n * s * d."""
    for model in workloads.tiny_models(45, 30, max_cu=1):
        model = dict(model, m=1)
        s = 3
        r = oracle.explore(workloads.with_speeds(model, [s]), trace=False)
        assert r["tc"] == [pc["n"] * s * pc["d"] for pc in cf.per_config(model)]


def test_invariants_and_queries(oracle_lib):
    for model in workloads.tiny_hetero_models(46, 40, max_cu=5):
        d = workloads.describe(model)
        r = oracle.explore(model, self_check=True)
        # the graph need not be graded (tails meet at different depths); the rest holds
        assert r["self_check"] & ~oracle.CHK_GRADED == 0, (d, r["self_check"])
        states = oracle.reach(model)
        t_min = r["t_min"]
        prev = -1
        for T in sorted({0, t_min // 2, t_min - 1, t_min, t_min + 1, max(r["tc"])}):
            if T < 0:
                continue
            q = oracle.explore(model, T=T)
            want = sum(1 for x in states if x[0] == oracle.ROOT or x[1] <= T)
            assert q["reachable"] == want, (d, T)
            assert q["reachable"] >= prev
            prev = q["reachable"]
            assert q["violated"] == (T >= t_min)
            if q["violated"]:
                oracle.check_trace(model, q["trace"], max_clock=T)
        oracle.check_trace(model, r["trace"], target_clock=t_min, cfgs=r["argmin"])


def test_tick_clock_same_optimum(oracle_lib):
    for model in workloads.tiny_hetero_models(47, 25, max_cu=3):
        a = oracle.explore(model, trace=False)
        b = oracle.explore(model, trace=False, tick=True)
        assert a["tc"] == b["tc"], workloads.describe(model)


def test_walk_matches_oracle_successors(oracle_lib):
    """The seeded simulation run on unequal units ends at a terminal clock of its
    configuration."""
    for model in workloads.tiny_hetero_models(48, 20, max_cu=4):
        t, c = oracle.simulate(model, 99)
        clocks = {x[1] for x in oracle.reach(model) if x[0] == c and x[2] == 0
                  and not any(x[3:])}
        assert t in clocks


# --- planted mistakes in the speed handling of a copy of the oracle ------------------

HETERO_MUTANTS = {
    # a dispatched workgroup gets the full-speed duration
    "dispatch_ignores_speed": ("            y[3 + i] = unit_speed(mo, i) * cf->d;",
                               "            y[3 + i] = cf->d + 0 * unit_speed(mo, i);"),
    # the next operation end is taken on the full-speed grid
    "advance_ignores_speed": ("            uint32_t di = next_end(cf, s, e) - e;",
                              "            uint32_t di = (next_end(cf, 1, e % cf->d) - e % cf->d);"),
    # every unit takes the speed of unit 0
    "speed_of_unit0": ("static uint32_t unit_speed(const or_model *mo, uint32_t i) {\n    return mo->speed[i] ? mo->speed[i] : 1u;",
                       "static uint32_t unit_speed(const or_model *mo, uint32_t i) {\n    return mo->speed[0 * i] ? mo->speed[0 * i] : 1u;"),
}


def _hetero_pins_pass() -> bool:
    try:
        test_hand_worked_two_workgroups()
        test_hand_worked_choice()
        for model, b in brute_cases()[:12]:
            r = oracle.explore(model, trace=False)
            if r["tc"] != b["tc"] or r["reachable"] != len(b["states"]):
                return False
    except (oracle.OracleError, AssertionError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(HETERO_MUTANTS))
def test_hetero_mutants(oracle_lib, name):
    tmp = tempfile.mkdtemp(prefix="mchmut")
    try:
        src = open(os.path.join(os.path.dirname(oracle.__file__), "mc_oracle.c")).read()
        old, new = HETERO_MUTANTS[name]
        assert src.count(old) == 1, name
        path = os.path.join(tmp, f"mut_{name}.c")
        open(path, "w").write(src.replace(old, new))
        so = os.path.join(tmp, f"libmut_{name}.so")
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-shared", "-fPIC", "-w", "-o", so, path])
        saved_path, saved_lib = oracle.LIB_PATH, oracle._lib
        try:
            oracle.LIB_PATH, oracle._lib = so, None
            assert not _hetero_pins_pass(), f"mutant {name} survived the pins"
        finally:
            oracle.LIB_PATH, oracle._lib = saved_path, saved_lib
        assert _hetero_pins_pass()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
