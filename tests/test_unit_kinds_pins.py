"""Pins of the oracle's two unit-model kinds (CPU only): the abstract kernel of Sec. 4
(Listings 6 and 8) and the Minimum problem model of Sec. 7 (Listings 10, 14 and 15),
both on units of NP processing elements that run a workgroup of WG > NP items in WG/NP
waves.

What fixes them, other than the oracle itself:
  * Table 1's printed model times (tests/golden/table1_abstract.txt): the per-item
    operation lengths of the abstract pex and the wave count, with GMT = 4;
  * three derivations of the operation lists that share nothing: the oracle's
    start-time bookkeeping, closed_form's formulas and brute's one-tick-at-a-time runs
    (of long_work for the abstract pex; of the Minimum model's unit and elements, with
    their relaunch bookkeeping, for the Minimum kind);
  * brute-force enumeration of every configuration x dispatch order on tiny models;
  * the closed-form round structure on the full paper-shaped workloads;
and planted mistakes in a copy of the oracle must fail one of these.
"""
import os
import shutil
import subprocess
import tempfile
from math import factorial

import pytest

import oracle
import workloads
from oracle import brute
from oracle import closed_form as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "table1_abstract.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        n, size, t, ts, wg = (int(v) for v in line.split())
        rows.append({"N": n, "S": size, "T": t, "TS": ts, "WG": wg})
    assert [r["N"] for r in rows] == list(range(1, 9))
    return rows


def _table1_model(row, gmt=workloads.PAPER_GMT):
    # one device, one unit of four elements; the printed configuration only
    return workloads.unit_model(workloads.KIND_ABSTRACT, row["S"], workloads.PAPER_NP, 1,
                                [row["WG"]], [row["TS"]], gmt, workloads.PAPER_LOCAL)


def test_table1_single_workgroup_rows_exact(oracle_lib):
    """Rows 1-5 (WG*TS > S: one workgroup) come out exactly: model time = T_min of the
    one-configuration model on one unit of four elements."""
    for row in _table1()[:5]:
        r = oracle.explore(_table1_model(row), trace=False)
        assert r["t_min"] == row["T"], row


def test_table1_rows_are_whole_workgroups(oracle_lib):
    """Every printed time, rows 6-8 included, is a whole number of workgroup
    durations of the printed (WG, TS)."""
    quotients = []
    for row in _table1():
        d = oracle.derive(_table1_model(row), 0)["d"]
        assert row["T"] % d == 0, row
        quotients.append(row["T"] // d)
    assert quotients == [1, 1, 1, 1, 1, 33, 65, 33]
    # every row runs 2*floor(S/(WG*NP)) + 1 workgroups of its printed (WG, TS): a count
    # that fits all eight rows but that the printed host and device processes do not
    # give (with one unit they run WGs + 1 workgroups per device activation and
    # activate the device WGs + 1 times), so rows 6-8 pin the workgroup time only
    assert quotients == [2 * (r["S"] // (r["WG"] * workloads.PAPER_NP)) + 1 for r in _table1()]


def test_table1_fixes_gmt(oracle_lib):
    """GMT is not printed; 4 is the only value in 1..64 for which rows 1-5 come out."""
    good = []
    for gmt in range(1, 65):
        if all(oracle.derive(_table1_model(row, gmt), 0)["d"] == row["T"]
               for row in _table1()[:5]):
            good.append(gmt)
    assert good == [4]


def test_wave_closed_form(oracle_lib):
    """One wave of the abstract kernel lasts (S/TS)(GMT*TS + 1) + Ll*TS + 1 + GMT + 1
    when Ll <= GMT, and a workgroup runs max(1, WG/NP) waves."""
    for S in (4, 8, 32, 128):
        for NP in (1, 2, 4, 8):
            for gmt, loc in ((1, 1), (4, 1), (5, 2), (9, 3)):
                params = [[wg, ts, 0, 0] for wg in (1, 2, 4, 8, 16) for ts in (1, 2, 4)
                          if wg <= S and ts <= S]
                model = workloads.unit_model(workloads.KIND_ABSTRACT, S, NP, 2,
                                             [1], [1], gmt, loc)
                model["params"] = params
                for c, (wg, ts, _, _) in enumerate(params):
                    got = oracle.derive(model, c)
                    waves = max(1, wg // NP)
                    assert got["d"] == waves * cf.abstract_wave_time(S, ts, gmt, loc)
                    assert got["n"] == max(1, S // (wg * ts))


def _sweep_models():
    out = []
    for kind in (workloads.KIND_ABSTRACT, workloads.KIND_MINIMUM):
        for S in (4, 8, 16, 32):
            for NP in (1, 2, 4):
                for gmt, loc in ((4, 1), (1, 1), (2, 3), (3, 1), (1, 2)):
                    params = [[wg, ts, 0, 0] for wg in (1, 2, 4, 8) for ts in (1, 2, 4, 8)
                              if wg <= S and ts <= S]
                    out.append(workloads.unit_model(kind, S, NP, 2, [1], [1], gmt, loc))
                    out[-1]["params"] = params
    return out


def _ends(prog):
    t, E = 0, []
    for lat in prog:
        t += lat
        if lat:
            E.append(t)
    return E


def test_three_derivations_agree(oracle_lib):
    """Operation ends from the oracle's start-time bookkeeping, from closed_form's
    formulas and from brute's one-tick clock are the same lists."""
    n_cfg = 0
    for model in _sweep_models():
        for c, row in enumerate(model["params"]):
            o = oracle.derive(model, c)
            n_c, ol = cf.ops(model, row)
            n_b, prog = brute.workgroup_program(model, row)
            assert o["n"] == n_c == n_b
            assert o["E"] == cf.end_times(ol) == _ends(prog), (workloads.describe(model), row)
            assert o["d"] == o["E"][-1] and o["b"] == len(o["E"])
            n_cfg += 1
    assert n_cfg > 1000


def _paths_ok(model, limit=3000):
    est = 0
    for pc in cf.per_config(model):
        # dispatch orders: at most m! per round
        est += factorial(min(model["m"], pc["n"])) ** max(1, pc["rounds"])
    return est <= limit


def test_brute_force_unit_tiny(oracle_lib):
    cases = [m for seed in (11, 12, 13, 14) for m in workloads.tiny_unit_models(seed, 40)
             if _paths_ok(m)]
    assert len(cases) >= 60
    kinds = set()
    for model in cases:
        b = brute.summary(model)
        r = oracle.explore(model)
        d = workloads.describe(model)
        assert oracle.reach(model) == b["states"], d
        assert r["tc"] == b["tc"], d
        assert r["argmin"] == b["argmin"], d
        assert r["levels"] == b["levels"], d
        kinds.add(model["kind"])
    assert kinds == {"abstract", "minimum"}


def test_unit_invariants_and_queries(oracle_lib):
    for model in workloads.tiny_unit_models(21, 60):
        r = oracle.explore(model, self_check=True)
        assert r["self_check"] == 0, workloads.describe(model)
        s = cf.summary(model)
        assert (r["reachable"], r["tc"], r["levels"]) == (s["reachable"], s["tc"], s["levels"])
        t_min = r["t_min"]
        for T in sorted({0, t_min // 2, t_min - 1, t_min, t_min + 1}):
            if T < 0:
                continue
            q = oracle.explore(model, T=T)
            assert q["reachable"] == cf.count_le(model, T)
            assert q["violated"] == (T >= t_min)
            if q["violated"]:
                oracle.check_trace(model, q["trace"], max_clock=T)


def test_tick_clock_same_optimum_unit(oracle_lib):
    for model in workloads.tiny_unit_models(22, 40):
        a = oracle.explore(model, trace=False)
        b = oracle.explore(model, trace=False, tick=True)
        assert a["tc"] == b["tc"]


@pytest.mark.parametrize("name", sorted(workloads.UNIT_WORKLOADS))
def test_unit_workloads_closed_form(oracle_lib, name):
    """The full paper-shaped unit workloads: the oracle's search against the round
    structure's closed forms."""
    model = workloads.UNIT_WORKLOADS[name]()
    r = oracle.explore(model)
    s = cf.summary(model)
    assert r["reachable"] == s["reachable"]
    assert r["tc"] == s["tc"]
    assert r["t_min"] == s["t_min"] and r["argmin"] == s["argmin"]
    assert r["levels"] == s["levels"]
    assert len(r["trace"]) == s["trace_len"]
    oracle.check_trace(model, r["trace"], target_clock=s["t_min"], cfgs=s["argmin"])


def test_np_beyond_wg_changes_nothing(oracle_lib):
    """With NP >= WG every item has its own element: more elements change no time."""
    for kind in (workloads.KIND_ABSTRACT, workloads.KIND_MINIMUM):
        base = workloads.unit_model(kind, 64, 8, 2, [1, 2, 4, 8], [1, 4, 16], 4, 1)
        wide = dict(base, NP=64)
        assert oracle.explore(base, trace=False)["tc"] == oracle.explore(wide, trace=False)["tc"]


# --- planted mistakes in the unit kinds of a copy of the oracle -----------------------

UNIT_MUTANTS = {
    # every global load waits its full GMT*TS + 1 (start time also reset before loads)
    "load_resets_start": ("        uint64_t until = start_time + GMT * TS + 1;     /* global load of tile i */",
                          "        start_time = time;\n        uint64_t until = start_time + GMT * TS + 1;"),
    # long_work returns at start_time + gt*tz (not one tick later)
    "long_work_no_extra_tick": ("        if ((rc = ops_push(o, LOC * TS + 1)) != OR_OK) return rc;\n        time = start_time + LOC * TS + 1;",
                                "        if ((rc = ops_push(o, LOC * TS)) != OR_OK) return rc;\n        time = start_time + LOC * TS;"),
    # the unit's final collection read as one more wave
    "extra_wave": ("    uint64_t waves = WG > NP ? WG / NP : 1;",
                   "    uint64_t waves = WG > NP ? WG / NP + 1 : 1;"),
    # element 0 folds all NWE local minima, its own included
    "reduce_nwe_steps": ("    for (uint64_t i = 1; i < nwe; i++)              /* REDUCE local by element 0 */",
                         "    for (uint64_t i = 0; i < nwe; i++)              /* REDUCE local by element 0 */"),
    # the map costs one access per item, not TS
    "map_one_access": ("        for (uint64_t i = 0; i < TS; i++)",
                       "        for (uint64_t i = 0; i < 1; i++)"),
    # element 0 folds the minima of all WG items, not of the min(WG, NP) elements
    "reduce_wg_steps": ("    uint64_t nwe = WG < NP ? WG : NP;", "    uint64_t nwe = WG;"),
    # the workgroup's minimum is never written to global memory
    "write_dropped": ("    return ops_push(o, mo->Lg);                     /* the minimum to global memory */",
                      "    return OR_OK;"),
    # one MAP per workgroup instead of one per wave
    "map_once_per_workgroup": ("    for (uint64_t w = 0; w < waves; w++)            /* MAP, wave by wave */",
                               "    for (uint64_t w = 0; w < 1; w++)"),
}


def _unit_pins_pass() -> bool:
    try:
        for row in _table1()[:5]:
            if oracle.explore(_table1_model(row), trace=False)["t_min"] != row["T"]:
                return False
        for model in _sweep_models()[::7]:
            for c, row in enumerate(model["params"]):
                n_b, prog = brute.workgroup_program(model, row)
                o = oracle.derive(model, c)
                if (o["n"], o["E"]) != (n_b, _ends(prog)):
                    return False
    except (oracle.OracleError, AssertionError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(UNIT_MUTANTS))
def test_unit_mutants(oracle_lib, name):
    tmp = tempfile.mkdtemp(prefix="mcumut")
    try:
        src = open(os.path.join(os.path.dirname(oracle.__file__), "mc_oracle.c")).read()
        old, new = UNIT_MUTANTS[name]
        assert src.count(old) == 1, name
        path = os.path.join(tmp, f"mut_{name}.c")
        open(path, "w").write(src.replace(old, new))
        so = os.path.join(tmp, f"libmut_{name}.so")
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-shared", "-fPIC", "-w", "-o", so, path])
        saved_path, saved_lib = oracle.LIB_PATH, oracle._lib
        try:
            oracle.LIB_PATH, oracle._lib = so, None
            assert not _unit_pins_pass(), f"mutant {name} survived the pins"
        finally:
            oracle.LIB_PATH, oracle._lib = saved_path, saved_lib
        assert _unit_pins_pass()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
