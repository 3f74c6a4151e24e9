"""Pins of the CPU oracle against what the method and mathematics fix (CPU only).

The oracle (oracle/mc_oracle.c) is trusted only after it matches:
  * hand-worked derivations and a hand-enumerated tiny model (tests/golden/);
  * closed forms of the lock-step round structure (oracle/closed_form.py);
  * brute-force enumeration of every configuration x every dispatch order with a
    one-cycle clock (oracle/brute.py);
  * structural invariants and query laws;
and after planted mistakes in a copy of it are caught by these pins (test_mutants).
"""
import math
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads
from oracle import brute
from oracle import closed_form as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _expand(spec: str) -> list[int]:
    toks = spec.split(",")
    out = []
    i = 0
    while i < len(toks):
        if toks[i] == "...":
            step = out[-1] - out[-2]
            stop = int(toks[i + 1])
            v = out[-1] + step
            while v <= stop:
                out.append(v)
                v += step
            i += 2
            continue
        out.append(int(toks[i]))
        i += 1
    return out


def _parse_sizes(kind, s):
    if kind == "reduction":
        return {"G": int(s.split("=")[1])}
    v = int(s.split("=")[-1])
    return {"M": v, "N": v, "K": v}


def _derivation_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "derivation.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        left, right = line.split("|")
        kind, sizes, params, lg, ll, lc, lb = left.split()
        n, b, d, E = right.split()
        model = {"kind": kind, "m": 1, "Lg": int(lg), "Ll": int(ll), "Lc": int(lc),
                 "Lb": int(lb), "params": [[int(x) for x in params.split(",")]]}
        model.update(_parse_sizes(kind, sizes))
        rows.append((model, int(n), int(b), int(d), _expand(E)))
    return rows


@pytest.mark.parametrize("row", _derivation_rows(), ids=lambda r: str(r[0]["params"][0]))
def test_derivation_golden(oracle_lib, row):
    model, n, b, d, E = row
    got = oracle.derive(model, 0)
    assert (got["n"], got["b"], got["d"]) == (n, b, d)
    assert got["E"] == E
    pc = cf.per_config(model)[0]
    assert (pc["n"], pc["b"], pc["d"], pc["E"]) == (n, b, d, E)


def _tiny_golden():
    spec = {"states": set()}
    for line in open(os.path.join(GOLDEN, "tiny_reduction_g4.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        key, *rest = line.split()
        if key == "model":
            kv = dict(x.split("=") for x in rest[1:])
            spec["model"] = {"kind": rest[0], "m": int(kv["m"]), "G": int(kv["G"]),
                             "Lg": int(kv["Lg"]), "Ll": int(kv["Ll"]), "Lc": int(kv["Lc"]),
                             "Lb": int(kv["Lb"]),
                             "params": [[int(a), int(b), 0, 0] for a, b in
                                        (p.split(",") for p in kv["params"].split(";"))]}
        elif key == "state":
            spec["states"].add(tuple(int(v) for v in rest))
        elif key in ("count_le", "violated"):
            spec.setdefault(key, {})[int(rest[0])] = int(rest[1])
        else:
            spec[key] = [int(v) for v in rest]
    return spec


def test_tiny_model_by_hand(oracle_lib):
    g = _tiny_golden()
    model = g["model"]
    r = oracle.explore(model, self_check=True)
    assert r["reachable"] == g["reachable"][0] == len(g["states"])
    assert r["levels"] == g["levels"][0]
    assert r["tc"] == g["tc"]
    assert r["t_min"] == g["t_min"][0]
    assert r["argmin"] == g["argmin"]
    assert oracle.reach(model) == g["states"]
    for T, cnt in g["count_le"].items():
        assert oracle.explore(model, T=T)["reachable"] == cnt
    for T, v in g["violated"].items():
        assert oracle.explore(model, T=T)["violated"] == bool(v)
    assert r["self_check"] == 0


def _workload_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "workloads.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        name, lg, ll, t_min, argmin, reach = line.split()
        rows.append((name, int(lg), int(ll), int(t_min), [int(a) for a in argmin.split(",")],
                     int(reach)))
    return rows


@pytest.mark.parametrize("row", _workload_rows(), ids=lambda r: r[0])
def test_workload_golden(oracle_lib, row):
    name, lg, ll, t_min, argmin, reach = row
    model = workloads.WORKLOADS[name]()
    assert (model["Lg"], model["Ll"]) == (lg, ll)
    s = cf.summary(model)
    assert (s["t_min"], s["argmin"], s["reachable"]) == (t_min, argmin, reach)
    if s["reachable"] < 200_000:
        r = oracle.explore(model, self_check=True)
        assert (r["t_min"], r["argmin"], r["reachable"]) == (t_min, argmin, reach)
        assert r["self_check"] == 0


@pytest.mark.slow
def test_matmul64_full_oracle_vs_closed_form(oracle_lib):
    model = workloads.matmul_64()
    r = oracle.explore(model)
    s = cf.summary(model)
    assert r["reachable"] == s["reachable"] == 5151061
    assert r["levels"] == s["levels"] == 331778
    assert r["tc"] == s["tc"]
    assert r["argmin"] == s["argmin"] == [96, 97, 98, 99]
    assert len(r["trace"]) == s["trace_len"]
    oracle.check_trace(model, r["trace"], target_clock=s["t_min"], cfgs=s["argmin"])


def _tiny_sweep():
    return workloads.tiny_models(11, 200)


def test_closed_form_tiny_sweep(oracle_lib):
    for model in _tiny_sweep():
        r = oracle.explore(model)
        s = cf.summary(model)
        assert r["reachable"] == s["reachable"], workloads.describe(model)
        assert r["levels"] == s["levels"], workloads.describe(model)
        assert r["tc"] == s["tc"], workloads.describe(model)
        assert r["argmin"] == s["argmin"]
        assert r["trace"] is not None and len(r["trace"]) == s["trace_len"]
        if model["m"] == 1:
            assert r["reachable"] == cf.single_cu_count(model)


def _paths_estimate(model):
    m = model["m"]
    tot = 0
    for c in cf.per_config(model):
        full = math.factorial(m) ** c["q"]
        part = math.perm(m, c["p"]) if c["p"] else 1
        tot += full * part
    return tot


def _brute_cases():
    out = []
    for seed in (3, 5, 7, 9):
        for model in workloads.tiny_models(seed, 40):
            if _paths_estimate(model) <= 3000:
                out.append(model)
    return out


def test_brute_force_tiny(oracle_lib):
    cases = _brute_cases()
    assert len(cases) >= 60
    seen_partial = False
    for model in cases:
        b = brute.summary(model)
        r = oracle.explore(model)
        d = workloads.describe(model)
        assert oracle.reach(model) == b["states"], d
        assert r["tc"] == b["tc"], d
        assert r["argmin"] == b["argmin"], d
        assert r["levels"] == b["levels"], d
        # every run of one configuration ends at the same clock and has the same length
        for c, clocks in b["terminal_clocks"].items():
            assert len(set(clocks)) == 1, d
            assert len(b["lengths"][c]) == 1, d
        seen_partial |= any(pc["p"] for pc in cf.per_config(model))
    assert seen_partial


def test_invariants(oracle_lib):
    for model in _tiny_sweep()[:80] + [workloads.reduction_g256()]:
        r = oracle.explore(model, self_check=True)
        assert r["self_check"] == 0, (workloads.describe(model), r["self_check"])


def test_counts_do_not_depend_on_latencies(oracle_lib):
    base = workloads.reduction_g256()
    counts = set()
    for lg, ll in ((20, 2), (40, 4), (20, 4), (40, 2), (37, 3)):
        m = dict(base, Lg=lg, Ll=ll)
        counts.add(oracle.explore(m, trace=False)["reachable"])
    assert counts == {81175}


def test_tick_clock_same_optimum(oracle_lib):
    """Ticking the clock one cycle per step (the paper's clock process) gives the same
    least terminal times as jumping to the next operation end."""
    for model in _tiny_sweep()[:60]:
        a = oracle.explore(model, trace=False)
        b = oracle.explore(model, trace=False, tick=True)
        assert a["tc"] == b["tc"]
        assert b["reachable"] >= a["reachable"]


def test_query_laws(oracle_lib):
    for model in _tiny_sweep()[:60] + [workloads.reduction_g256()]:
        r = oracle.explore(model, trace=False)
        t_min = r["t_min"]
        clocks = sorted({c for c in (t_min - 1, t_min, t_min + 1, 0, 1, t_min // 2)
                         if c >= 0})
        prev = -1
        for T in clocks:
            q = oracle.explore(model, T=T)
            assert q["reachable"] == cf.count_le(model, T), (workloads.describe(model), T)
            assert q["reachable"] >= prev
            prev = q["reachable"]
            assert q["violated"] == (T >= t_min)
            if q["violated"]:
                oracle.check_trace(model, q["trace"], max_clock=T)
        full = oracle.explore(model, T=2 ** 31)
        assert full["reachable"] == r["reachable"]


def test_bisection_equals_min_time(oracle_lib):
    for model in _tiny_sweep()[:30] + [workloads.reduction_g256()]:
        r = oracle.explore(model, trace=False)
        t_ini, c = oracle.simulate(model, 12345)
        assert t_ini == r["tc"][c]
        t_min, n = oracle.bisect_t_min(model, t_ini)
        assert t_min == r["t_min"]
        assert n <= max(1, t_ini).bit_length() + 1


def test_trace_laws(oracle_lib):
    for model in _tiny_sweep()[:60] + [workloads.reduction_g256()]:
        r = oracle.explore(model)
        s = cf.summary(model)
        assert r["trace_cfg"] == min(s["argmin"])
        assert len(r["trace"]) == s["trace_len"]
        oracle.check_trace(model, r["trace"], target_clock=s["t_min"], cfgs=s["argmin"])


# --- planted mistakes in a copy of the oracle must be caught by the pins -------------

MUTANTS = {
    # only the first free unit may take a workgroup (drops dispatch interleavings)
    "one_dispatch_order": ("if (rem[i] != 0) continue;", "if (rem[i] != 0 || k) continue;"),
    # pruning keeps clock == T out (off by one in the threshold)
    "prune_off_by_one": ("if (prune && y[1] > T) continue;", "if (prune && y[1] >= T) continue;"),
    # the advance jumps straight to the end of the workgroup
    "advance_to_end": ("uint32_t di = next_end(cf, s, e) - e;", "uint32_t di = s * cf->d - e;"),
    # workgroup count uses the tile size too
    "wrong_workgroups": ("n = mo->G / WG;", "n = mo->G / (WG * TS) ? mo->G / (WG * TS) : 1;"),
    # zero-latency operations are counted as end times
    "zero_latency_entries": ("if (lat[j]) out->E[k++] = (uint32_t)t;", "out->E[k++] = (uint32_t)t;"),
    # a state with work still pending but every unit idle counts as terminal
    "terminal_ignores_pending": ("if (x[0] == OR_ROOT || x[2] != 0) return 0;",
                                 "if (x[0] == OR_ROOT) return 0;"),
}


def _build_mutant(tmp, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "mc_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    src = src.replace(old, new)
    if name == "zero_latency_entries":
        src = src.replace("for (int j = 0; j < 4; j++) if (lat[j]) b += cnt[j];",
                          "for (int j = 0; j < 4; j++) b += cnt[j];")
    path = os.path.join(tmp, f"mut_{name}.c")
    open(path, "w").write(src)
    so = os.path.join(tmp, f"libmut_{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-shared",
                           "-fPIC", "-w", "-o", so, path])
    return so


def _pins_pass() -> bool:
    """The cheap pins: closed form on a small sweep, the golden tiny model, count_T."""
    try:
        for model, n, b, d, E in _derivation_rows():
            got = oracle.derive(model, 0)
            if (got["n"], got["b"], got["d"], got["E"]) != (n, b, d, E):
                return False
        g = _tiny_golden()
        r = oracle.explore(g["model"])
        if (r["reachable"], r["tc"]) != (g["reachable"][0], g["tc"]):
            return False
        for T, cnt in g["count_le"].items():
            if oracle.explore(g["model"], T=T)["reachable"] != cnt:
                return False
        for model in _tiny_sweep()[:40]:
            r = oracle.explore(model, trace=False)
            s = cf.summary(model)
            if (r["reachable"], r["tc"], r["levels"]) != (s["reachable"], s["tc"], s["levels"]):
                return False
    except (oracle.OracleError, AssertionError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants(oracle_lib, name):
    tmp = tempfile.mkdtemp(prefix="mcmut")
    try:
        so = _build_mutant(tmp, name)
        saved_path, saved_lib = oracle.LIB_PATH, oracle._lib
        try:
            oracle.LIB_PATH, oracle._lib = so, None
            assert not _pins_pass(), f"planted mistake {name} went unnoticed"
        finally:
            oracle.LIB_PATH, oracle._lib = saved_path, saved_lib
        assert _pins_pass()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
