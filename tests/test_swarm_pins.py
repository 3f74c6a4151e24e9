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


# --- the bitstate, member by member, against an independent walk ------------------------
#
# A second implementation of the swarm member (the reading of Sec. 5 written down for the
# explorer: member i walks from the root with seed splitmix64(base + i); its step t picks
# successor splitmix64(seed ^ splitmix64(t)) mod k in the order configuration, then unit;
# at a state with other than one successor the state's hash h, a splitmix64 chain over
# (cfg, clock, pending, rem_0..rem_{m-1}), names the two bits h mod B and (h >> 32) mod B;
# both set ends the walk, else both are set).  Its successor function is built from the
# transition system's definition and brute's one-tick operation lists, not from the
# oracle.  With B = 2^6 bits the arrays fill within a few walks, so walks end on
# collisions and every member's counters depend on both bit positions.

def _succ_fn(model):
    from oracle import brute
    m = model["m"]
    progs = []
    for row in model["params"]:
        n, prog = brute.workgroup_program(model, row)
        E, t = [], 0
        for lat in prog:
            t += lat
            if lat:
                E.append(t)
        progs.append((n, E))

    def succ(x):
        if x[0] == oracle.ROOT:
            return [(c, 0, progs[c][0]) + (0,) * m for c in range(len(progs))]
        c, clock, pending, rem = x[0], x[1], x[2], list(x[3:])
        n, E = progs[c]
        d = E[-1]
        free = [i for i in range(m) if rem[i] == 0]
        if pending and free:
            out = []
            for i in free:
                r = list(rem)
                r[i] = d
                out.append((c, clock, pending - 1) + tuple(r))
            return out
        busy = [i for i in range(m) if rem[i]]
        if not busy:
            return []
        delta = min(min(e for e in E if e > d - rem[i]) - (d - rem[i]) for i in busy)
        return [(c, clock + delta, pending) + tuple(r - delta if r else 0 for r in rem)]
    return succ


def _state_hash(x):
    h = 0
    for j, v in enumerate(x):
        h = _splitmix64(v if j == 0 else h ^ v)
    return h


def _members(model, base, members, budget, bits_log2, T=None):
    succ = _succ_fn(model)
    B = 1 << bits_log2
    out = []
    collisions = 0
    for i in range(members):
        seed = _splitmix64(base + i)
        bits = set()
        r = {"walks": 0, "trails": 0, "best_clock": oracle.NONE, "best_cfg": oracle.NONE,
             "first_clock": oracle.NONE, "first_cfg": oracle.NONE, "first_step": M64,
             "best_walk_start": 0}
        t = 0
        while t < budget:
            r["walks"] += 1
            start = t
            nxt = succ((oracle.ROOT, 0, 0) + (0,) * model["m"])
            while True:
                x = nxt[_splitmix64(seed ^ _splitmix64(t)) % len(nxt)]
                t += 1
                if T is not None and x[1] > T:
                    break
                nxt = succ(x)
                if len(nxt) != 1:
                    h = _state_hash(x)
                    p0, p1 = h % B, (h >> 32) % B
                    if p0 in bits and p1 in bits:
                        collisions += 1
                        break
                    bits.update((p0, p1))
                if not nxt:
                    r["trails"] += 1
                    if r["first_step"] == M64:
                        r["first_step"], r["first_clock"], r["first_cfg"] = t, x[1], x[0]
                    if r["best_clock"] == oracle.NONE or x[1] < r["best_clock"]:
                        r["best_clock"], r["best_cfg"], r["best_walk_start"] = x[1], x[0], start
                    break
        r["steps"] = t
        out.append(r)
    return out, collisions


SMALL = [workloads.reduction_model(16, 2, [1, 2, 4], [1, 2], 5, 2),
         workloads.matmul_model(4, 4, 4, 3, [1, 2], [1, 2], [1, 2], [1], 3, 2, Lb=1),
         workloads.unit_model(workloads.KIND_MINIMUM, 16, 2, 2, [2, 4, 8], [1, 2], 3, 1)]


@pytest.mark.parametrize("k", range(len(SMALL)))
@pytest.mark.parametrize("T", [None, "tmin"])
def test_members_equal_an_independent_walk_with_64_bits(k, T):
    model = SMALL[k]
    thr = None if T is None else cf.summary(model, with_E=False)["t_min"]
    ref, collisions = _members(model, 41, 6, 400, 6, thr)
    assert collisions >= 6, "the 64-bit arrays must fill and end walks"
    got = oracle.swarm(model, 41, 6, 400, 6, thr)
    keys = ("walks", "trails", "steps", "best_clock", "best_cfg", "first_clock", "first_cfg",
            "first_step", "best_walk_start")
    assert [{q: g[q] for q in keys} for g in got] == [{q: r[q] for q in keys} for r in ref]


def test_hand_worked_collision():
    """The worked case of tests/golden/swarm_bits64.txt: member 0 of a one-unit model
    whose only branching state is the root's child.  Its state hash lands on bits
    (p0, p1) of the 64; the first walk sets both and ends in a trail, the second walk
    finds both set at that state and ends there, without a trail."""
    model = workloads.reduction_model(4, 1, [2], [1, 2], 3, 1)
    rows = {}
    for line in open(__import__("os").path.join(__import__("os").path.dirname(__file__),
                                                "golden", "swarm_bits64.txt")):
        if line.strip() and not line.startswith("#"):
            key, *vals = line.split()
            rows[key] = [int(v) for v in vals]
    x = tuple(rows["state"])
    h = _state_hash(x)
    assert [h % 64, (h >> 32) % 64] == rows["bits"]
    ref, _ = _members(model, 0, 1, rows["budget"][0], 6)
    got = oracle.swarm(model, 0, 1, rows["budget"][0], 6)[0]
    for q, v in zip(("walks", "trails", "steps"), rows["member0"]):
        assert got[q] == v == ref[0][q], q


# --- planted mistakes in the bitstate of a copy of the oracle ----------------------------

SWARM_MUTANTS = {
    # one bit per state instead of two
    "one_bit": ("if (b0 && b1) break;", "if (b0) break;"),
    # the second bit from the wrong half of the hash
    "second_bit_shift": ("p1 = (h >> 32) & (B - 1);", "p1 = (h >> 31) & (B - 1);"),
    # the bitstate consulted inside lock-step runs too (states with one successor)
    "hash_every_state": ("                if (k != 1) {", "                if (1) {"),
}


def _swarm_pins_pass() -> bool:
    keys = ("walks", "trails", "steps", "best_clock", "best_cfg", "first_step")
    for model in SMALL:
        ref, _ = _members(model, 41, 6, 400, 6)
        got = oracle.swarm(model, 41, 6, 400, 6)
        if [{q: g[q] for q in keys} for g in got] != [{q: r[q] for q in keys} for r in ref]:
            return False
    return True


@pytest.mark.parametrize("name", sorted(SWARM_MUTANTS))
def test_swarm_mutants(name):
    import os
    import shutil
    import subprocess
    import tempfile
    tmp = tempfile.mkdtemp(prefix="mcsmut")
    try:
        src = open(os.path.join(os.path.dirname(oracle.__file__), "mc_oracle.c")).read()
        old, new = SWARM_MUTANTS[name]
        assert src.count(old) == 1, name
        path = os.path.join(tmp, f"mut_{name}.c")
        open(path, "w").write(src.replace(old, new))
        so = os.path.join(tmp, f"libmut_{name}.so")
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-shared", "-fPIC", "-w", "-o", so, path])
        saved_path, saved_lib = oracle.LIB_PATH, oracle._lib
        try:
            oracle.LIB_PATH, oracle._lib = so, None
            assert not _swarm_pins_pass(), f"mutant {name} survived the pins"
        finally:
            oracle.LIB_PATH, oracle._lib = saved_path, saved_lib
        assert _swarm_pins_pass()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
