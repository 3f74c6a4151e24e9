"""CPU oracle of the explicit-state auto-tuning checker.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.  It shares
no code with the GPU path (it imports nothing from it).

Three independent pieces, each written from the method's definition:
  * ``mc_oracle.c`` (loaded here through ctypes): plain sequential BFS with an exact
    hash set over explicit states -- reachable set, per-configuration least terminal
    clock, T_min and its configurations, the over-time verdict, a counterexample path.
  * ``closed_form``: the same quantities from formulas for the lock-step model kinds.
  * ``brute``: enumeration of every configuration x every dispatch order on tiny
    models, stepping the clock one cycle at a time.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcoracle.so")
ROOT = 0xFFFFFFFF
NONE = 0xFFFFFFFF

CHK_MEASURE, CHK_DEADLOCK, CHK_GRADED, CHK_PERMUTE = 1, 2, 4, 8
KINDS = {"reduction": 0, "matmul": 1, "abstract": 2, "minimum": 3}


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/libmcoracle.so`` with gcc."""
    if force or not os.path.exists(LIB_PATH):
        src = os.path.join(HERE, "mc_oracle.c")
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_uint32),
                ("G", ctypes.c_uint32), ("M", ctypes.c_uint32), ("N", ctypes.c_uint32),
                ("K", ctypes.c_uint32), ("S", ctypes.c_uint32), ("NP", ctypes.c_uint32),
                ("Lg", ctypes.c_uint32), ("Ll", ctypes.c_uint32),
                ("Lc", ctypes.c_uint32), ("Lb", ctypes.c_uint32),
                ("n_cfg", ctypes.c_uint32), ("params", ctypes.POINTER(ctypes.c_uint32)),
                ("tick", ctypes.c_int32), ("speed", ctypes.c_uint32 * 16)]


class _Result(ctypes.Structure):
    _fields_ = [("reachable", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("levels", ctypes.c_uint64), ("terminals", ctypes.c_uint64),
                ("violated", ctypes.c_int32), ("t_min", ctypes.c_uint32),
                ("self_check", ctypes.c_uint32), ("trace_cfg", ctypes.c_uint32),
                ("seconds", ctypes.c_double)]


class _SwarmMember(ctypes.Structure):
    _fields_ = [("walks", ctypes.c_uint64), ("trails", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("best_walk_start", ctypes.c_uint64),
                ("first_step", ctypes.c_uint64), ("best_clock", ctypes.c_uint32),
                ("best_cfg", ctypes.c_uint32), ("first_clock", ctypes.c_uint32),
                ("first_cfg", ctypes.c_uint32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        u32p = P(ctypes.c_uint32)
        lib.or_explore.argtypes = [P(_Model), ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                                   P(_Result), u32p, u32p, ctypes.c_uint64,
                                   P(ctypes.c_uint64), u32p, ctypes.c_uint64]
        lib.or_derive.argtypes = [P(_Model), ctypes.c_uint32, u32p, u32p, u32p, u32p,
                                  ctypes.c_uint64]
        lib.or_successors.argtypes = [P(_Model), u32p, u32p, ctypes.c_uint64]
        lib.or_simulate.argtypes = [P(_Model), ctypes.c_uint64, u32p, u32p]
        lib.or_swarm.argtypes = [P(_Model), ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                 P(_SwarmMember)]
        _lib = lib
    return _lib


def _u32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _model(model: dict, tick: bool = False):
    params = np.ascontiguousarray(np.asarray(model["params"], dtype=np.uint32).reshape(-1, 4))
    kind = KINDS[model["kind"]]
    mo = _Model(kind, model["m"], model.get("G", 0), model.get("M", 0), model.get("N", 0),
                model.get("K", 0), model.get("S", 0), model.get("NP", 0),
                model["Lg"], model["Ll"], model.get("Lc", 1), model.get("Lb", 0),
                params.shape[0], _u32p(params), 1 if tick else 0)
    for i, v in enumerate(model.get("speed") or []):
        mo.speed[i] = int(v)
    return mo, params  # keep params alive


class OracleError(RuntimeError):
    pass


def explore(model: dict, T: int | None = None, self_check: bool = False,
            trace: bool = True, tick: bool = False) -> dict:
    """Explore the model; with ``T`` given, states with clock > T are pruned (check(T)).

    Returns reachable (count_T under pruning), edges, levels, terminals, t_min, argmin,
    tc (per-configuration least terminal clock, None if no terminal), violated,
    self_check flags, seconds (exploration wall time) and the trace (rows of 3+m
    integers, root first) with its configuration.
    """
    lib = _load()
    mo, keep = _model(model, tick)
    res = _Result()
    n = len(model["params"])
    tc = np.zeros(n, dtype=np.uint32)
    tlen = ctypes.c_uint64(0)
    cap = 1 << 16 if trace else 0
    while True:
        tr = np.zeros((max(cap, 1), 3 + model["m"]), dtype=np.uint32)
        rc = lib.or_explore(ctypes.byref(mo), 1 if T is not None else 0,
                            0 if T is None else int(T), 1 if self_check else 0,
                            ctypes.byref(res), _u32p(tc), _u32p(tr) if trace else None,
                            cap, ctypes.byref(tlen), None, 0)
        if rc == -3 and trace and tlen.value > cap:   # buffer too small: explore again
            cap = tlen.value
            continue
        if rc != 0:
            raise OracleError(f"or_explore failed: {rc}")
        break
    tr = tr[:tlen.value] if (trace and tlen.value) else None
    tcl = [None if int(v) == NONE else int(v) for v in tc]
    t_min = None if res.t_min == NONE else int(res.t_min)
    argmin = [c for c, v in enumerate(tcl) if v is not None and v == t_min]
    return {"reachable": int(res.reachable), "edges": int(res.edges),
            "levels": int(res.levels), "terminals": int(res.terminals),
            "violated": bool(res.violated), "t_min": t_min, "argmin": argmin, "tc": tcl,
            "self_check": int(res.self_check), "seconds": float(res.seconds),
            "trace": tr, "trace_cfg": None if res.trace_cfg == NONE else int(res.trace_cfg)}


def reach(model: dict) -> set:
    """The reachable set itself (tuples of 3+m integers), for small models."""
    lib = _load()
    mo, keep = _model(model)
    res = _Result()
    tc = np.zeros(len(model["params"]), dtype=np.uint32)
    tlen = ctypes.c_uint64(0)
    first = explore(model, trace=False)["reachable"]
    out = np.zeros((first, 3 + model["m"]), dtype=np.uint32)
    rc = lib.or_explore(ctypes.byref(mo), 0, 0, 0, ctypes.byref(res), _u32p(tc), None, 0,
                        ctypes.byref(tlen), _u32p(out), first)
    if rc != 0:
        raise OracleError(f"or_explore failed: {rc}")
    return {tuple(int(v) for v in r) for r in out}


def derive(model: dict, c: int) -> dict:
    """Workgroup count n, |E| = b, duration d and the end-time list E of configuration c."""
    lib = _load()
    mo, keep = _model(model)
    n, b, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib.or_derive(ctypes.byref(mo), c, ctypes.byref(n), ctypes.byref(b), ctypes.byref(d),
                       None, 0)
    if rc != 0:
        raise OracleError(f"or_derive failed: {rc}")
    E = np.zeros(max(1, b.value), dtype=np.uint32)
    rc = lib.or_derive(ctypes.byref(mo), c, ctypes.byref(n), ctypes.byref(b), ctypes.byref(d),
                       _u32p(E), E.shape[0])
    if rc != 0:
        raise OracleError(f"or_derive failed: {rc}")
    return {"n": n.value, "b": b.value, "d": d.value, "E": [int(v) for v in E[:b.value]]}


def successors(model: dict, state) -> list[tuple]:
    """Successor states (tuples of 3+m integers) of one state; root = (ROOT, 0, 0, 0..)."""
    lib = _load()
    mo, keep = _model(model)
    m = model["m"]
    x = np.ascontiguousarray(np.asarray(state, dtype=np.uint32).reshape(3 + m))
    cap = max(len(model["params"]), m)
    out = np.zeros((cap, 3 + m), dtype=np.uint32)
    k = lib.or_successors(ctypes.byref(mo), _u32p(x), _u32p(out), cap)
    if k < 0:
        raise OracleError(f"or_successors failed: {k}")
    return [tuple(int(v) for v in out[i]) for i in range(k)]


def is_terminal(state, m: int) -> bool:
    return state[0] != ROOT and state[2] == 0 and all(v == 0 for v in state[3:3 + m])


def check_trace(model: dict, rows, target_clock: int | None = None,
                max_clock: int | None = None, cfgs=None) -> None:
    """Raise AssertionError unless ``rows`` is a path root -> ... -> terminal of the
    model in which every step is a successor (replayed through the oracle)."""
    m = model["m"]
    rows = [tuple(int(v) for v in r) for r in rows]
    assert len(rows) >= 2, "trace too short"
    assert rows[0][0] == ROOT, "trace does not start at the root"
    for a, b in zip(rows, rows[1:]):
        assert b in successors(model, a), f"step {a} -> {b} is not a transition"
    last = rows[-1]
    assert is_terminal(last, m), f"trace ends at a non-terminal {last}"
    if target_clock is not None:
        assert last[1] == target_clock, f"trace ends at clock {last[1]} != {target_clock}"
    if max_clock is not None:
        assert last[1] <= max_clock
    if cfgs is not None:
        assert last[0] in cfgs


def simulate(model: dict, seed: int) -> tuple[int, int]:
    lib = _load()
    mo, keep = _model(model)
    t, c = ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib.or_simulate(ctypes.byref(mo), seed, ctypes.byref(t), ctypes.byref(c))
    if rc != 0:
        raise OracleError(f"or_simulate failed: {rc}")
    return t.value, c.value


def bisect_t_min(model: dict, t_ini: int) -> tuple[int, int]:
    """Integer bisection over the oracle's check(T) (the search of Sec. 2, Fig. 1 read as
    plain bisection): keeps check(lo) holding and check(hi) violated; returns
    (T_min, number of checks)."""
    lo, hi, n = 0, int(t_ini), 0
    while hi - lo > 1:
        mid = (lo + hi) // 2
        n += 1
        if explore(model, T=mid, trace=False)["violated"]:
            hi = mid
        else:
            lo = mid
    return hi, n


def swarm(model: dict, seed: int, members: int, budget: int, bits_log2: int,
          T: int | None = None) -> list[dict]:
    """Swarm search members (Sec. 5): independent random walks from the root with a
    bitstate array per member, against G(!FIN) (T None) or the over-time property with
    threshold T.  One dict per member: walks, trails, steps, best/first trail clock and
    configuration (NONE without trails), the member step where the best walk began and
    where the first trail ended."""
    lib = _load()
    mo, keep = _model(model)
    out = (_SwarmMember * members)()
    rc = lib.or_swarm(ctypes.byref(mo), seed, members, budget, bits_log2,
                      0 if T is None else 1, 0 if T is None else T, out)
    if rc != 0:
        raise OracleError(f"or_swarm failed: {rc}")
    return [{n: int(getattr(r, n)) for n, _ in _SwarmMember._fields_} for r in out]
