"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's harness.

This module only draws numbers: latencies, parameter domains, instance mixes and
arrival times.  It holds none of the checker's arithmetic (no workgroup counts, no
operation costs, no state counts); where a draw must be filtered by model size the
caller passes the filter in.

A model is a plain dict:

    {"kind": "reduction" | "matmul" | "abstract" | "minimum", "m": CU count,
     "G": global size (reduction) | "M","N","K": matrix sizes (matmul) |
     "S", "NP": data size and processing elements per unit (abstract, minimum),
     "Lg", "Ll", "Lc", "Lb": integer latencies,
     "params": [[p0, p1, p2, p3], ...]}     # one row per configuration

Reduction, abstract and minimum rows are (WG, TS, 0, 0); matmul rows are
(WGx, WGy, TS, VW).  Rows are in lexicographic order of the parameter domains unless a
subset was drawn.
"""
from __future__ import annotations

import itertools

import numpy as np

KIND_REDUCTION = "reduction"
KIND_MATMUL = "matmul"
KIND_ABSTRACT = "abstract"
KIND_MINIMUM = "minimum"


def latencies(seed: int) -> tuple[int, int]:
    """One global-memory latency in [20, 40] and one local-memory latency in [2, 4]
    (inclusive), drawn once per model instance from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    lg = int(rng.integers(20, 41))
    ll = int(rng.integers(2, 5))
    return lg, ll


def pow2_range(lo_exp: int, hi_exp: int) -> list[int]:
    return [1 << e for e in range(lo_exp, hi_exp + 1)]


def reduction_model(G, m, wg_values, ts_values, Lg, Ll, Lc=1, Lb=0) -> dict:
    params = [[wg, ts, 0, 0] for wg, ts in itertools.product(wg_values, ts_values)]
    return {"kind": KIND_REDUCTION, "m": m, "G": G, "Lg": Lg, "Ll": Ll, "Lc": Lc,
            "Lb": Lb, "params": params}


def matmul_model(M, N, K, m, wgx_values, wgy_values, ts_values, vw_values, Lg, Ll,
                 Lc=1, Lb=0) -> dict:
    params = [[x, y, t, v] for x, y, t, v in
              itertools.product(wgx_values, wgy_values, ts_values, vw_values)]
    return {"kind": KIND_MATMUL, "m": m, "M": M, "N": N, "K": K, "Lg": Lg, "Ll": Ll,
            "Lc": Lc, "Lb": Lb, "params": params}


# --- the three single-query workloads -------------------------------------------------

def reduction_g256(seed: int = 0) -> dict:
    """1D reduction-shaped model: G=256 work-items, 2 CUs, WG in {1..32}, TS in {1,2,4}."""
    lg, ll = latencies(seed)
    return reduction_model(256, 2, pow2_range(0, 5), pow2_range(0, 2), lg, ll)


def matmul_64(seed: int = 1) -> dict:
    """2D matmul-shaped model: M=N=K=64, 4 CUs, WGx,WGy in {1..16}, TS in {1..8}."""
    lg, ll = latencies(seed)
    return matmul_model(64, 64, 64, 4, pow2_range(0, 4), pow2_range(0, 4),
                        pow2_range(0, 3), [1], lg, ll)


def matmul_128_vw(seed: int = 2) -> dict:
    """Large matmul-shaped model: M=N=K=128, 8 CUs, plus vector width in {1,2,4}."""
    lg, ll = latencies(seed)
    return matmul_model(128, 128, 128, 8, pow2_range(0, 4), pow2_range(0, 4),
                        pow2_range(0, 3), pow2_range(0, 2), lg, ll)


WORKLOADS = {
    "reduction_g256_cu2": reduction_g256,
    "matmul64_cu4": matmul_64,
    "matmul128_vw_cu8": matmul_128_vw,
}


# --- the paper's own unit models (abstract kernel, Minimum problem) ----------------------

# Platform constants of the paper's abstract-model experiments: one device, units of
# four processing elements, a global access GMT = 4 local steps of 1 (GMT is not
# printed; 4 is the value under which the printed model times come out).
PAPER_NP, PAPER_GMT, PAPER_LOCAL = 4, 4, 1


def unit_model(kind: str, S: int, NP: int, m: int, wg_values, ts_values, Lg: int,
               Ll: int = 1) -> dict:
    params = [[wg, ts, 0, 0] for wg, ts in itertools.product(wg_values, ts_values)]
    return {"kind": kind, "m": m, "S": S, "NP": NP, "Lg": Lg, "Ll": Ll, "Lc": 1, "Lb": 0,
            "params": params}


def paper_domain(S: int) -> list[int]:
    """WG and TS values the parameter-selecting process picks from: 2 .. S/2."""
    return pow2_range(1, S.bit_length() - 2)


def abstract_paper(S: int = 1024, m: int = 1) -> dict:
    """The abstract kernel on the paper's platform (units of 4 elements, GMT 4), every
    (WG, TS) pair of the paper's domain; m = 1 is the single unit of its experiments."""
    dom = paper_domain(S)
    return unit_model(KIND_ABSTRACT, S, PAPER_NP, m, dom, dom, PAPER_GMT, PAPER_LOCAL)


def minimum_paper(S: int = 1024, m: int = 4) -> dict:
    """The Minimum problem model on the same platform and domain."""
    dom = paper_domain(S)
    return unit_model(KIND_MINIMUM, S, PAPER_NP, m, dom, dom, PAPER_GMT, PAPER_LOCAL)


UNIT_WORKLOADS = {
    "abstract_s1024_np4_cu1": lambda: abstract_paper(1024, 1),
    "abstract_s1024_np4_cu4": lambda: abstract_paper(1024, 4),
    "minimum_s1024_np4_cu4": lambda: minimum_paper(1024, 4),
}


# --- batched and served mixes -----------------------------------------------------------

def _instance_candidate(rng: np.random.Generator, kind: str) -> dict:
    """One candidate instance of the batched mix (kind fixed by the caller)."""
    e = int(rng.integers(6, 13))            # size 2^6 .. 2^12
    m = int(rng.choice([2, 4, 8]))
    lg = int(rng.integers(20, 41))
    ll = int(rng.integers(2, 5))
    if kind == KIND_REDUCTION:
        size = 1 << e
        domain = [[wg, ts, 0, 0] for wg, ts in
                  itertools.product(pow2_range(0, min(e, 10)), pow2_range(0, 6))]
        base = {"kind": kind, "m": m, "G": size}
    else:
        size = 1 << e
        domain = [[x, y, t, v] for x, y, t, v in
                  itertools.product(pow2_range(0, 4), pow2_range(0, 4),
                                    [t for t in pow2_range(0, 3) if t <= size],
                                    pow2_range(0, 2))]
        base = {"kind": kind, "m": m, "M": size, "N": size, "K": size}
    s = int(rng.integers(12, 201))
    s = min(s, len(domain))
    pick = np.sort(rng.choice(len(domain), size=s, replace=False))
    base.update({"Lg": lg, "Ll": ll, "Lc": 1, "Lb": 0,
                 "params": [domain[int(i)] for i in pick]})
    return base


def draw_batch(seed: int, n: int, accept) -> tuple[list[dict], int]:
    """Draw ``n`` instances of the uneven batched mix.

    Each instance picks its kind 50/50, then a size 2^e (e in 6..12), a CU count in
    {2,4,8}, latencies as above and a random subset of 12..200 configurations of its
    kind's domain.  ``accept(model) -> bool`` is the caller's size filter; a rejected
    candidate is redrawn with the same kind.  Returns (instances, rejections).
    """
    rng = np.random.default_rng(seed)
    out, rejected = [], 0
    while len(out) < n:
        kind = KIND_REDUCTION if rng.random() < 0.5 else KIND_MATMUL
        while True:
            cand = _instance_candidate(rng, kind)
            if accept(cand):
                out.append(cand)
                break
            rejected += 1
    return out, rejected


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    """Arrival times (seconds, ascending) of a Poisson stream at ``qps``."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def query_mix(seed: int, n: int, pool_size: int) -> list[tuple[int, str, float]]:
    """(model index, query kind, threshold factor) triples of the served stream: the
    model is uniform over the pool, the kind is 'check' or 'min_time' 50/50, and the
    threshold factor u is uniform in [0.8, 1.5) (the caller sets T = floor(u*T_min))."""
    rng = np.random.default_rng(seed + 1)
    idx = rng.integers(0, pool_size, size=n)
    kinds = rng.random(n) < 0.5
    us = rng.uniform(0.8, 1.5, size=n)
    return [(int(i), "check" if k else "min_time", float(u))
            for i, k, u in zip(idx, kinds, us)]


def tiny_models(seed: int, count: int, max_cu: int = 4) -> list[dict]:
    """Random tiny models for sweeps: small sizes, few configurations, latencies
    1..6, barrier latency 0 or 1, CU counts 1..max_cu (partial rounds included)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.integers(1, max_cu + 1))
        lg = int(rng.integers(1, 7))
        ll = int(rng.integers(1, 4))
        lb = int(rng.integers(0, 2))
        if rng.random() < 0.5:
            e = int(rng.integers(2, 6))
            dom = [[wg, ts, 0, 0] for wg, ts in
                   itertools.product(pow2_range(0, min(e, 3)), pow2_range(0, 2))]
            base = {"kind": KIND_REDUCTION, "m": m, "G": 1 << e}
        else:
            e = int(rng.integers(1, 3))
            s = 1 << e
            dom = [[x, y, t, v] for x, y, t, v in
                   itertools.product(pow2_range(0, e), pow2_range(0, e),
                                     pow2_range(0, e), [1, 2])
                   if y * v <= s]
            base = {"kind": KIND_MATMUL, "m": m, "M": s, "N": s, "K": s}
        k = int(rng.integers(1, min(len(dom), 6) + 1))
        pick = np.sort(rng.choice(len(dom), size=k, replace=False))
        base.update({"Lg": lg, "Ll": ll, "Lc": 1, "Lb": lb,
                     "params": [dom[int(i)] for i in pick]})
        out.append(base)
    return out


def tiny_unit_models(seed: int, count: int, max_cu: int = 3) -> list[dict]:
    """Random tiny abstract / minimum models: S in 4..32, NP in {1,2,4}, GMT 1..5, local
    step 1..3 (so GMT below, at and above it), CU counts 1..max_cu, a few (WG, TS)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = KIND_ABSTRACT if rng.random() < 0.5 else KIND_MINIMUM
        e = int(rng.integers(2, 6))
        S = 1 << e
        dom = [[wg, ts, 0, 0] for wg, ts in
               itertools.product(pow2_range(0, min(e, 3)), pow2_range(0, min(e, 3)))]
        k = int(rng.integers(1, min(len(dom), 5) + 1))
        pick = np.sort(rng.choice(len(dom), size=k, replace=False))
        out.append({"kind": kind, "m": int(rng.integers(1, max_cu + 1)), "S": S,
                    "NP": int(rng.choice([1, 2, 4])), "Lg": int(rng.integers(1, 6)),
                    "Ll": int(rng.integers(1, 4)), "Lc": 1, "Lb": 0,
                    "params": [dom[int(i)] for i in pick]})
    return out


def with_speeds(model: dict, speeds) -> dict:
    """The model on units of unequal speed: unit i runs every operation speeds[i] times as
    long (speeds[i] >= 1)."""
    out = dict(model)
    out["speed"] = [int(v) for v in speeds]
    assert len(out["speed"]) == model["m"]
    return out


def hetero_workloads() -> dict:
    """Models on units of unequal speed (speeds 1, 1, 2, 3): the reduction-shaped model of
    G = 256 on four units and the matmul-shaped model of M = N = K = 32 on four units,
    with the latencies of the single-query workloads (seeds 0 and 1)."""
    return {
        "reduction_g256_cu4_s1123": with_speeds(
            reduction_model(256, 4, pow2_range(0, 5), pow2_range(0, 2), *latencies(0)),
            [1, 1, 2, 3]),
        "matmul32_cu4_s1123": with_speeds(
            matmul_model(32, 32, 32, 4, pow2_range(0, 4), pow2_range(0, 4), pow2_range(0, 3),
                         [1], *latencies(1)),
            [1, 1, 2, 3]),
    }


def tiny_hetero_models(seed: int, count: int, max_cu: int = 4, max_speed: int = 3) -> list[dict]:
    """Tiny models of every kind on 2..max_cu units whose speeds are drawn from
    1..max_speed (at least two distinct speeds)."""
    rng = np.random.default_rng(seed)
    pool = tiny_models(seed + 1, count, max_cu) + tiny_unit_models(seed + 2, count, max_cu)
    out = []
    for k in range(count):
        base = pool[int(rng.integers(0, len(pool)))]
        m = max(2, base["m"])
        speeds = [int(v) for v in rng.integers(1, max_speed + 1, size=m)]
        if len(set(speeds)) == 1:
            speeds[int(rng.integers(0, m))] = 1 + speeds[0] % max_speed
        out.append(with_speeds(dict(base, m=m), speeds))
    return out


def describe(model: dict) -> str:
    if model.get("speed") and len(set(model["speed"])) > 1:
        base = describe({k: v for k, v in model.items() if k != "speed"})
        return base[:-1] + f", speeds={model['speed']})"
    if model["kind"] in (KIND_ABSTRACT, KIND_MINIMUM):
        return (f"{model['kind']}(S={model['S']}, NP={model['NP']}, m={model['m']}, "
                f"GMT={model['Lg']}, local={model['Ll']}, #P={len(model['params'])})")
    if model["kind"] == KIND_REDUCTION:
        sz = f"G={model['G']}"
    else:
        sz = f"M={model['M']},N={model['N']},K={model['K']}"
    return (f"{model['kind']}({sz}, m={model['m']}, Lg={model['Lg']}, Ll={model['Ll']}, "
            f"Lc={model['Lc']}, Lb={model['Lb']}, #P={len(model['params'])})")

