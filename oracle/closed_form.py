"""Closed forms for the lock-step model kinds (test infrastructure only).

Independent of ``mc_oracle.c``: its own derivation of the per-configuration operation
lists (written from the same reading of the model), then formulas instead of search.

Why the formulas hold.  Workgroups of one configuration all have the same duration d
and dispatch is eager (no time passes while a free unit could take pending work; the
clock process of the paper's Listing 9 ticks only after every active processing element
has reported).  So every run proceeds in rounds: at a round start all m units are idle;
min(pending, m) of them are given a workgroup in any order (zero time), those run in
lock step through the b distinct operation end times E_1 < ... < E_b = d, and all become
idle together.  With q = floor(n/m) full rounds and p = n mod m workgroups left over:

  * every terminal of configuration c has clock T_c = ceil(n/m) * d;
  * the states of a full round are the 2^m - 1 non-empty sets of started units plus the
    b states after each advance (the last is the next round start);
  * the partial round has sum_{j=1..p} C(m,j) dispatch states, C(m,p) lock-step runs of
    b-1 intermediate states, and one shared terminal;
  * reachable = 1 (root) + sum_c [1 + q(2^m - 1 + b) + [p>0](sum_j C(m,j) + C(m,p)(b-1) + 1)];
  * the depth of the terminal (and of every path to it) is 1 + n + ceil(n/m) * b.
"""
from __future__ import annotations

from math import comb


def _unit_shape(model: dict, row) -> tuple[int, int, int]:
    """(workgroups, waves, working elements) of the abstract and minimum kinds: n =
    S/(WG*TS), at least one; WG items on NP elements run in WG/NP waves."""
    S, NP, wg, ts = model["S"], model["NP"], row[0], row[1]
    return max(1, S // (wg * ts)), max(1, wg // NP), min(wg, NP)


def ops(model: dict, row) -> tuple[int, list[tuple[int, int]]]:
    """(workgroups, [(count, latency), ...]) of one configuration."""
    if model["kind"] == "abstract":
        # one wave: the first tile's global load lasts GMT*TS + 1 ticks, every local step
        # Ll*TS + 1, every later global load only the part of GMT*TS + 1 not already
        # spent in the previous local step, the final write GMT + 1
        n, waves, _ = _unit_shape(model, row)
        ts, tiles, gmt, loc = row[1], model["S"] // row[1], model["Lg"], model["Ll"]
        later = max(0, gmt * ts + 1 - (loc * ts + 1))
        wave = [(1, gmt * ts + 1), (1, loc * ts + 1)]
        wave += [(1, later), (1, loc * ts + 1)] * (tiles - 1)
        wave += [(1, gmt + 1)]
        return n, wave * waves
    if model["kind"] == "minimum":
        n, waves, nwe = _unit_shape(model, row)
        return n, [(waves * row[1], model["Lg"]), (nwe - 1, model["Ll"]), (1, model["Lg"])]
    if model["kind"] == "reduction":
        G = model["G"]
        wg, ts = row[0], row[1]
        n = G // wg
        loads = -(-G // (wg * ts))
        return n, [(loads, model["Lg"]), (wg.bit_length() - 1, model["Ll"]),
                   (1, model["Lb"]), (ts, model["Lc"])]
    M, N, K = model["M"], model["N"], model["K"]
    x, y, ts, vw = row[0], row[1], row[2], (row[3] or 1)
    n = (M // x) * (N // (y * vw))
    return n, [(2 * K, model["Lg"]), (K * (1 + vw), model["Ll"]),
               ((K // ts) * 2, model["Lb"]), (K * vw, model["Lc"])]


def abstract_wave_time(S: int, TS: int, gmt: int, loc: int = 1) -> int:
    """Duration of one wave of the abstract kernel for loc <= gmt.  Every global load
    ends gmt*TS + 1 ticks after the previous load ended (the start time it waits from is
    set when the previous local step starts, i.e. when the previous load ended), so load
    k ends at k*(gmt*TS + 1); the last local step adds loc*TS + 1 and the final write
    gmt + 1: (S/TS)*(gmt*TS + 1) + loc*TS + 1 + gmt + 1."""
    assert loc <= gmt
    return (S // TS) * (gmt * TS + 1) + loc * TS + 1 + gmt + 1


def end_times(oplist) -> list[int]:
    """Distinct cumulative end times of the operations, in order."""
    out, t = [], 0
    for count, lat in oplist:
        for _ in range(count):
            t += lat
            if not out or out[-1] != t:
                out.append(t)
    return out


def per_config(model: dict, with_E: bool = True) -> list[dict]:
    m = model["m"]
    res = []
    for row in model["params"]:
        n, ol = ops(model, row)
        E = end_times(ol) if with_E else None
        b = len(E) if E is not None else sum(cnt for cnt, lat in ol if lat > 0)
        d = sum(cnt * lat for cnt, lat in ol)
        q, p = divmod(n, m)
        rounds = -(-n // m)
        count = 1 + q * ((1 << m) - 1 + b)
        if p:
            count += sum(comb(m, j) for j in range(1, p + 1)) + comb(m, p) * (b - 1) + 1
        res.append({"n": n, "b": b, "d": d, "E": E, "q": q, "p": p, "rounds": rounds,
                    "tc": rounds * d, "count": count, "depth": 1 + n + rounds * b})
    return res


def summary(model: dict, with_E: bool = True) -> dict:
    pc = per_config(model, with_E)
    tcs = [c["tc"] for c in pc]
    t_min = min(tcs)
    return {"reachable": 1 + sum(c["count"] for c in pc),
            "levels": 1 + max(c["depth"] for c in pc),
            "tc": tcs, "t_min": t_min,
            "argmin": [i for i, t in enumerate(tcs) if t == t_min],
            "trace_len": 1 + pc[min(i for i, t in enumerate(tcs) if t == t_min)]["depth"],
            "per_config": pc}


def count_le(model: dict, T: int) -> int:
    """Number of reachable states with clock <= T (root clock 0), summed round by round
    from the clocks of the states of each round."""
    m = model["m"]
    total = 1
    for c in per_config(model):
        n, E, d, q, p = c["n"], c["E"], c["d"], c["q"], c["p"]
        total += 1 if T >= 0 else 0                     # the selected start state
        for r in range(q):                              # full rounds
            start = r * d
            if start <= T:
                total += (1 << m) - 1
            total += sum(1 for e in E if start + e <= T)
        if p:
            start = q * d
            if start <= T:
                total += sum(comb(m, j) for j in range(1, p + 1))
            total += comb(m, p) * sum(1 for e in E[:-1] if start + e <= T)
            total += 1 if start + d <= T else 0
    return total


def single_cu_count(model: dict) -> int:
    """Reachable count of a one-unit model: 1 + sum_c (1 + n_c (1 + b_c))."""
    assert model["m"] == 1
    return 1 + sum(1 + c["n"] * (1 + c["b"]) for c in per_config(model))
