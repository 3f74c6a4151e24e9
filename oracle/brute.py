"""Brute-force path enumeration on tiny models (test infrastructure only).

Independent of ``mc_oracle.c`` and of ``closed_form``: it unfolds the model as a tree
(no visited set), branching over every configuration and, at every dispatch point, over
every free unit, and it runs time one cycle at a time with each unit executing its
workgroup's operation list op by op (like the clock process of the paper's Listing 9
ticking ``time++`` and the pex processes of Listing 8 counting down their work).

A state of the checked transition system exists at the root, after each selection or
dispatch, and after each cycle in which some busy unit finishes an operation of positive
latency; the jump-clock system visits exactly those.  The enumeration records them with
the same fields (cfg, clock, pending, rem_0..rem_{m-1}), rem being the cycles left in the
unit's workgroup.
"""
from __future__ import annotations

ROOT = 0xFFFFFFFF


def _ticked_pex(S: int, TS: int, gmt: int, loc: int) -> list[int]:
    """Ticks spent in each long_work of one abstract work item (the pex of Listing 8),
    found by running its clock one tick at a time: a long_work keeps reporting work,
    and the clock keeps ticking, while time has not passed its start time + gt*tz."""
    time = 0
    spent = []

    def long_work(start, budget):
        nonlocal time
        t0 = time
        while time <= start + budget:
            time += 1
        spent.append(time - t0)

    start = time
    for _tile in range(S // TS):
        long_work(start, gmt * TS)          # global load of the tile
        start = time
        long_work(start, loc * TS)          # local step on the tile
    start = time
    long_work(start, gmt)                   # the result to global memory
    return spent


def _ticked_minimum(WG: int, TS: int, NP: int, gmt: int, loc: int) -> list[int]:
    """Ticks between consecutive operation ends of one workgroup of the Minimum model,
    found by running its unit (Listing 14) and processing elements (Listing 15) one
    tick at a time.

    The unit starts min(WG, NP) elements on iteration 0.  While WG > NP it answers
    WG - NP status messages: an element that has not reached its last iteration,
    (iter + 1) >= WG/NP, is launched again on the unit's current iteration number,
    which advances after every NP answers; the last statuses are collected by its
    final loop.  An element's MAP makes TS global accesses, one after another, each
    a wait of GMT ticks (the reading of its long_work(GMT) per access); the running
    elements report every tick together, so the clock moves with all of them.  After
    the workgroup, element 0 folds the minima that the other elements left in local
    memory, Ll ticks per element, and writes the result to global memory in GMT."""
    time = 0
    ends = []
    nwe = WG if WG <= NP else NP
    last_iter = WG // NP                      # the listing's integer WG/NP
    running = {e: 0 for e in range(nwe)}      # element -> iteration it runs
    answers_left = WG - NP if WG > NP else 0  # statuses the unit's loop receives
    it, num = 1, 0
    while running:
        left = {e: TS * gmt for e in running}  # ticks of global access work left
        while any(left.values()):
            time += 1                          # every running element reported: tick
            ended = False
            for e in left:
                if left[e]:
                    left[e] -= 1
                    ended = ended or left[e] % gmt == 0
            if ended:
                ends.append(time)              # an access ended
        relaunch = {}
        for e in sorted(running):
            done_wg = running[e] + 1 >= last_iter
            if answers_left:
                answers_left -= 1
                if not done_wg:
                    relaunch[e] = it
                num += 1
                if num >= NP:
                    it, num = it + 1, 0
        running = relaunch
    for other in range(1, nwe):                # element 0 folds loc[myloc + other]
        time += loc
        ends.append(time)
    time += gmt                                # the workgroup's minimum to global memory
    ends.append(time)
    return [b - a for a, b in zip([0] + ends[:-1], ends)]


def workgroup_program(model: dict, row) -> tuple[int, list[int]]:
    """(number of workgroups, latency of every operation of one workgroup, in order)."""
    if model["kind"] in ("abstract", "minimum"):
        S, NP, wg, ts = model["S"], model["NP"], row[0], row[1]
        n = max(1, S // (wg * ts))
        waves = max(1, wg // NP)
        if model["kind"] == "abstract":
            return n, _ticked_pex(S, ts, model["Lg"], model["Ll"]) * waves
        return n, _ticked_minimum(wg, ts, NP, model["Lg"], model["Ll"])
    if model["kind"] == "reduction":
        G, wg, ts = model["G"], row[0], row[1]
        local_steps = 0
        while (1 << local_steps) < wg:
            local_steps += 1
        loads = (G + wg * ts - 1) // (wg * ts)
        prog = ([model["Lg"]] * loads + [model["Ll"]] * local_steps + [model["Lb"]]
                + [model["Lc"]] * ts)
        return G // wg, prog
    M, N, K = model["M"], model["N"], model["K"]
    x, y, ts, vw = row[0], row[1], row[2], (row[3] or 1)
    prog = ([model["Lg"]] * (2 * K) + [model["Ll"]] * (K * (1 + vw))
            + [model["Lb"]] * (2 * (K // ts)) + [model["Lc"]] * (K * vw))
    return (M // x) * (N // (y * vw)), prog


def _skip_free(prog, op):
    while op < len(prog) and prog[op] == 0:
        op += 1
    return op


def enumerate_model(model: dict, max_paths: int = 2_000_000) -> dict:
    """Walk every path.  Returns the set of states on any path, the terminal clocks per
    configuration (as sorted lists with multiplicity per path), the set of path lengths
    per configuration, and the number of paths."""
    m = model["m"]
    states = {(ROOT, 0, 0) + (0,) * m}
    term = {}
    lengths = {}
    npaths = 0

    speed = list(model.get("speed") or [1] * m)  # unit i runs every operation speed[i] times as long
    for c, row in enumerate(model["params"]):
        n, prog = workgroup_program(model, row)
        total = sum(prog)

        def rem_of(i, u):
            if u is None:
                return 0
            op, left = u
            return left + speed[i] * sum(prog[op + 1:])

        def snap(clock, pending, units):
            return (c, clock, pending) + tuple(rem_of(i, u) for i, u in enumerate(units))

        # iterative DFS; frame = (clock, pending, units tuple, depth)
        start = (0, n, (None,) * m, 1)
        states.add(snap(0, n, start[2]))
        stack = [start]
        while stack:
            clock, pending, units, depth = stack.pop()
            free = [i for i, u in enumerate(units) if u is None]
            if pending > 0 and free:
                for i in free:
                    op = _skip_free(prog, 0)
                    nu = list(units)
                    nu[i] = (op, speed[i] * prog[op]) if op < len(prog) else None
                    nu = tuple(nu)
                    states.add(snap(clock, pending - 1, nu))
                    stack.append((clock, pending - 1, nu, depth + 1))
                continue
            if all(u is None for u in units):
                term.setdefault(c, []).append(clock)
                lengths.setdefault(c, set()).add(depth)
                npaths += 1
                if npaths > max_paths:
                    raise RuntimeError("model too large for brute force")
                continue
            # run cycles until some busy unit finishes a timed operation
            us = list(units)
            while True:
                clock += 1
                event = False
                for i, u in enumerate(us):
                    if u is None:
                        continue
                    op, left = u
                    left -= 1
                    if left == 0:
                        event = True
                        op = _skip_free(prog, op + 1)
                        us[i] = (op, speed[i] * prog[op]) if op < len(prog) else None
                    else:
                        us[i] = (op, left)
                if event:
                    break
            nu = tuple(us)
            assert clock <= n * total * max(speed)
            states.add(snap(clock, pending, nu))
            stack.append((clock, pending, nu, depth + 1))
    return {"states": states,
            "terminal_clocks": {c: sorted(v) for c, v in term.items()},
            "lengths": lengths, "paths": npaths}


def summary(model: dict, max_paths: int = 2_000_000) -> dict:
    e = enumerate_model(model, max_paths)
    tc = [min(e["terminal_clocks"][c]) for c in range(len(model["params"]))]
    t_min = min(tc)
    return {"reachable": len(e["states"]), "tc": tc, "t_min": t_min,
            "argmin": [c for c, t in enumerate(tc) if t == t_min],
            "levels": 1 + max(max(s) for s in e["lengths"].values()),
            "states": e["states"], "lengths": e["lengths"],
            "terminal_clocks": e["terminal_clocks"], "paths": e["paths"]}
