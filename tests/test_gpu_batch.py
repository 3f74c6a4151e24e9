"""GPU parity of the batched engine: many models in one persistent launch.

Every model's T_min, reachable count and per-configuration clocks must equal the oracle
(small models) or the oracle-pinned closed forms (the full 512-instance mix), and equal
the same model explored alone.  The hipGraph replay must reproduce the eager result on
every replay.
"""
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


def _mix(n, seed=3):
    import paper_2305_09130_amd as mc
    ms, _ = workloads.draw_batch(seed, n, lambda x: (mc.state_count(x) or BUDGET + 1) <= BUDGET)
    return ms


def test_batch_small_models_vs_oracle(mc):
    models = workloads.tiny_models(301, 40, max_cu=8) + [workloads.reduction_g256()]
    _say(f"batch of {len(models)} small models")
    b = mc.Batch(models, mc.make_batch_opts(block=256))
    t_min, states = b.mc_batch_min_time()
    for i, m in enumerate(models):
        r = oracle.explore(m, trace=False)
        assert t_min[i] == r["t_min"], (i, workloads.describe(m))
        assert states[i] == r["reachable"], (i, workloads.describe(m))
        assert b.mc_batch_terminal_clocks(i) == r["tc"]
    b.close()


def test_batch_round_blocks_vs_oracle(mc):
    """Models with many rounds per configuration, every subgraph cut into 8-round blocks,
    in one batch (three key widths, so three concurrent launches) against the oracle."""
    models = [
        workloads.reduction_model(256, 2, [1, 2, 4, 8], [1, 2], 5, 2, Lb=1),
        workloads.matmul_model(16, 16, 16, 4, [1, 2], [1, 2], [1, 4], [1, 2], 3, 2),
        workloads.reduction_model(64, 3, [1, 2], [1, 2], 4, 3),
        workloads.matmul_model(16, 16, 8, 8, [1], [1], [1, 2], [1], 2, 1),
        workloads.matmul_64(),
    ]
    _say("batch of round-block models")
    b = mc.Batch(models, mc.make_batch_opts(block=512, part_states=1))
    t_min, states = b.mc_batch_min_time()
    assert b.last_stats["parts"] > sum(len(m["params"]) for m in models)
    for i, m in enumerate(models):
        r = oracle.explore(m, trace=False)
        assert (t_min[i], states[i]) == (r["t_min"], r["reachable"]), workloads.describe(m)
        assert b.mc_batch_terminal_clocks(i) == r["tc"]
    b.close()


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_batch_equals_alone(mc, block):
    models = _mix(24)
    _say(f"mix of 24, block={block}")
    b = mc.Batch(models, mc.make_batch_opts(block=block, load_factor=0.5))
    t_min, states = b.mc_batch_min_time()
    for i, m in enumerate(models):
        s = cf.summary(m, with_E=False)
        assert (t_min[i], states[i]) == (s["t_min"], s["reachable"]), workloads.describe(m)
        assert b.mc_batch_terminal_clocks(i) == s["tc"]
    b.close()
    for i in (0, 5, 11):
        g = mc.Model(models[i])
        assert g.mc_min_time()[0] == t_min[i]
        assert g.last_stats["states"] == states[i]
        g.close()


def test_batch_graph_replay_matches_eager(mc):
    import torch
    models = _mix(16, seed=5)
    eager = mc.Batch(models, mc.make_batch_opts(block=512))
    ref = eager.mc_batch_min_time()
    ref_tc = [eager.mc_batch_terminal_clocks(i) for i in range(len(models))]
    eager.close()
    g = mc.Batch(models, mc.make_batch_opts(block=512, use_graph=True))
    other = mc.Model(workloads.reduction_g256())
    for rep in range(4):
        _say(f"graph replay {rep}")
        got = g.mc_batch_min_time()
        assert got == ref
        assert [g.mc_batch_terminal_clocks(i) for i in range(len(models))] == ref_tc
        # the program's own eager work between replays
        other.mc_min_time()
        x = torch.arange(1 << 20, device="cuda:0", dtype=torch.int64).sum().item()
        assert x == (1 << 20) * ((1 << 20) - 1) // 2
        torch.cuda.synchronize()
    g.close()
    other.close()


def test_batch_autotune(mc):
    import torch
    models = _mix(8, seed=7)
    need = mc.mc_batch_workspace_bytes(models, mc.make_batch_opts(load_factor=0.25))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    best, ms = mc.mc_batch_autotune(models, ws)
    assert best.block in (256, 512, 1024) and 0.0 < best.load_factor < 1.0 and ms > 0
    best2, ms2 = mc.mc_batch_autotune(models, ws)
    assert best2.as_dict() == best.as_dict() and ms2 < 0   # cached
    b = mc.Batch(models, best, workspace=ws)
    t_min, states = b.mc_batch_min_time()
    for i, m in enumerate(models):
        s = cf.summary(m, with_E=False)
        assert (t_min[i], states[i]) == (s["t_min"], s["reachable"])
    b.close()


def test_batch_512_full_mix(mc):
    """The full seeded mix of 512 uneven instances in one launch, against the pinned
    closed forms; the smallest instances also against the oracle itself."""
    models = _mix(512)
    _say("batch of 512")
    b = mc.Batch(models, mc.make_batch_opts(block=512, use_graph=True))
    t_min, states = b.mc_batch_min_time()
    sizes = []
    for i, m in enumerate(models):
        s = cf.summary(m, with_E=False)
        assert (t_min[i], states[i]) == (s["t_min"], s["reachable"]), (i, workloads.describe(m))
        sizes.append((s["reachable"], i))
    for _, i in sorted(sizes)[:6]:
        r = oracle.explore(models[i], trace=False)
        assert (r["t_min"], r["reachable"], r["tc"]) == \
            (t_min[i], states[i], b.mc_batch_terminal_clocks(i))
    b.close()
