"""Stress tier of the visited set on the GPU: with a test option that keeps only a few
bits of the key hash, keys crowd into 2^k probe sequences, so inserts walk long probe
chains and keys of two and four words that share word 0 meet in the same slots (the
claim on word 0, then the wait for and comparison of the other words).  Counts, clocks,
verdicts and traces must stay the oracle's, on both engines and with one or two keys per
lane; a nearly full table (load 0.9) is exercised too."""
import sys

import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available()
    import paper_2305_09130_amd as mc
    return mc


def _models():
    w = workloads
    return [
        w.reduction_model(64, 4, [1, 2, 4, 8], [1, 2], 7, 3),                     # 1 word
        w.with_speeds(w.reduction_model(64, 4, [1, 2, 4], [1, 2], 37, 3), [1, 2, 3, 4]),
        w.with_speeds(w.reduction_model(64, 8, [1, 2, 4], [1, 2], 37, 3),
                      [1, 2, 3, 4, 5, 6, 7, 8]),                                      # 4 words
        w.matmul_model(8, 8, 8, 4, [1, 2], [1, 2], [1, 2], [1, 2], 5, 2),
    ]


@pytest.mark.parametrize("bits", [3, 8])
@pytest.mark.parametrize("engine", [0, 1])
def test_low_entropy_hash(mc, bits, engine):
    for model in _models():
        d = mc.mc_describe(model)
        _say(f"hash bits {bits} engine {engine} W={d['key_words']} {workloads.describe(model)}")
        r = oracle.explore(model, trace=False)
        for lane_items in ((1, 2) if engine == 0 else (0,)):
            g = mc.Model(model, engine=engine, test_hash_bits=bits, lane_items=lane_items)
            t_min, argmin = g.mc_min_time()
            st = g.last_stats
            assert (t_min, argmin) == (r["t_min"], r["argmin"])
            assert st["states"] == r["reachable"]
            assert g.mc_terminal_clocks() == r["tc"]
            assert st["cas_fail"] == st["probes"] - st["states"] - st["dups"] >= 0
            if bits == 3:
                assert st["max_probe"] > 16   # the chains really are long
                assert st["cas_fail"] > st["states"]
            oracle.check_trace(model, g.mc_trace(), target_clock=r["t_min"], cfgs=r["argmin"])
            q = oracle.explore(model, T=r["t_min"] - 1, trace=False)
            assert g.mc_check(r["t_min"] - 1) is False
            assert g.last_stats["states"] == q["reachable"]
            g.close()


def test_key_widths_covered(mc):
    assert sorted({mc.mc_describe(m)["key_words"] for m in _models()}) == [1, 2, 4]


@pytest.mark.parametrize("engine", [0, 1])
def test_nearly_full_table(mc, engine):
    """Load factor 0.9: long probe sequences over the whole table."""
    model = workloads.reduction_g256()
    r = oracle.explore(model, trace=False)
    g = mc.Model(model, engine=engine, load_factor=0.9)
    info = g.mc_model_info_get()
    assert r["reachable"] / info["slots"] > 0.6
    assert g.mc_min_time() == (r["t_min"], r["argmin"])
    assert g.last_stats["states"] == r["reachable"]
    g.close()
