"""The bench's command line on the CPU: more than one GPU is refused with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_graph_edges_match_the_oracle(oracle_lib):
    """The edge count behind the bench's algorithmic bytes per state (its round formula)
    equals the edges the oracle's breadth-first search generates, and the duplicate
    edges of the 58M-state workload are those its rounds give (769 per round of eight
    units, 53,816 rounds)."""
    import bench
    import workloads
    import paper_2305_09130_amd as mc
    models = (workloads.tiny_models(5, 40, max_cu=5) + workloads.tiny_unit_models(6, 20)
              + [workloads.reduction_g256()])
    for m in models:
        assert bench.graph_edges(mc, m) == oracle_lib.explore(m, trace=False)["edges"], \
            workloads.describe(m)
    big = workloads.matmul_128_vw()
    assert bench.graph_edges(mc, big) - (58_006_261 - 1) == 769 * 53_816
    assert bench.graph_edges(mc, workloads.with_speeds(workloads.reduction_g256(), [1, 2])) is None


def test_bytes_per_state():
    import bench
    # 2L + 2S + r_dup L with L = 64: two-word keys and the 58M-state workload's r_dup
    r = 41_384_504 / 58_006_261
    assert abs(bench.bytes_per_state(16, r) - (128 + 32 + 64 * r)) < 1e-9
