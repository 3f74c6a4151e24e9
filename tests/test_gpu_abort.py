"""A stop request from the host (mc_abort) ends a query early with MC_E_ABORTED, every
kernel of it exits normally, and the handle answers the next query exactly."""
import sys
import threading
import time

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


@pytest.mark.parametrize("engine", [0, 1])
def test_abort_before_the_query(mc, engine):
    """A request made while no query runs stops the next one; the one after is exact."""
    model = workloads.reduction_g256()
    ref = oracle.explore(model, trace=False)
    _say(f"abort before min_time, engine {engine}")
    g = mc.Model(model, engine=engine)
    g.mc_abort()
    with pytest.raises(mc.McError) as e:
        g.mc_min_time()
    assert e.value.code == mc.MC_E_ABORTED
    t_min, argmin = g.mc_min_time()
    assert (t_min, argmin) == (ref["t_min"], ref["argmin"])
    assert g.last_stats["states"] == ref["reachable"]
    g.mc_abort()
    with pytest.raises(mc.McError) as e:
        g.mc_check(ref["t_min"])
    assert e.value.code == mc.MC_E_ABORTED
    assert g.mc_check(ref["t_min"]) is True
    g.close()


def test_abort_from_another_thread_stops_a_long_query(mc):
    """The plain level engine needs one launch per BFS level (331,777 levels, seconds);
    a request from another thread 50 ms in stops it within a batch of launches."""
    import torch
    model = workloads.matmul_64()
    g = mc.Model(model, engine=mc.MC_ENGINE_LEVEL)
    _say("level engine on matmul64_cu4, abort after 50 ms")
    timer = threading.Timer(0.05, g.mc_abort)
    t0 = time.perf_counter()
    timer.start()
    with pytest.raises(mc.McError) as e:
        g.mc_min_time()
    dt = time.perf_counter() - t0
    timer.join()
    assert e.value.code == mc.MC_E_ABORTED
    assert dt < 1.0, dt
    torch.cuda.synchronize()
    # the handle still answers exactly (the super-step engine, for speed)
    g.mc_set_engine(mc.MC_ENGINE_SUPERSTEP)
    t_min, argmin = g.mc_min_time()
    assert g.last_stats["states"] == 5_151_061
    assert t_min == 512 * model["Lg"] + 512 * model["Ll"] + 256
    g.close()
