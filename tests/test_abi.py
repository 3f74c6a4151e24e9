"""The C-ABI library loads on the CPU, exports every declared symbol, and its host-side
model logic (validation, sizing) agrees with the oracle's closed forms.  No compute
call touches a GPU here."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import closed_form as cf


@pytest.fixture(scope="module")
def mc():
    import paper_2305_09130_amd as mc
    return mc


def test_every_declared_symbol_is_exported(mc):
    names = mc.exported_symbols()
    assert len(names) >= 14
    lib = ctypes.CDLL(mc.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/mctune.h but not exported"


def test_strerror(mc):
    assert mc.mc_strerror(0) == "ok"
    for code in range(-9, 0):
        assert mc.mc_strerror(code) != "unknown error"


@pytest.mark.parametrize("name", sorted(workloads.WORKLOADS))
def test_describe_matches_closed_form(mc, name):
    model = workloads.WORKLOADS[name]()
    d = mc.mc_describe(model)
    s = cf.summary(model)
    assert d["states"] == s["reachable"]
    assert d["max_depth"] + 1 == s["levels"]
    assert d["key_words"] == {"reduction_g256_cu2": 1, "matmul64_cu4": 2,
                              "matmul128_vw_cu8": 4}[name]


def test_describe_tiny_sweep(mc):
    for model in workloads.tiny_models(21, 200, max_cu=8):
        d = mc.mc_describe(model)
        s = cf.summary(model)
        assert d["states"] == s["reachable"], workloads.describe(model)
        assert d["max_depth"] + 1 == s["levels"]


def test_workspace_sizes(mc):
    m = workloads.matmul_128_vw()
    n = mc.mc_workspace_bytes(m)
    # 58M states at load factor <= 0.5 in 64-byte slots: 2^27 slots = 8 GiB
    assert 8 * 2**30 <= n < 9 * 2**30
    small = mc.mc_workspace_bytes(m, mc.make_opts(load_factor=0.25))
    assert small > n


@pytest.mark.parametrize("bad", [
    {"m": 0}, {"m": 9}, {"Lg": 0}, {"Ll": 0}, {"Lc": 0}, {"params": []},
    {"params": [[3, 1, 0, 0]]}, {"params": [[512, 1, 0, 0]]}, {"G": 100},
])
def test_invalid_descriptors(mc, bad):
    model = dict(workloads.reduction_g256(), **bad)
    if "params" in bad and bad["params"] == []:
        model["params"] = np.zeros((0, 4), dtype=np.uint32)
    with pytest.raises(mc.McError) as e:
        mc.mc_describe(model)
    assert e.value.code == mc.MC_E_INVAL


def test_invalid_matmul(mc):
    base = workloads.matmul_64()
    for params in ([[128, 1, 1, 1]], [[1, 32, 1, 4]], [[1, 1, 128, 1]], [[1, 1, 3, 1]]):
        with pytest.raises(mc.McError):
            mc.mc_describe(dict(base, params=params))


def test_batch_draws_agree(mc):
    """The batched mix drawn with the library's size filter equals the mix drawn with
    the oracle's closed form."""
    budget = 1 << 20
    a, ra = workloads.draw_batch(3, 64, lambda x: (mc.state_count(x) or budget + 1) <= budget)
    b, rb = workloads.draw_batch(3, 64, lambda x: cf.summary(x, with_E=False)["reachable"] <= budget)
    assert a == b and ra == rb
