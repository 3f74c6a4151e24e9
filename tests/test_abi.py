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
    # equal units: cfg, pending, busy mask and one shared time left (the clock follows
    # from them): 9 + 15 + 8 + 14 = 46 bits for the 58M-state workload
    assert d["key_words"] == {"reduction_g256_cu2": 1, "matmul64_cu4": 1,
                              "matmul128_vw_cu8": 1}[name]


def test_describe_tiny_sweep(mc):
    for model in workloads.tiny_models(21, 200, max_cu=8):
        d = mc.mc_describe(model)
        s = cf.summary(model)
        assert d["states"] == s["reachable"], workloads.describe(model)
        assert d["max_depth"] + 1 == s["levels"]


def test_workspace_sizes(mc):
    m = workloads.matmul_128_vw()
    n = mc.mc_workspace_bytes(m)
    # 58M states at the automatic load factor (at most 3/8 after rounding up to a power of
    # two) in 16-byte slots (one key word): 2^28 slots = 4 GiB
    assert 4 * 2**30 <= n < 4.5 * 2**30
    half = mc.mc_workspace_bytes(m, mc.make_opts(load_factor=0.5))
    assert 2 * 2**30 <= half < 2.5 * 2**30
    small = mc.mc_workspace_bytes(m, mc.make_opts(load_factor=0.125))
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


# --- the unit-model kinds (abstract kernel, Minimum problem) --------------------------

def _unit_sweep():
    out = []
    for seed in (31, 32):
        out += workloads.tiny_unit_models(seed, 100, max_cu=8)
    for kind in (workloads.KIND_ABSTRACT, workloads.KIND_MINIMUM):
        for S, NP, gmt, loc in ((64, 4, 4, 1), (256, 2, 1, 3), (1024, 8, 9, 2)):
            dom = workloads.pow2_range(0, 6)
            out.append(workloads.unit_model(kind, S, NP, 3, dom, dom, gmt, loc))
    return out


def test_unit_kinds_config_ends_match_closed_form(mc):
    """The library's per-configuration phase tables (waves, two-operation periods,
    offset grids) give exactly the operation ends of the closed-form lists."""
    n_cfg = 0
    for model in _unit_sweep() + [f() for f in workloads.UNIT_WORKLOADS.values()]:
        for c, row in enumerate(model["params"]):
            n, ol = cf.ops(model, row)
            E = cf.end_times(ol)
            got = mc.mc_config_ends(model, c)
            assert (got["n"], got["b"], got["d"]) == (n, len(E), E[-1]), workloads.describe(model)
            assert got["E"] == E, (workloads.describe(model), row)
            n_cfg += 1
    assert n_cfg > 500


def test_config_ends_uniform_kinds(mc):
    for name, f in workloads.WORKLOADS.items():
        model = f()
        for c in range(0, len(model["params"]), 7):
            n, ol = cf.ops(model, model["params"][c])
            got = mc.mc_config_ends(model, c)
            assert got["E"] == cf.end_times(ol) and got["n"] == n, name


def test_unit_kinds_describe(mc):
    for model in _unit_sweep():
        d = mc.mc_describe(model)
        s = cf.summary(model, with_E=False)
        assert d["states"] == s["reachable"], workloads.describe(model)
        assert d["max_depth"] + 1 == s["levels"]
    want = {"abstract_s1024_np4_cu1": (1868340, 1), "abstract_s1024_np4_cu4": (2266564, 1),
            "minimum_s1024_np4_cu4": (1052986, 1)}
    for name, f in workloads.UNIT_WORKLOADS.items():
        d = mc.mc_describe(f())
        assert (d["states"], d["key_words"]) == want[name]
        assert d["states"] == cf.summary(f(), with_E=False)["reachable"]


@pytest.mark.parametrize("bad", [
    {"S": 100}, {"NP": 3}, {"NP": 0}, {"params": [[3, 1, 0, 0]]}, {"params": [[1, 2048, 0, 0]]},
    {"params": [[2048, 1, 0, 0]]},
])
def test_invalid_unit_descriptors(mc, bad):
    model = dict(workloads.minimum_paper(1024, 2), **bad)
    with pytest.raises(mc.McError) as e:
        mc.mc_describe(model)
    assert e.value.code == mc.MC_E_INVAL
    with pytest.raises(mc.McError):
        mc.mc_config_ends(model, 0)


def test_unequal_units_describe_bounds_the_oracle(mc):
    """On units of unequal speed the library sizes each configuration by walking its
    determined run and every tail: an upper bound on the reachable count (tails that
    meet are counted twice) and the exact longest path."""
    import oracle
    exact = 0
    for model in workloads.tiny_hetero_models(51, 60, max_cu=6):
        d = mc.mc_describe(model)
        r = oracle.explore(model)
        assert d["states"] >= r["reachable"], workloads.describe(model)
        assert d["max_depth"] + 1 >= len(r["trace"])
        exact += d["states"] == r["reachable"]
    assert exact >= 10
    for name, model in workloads.hetero_workloads().items():
        assert mc.mc_describe(model)["states"] >= 86474


def test_invalid_speeds(mc):
    base = workloads.reduction_g256()
    for speeds in ([0, 1], [1, 65]):
        with pytest.raises(mc.McError) as e:
            mc.mc_describe(workloads.with_speeds(base, speeds))
        assert e.value.code == mc.MC_E_INVAL


def test_peak_library_exports_its_header():
    from paper_2305_09130_amd import peak
    names = peak.exported_symbols()
    assert names == ["mcp_random_cas", "mcp_random_read"]
    lib = ctypes.CDLL(peak.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/mcpeak.h but not exported"


def test_abort_code(mc):
    assert mc.MC_E_ABORTED == -11
    assert "abort" in mc.mc_strerror(mc.MC_E_ABORTED)


def test_test_hash_bits_bounded(mc):
    m = workloads.reduction_g256()
    assert mc.mc_workspace_bytes(m, mc.make_opts(test_hash_bits=24)) > 0
    with pytest.raises(mc.McError) as e:
        mc.mc_workspace_bytes(m, mc.make_opts(test_hash_bits=25))
    assert e.value.code == mc.MC_E_INVAL
