"""Python binding of libmctune, the MI355X explicit-state auto-tuning checker.

Argument marshalling only: every step of the exploration runs in the HIP kernels of
``csrc/``.  PyTorch provides the device workspace and the stream.  The C names
(``mc_*``) are exposed one-to-one; ``Model`` bundles a loaded model with its workspace.

Importing the package never falls back to anything: if ``libmctune.so`` has not been
built the import raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmctune.so")

MC_OK = 0
MC_E_INVAL, MC_E_NOMEM, MC_E_DEVICE, MC_E_TABLE_FULL = -1, -2, -3, -4
MC_E_BUFFER, MC_E_STATE, MC_E_OVERFLOW, MC_E_ADMIT, MC_E_NOTFOUND = -5, -6, -7, -8, -9
MC_E_INTERNAL, MC_E_ABORTED = -10, -11
MC_REUSE_NONE, MC_REUSE_RESUMED, MC_REUSE_ANSWERED = 0, 1, 2
NEVER_CUT = 0xFFFFFFFF
MC_KIND_REDUCTION, MC_KIND_MATMUL, MC_KIND_ABSTRACT, MC_KIND_MINIMUM = 0, 1, 2, 3
MC_ENGINE_SUPERSTEP, MC_ENGINE_LEVEL = 0, 1
MC_MAX_CU = 8
ROOT = 0xFFFFFFFF
NO_CLOCK = 0xFFFFFFFF

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2305_09130_amd/build.py "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class McDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("n_cu", ctypes.c_uint32),
                ("size", ctypes.c_uint32 * 3), ("lat_global", ctypes.c_uint32),
                ("lat_local", ctypes.c_uint32), ("lat_compute", ctypes.c_uint32),
                ("lat_barrier", ctypes.c_uint32), ("n_cfg", ctypes.c_uint32),
                ("params", _u32p), ("unit_speed", _u32p)]


class McOpts(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("log2_slots", ctypes.c_uint32), ("load_factor", ctypes.c_float),
                ("grid", ctypes.c_uint32), ("batch_items", ctypes.c_uint32),
                ("lane_items", ctypes.c_uint32), ("part_states", ctypes.c_uint32),
                ("test_hash_bits", ctypes.c_uint32)]


class McStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("states", "levels", "terminals", "edges", "dups", "probes", "launches",
                 "explore_ns", "total_ns", "clear_ns", "engine_ns", "supersteps",
                 "batches", "max_probe", "critical_ns", "critical_cfg", "parts",
                 "cas_fail")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class McModelInfo(ctypes.Structure):
    _fields_ = [("n_cu", ctypes.c_uint32), ("n_cfg", ctypes.c_uint32),
                ("key_words", ctypes.c_uint32), ("key_bits", ctypes.c_uint32),
                ("slots", ctypes.c_uint64), ("slot_bytes", ctypes.c_uint64),
                ("bound_states", ctypes.c_uint64), ("max_depth", ctypes.c_uint64)]


class McBatchOpts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("load_factor", ctypes.c_float), ("chunk", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("lane_items", ctypes.c_uint32),
                ("part_states", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 1)]

    def as_dict(self) -> dict:
        return {"block": int(self.block), "grid": int(self.grid),
                "load_factor": float(self.load_factor), "chunk": int(self.chunk),
                "use_graph": int(self.use_graph), "lane_items": int(self.lane_items),
                "part_states": int(self.part_states)}


class McEngineOpts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_uint32), ("max_cfg", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("slice", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("load_factor", ctypes.c_float), ("lane_items", ctypes.c_uint32),
                ("part_states", ctypes.c_uint32), ("no_reuse", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class McSwarmOpts(ctypes.Structure):
    _fields_ = [("members", ctypes.c_uint32), ("bits_log2", ctypes.c_uint32),
                ("budget", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("prune", ctypes.c_uint32), ("T", ctypes.c_uint32)]


class McSwarmResult(ctypes.Structure):
    _fields_ = [("best_clock", ctypes.c_uint32), ("best_cfg", ctypes.c_uint32),
                ("best_member", ctypes.c_uint32), ("first_clock", ctypes.c_uint32),
                ("first_cfg", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("trails", ctypes.c_uint64), ("walks", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("first_trail_ns", ctypes.c_uint64),
                ("swarm_ns", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "pad"}


class McSwarmMember(ctypes.Structure):
    _fields_ = [("walks", ctypes.c_uint64), ("trails", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("best_walk_start", ctypes.c_uint64),
                ("first_step", ctypes.c_uint64), ("start_ticks", ctypes.c_uint64),
                ("first_ticks", ctypes.c_uint64), ("best_clock", ctypes.c_uint32),
                ("best_cfg", ctypes.c_uint32), ("first_clock", ctypes.c_uint32),
                ("first_cfg", ctypes.c_uint32), ("pad", ctypes.c_uint32 * 2)]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "pad"}


class McQueryResult(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("T", ctypes.c_uint32), ("status", ctypes.c_int),
                ("done", ctypes.c_int), ("violated", ctypes.c_int), ("t_min", ctypes.c_uint32),
                ("n_argmin", ctypes.c_uint32), ("argmin_first", ctypes.c_uint32),
                ("states", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("steps", ctypes.c_uint32),
                ("reuse", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "pad"}


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_SIGS = {
    "mc_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "mc_describe": ([_P(McDesc), _u64p, _u64p, _u32p], ctypes.c_int),
    "mc_config_ends": ([_P(McDesc), ctypes.c_uint32, _u32p, _u32p, _u32p, _u32p,
                        ctypes.c_uint64], ctypes.c_int),
    "mc_workspace_bytes": ([_P(McDesc), _P(McOpts), _P(ctypes.c_size_t)], ctypes.c_int),
    "mc_model_load": ([_P(McDesc), _P(McOpts), _vp, ctypes.c_size_t, _vp, _P(_vp)], ctypes.c_int),
    "mc_model_free": ([_vp], ctypes.c_int),
    "mc_model_reload": ([_vp, _P(McDesc)], ctypes.c_int),
    "mc_model_info_get": ([_vp, _P(McModelInfo)], ctypes.c_int),
    "mc_set_engine": ([_vp, ctypes.c_uint32], ctypes.c_int),
    "mc_abort": ([_vp], ctypes.c_int),
    "mc_min_time_static": ([_P(McDesc), _P(McOpts), _vp, _u32p, _u32p, ctypes.c_size_t,
                            _P(ctypes.c_size_t), _P(McStats)], ctypes.c_int),
    "mc_min_time": ([_vp, _u32p, _u32p, ctypes.c_size_t, _P(ctypes.c_size_t), _P(McStats)],
                    ctypes.c_int),
    "mc_check": ([_vp, ctypes.c_uint32, _P(ctypes.c_int), _P(McStats)], ctypes.c_int),
    "mc_min_time_bb": ([_vp, ctypes.c_uint32, _u32p, _u32p, ctypes.c_size_t,
                        _P(ctypes.c_size_t), _P(McStats)], ctypes.c_int),
    "mc_terminal_clocks": ([_vp, _u32p, ctypes.c_size_t], ctypes.c_int),
    "mc_trace": ([_vp, _u32p, ctypes.c_size_t, _P(ctypes.c_size_t)], ctypes.c_int),
    "mc_simulate": ([_vp, ctypes.c_uint64, _u32p, _u32p], ctypes.c_int),
    "mc_tune_bisect": ([_vp, ctypes.c_uint64, _u32p, _u32p, _P(McStats)], ctypes.c_int),
    "mc_config": ([_vp, ctypes.c_uint32, _u32p], ctypes.c_int),
    "mc_batch_workspace_bytes": ([_P(McDesc), ctypes.c_uint32, _P(McBatchOpts),
                                  _P(ctypes.c_size_t)], ctypes.c_int),
    "mc_batch_create": ([_P(McDesc), ctypes.c_uint32, _P(McBatchOpts), _vp, ctypes.c_size_t,
                         _vp, _P(_vp)], ctypes.c_int),
    "mc_batch_min_time": ([_vp, _u32p, _u64p, _P(McStats)], ctypes.c_int),
    "mc_batch_terminal_clocks": ([_vp, ctypes.c_uint32, _u32p, ctypes.c_size_t], ctypes.c_int),
    "mc_batch_free": ([_vp], ctypes.c_int),
    "mc_batch_autotune": ([_P(McDesc), ctypes.c_uint32, _vp, ctypes.c_size_t, _vp,
                           _P(McBatchOpts), _P(ctypes.c_float)], ctypes.c_int),
    "mc_engine_bytes": ([_P(McEngineOpts), ctypes.c_size_t, _P(ctypes.c_size_t)], ctypes.c_int),
    "mc_engine_create": ([_P(McEngineOpts), _vp, ctypes.c_size_t, _vp, _P(_vp)], ctypes.c_int),
    "mc_engine_submit": ([_vp, _P(McDesc), ctypes.c_uint32, ctypes.c_uint32, _u64p],
                         ctypes.c_int),
    "mc_engine_step": ([_vp, _u32p, _u32p], ctypes.c_int),
    "mc_engine_poll": ([_vp, ctypes.c_uint64, _P(McQueryResult)], ctypes.c_int),
    "mc_engine_argmin": ([_vp, ctypes.c_uint64, _u32p, ctypes.c_size_t, _P(ctypes.c_size_t)],
                         ctypes.c_int),
    "mc_engine_trace": ([_vp, ctypes.c_uint64, _u32p, ctypes.c_size_t, _P(ctypes.c_size_t)],
                        ctypes.c_int),
    "mc_engine_release": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "mc_engine_destroy": ([_vp], ctypes.c_int),
    "mc_swarm": ([_vp, _P(McSwarmOpts), _P(McSwarmResult)], ctypes.c_int),
    "mc_swarm_members": ([_vp, _P(McSwarmMember), ctypes.c_size_t], ctypes.c_int),
    "mc_swarm_tune": ([_vp, _P(McSwarmOpts), _u32p, _u32p, _P(McSwarmResult)], ctypes.c_int),
    "mc_swarm_trace": ([_vp, _u32p, ctypes.c_size_t, _P(ctypes.c_size_t)], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class McError(RuntimeError):
    def __init__(self, where: str, code: int):
        super().__init__(f"{where}: {mc_strerror(code)} ({code})")
        self.code = code


def mc_strerror(code: int) -> str:
    return _lib.mc_strerror(code).decode()


def _check(where: str, rc: int) -> None:
    if rc != MC_OK:
        raise McError(where, rc)


def make_desc(model: dict) -> tuple[McDesc, tuple]:
    """McDesc of a model dict (see workloads); returns the arrays to keep alive."""
    params = np.ascontiguousarray(np.asarray(model["params"], dtype=np.uint32).reshape(-1, 4))
    d = McDesc()
    kind = model["kind"]
    if kind == "reduction":
        d.kind = MC_KIND_REDUCTION
        d.size[0], d.size[1], d.size[2] = model["G"], 0, 0
    elif kind == "matmul":
        d.kind = MC_KIND_MATMUL
        d.size[0], d.size[1], d.size[2] = model["M"], model["N"], model["K"]
    elif kind in ("abstract", "minimum"):
        d.kind = MC_KIND_ABSTRACT if kind == "abstract" else MC_KIND_MINIMUM
        d.size[0], d.size[1], d.size[2] = model["S"], model["NP"], 0
    else:
        raise ValueError(f"unknown model kind {kind!r}")
    d.n_cu = model["m"]
    d.lat_global, d.lat_local = model["Lg"], model["Ll"]
    d.lat_compute, d.lat_barrier = model.get("Lc", 1), model.get("Lb", 0)
    d.n_cfg = params.shape[0]
    d.params = params.ctypes.data_as(_u32p)
    speed = None
    if model.get("speed") is not None:
        speed = np.ascontiguousarray(np.asarray(model["speed"], dtype=np.uint32))
        d.unit_speed = speed.ctypes.data_as(_u32p)
    return d, (params, speed)


def make_opts(engine: int = MC_ENGINE_SUPERSTEP, block: int = 0, log2_slots: int = 0,
              load_factor: float = 0.0, grid: int = 0, batch_items: int = 0,
              lane_items: int = 0, part_states: int = 0, test_hash_bits: int = 0) -> McOpts:
    o = McOpts()
    o.engine, o.block, o.log2_slots, o.load_factor, o.grid = engine, block, log2_slots, \
        load_factor, grid
    o.batch_items, o.lane_items, o.part_states = batch_items, lane_items, part_states
    o.test_hash_bits = test_hash_bits
    return o


def mc_describe(model: dict) -> dict:
    d, keep = make_desc(model)
    s, dep, w = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
    _check("mc_describe", _lib.mc_describe(ctypes.byref(d), ctypes.byref(s), ctypes.byref(dep),
                                           ctypes.byref(w)))
    return {"states": s.value, "max_depth": dep.value, "key_words": w.value}


def mc_config_ends(model: dict, cfg: int) -> dict:
    """Workgroups n, duration d and operation end times E of one configuration, as the
    library derives them (host only)."""
    d, keep = make_desc(model)
    n, b, dur = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = _lib.mc_config_ends(ctypes.byref(d), cfg, ctypes.byref(n), ctypes.byref(b),
                             ctypes.byref(dur), None, 0)
    if rc not in (MC_OK, MC_E_BUFFER):
        _check("mc_config_ends", rc)
    ends = np.zeros(max(1, b.value), dtype=np.uint32)
    _check("mc_config_ends", _lib.mc_config_ends(ctypes.byref(d), cfg, ctypes.byref(n),
                                                 ctypes.byref(b), ctypes.byref(dur),
                                                 ends.ctypes.data_as(_u32p), b.value))
    return {"n": n.value, "b": b.value, "d": dur.value, "E": ends[:b.value].tolist()}


def state_count(model: dict) -> int | None:
    """Reachable-state count of a model, or None if the library cannot represent it
    (invalid sizes, clocks beyond 32 bits, keys beyond 256 bits)."""
    try:
        return mc_describe(model)["states"]
    except McError:
        return None


MC_STATIC_SCRATCH_BYTES = 128 << 20


def mc_min_time_static(model: dict, opts: McOpts | None = None, stream=None) -> tuple:
    """min_time of a model in the library's static device scratch (no allocation):
    (T_min, argmin list, stats dict).  stream: a torch stream (default: the current
    stream of the current device)."""
    import torch
    d, keep = make_desc(model)
    if stream is None:
        stream = torch.cuda.current_stream()
    t = ctypes.c_uint32()
    n = ctypes.c_size_t()
    st = McStats()
    cap = len(model["params"])
    arg = (ctypes.c_uint32 * cap)()
    _check("mc_min_time_static",
           _lib.mc_min_time_static(ctypes.byref(d), ctypes.byref(opts) if opts else None,
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(t), arg,
                                   cap, ctypes.byref(n), ctypes.byref(st)))
    return t.value, [int(arg[i]) for i in range(n.value)], st.as_dict()


def mc_workspace_bytes(model: dict, opts: McOpts | None = None) -> int:
    d, keep = make_desc(model)
    n = ctypes.c_size_t()
    _check("mc_workspace_bytes",
           _lib.mc_workspace_bytes(ctypes.byref(d), ctypes.byref(opts) if opts else None,
                                   ctypes.byref(n)))
    return n.value


class Model:
    """A model loaded on the GPU with its own workspace (a torch uint8 tensor)."""

    def __init__(self, model: dict, engine: int = MC_ENGINE_SUPERSTEP, block: int = 0,
                 log2_slots: int = 0, load_factor: float = 0.0, grid: int = 0,
                 device: str = "cuda:0", stream=None, workspace=None, batch_items: int = 0,
                 lane_items: int = 0, part_states: int = 0, test_hash_bits: int = 0):
        import torch
        self.model = model
        self.m = model["m"]
        self.n_cfg = len(model["params"])
        self._desc, self._params = make_desc(model)
        self._opts = make_opts(engine, block, log2_slots, load_factor, grid, batch_items,
                               lane_items, part_states, test_hash_bits)
        self.device = torch.device(device)
        if workspace is None:
            workspace = torch.empty(mc_workspace_bytes(model, self._opts), dtype=torch.uint8,
                                    device=self.device)
        elif workspace.dtype != torch.uint8:
            raise ValueError("the workspace must be a uint8 tensor")
        self.workspace = workspace
        nbytes = workspace.numel()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        # a given workspace is sized by the load itself (MC_E_NOMEM when too small)
        rc = _lib.mc_model_load(ctypes.byref(self._desc), ctypes.byref(self._opts),
                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc == MC_E_NOMEM:
            need = mc_workspace_bytes(model, self._opts)
            if nbytes < need:
                raise ValueError(f"workspace needs {need} bytes of uint8, has {nbytes}")
        _check("mc_model_load", rc)
        self._h = h
        self.last_stats: dict = {}

    def mc_model_reload(self, model: dict) -> None:
        """The next model on this handle, its workspace and its stream (the options given
        at construction)."""
        desc, params = make_desc(model)
        _check("mc_model_reload", _lib.mc_model_reload(self._h, ctypes.byref(desc)))
        self.model = model
        self.m = model["m"]
        self.n_cfg = len(model["params"])
        self._desc, self._params = desc, params
        self.last_stats = {}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.mc_model_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def mc_model_info_get(self) -> dict:
        info = McModelInfo()
        _check("mc_model_info_get", _lib.mc_model_info_get(self._h, ctypes.byref(info)))
        return {n: int(getattr(info, n)) for n, _ in info._fields_}

    def mc_set_engine(self, engine: int) -> None:
        _check("mc_set_engine", _lib.mc_set_engine(self._h, engine))

    def mc_abort(self) -> None:
        """Stop request for the running (or the next) query of this model; safe to call
        from another thread while a query runs."""
        _check("mc_abort", _lib.mc_abort(self._h))

    def mc_min_time(self) -> tuple[int, list[int]]:
        t = ctypes.c_uint32()
        n = ctypes.c_size_t()
        st = McStats()
        arg = np.zeros(self.n_cfg, dtype=np.uint32)
        _check("mc_min_time", _lib.mc_min_time(self._h, ctypes.byref(t),
                                               arg.ctypes.data_as(_u32p), arg.shape[0],
                                               ctypes.byref(n), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return t.value, [int(v) for v in arg[:n.value]]

    def mc_min_time_bb(self, T_init: int = 0) -> tuple[int, list[int]]:
        """Branch-and-bound min_time (exact T_min and argmin; last_stats counts the states
        the pruned search claimed).  T_init: initial incumbent, 0 = none."""
        t = ctypes.c_uint32()
        n = ctypes.c_size_t()
        st = McStats()
        arg = np.zeros(self.n_cfg, dtype=np.uint32)
        _check("mc_min_time_bb", _lib.mc_min_time_bb(self._h, int(T_init), ctypes.byref(t),
                                                     arg.ctypes.data_as(_u32p), arg.shape[0],
                                                     ctypes.byref(n), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return t.value, [int(v) for v in arg[:n.value]]

    def mc_check(self, T: int) -> bool:
        v = ctypes.c_int()
        st = McStats()
        _check("mc_check", _lib.mc_check(self._h, int(T), ctypes.byref(v), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return bool(v.value)

    def mc_terminal_clocks(self) -> list[int | None]:
        tc = np.zeros(self.n_cfg, dtype=np.uint32)
        _check("mc_terminal_clocks",
               _lib.mc_terminal_clocks(self._h, tc.ctypes.data_as(_u32p), tc.shape[0]))
        return [None if int(v) == NO_CLOCK else int(v) for v in tc]

    def mc_trace(self) -> np.ndarray:
        n = ctypes.c_size_t()
        _check("mc_trace", _lib.mc_trace(self._h, None, 0, ctypes.byref(n)))
        rows = np.zeros((n.value, 3 + self.m), dtype=np.uint32)
        _check("mc_trace", _lib.mc_trace(self._h, rows.ctypes.data_as(_u32p), n.value,
                                         ctypes.byref(n)))
        return rows

    def mc_simulate(self, seed: int) -> tuple[int, int]:
        t, c = ctypes.c_uint32(), ctypes.c_uint32()
        _check("mc_simulate", _lib.mc_simulate(self._h, seed, ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    def mc_tune_bisect(self, seed: int) -> tuple[int, int]:
        t, n = ctypes.c_uint32(), ctypes.c_uint32()
        st = McStats()
        _check("mc_tune_bisect", _lib.mc_tune_bisect(self._h, seed, ctypes.byref(t),
                                                     ctypes.byref(n), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return t.value, n.value

    def _swarm_opts(self, members, bits_log2, budget, seed, T):
        o = McSwarmOpts()
        o.members, o.bits_log2, o.budget, o.seed = members, bits_log2, budget, seed
        o.prune, o.T = (0, 0) if T is None else (1, T)
        return o

    def mc_swarm(self, members: int, bits_log2: int, budget: int, seed: int,
                 T: int | None = None) -> dict:
        """One swarm against G(!FIN) (T None) or the over-time property with threshold
        T; the aggregate result (see mc_swarm_result)."""
        r = McSwarmResult()
        _check("mc_swarm", _lib.mc_swarm(self._h, ctypes.byref(
            self._swarm_opts(members, bits_log2, budget, seed, T)), ctypes.byref(r)))
        return r.as_dict()

    def mc_swarm_members(self, members: int) -> list[dict]:
        out = (McSwarmMember * members)()
        _check("mc_swarm_members", _lib.mc_swarm_members(self._h, out, members))
        return [x.as_dict() for x in out]

    def mc_swarm_tune(self, members: int, bits_log2: int, budget: int,
                      seed: int) -> tuple[int, int, dict]:
        """The swarm search of Sec. 5: (T found, swarms run, the result of the last swarm
        that found a trail)."""
        t, n = ctypes.c_uint32(), ctypes.c_uint32()
        r = McSwarmResult()
        _check("mc_swarm_tune", _lib.mc_swarm_tune(
            self._h, ctypes.byref(self._swarm_opts(members, bits_log2, budget, seed, None)),
            ctypes.byref(t), ctypes.byref(n), ctypes.byref(r)))
        return t.value, n.value, r.as_dict()

    def mc_swarm_trace(self) -> np.ndarray:
        n = ctypes.c_size_t()
        _check("mc_swarm_trace", _lib.mc_swarm_trace(self._h, None, 0, ctypes.byref(n)))
        rows = np.zeros((n.value, 3 + self.m), dtype=np.uint32)
        _check("mc_swarm_trace", _lib.mc_swarm_trace(self._h, rows.ctypes.data_as(_u32p),
                                                     n.value, ctypes.byref(n)))
        return rows

    def mc_config(self, cfg: int) -> list[int]:
        p = np.zeros(4, dtype=np.uint32)
        _check("mc_config", _lib.mc_config(self._h, cfg, p.ctypes.data_as(_u32p)))
        return [int(v) for v in p]


def _desc_array(models: list[dict]):
    arr = (McDesc * len(models))()
    keep = []
    for i, m in enumerate(models):
        d, p = make_desc(m)
        arr[i] = d
        keep.append(p)
    return arr, keep


def make_batch_opts(block: int = 0, grid: int = 0, load_factor: float = 0.0, chunk: int = 0,
                    use_graph: bool = False, lane_items: int = 0,
                    part_states: int = 0) -> McBatchOpts:
    o = McBatchOpts()
    o.block, o.grid, o.load_factor, o.chunk = block, grid, load_factor, chunk
    o.use_graph = 1 if use_graph else 0
    o.lane_items, o.part_states = lane_items, part_states
    return o


def mc_batch_workspace_bytes(models: list[dict], opts: McBatchOpts | None = None) -> int:
    arr, keep = _desc_array(models)
    n = ctypes.c_size_t()
    _check("mc_batch_workspace_bytes",
           _lib.mc_batch_workspace_bytes(arr, len(models), ctypes.byref(opts) if opts else None,
                                         ctypes.byref(n)))
    return n.value


def mc_batch_autotune(models: list[dict], workspace, stream=None) -> tuple[McBatchOpts, float]:
    """Fastest batch options for these models on this GPU (cached per process)."""
    import torch
    arr, keep = _desc_array(models)
    st = stream if stream is not None else torch.cuda.current_stream(workspace.device)
    best = McBatchOpts()
    ms = ctypes.c_float()
    _check("mc_batch_autotune",
           _lib.mc_batch_autotune(arr, len(models), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), ctypes.c_void_p(st.cuda_stream),
                                  ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value


class Batch:
    """Many models explored together in one persistent launch (mc_batch_*)."""

    def __init__(self, models: list[dict], opts: McBatchOpts | None = None,
                 device: str = "cuda:0", stream=None, workspace=None):
        import torch
        self.models = models
        self.n = len(models)
        self._arr, self._keep = _desc_array(models)
        self._opts = opts if opts is not None else McBatchOpts()
        nbytes = mc_batch_workspace_bytes(models, self._opts)
        self.device = torch.device(device)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif workspace.numel() < nbytes:
            raise ValueError(f"batch workspace needs {nbytes} bytes")
        self.workspace = workspace
        if stream is None:
            # a graph needs a capturable stream of its own (default priority)
            stream = (torch.cuda.Stream(self.device) if self._opts.use_graph
                      else torch.cuda.current_stream(self.device))
        self.stream = stream
        if self._opts.use_graph:
            # the workspace was allocated on the current stream: order it before ours
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = ctypes.c_void_p()
        _check("mc_batch_create",
               _lib.mc_batch_create(self._arr, self.n, ctypes.byref(self._opts),
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.last_stats: dict = {}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.mc_batch_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def mc_batch_min_time(self) -> tuple[list[int], list[int]]:
        t = np.zeros(self.n, dtype=np.uint32)
        st_ = np.zeros(self.n, dtype=np.uint64)
        st = McStats()
        _check("mc_batch_min_time",
               _lib.mc_batch_min_time(self._h, t.ctypes.data_as(_u32p),
                                      st_.ctypes.data_as(_u64p), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return [int(v) for v in t], [int(v) for v in st_]

    def mc_batch_terminal_clocks(self, i: int) -> list[int | None]:
        nc = len(self.models[i]["params"])
        tc = np.zeros(nc, dtype=np.uint32)
        _check("mc_batch_terminal_clocks",
               _lib.mc_batch_terminal_clocks(self._h, i, tc.ctypes.data_as(_u32p), nc))
        return [None if int(v) == NO_CLOCK else int(v) for v in tc]


MC_QUERY_MIN_TIME, MC_QUERY_CHECK = 0, 1


class Engine:
    """Continuous-batching query server (mc_engine_*) on its own device buffer."""

    def __init__(self, arena_bytes: int, max_active: int = 64, max_cfg: int = 512,
                 block: int = 512, slice: int = 16, chunk: int = 0, grid: int = 0,
                 load_factor: float = 0.5, device: str = "cuda:0", stream=None,
                 lane_items: int = 0, part_states: int = 0, no_reuse: bool = False):
        import torch
        o = McEngineOpts()
        o.max_active, o.max_cfg, o.block, o.slice = max_active, max_cfg, block, slice
        o.chunk, o.grid, o.load_factor = chunk, grid, load_factor
        o.lane_items, o.part_states = lane_items, part_states
        o.no_reuse = 1 if no_reuse else 0
        self._o = o
        n = ctypes.c_size_t()
        _check("mc_engine_bytes", _lib.mc_engine_bytes(ctypes.byref(o), arena_bytes,
                                                       ctypes.byref(n)))
        self.device = torch.device(device)
        self.buffer = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check("mc_engine_create",
               _lib.mc_engine_create(ctypes.byref(o), ctypes.c_void_p(self.buffer.data_ptr()),
                                     n.value, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.mc_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def mc_engine_submit(self, model: dict, kind: int, T: int = 0) -> int:
        d, p = make_desc(model)
        t = ctypes.c_uint64()
        _check("mc_engine_submit", _lib.mc_engine_submit(self._h, ctypes.byref(d), kind, int(T),
                                                         ctypes.byref(t)))
        return t.value

    def mc_engine_step(self) -> tuple[int, int]:
        a, w = ctypes.c_uint32(), ctypes.c_uint32()
        _check("mc_engine_step", _lib.mc_engine_step(self._h, ctypes.byref(a), ctypes.byref(w)))
        return a.value, w.value

    def mc_engine_poll(self, ticket: int) -> dict | None:
        r = McQueryResult()
        rc = _lib.mc_engine_poll(self._h, ticket, ctypes.byref(r))
        if rc == MC_E_STATE:
            return None
        _check("mc_engine_poll", rc)
        return r.as_dict()

    def mc_engine_argmin(self, ticket: int) -> list[int]:
        n = ctypes.c_size_t()
        _check("mc_engine_argmin", _lib.mc_engine_argmin(self._h, ticket, None, 0,
                                                         ctypes.byref(n)))
        out = (ctypes.c_uint32 * max(1, n.value))()
        _check("mc_engine_argmin", _lib.mc_engine_argmin(self._h, ticket, out, n.value,
                                                         ctypes.byref(n)))
        return [int(out[i]) for i in range(n.value)]

    def mc_engine_trace(self, ticket: int, m: int) -> np.ndarray:
        """Counterexample rows (cfg, clock, pending, rem...) root first, as mc_trace;
        m = the model's unit count."""
        n = ctypes.c_size_t()
        _check("mc_engine_trace", _lib.mc_engine_trace(self._h, ticket, None, 0,
                                                       ctypes.byref(n)))
        rows = np.zeros((max(1, n.value), 3 + m), dtype=np.uint32)
        _check("mc_engine_trace", _lib.mc_engine_trace(self._h, ticket,
                                                       rows.ctypes.data_as(_u32p), n.value,
                                                       ctypes.byref(n)))
        return rows[:n.value]

    def mc_engine_release(self, ticket: int) -> None:
        _check("mc_engine_release", _lib.mc_engine_release(self._h, ticket))

    def drain(self, max_steps: int = 1 << 20) -> None:
        for _ in range(max_steps):
            a, w = self.mc_engine_step()
            if a == 0 and w == 0:
                return
        raise RuntimeError("engine did not drain")


def exported_symbols() -> list[str]:
    """Names declared in include/mctune.h (the ABI test checks they are exported)."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "mctune.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(mc_\w+)\s*\(", text, re.M)))
