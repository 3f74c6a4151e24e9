"""Python binding of libmcpeak.so, the random-access peak probes (include/mcpeak.h).

Argument marshalling only: the probes are HIP kernels.  ``measure`` times them with
events on the stream they are launched on and returns the rates that bound the
explorer's visited-set traffic: random 64-bit CAS per second and random 64-byte line
reads per second on a buffer of the given size, plus a streaming copy for scale.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcpeak.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mcpeak.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2305_09130_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib.mcp_random_cas.argtypes = [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint64, _vp, _vp, _u64p]
_lib.mcp_random_cas.restype = ctypes.c_int
_lib.mcp_random_read.argtypes = [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint64, _vp, _vp, _u64p]
_lib.mcp_random_read.restype = ctypes.c_int


def exported_symbols() -> list[str]:
    """Names declared in include/mcpeak.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*int\s+(mcp_\w+)\s*\(", text, re.M)))


def _check(where: str, rc: int) -> None:
    if rc != 0:
        raise RuntimeError(f"{where} failed ({rc})")


def random_cas(buf, sink, grid: int, rounds: int, seed: int, stream) -> int:
    """Enqueues the random-CAS probe over the uint64 tensor ``buf`` (a power-of-two
    number of words); returns the number of CAS issued."""
    n = ctypes.c_uint64()
    _check("mcp_random_cas", _lib.mcp_random_cas(
        ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size() // 8, grid, rounds,
        seed, ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(stream.cuda_stream),
        ctypes.byref(n)))
    return n.value


def random_read(buf, sink, grid: int, rounds: int, seed: int, stream) -> int:
    """Enqueues the random 64-byte line read probe over ``buf`` (a power-of-two number
    of 64-byte lines); returns the number of lines read."""
    n = ctypes.c_uint64()
    _check("mcp_random_read", _lib.mcp_random_read(
        ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size() // 64, grid, rounds,
        seed, ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(stream.cuda_stream),
        ctypes.byref(n)))
    return n.value


def measure(buf_bytes: int = 8 << 30, grid: int = 16384, rounds: int = 16, reps: int = 5,
            device: str = "cuda:0") -> dict:
    """Random-access peaks on a buffer of ``buf_bytes`` (a power of two, far beyond the
    256 MB Infinity Cache): the median over ``reps`` launches of each probe, timed with
    events on the launch stream, and a device copy of half the buffer."""
    import torch
    assert buf_bytes & (buf_bytes - 1) == 0
    stream = torch.cuda.current_stream(device)
    buf = torch.full((buf_bytes // 8,), -1, dtype=torch.int64, device=device)
    sink = torch.zeros(1, dtype=torch.int64, device=device)

    def timed(fn):
        ts, n = [], 0
        fn()  # warm
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            n = fn()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return n, sorted(ts)[len(ts) // 2]

    seeds = iter(range(1, 1 + 4 * (reps + 1)))
    n_cas, t_cas = timed(lambda: random_cas(buf, sink, grid, rounds, next(seeds), stream))
    buf.fill_(-1)
    n_rd, t_rd = timed(lambda: random_read(buf, sink, grid, rounds, next(seeds), stream))
    half = buf_bytes // 16
    src, dst = buf[:half], buf[half:2 * half]

    def copy():
        dst.copy_(src)
        return half * 8

    n_cp, t_cp = timed(copy)
    out = {
        "buffer_bytes": buf_bytes,
        "random_cas_per_s": n_cas / t_cas,
        "random_cas_ms": 1e3 * t_cas, "random_cas_ops": n_cas,
        "random_read_lines_per_s": n_rd / t_rd,
        "random_read_GBps": 64.0 * n_rd / t_rd / 1e9,
        "random_read_ms": 1e3 * t_rd, "random_read_lines": n_rd,
        "copy_GBps": 2.0 * n_cp / t_cp / 1e9,
        "grid": grid, "rounds": rounds, "reps": reps,
    }
    del buf, sink
    torch.cuda.empty_cache()
    return out
