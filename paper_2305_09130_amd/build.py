"""Build step of the HIP libraries for gfx950: csrc/ into libmctune.so (the explorer)
and libmcpeak.so (the random-access peak probes used by the benchmark)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmctune.so")
PEAK_LIB = os.path.join(HERE, "libmcpeak.so")
SOURCES = ["mc_model.cpp", "mc_host_pool.cpp", "mc_kernels.hip", "mc_walks.hip", "mc_trace.hip",
           "mc_api.hip", "mc_batch.hip", "mc_engine.hip", "mc_static.hip"]
PEAK_SOURCES = ["mc_peak.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Wno-unused-command-line-argument"]
DEV = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# mc_kernels.hip is compiled once per part (MC_PART): the k_superstep instances of each
# key width in a part of their own, everything else in part 0
KERNEL_PARTS = (0, 1, 2, 4)


def _units(srcs: list[str]) -> list[tuple[str, int | None]]:
    out = []
    for s in srcs:
        if s == "mc_kernels.hip":
            out += [(s, p) for p in KERNEL_PARTS]
        else:
            out.append((s, None))
    return out


def _compile(unit: tuple[str, int | None], outdir: str, verbose: bool) -> str:
    src, part = unit
    path = os.path.join(CSRC, src)
    obj = os.path.join(outdir, src + ("" if part is None else f".part{part}") + ".o")
    extra = [] if part is None else [f"-DMC_PART={part}"]
    if src.endswith(".hip"):
        cmd = [HIPCC, *COMMON, *DEV, *extra, "-x", "hip", "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, *DEV, *extra, "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def _link(objs: list[str], lib: str, verbose: bool) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source (in parallel: the kernel file dominates) and links both
    libraries.  Returns the explorer library's path."""
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    units = _units(SOURCES)
    peak_units = _units(PEAK_SOURCES)
    jobs = jobs or min(len(units) + len(peak_units), max(1, (os.cpu_count() or 2) - 1), 8)
    # the heaviest units first, so that they start at once
    order = sorted(units + peak_units, key=lambda u: u[1] is None)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = dict(zip(order, ex.map(lambda u: _compile(u, outdir, verbose), order)))
    _link([objs[u] for u in units], LIB, verbose)
    _link([objs[u] for u in peak_units], PEAK_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
