"""Host code under the sanitizers (CPU only): the oracle (oracle/mc_oracle.c) under
AddressSanitizer + UndefinedBehaviorSanitizer, and the library's host-side model code
(csrc/mc_model.cpp: validation, operation lists, layouts, sizes, the multithreaded walk of
units of unequal speed, partition plans, the key codec) under ASan + UBSan and under
ThreadSanitizer.  Each is built with gcc/g++ (host code only, no GPU code) together with a
driver in tests/sanitize/ that calls it on a spread of valid and invalid models; a report
or a failed expectation fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_09130_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")


def _build_and_run(cmd, exe, env=None):
    subprocess.check_call(cmd)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for word in ("ERROR: AddressSanitizer", "runtime error", "WARNING: ThreadSanitizer",
                 "FAILED"):
        assert word not in out, out[-4000:]
    return out


@pytest.fixture
def tmp():
    d = tempfile.mkdtemp(prefix="mcsan")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_oracle_asan_ubsan(tmp):
    exe = os.path.join(tmp, "oracle_asan")
    out = _build_and_run(["gcc", "-O1", "-g", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                          "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                          "-fno-sanitize-recover=all", "-w", "-o", exe,
                          os.path.join(SAN, "oracle_driver.c"), "-lm"], exe)
    assert "0 failures" in out


def test_host_model_asan_ubsan(tmp):
    exe = os.path.join(tmp, "host_asan")
    out = _build_and_run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                          "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                          "-I", CSRC, "-o", exe, os.path.join(SAN, "host_driver.cpp"),
                          os.path.join(CSRC, "mc_model.cpp"), "-pthread"], exe)
    assert "0 failures" in out


def test_host_model_tsan(tmp):
    exe = os.path.join(tmp, "host_tsan")
    out = _build_and_run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread",
                          "-I", CSRC, "-o", exe, os.path.join(SAN, "host_driver.cpp"),
                          os.path.join(CSRC, "mc_model.cpp"), "-pthread"], exe)
    assert "0 failures" in out
