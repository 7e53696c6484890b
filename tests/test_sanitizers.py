"""Host code under the sanitizers (no GPU).

- The projector server's scheduler and its C entry points (sh_server.cpp,
  sh_server_api.cpp) with the simulated executor, driven from several threads by
  tests/host/server_stress.cpp: once under ThreadSanitizer, once under
  AddressSanitizer + UndefinedBehaviorSanitizer.  They are built with the LLVM
  toolchain of the ROCm install: GCC 11's ThreadSanitizer does not intercept
  pthread_cond_clockwait (which libstdc++ uses for timed waits on the steady
  clock) and reports false races for it.  The driver also checks that the
  scheduler thread sleeps while long batches run.
- The C oracle (oracle/sh_oracle.c) under AddressSanitizer + UBSan with OpenMP,
  every entry point on inputs with its special cases (tests/host/oracle_san.c).

Each build must run to completion, print OK and produce no sanitizer report."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_05282_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
REPORTS = ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run(cmd_build, exe, env=None, timeout=240):
    b = subprocess.run(cmd_build, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    print(out)
    assert r.returncode == 0, out
    assert "OK" in r.stdout
    for rep in REPORTS:
        assert rep not in out, rep
    return out


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_under_sanitizer(tmp_path, san):
    if not os.path.exists(CLANG):
        pytest.skip("LLVM clang++ of the ROCm install not found")
    exe = str(tmp_path / "server_stress")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}",
           "-fno-sanitize-recover=undefined" if "undefined" in san else "-g",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host", "server_stress.cpp"), os.path.join(CSRC, "sh_server.cpp"),
           os.path.join(CSRC, "sh_server_api.cpp"), "-o", exe, "-lpthread"]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    out = _run(cmd, exe, env=env)
    assert "scheduler thread" in out


def test_oracle_under_sanitizer(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    cmd = [cc, "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "host", "oracle_san.c"), os.path.join(ROOT, "oracle", "sh_oracle.c"),
           "-o", exe, "-lm"]
    _run(cmd, exe, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
