"""Builds libshmi.so (the HIP kernels and the C ABI) in-tree with hipcc for gfx950.

    python -m paper_2510_05282_amd.build        # or build() from Python

Every HIP source is compiled with packed-FP32 instruction selection disabled,
then linked into one shared library next to this file.  The store-pattern
probes that bench.py times beside the forward kernel go into a second library,
libshprobe.so, which nothing else loads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libshmi.so")
SOURCES = ["sh_api.hip", "sh_eval.hip", "sh_grad.hip", "sh_proj.hip", "sh_rec.hip", "sh_serve.hip",
           "sh_server.cpp", "sh_server_api.cpp"]
PROBE_SOURCES = ["sh_probe.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def compile_flags() -> list[str]:
    # -ffp-contract=on: multiply-adds are fused only within one source expression,
    # so a value does not depend on whether its point was evaluated alone or as a
    # lane of a vector (the default lets the back end fuse across statements,
    # differently in scalar and vector code)
    return ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-ffp-contract=on",
            "-Wno-unused-parameter",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, obj: str, extra: list[str]) -> None:
    cmd = [hipcc(), *compile_flags(), *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature and says so; keep other warnings
    for ln in (r.stdout + r.stderr).splitlines():
        if ln.strip() and "packed-fp32-ops" not in ln and "not a recognized feature" not in ln:
            print(ln, file=sys.stderr)


def _link(objs: list[str], lib: str) -> None:
    tmp = lib + ".tmp"
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(out_dir: str | None = None, extra: list[str] | None = None) -> str:
    """Compile every source, link libshmi.so and libshprobe.so; returns libshmi's path."""
    extra = list(extra or [])
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    objs = {s: os.path.join(bdir, os.path.splitext(s)[0] + ".o") for s in srcs}
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        futs = [ex.submit(_compile, os.path.join(CSRC, s), objs[s], extra) for s in srcs]
        for f in futs:
            f.result()
    lib = os.path.join(out_dir or HERE, "libshmi.so")
    _link([objs[s] for s in SOURCES], lib)
    _link([objs[s] for s in PROBE_SOURCES], os.path.join(out_dir or HERE, "libshprobe.so"))
    return lib


if __name__ == "__main__":
    print(build())
