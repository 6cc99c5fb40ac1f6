"""Builds libmsgpm.so (HIP, gfx950) in the package directory with hipcc, and
libmsgpm_ceiling.so, the benchmark's gather-ceiling measurement kernel.

Every translation unit is compiled with contraction off (explicit fmaf where a
fused multiply-add is wanted) and without packed-FP32 instruction selection.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmsgpm.so")
SOURCES = ["host.hip", "init.hip", "patchmatch.hip", "planes.hip"]
CEILING_OUT = os.path.join(HERE, "libmsgpm_ceiling.so")
CEILING_SOURCE = "ceiling.hip"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, build_dir: str, verbose: bool) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def _link(objs, out: str, libs, verbose: bool) -> None:
    tmp = out + ".tmp"
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-L", os.path.join(rocm, "lib"), *libs,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, verbose), SOURCES + [CEILING_SOURCE]))
    _link(objs[:-1], OUT, ["-lrocprofiler-sdk-roctx"], verbose)
    _link(objs[-1:], CEILING_OUT, [], verbose)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
