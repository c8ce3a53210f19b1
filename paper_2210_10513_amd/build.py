"""Build libpns.so (HIP kernels + C-ABI runtime) for gfx950 in-tree.

    python -m paper_2210_10513_amd.build

Compiles every source with hipcc for gfx950 into ``paper_2210_10513_amd/lib``.
Packed FP32 instructions are disabled on every HIP compile line.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libpns.so")
ARCH = os.environ.get("PNS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["pns_step_i16.hip", "pns_step_i32.hip", "pns_step_i64.hip", "pns_step_f32.hip", "pns_wave_i16.hip",
           "pns_wave_i32.hip", "pns_kernels.hip", "pns_moments.hip", "pns_cont.hip", "pns_runtime.cpp"]

# Per-source additions: the moment kernel adds FP64 partial sums with the
# hardware atomic add (device memory only); the window kernels keep the
# constants of their rare paths where they are used instead of in registers
# across the step loop (machine loop-invariant code motion off).
EXTRA_FLAGS = {"pns_moments.hip": ["-munsafe-fp-atomics"],
               "pns_wave_i16.hip": ["-mllvm", "-disable-machine-licm"],
               "pns_wave_i32.hip": ["-mllvm", "-disable-machine-licm"]}

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(LIBDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
