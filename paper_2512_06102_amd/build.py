"""Build the HIP library libfiresim.so (gfx950) in-tree with hipcc.

fp32 arithmetic of the stochastic step is defined bit for bit, so the device
code is compiled without FMA contraction and with fp32 denormals kept; packed
fp32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfiresim.so")
SOURCES = ["capi.cpp", "stoch.hip", "relaxed.hip", "rl.hip", "resident.hip", "groups.hip", "probe.hip"]
HEADERS = ["devmath.hpp", "internal.hpp", "stepcell.hpp", "framed.hpp", "relaxed.hpp", "resident.hpp", "rl.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# roctx ranges around every C-ABI call
LINK_FLAGS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library; with force=False reuse a build newer than its sources.
    Each source compiles to its own object in parallel, then one link."""
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [
        os.path.join(HERE, "..", "include", "firesim.h")]
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(obj_dir, os.path.basename(src) + "." + tag + ".o") for src in sources()]
    cmds = [[hipcc(), *[f for f in HIPCC_FLAGS if f != "-shared"], "-x", "hip", "-c", src, "-o", obj]
            for src, obj in zip(sources(), objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c))
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp" + tag
    subprocess.check_call([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, *LINK_FLAGS])
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
