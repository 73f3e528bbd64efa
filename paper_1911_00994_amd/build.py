"""Build of the HIP library (gfx950) in-tree: paper_1911_00994_amd/libgpmg.so.

Every .hip source under csrc/ is compiled to an object with hipcc and linked into one shared library.  The
geometry file is compiled with FMA contraction off (branch decisions of the boundary-point bisection), and so is the
level-set file (its arithmetic then matches the plain C oracle's operation for operation).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgpmg.so")
ARCH = os.environ.get("GPMG_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]
PER_FILE = {"geom.hip": ["-ffp-contract=off"], "levelset.hip": ["-ffp-contract=off"], "mg3d.hip": ["-ffp-contract=off"]}
SOURCES = ["geom.hip", "mg.hip", "cn.hip", "adjoint.hip", "levelset.hip", "mg3d.hip", "api.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link the library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    for s in srcs:
        obj = os.path.join(BUILD, s.replace(".hip", ".o"))
        cmd = [hipcc()] + COMMON + PER_FILE.get(s, []) + ["-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((s, out.decode(errors="replace")))
        elif verbose and out:
            print(out.decode(errors="replace"))
    if failed:
        raise RuntimeError("HIP build failed:\n" + "\n".join(f"--- {s}\n{o}" for s, o in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
