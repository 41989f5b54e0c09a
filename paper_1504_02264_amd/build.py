"""Build the gfx950 HIP library ``libles.so`` in-tree with hipcc.

Every source is compiled to its own object in parallel (each translation
unit launches only its own kernels, so no relocatable device code is
needed), then the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libles.so")
SOURCES = ["kernels_step.hip", "kernels_sor.hip", "ensemble.hip", "les_api.hip", "lesnet.hip",
           "warm.hip", "twinned.hip", "noalloc.hip", "netdata.hip"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # no packed-fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, r.stdout + r.stderr


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
             os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = [(s, out) for s, (rc, out) in zip(SOURCES, results) if rc != 0]
    if failed:
        for s, out in failed:
            sys.stderr.write(f"---- {s}\n{out}")
        raise RuntimeError("hipcc failed building libles.so: " + ", ".join(s for s, _ in failed))
    rc, out = _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", LIB + ".tmp"],
                   verbose)
    if rc != 0:
        sys.stderr.write(out)
        raise RuntimeError("linking libles.so failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
