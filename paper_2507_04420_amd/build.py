"""Builds the gfx950 shared library libmm_hip.so in-tree with hipcc: every
source compiles to an object in _build/ (in parallel), then one link."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmm_hip.so")
SOURCES = [os.path.join(CSRC, f) for f in ("mm.hip", "batch.hip", "check.hip", "pairs.hip", "ems.hip",
                                           "relabel.hip", "hubs.hip", "order.hip", "probe.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("protocol.h", "sweep.h", "batch.h", "internal.h",
                                           "pieces.h", "whole.h")] + [
    os.path.join(ROOT, "include", "mm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
OBJDIR = os.path.join(ROOT, "_build")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off in all device code of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles every source into libmm_hip.so (always, when force is set)."""
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(OBJDIR, os.path.basename(src) + "." + tag + ".o") for src in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, zip(SOURCES, objs)))
    try:
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building %s" % LIB)
        tmp = LIB + ".tmp" + tag
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp],
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking %s" % LIB)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
