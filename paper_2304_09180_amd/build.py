"""Builds the clotting-step library in-tree with hipcc for gfx950, once per tile size.

A tile is the group of cells one 256-thread block owns (its partial sums, its
channel); the tile size is fixed at compile time, so each candidate size is its own
library: libclot.so (256 cells, one per thread), libclot_t512.so and
libclot_t1024.so (two and four cells per thread).  The autotuner picks among them.
libclot_inh.so (256 cells) is the model with the inhibitor of section 3.4's
extensibility example (I + E2 -> E2i), built from the same sources with
CLOT_INHIBITOR defined.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", "clot_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # no packed-FP32 instructions anywhere in this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]
TILES = (256, 512, 1024)
LIBS = [(t, False) for t in TILES] + [(256, True)]     # (cells per tile, inhibitor model)


def lib_name(tile: int, inhibitor: bool = False) -> str:
    stem = "libclot_inh" if inhibitor else "libclot"
    return f"{stem}.so" if tile == 256 else f"{stem}_t{tile}.so"


def build(verbose: bool = False, libs=LIBS) -> list[str]:
    procs = []
    for tile, inh in libs:
        out = os.path.join(HERE, lib_name(tile, inh))
        cmd = [HIPCC, *FLAGS, f"-DCLOT_CPT={tile // 256}", *(["-DCLOT_INHIBITOR"] if inh else []),
               "-o", out + ".tmp", *SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for out, p in procs:
        log, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(log)
            failed.append(out)
        else:
            os.replace(out + ".tmp", out)
    if failed:
        raise RuntimeError("hipcc failed building " + ", ".join(os.path.basename(f) for f in failed))
    return [out for out, _ in procs]


if __name__ == "__main__":
    print(build(verbose=True))
