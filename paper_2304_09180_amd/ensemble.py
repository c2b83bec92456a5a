"""The batched ensemble of uneven 2-D channels in one context: every member steps in the
same launches, each with its own time step, solver scalars and convergence.

    python -m paper_2304_09180_amd.ensemble --members 64 --steps 20 [--graph] [--tile 256]

Members are the seeded synthetic ensemble of `clot_inputs.ensemble` (sizes 128x32,
256x64 and 512x128, shear log-uniform in [100, 2000] 1/s, injury 0.1-0.5 of the length).
Prints one JSON line: the step time after the warm-up steps, cell-timesteps per second
over all members, and the iteration counts of the first member of each size.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", type=int, default=256, choices=[256, 512, 1024])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--graph", action="store_true", help="replay recorded steps as HIP graphs")
    args = ap.parse_args(argv)

    import torch
    import clot_inputs as ci
    from . import clot

    descs = ci.ensemble(args.members)
    prec = clot.FP32_MIXED if args.precision == "fp32" else clot.FP64
    s = clot.Solver(descs, prec, clot.default_params(prec), tile=args.tile)
    for c, d in enumerate(descs):
        s.init_state(c, *ci.noise(d))
    if args.graph:
        s.set_graph_mode(True)
    for _ in range(max(args.warmup, 3) if args.graph else args.warmup):
        s.step(1)                  # graph mode: two calibrating steps, then the recording
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    cells = sum(ci.ncell(d) for d in descs)
    first = {}
    for c, d in enumerate(descs):
        first.setdefault(f"{d['nx']}x{d['ny']}", c)
    stats = {k: s.stats(c) for k, c in sorted(first.items())}
    status = sorted({s.stats(c)["status"] for c in range(len(descs))})
    s.close()
    print(json.dumps({"members": len(descs), "cells": cells, "steps": args.steps, "tile": args.tile,
                      "graph": args.graph, "ms_per_step": round(ms, 3),
                      "cell_timesteps_per_s": cells * 1e3 / ms, "status": status,
                      "solver": {k: {"it_mom": v["it_mom"], "it_p": v["it_p"][:3], "it_eta": v["it_eta"],
                                     "it_tr": v["it_tr"]} for k, v in stats.items()}}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
