"""The paper's 2-D thrombosis example (section 4.1): a 240 x 60 um channel on a
uniform 128 x 32 mesh with a ~90 um adhesive, reactive patch centred on the bottom
wall, wall shear 1000 1/s, Crank-Nicolson 0.9 and a variable step at Courant 0.75
(Appendix D).  Reports over time the clot 'areas' used in the paper's quantitative
validation: the number of cells whose bound-platelet fraction theta_B exceeds 10%,
50% and 90% of P_max, next to the number of cells of the adhesion region
(k_adh H_adh > 0).

    python -m paper_2304_09180_amd.thrombus2d --seconds 5 --every 0.25 [--load A.npy] [--save B.npy]

Each report is one JSON line on stdout.  --save writes the context's state (a checkpoint)
at the end and --load starts from one, so a long run can span several processes.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def channel(shear: float = 1000.0, dt_max: float = 1e-4) -> dict:
    """Channel descriptor of the example: 0.24 x 0.06 mm, 128 x 32 cells, patch 0.09 mm."""
    import clot_inputs as ci
    return ci.channel(2, 128, 32, shear=shear, dt=dt_max, Lx=0.24, Ly=0.06, inj_frac=0.09 / 0.24)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=5.0, help="simulated time")
    ap.add_argument("--every", type=float, default=0.25, help="report interval (simulated s)")
    ap.add_argument("--shear", type=float, default=1000.0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--chunk", type=int, default=200, help="steps per library call")
    ap.add_argument("--load", default=None, help="start from this saved state (.npy)")
    ap.add_argument("--save", default=None, help="save the final state here (.npy)")
    args = ap.parse_args(argv)

    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    from . import clot

    d = channel(args.shear)
    prec = clot.FP32_MIXED if args.precision == "fp32" else clot.FP64
    s = clot.Solver([d], prec, clot.default_params(prec, ddt_psi=0.9, max_co=0.75))
    n = d["nx"] * d["ny"]
    s.init_state(0, np.zeros((15, n)), np.zeros((2, s.count(0, "E0"))))
    adh = (s.get(0, "HADH") > 0).reshape(d["ny"], d["nx"])
    n_adh = int(adh.sum())
    if args.load:
        s.load_state(np.load(args.load))
    t0 = s.stats(0)["t"]
    t_next = np.ceil(t0 / args.every - 1e-9) * args.every
    steps = int(s.stats(0)["steps"])
    wall0 = time.perf_counter()
    while True:
        st = s.stats(0)
        if st["t"] >= t_next - 1e-12 or st["t"] >= args.seconds:
            th = s.get(0, "THETAB")
            rec = {"t": round(st["t"], 6), "steps": steps, "dt": st["dt"], "adhesion_cells": n_adh,
                   "area_10": int((th > 0.1).sum()), "area_50": int((th > 0.5).sum()),
                   "area_90": int((th > 0.9).sum()), "theta_b_max": float(th.max()),
                   # mean theta_B over the adhesion region, wall layer and the layer above
                   "theta_b_adh_layers": [float(th.reshape(d["ny"], d["nx"])[j][adh[j]].mean())
                                          for j in range(2) if adh[j].any()],
                   "adp_max": float(s.get(0, "ADP").max()), "pma_max": float(s.get(0, "PMA").max()),
                   "e2_max": float(s.get(0, "E2").max()), "status": st["status"],
                   "wall_s": round(time.perf_counter() - wall0, 2)}
            print(json.dumps(rec), flush=True)
            t_next += args.every
        if st["t"] >= args.seconds:
            break
        s.step(args.chunk)
        steps += args.chunk
    if args.save:
        np.save(args.save, s.save_state())
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
