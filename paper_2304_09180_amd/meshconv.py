"""Mesh convergence on the paper's rectangular test channel (supplement, "Mesh
convergence study"): a 120 x 30 um channel with a 45 um injury patch centred on the
bottom wall, wall shear 1000 1/s, uniform square cells of side h, Crank-Nicolson 0.9,
every mesh started from the species' initial values.  At one time the solution on each
coarser mesh is interpolated to the finest mesh's cell centres and its relative l2
error against the finest solution is taken for four quantities the paper plots: S1 and
E1 (fluid-phase biochemistry), P^{m,u} (mobile unactivated platelets) and E2 + E2^b
(total thrombin).  The convergence rate is the least-squares slope of log error
against log h.

The study's own step rule (Courant 0.75 on each mesh) puts the viscous diffusion number
nu dt / h^2 far above the range in which this solver's PISO step is stable on the fine
meshes, so every mesh here takes one common step small enough for the finest, and the
differences between meshes are spatial errors only.

    python -m paper_2304_09180_amd.meshconv --h 3 1.5 0.75 0.375 --dt 4e-6 --seconds 0.25

Progress goes to stderr; the result is one JSON line on stdout.  A long study can span
several processes: --max-steps stops after that many steps of this call and --save writes
the context's state (a checkpoint), which --load resumes; the result is printed by the
call that reaches the horizon.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

L_MM, H_MM, INJ_MM = 0.12, 0.03, 0.045
QUANTITIES = ("S1", "E1", "PMU", "E2+E2B")


def channel(h_um: float, dt: float) -> dict:
    """The test channel on a uniform mesh of side h_um micrometres."""
    import clot_inputs as ci
    h = h_um * 1e-3
    nx, ny = int(round(L_MM / h)), int(round(H_MM / h))
    return ci.channel(2, nx, ny, shear=1000.0, dt=dt, Lx=L_MM, Ly=H_MM, inj_frac=INJ_MM / L_MM)


def linear_resample(f: np.ndarray, nfine: int) -> np.ndarray:
    """Values of cell-centred f (n cells on [0, 1]) at the centres of nfine equal cells,
    by linear interpolation between centres and linear extrapolation beyond the first
    and last centre (exact for linear fields); along the last axis."""
    n = f.shape[-1]
    xc = (np.arange(n) + 0.5) / n
    xf = (np.arange(nfine) + 0.5) / nfine
    j = np.clip(np.searchsorted(xc, xf) - 1, 0, n - 2) if n > 1 else np.zeros(nfine, dtype=int)
    if n == 1:
        return np.repeat(f, nfine, axis=-1)
    w = (xf - xc[j]) / (xc[j + 1] - xc[j])
    return f[..., j] * (1.0 - w) + f[..., j + 1] * w


def to_fine(f: np.ndarray, shape: tuple) -> np.ndarray:
    """A (ny, nx) cell field interpolated to a finer (NY, NX) mesh of the same box."""
    g = linear_resample(f, shape[1])
    return linear_resample(g.T, shape[0]).T


def quantity(fields: dict, name: str) -> np.ndarray:
    if name == "E2+E2B":
        return fields["E2"] + fields["E2B"]
    return fields[name]


def errors_and_rates(hs, sols):
    """Relative l2 error of every mesh but the finest against the finest, and the
    least-squares slope of log error over log h, per quantity.  sols[i][name] is a
    (ny, nx) array on mesh i; the finest mesh is the last."""
    fine = sols[-1]
    out = {}
    for q in QUANTITIES:
        ref = quantity(fine, q)
        errs = []
        for sol in sols[:-1]:
            c = to_fine(quantity(sol, q), ref.shape)
            errs.append(float(np.linalg.norm(c - ref) / np.linalg.norm(ref)))
        rate = float(np.polyfit(np.log(hs[:-1]), np.log(errs), 1)[0]) if len(errs) >= 2 else None
        out[q] = {"errors": errs, "rate": rate}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=float, nargs="+", default=[3.0, 1.5, 0.75, 0.375], help="cell sizes, um, finest last")
    ap.add_argument("--dt", type=float, default=4e-6, help="the common time step, s")
    ap.add_argument("--seconds", type=float, default=0.25)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--chunk", type=int, default=2500, help="steps per library call")
    ap.add_argument("--max-steps", type=int, default=0, help="stop after this many steps of this call (0: none)")
    ap.add_argument("--load", default=None, help="resume from this saved state (.npy)")
    ap.add_argument("--save", default=None, help="save the state here (.npy) when this call stops")
    args = ap.parse_args(argv)

    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    from . import clot

    hs = sorted(args.h, reverse=True)
    descs = [channel(h, args.dt) for h in hs]
    prec = clot.FP32_MIXED if args.precision == "fp32" else clot.FP64
    s = clot.Solver(descs, prec, clot.default_params(prec, ddt_psi=0.9))
    for i, d in enumerate(descs):
        n = d["nx"] * d["ny"]
        s.init_state(i, np.zeros((15, n)), np.zeros((2, s.count(i, "E0"))))
    nsteps = int(round(args.seconds / args.dt))
    done = 0
    if args.load:
        s.load_state(np.load(args.load))
        done = int(s.stats(len(descs) - 1)["steps"])
    stop = nsteps if args.max_steps <= 0 else min(nsteps, done + args.max_steps)
    wall0 = time.perf_counter()
    while done < stop:
        k = min(args.chunk, stop - done)
        s.step(k)
        done += k
        st = s.stats(len(descs) - 1)
        print(json.dumps({"steps": done, "t": st["t"], "status": st["status"], "it_p": st["it_p"][:2],
                          "wall_s": round(time.perf_counter() - wall0, 1)}), file=sys.stderr, flush=True)
    if args.save:
        np.save(args.save, s.save_state())
    if done < nsteps:
        print(json.dumps({"stopped_at": done, "of": nsteps, "saved": args.save}), flush=True)
        s.close()
        return 0
    sols = []
    for i, d in enumerate(descs):
        sols.append({n: s.get(i, n).reshape(d["ny"], d["nx"]) for n in ("S1", "E1", "PMU", "E2", "E2B")})
    stats = [s.stats(i) for i in range(len(descs))]
    s.close()
    res = {"h_um": hs, "grids": [[d["nx"], d["ny"]] for d in descs], "dt": args.dt, "seconds": args.seconds,
           "steps": nsteps, "t": [st["t"] for st in stats], "status": [st["status"] for st in stats],
           "wall_s": round(time.perf_counter() - wall0, 1), "quantities": errors_and_rates(hs, sols)}
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
