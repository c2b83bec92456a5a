"""Throughput benchmark of the clotting step on one MI355X.

Prints ONE JSON line: cell-timesteps/s of whole steps of the workload (inputs
resident in HBM), the roofline of the dominant kernel measured live with HIP
events on the library's stream, and the FP64 CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision fp32|fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s

# Algorithmic bytes per cell for each timed phase (compulsory reads + writes of one
# launch, stencil neighbours counted once), in cell-sized FP32 arrays (x2 for FP64).
# c = velocity components (= dim), a = transport systems still iterating (the last
# step's sysit_tr / it_tr: a system leaves the batched solve once it converges).
#   p_cg_a   : z, p_old, diag, rAU read; p_new, q written                       -> 6
#   p_cg_b   : x, p_new, r, q, diag read; x, r written                          -> 7
#   tr_b1    : per system r, p_old, v_old, diag, rhat and the six stored couplings
#              read; p, v written                                              -> 13 a
#   tr_b2    : per system r, v, diag and the six couplings read; t written       -> 10 a
#   tr_b3    : per system x, r, rhat, p, v, t, diag read; x, r written          -> 9 a
#   rxn      : 14 species and their low parts + ADP + eta read; 14 species and
#              their low parts written                                          -> 58
#   momentum BiCGStab with the multigrid V-cycle (the default):
#   mom_b1   : y, rhat per component + a_P + dim face fluxes read; v written   -> 3c + 1 + dim
#   mom_b2   : z, s per component + a_P + fluxes read; t written               -> 3c + 1 + dim
#   mom_b3   : x, y, z, s, t, rhat read; x, r written per component             -> 8c
#   mom_mg_r : finest restriction, averaged over its two forms (r, p, v or r, v
#              read; the formed right-hand side and the coarse one (1/8) written)
#              + a_P + fluxes                                                   -> 3.5c + 1 + dim + c/8
#   mom_mg_p1: b, coarse x (1/8), a_P, fluxes read; y written                  -> 2c + 1 + dim + c/8
#   mom_mg_p2: b, y, a_P, fluxes read; x written                                -> 3c + 1 + dim
def probe_arrays(probe, dim, st):
    c = dim
    a = st["sysit_tr"] / st["it_tr"] if st.get("it_tr") else 7.0
    table = {"p_cg_a": 6, "p_cg_b": 7, "tr_b1": 13 * a, "tr_b2": 10 * a, "tr_b3": 9 * a, "rxn": 58,
             "mom_b1": 3 * c + 1 + dim, "mom_b2": 3 * c + 1 + dim, "mom_b3": 8 * c,
             "mom_mg_r": 3.5 * c + 1 + dim + c / 8, "mom_mg_p1": 2 * c + 1 + dim + c / 8,
             "mom_mg_p2": 3 * c + 1 + dim}
    return table[probe]


def step_arrays(dim, st, ns):
    """Algorithmic traffic of one whole step, in cell-sized FP32 arrays per cell (an FP64
    array counts 2), from the solver's iteration counts of that step: every pass over the
    mesh counted once with its compulsory reads and writes (stencil neighbours once; the
    multigrid levels below the mesh at their own sizes).  ns: multigrid sweeps each way."""
    c = dim                                           # velocity components
    fixed = (6                                        # k_derive: 4 platelet fields -> theta_B, W
             + (2 * c + 2 + dim + 1) + (1 + 2 * c)    # k_mom_assemble: u, p, fluxes, theta_B -> a_P, src, b
             + 1 + 5 / 8.0                            # momentum levels: theta_B -> coarse mass, coefficients
             + (2 * c + 1 + dim) + 4 * c)             # momentum BiCGStab start: x, b, a_P, fluxes -> r, rh, p, v
    # momentum iteration: two V-cycles (finest: restriction, prolongation sweep, sweep; the
    # coarse levels at 1/8 the cells each, three passes over b, x, y and four coefficient
    # arrays) and the three BiCGStab phases
    fine = ((3.5 * c + 1 + dim + c / 8) + (2 * c + 1 + dim + c / 8) + (3 * c + 1 + dim))
    coarse = ((c + 4 + c / 8) + (2 * c + 4 + c / 8) + (3 * c + 4)) / 8.0 * 8.0 / 7.0
    mom_it = 2 * (fine + coarse) + (3 * c + 1 + dim) + (3 * c + 1 + dim) + 8 * c
    corr = (2 * c + 1 + dim) + c                      # k_hbya: u, src, a_P, fluxes -> HbyA
    corr += (c + 1) + 2 + 1                           # k_prhs: HbyA, rAU -> rhs (FP64), diagonal
    corr += (2 + c + 1) + (c + dim)                   # k_correct: p, HbyA, rAU -> u, flux
    per_pass = 8 + 6 + 5                              # FP64 residual, MG-CG start, p += e
    cg_it = 6 + 6                                     # k_mgcg_a, k_mgcg_b
    fine = 4 + 5 * (ns - 2) + 4.125 + 5.125 + 5 * (ns - 1)   # V-cycle on the mesh (pre, sweeps, restrict, up)
    lvl = (7 + 8 * (ns - 2) + 7.125 + 8.125 + 8 * (ns - 1)) / 8.0   # coefficient levels, 1/8 the cells each
    vcyc = fine + lvl * 8.0 / 7.0                     # geometric sum over the coarser levels
    eta = 3 + 5 + st["it_eta"] * 12                   # prep, CG start, per iteration cg_a + cg_b
    ntr = 7
    tr = ((7 + 7 + 1 + dim) + (7 + 14 + 14 + 6 * 7)   # assembly: C^n and low parts, W, fluxes -> diagonals
                                                      # (FP32 and FP64), FP64 right-hand sides, couplings
          + ntr * 17                                  # delta-form start: C^n, low part, FP64 diagonal and
                                                      # right-hand side, couplings -> r, rh, p, v, change
          + st["sysit_tr"] * (13 + 10 + 9)            # BiCGStab phases of the systems still iterating
          + ntr * 5)                                  # species + low part + change -> species, low part
    rxn = 58                                          # reactions on value + low part of 14 species
    total = fixed + st["it_mom"] * mom_it + eta + tr + rxn
    for k, passes in enumerate(st["refine_p"]):
        if passes <= 0:
            continue
        its = st["it_p"][k]
        total += corr + passes * (per_pass + vcyc) + its * (cg_it + vcyc)
    return total


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="channel3d_256x64x64")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tile", default="auto", choices=["auto", "256", "512", "1024"],
                    help="cells per block; auto runs the tile autotuner on each workload first")
    ap.add_argument("--probe", default="tr_b1",
                    help="kernel phase timed for the roofline (default: the transport BiCGStab's first phase, "
                         "the mesh-streaming kernel with the largest share of the step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brick-tune", action="store_true",
                    help="keep the default brick shape of the LDS-staged momentum kernels")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-reaction comparison")
    ap.add_argument("--train-samples", type=int, default=1_000_000)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-inhibitor", action="store_true",
                    help="skip the leg of the model with the inhibitor (section 3.4)")
    ap.add_argument("--no-time-scheme", action="store_true",
                    help="skip the Crank-Nicolson / variable-step leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    return ap.parse_args()


def recorded_traffic(workload, probe):
    """HBM bytes per launch of the probed kernel from the committed counter summary,
    or None when that summary was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{probe}_traffic.md")
    if not os.path.exists(path):
        return None
    from paper_2304_09180_amd.profsum import source_hash
    text = open(path).read()
    h = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("kernel source hash:")]
    t = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("traffic_bytes_per_launch:")]
    if not h or not t or h[0] != source_hash():
        return None
    return int(t[0])


def copy_calibration(mib):
    """A plain device-to-device copy of known size: its FETCH_SIZE/WRITE_SIZE counter
    readings calibrate the counters of the solver kernels."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(desc, steps=2):
    """FP64 oracle on a bounded sample of the workload: a slice of the same channel, 16
    cells long (its full cross-section at the same cell size, time step, shear, seed and
    injury patch proportions), `steps` timed steps (about 20-25 s of one core).  The
    oracle's sparse LU and Krylov solves run on one thread.  Reported in cell-timesteps/s."""
    import clot_inputs as ci
    from oracle import clot_oracle as oc
    d = dict(desc)
    nx = min(16, desc["nx"])
    d["nx"] = nx
    d["Lx"] = desc["Lx"] * nx / desc["nx"]
    d["inj_x0"], d["inj_x1"] = 0.25 * d["Lx"], 0.75 * d["Lx"]
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step()
    el = time.perf_counter() - t0
    cells = d["nx"] * d["ny"] * d["nz"]
    return {"value": cells * steps / el, "unit": "cell-timesteps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of a {d['nx']}x{d['ny']}x{d['nz']} slice of the same channel (the "
                      f"full {desc['ny']}x{desc['nz']} cross-section, same cell size, time step, shear and "
                      f"seed), FP64, sparse LU for momentum and pressure, Krylov for eta and transport",
            "grid": [d["nx"], d["ny"], d["nz"]], "steps": steps, "seconds": round(el, 3),
            "threads": 1, "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def timed_steps(s, steps, probe):
    """Runs `steps` steps between events on the library stream; returns (seconds,
    probe ms, probe launches)."""
    import torch
    stream = s.stream
    s.probe(probe)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step_async(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    pm, pn = s.probe_read()
    s.probe(None)
    return max(ms / 1e3, wall), pm, pn


def kernel_us(s, probe, steps=2):
    """Average launch time of one kernel phase over a few extra steps."""
    _, pm, pn = timed_steps(s, steps, probe)
    return round(1e3 * pm / pn, 3) if pn else None


def pick_tile(descs, prec, args):
    """The tile for a workload: given, or tuned (whole-step timing of each candidate)."""
    if args.tile != "auto":
        return int(args.tile), None
    from paper_2304_09180_amd import autotune
    e = autotune.tune(descs, prec, log=lambda m: print(m, file=sys.stderr, flush=True))
    return e["tile"], e


def pick_bricks(descs, prec, tile, args):
    """Brick shape of each LDS-staged momentum kernel: tuned (per-kernel launch times in
    each shape) unless --no-brick-tune."""
    if args.no_brick_tune:
        return None
    from paper_2304_09180_amd import autotune
    return autotune.tune_bricks(descs, prec, tile=tile, log=lambda m: print(m, file=sys.stderr, flush=True))


def surrogate_leg(desc, prec, args, xc, xf, tile):
    """Trains the reaction surrogate on the GPU (2-D channel states), then times the
    same workload with the learned reaction step."""
    from paper_2304_09180_amd import clot, surrogate
    t0 = time.perf_counter()
    states = surrogate.default_training_states(log=lambda m: print(m, file=sys.stderr, flush=True))
    rows = surrogate.sample_rows(states, args.train_samples)
    tr = surrogate.Trainer(rows, log=lambda m: print(m, file=sys.stderr, flush=True))
    l0 = tr.loss()
    hist = tr.train(epochs=12)
    held = surrogate.sample_rows(states, 50_000, seed=99, dt_range=(2e-4, 1e-3))
    held_net, held_zero = tr.heldout_gain(held)
    t_train = time.perf_counter() - t0
    blob = tr.blob()
    ncell = desc["nx"] * desc["ny"] * desc["nz"]

    def run(mode, m_rxn):
        s = clot.Solver([desc], prec, clot.default_params(prec, M_rxn=m_rxn), tile=tile)
        s.init_state(0, xc, xf)
        if mode == "surrogate":
            s.set_reaction_mode(clot.SURROGATE, blob, 1e-3)
        for _ in range(args.warmup):
            s.step(1)
        el, _, _ = timed_steps(s, args.steps, "rxn")
        r = {"value": ncell * args.steps / el, "ms_per_step": el * 1e3 / args.steps, "rxn_kernel_us": kernel_us(s, "rxn")}
        if mode == "surrogate":
            r["fallback_kernel_us"] = kernel_us(s, "rxn_fallback")
            r["fallback_frac"] = s.stats(0)["fallback_frac"]
        s.close()
        return r

    sweep = {}
    for m in (2, 8, 32):
        sweep[f"M_rxn={m}"] = {"plain": run("plain", m), "surrogate": run("surrogate", m)}
        print(f"# M_rxn={m}: {sweep[f'M_rxn={m}']}", file=sys.stderr, flush=True)
    out = dict(sweep["M_rxn=2"]["surrogate"])
    out.update({"resid_tol": 1e-3, "m_rxn_sweep": sweep,
                "training": {"samples": args.train_samples, "epochs": 12, "seconds": round(t_train, 2),
                             "loss_start": l0, "loss_end": hist[-1],
                             "heldout_mse_network": held_net, "heldout_mse_midpoint_alone": held_zero}})
    return out


def time_scheme_leg(desc, prec, args, xc, xf, tile):
    """The same workload with Crank-Nicolson 0.9 on every ddt term and the variable step
    at maxCo 0.75 (the channel's dt is the largest step): cost per step against the
    implicit-Euler fixed step, and the simulated time it covers."""
    import torch
    from paper_2304_09180_amd import clot
    prm = clot.default_params(prec, ddt_psi=0.9, max_co=0.75)
    s = clot.Solver([desc], prec, prm, tile=tile)
    s.init_state(0, xc, xf)
    for _ in range(max(1, args.warmup)):
        s.step(1)
    t0 = s.stats(0)["t"]
    el, _, _ = timed_steps(s, args.steps, args.probe)
    st = s.stats(0)
    s.close()
    torch.cuda.synchronize()
    return {"ddt": "CrankNicolson 0.9", "max_co": 0.75, "ms_per_step": round(el * 1e3 / args.steps, 4),
            "dt_last": st["dt"], "simulated_s_per_wall_s": round((st["t"] - t0) / el, 6), "status": st["status"],
            "solver": {k: st[k] for k in ("it_mom", "it_p", "it_eta", "it_tr", "refine_p")}}


def inhibitor_leg(desc, prec, args, xc, xf):
    """The same workload with the inhibitor of section 3.4's extensibility example
    (I + E2 -> E2i: 17 cell species, 9 transported, 16 reacting) from its own build:
    cost per step next to the base model's, and the kernels the two species widen."""
    import torch
    from paper_2304_09180_amd import clot
    s = clot.Solver([desc], prec, clot.default_params(prec), inhibitor=True)
    s.init_state(0, xc, xf)
    for _ in range(max(1, args.warmup)):
        s.step(1)
    el, _, _ = timed_steps(s, args.steps, args.probe)
    st = s.stats(0)
    us = {k: kernel_us(s, k) for k in ("rxn", "tr_asm", "tr_b1")}
    s.close()
    torch.cuda.synchronize()
    return {"species": 17, "transported": 9, "tile": 256, "ms_per_step": round(el * 1e3 / args.steps, 4),
            "kernel_us": us, "status": st["status"],
            "solver": {k: st[k] for k in ("it_mom", "it_p", "it_eta", "it_tr", "refine_p")}}


def ensemble_leg(args):
    """The 64-member uneven ensemble of 2-D channels in one context, FP32: eager steps,
    then the same steps replayed as HIP graphs."""
    import clot_inputs as ci
    from paper_2304_09180_amd import autotune, clot
    descs = ci.ensemble(64)
    ncell = sum(ci.ncell(d) for d in descs)
    tile, tuned = pick_tile(descs, clot.FP32_MIXED, args)
    bricks = pick_bricks(descs, clot.FP32_MIXED, tile, args)
    out = {"members": len(descs), "cells": ncell,
           "sizes": sorted({f"{d['nx']}x{d['ny']}" for d in descs}),
           "dt_range": [min(d["dt"] for d in descs), max(d["dt"] for d in descs)], "tile": tile}
    if tuned:
        out["autotune"] = {"ms_per_step": tuned["ms_per_step"], "kernel_us": tuned["kernel_us"]}
    if bricks:
        out.setdefault("autotune", {})["bricks"] = {k: bricks[k] for k in (*autotune.BRICK_PROBES, "us")}
    for mode in ("eager", "graph"):
        s = clot.Solver(descs, clot.FP32_MIXED, tile=tile)
        if bricks:
            autotune.apply_bricks(s, bricks)
        for c, d in enumerate(descs):
            xc, xf = ci.noise(d)
            s.init_state(c, xc, xf)
        if mode == "graph":
            s.set_graph_mode(True)
        for _ in range(max(args.warmup, 3)):   # graph mode: two calibrating steps, then recording
            s.step(1)
        el, _, _ = timed_steps(s, args.steps, None)
        s.sync()
        r = {"value": ncell * args.steps / el, "ms_per_step": el * 1e3 / args.steps}
        if mode == "graph":
            gi = s.graph_info()
            r.update({"replays": gi["replays"], "overflows": gi["overflows"], "budgets": gi["budgets"]})
        st = s.stats(0)
        r["solver_member0"] = {k: st[k] for k in ("it_mom", "it_p", "it_eta", "it_tr", "refine_p")}
        out[mode] = r
        print(f"# ensemble {mode}: {r}", file=sys.stderr, flush=True)
        s.close()
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the library solves every channel "
                                   "on one device (a slab decomposition over several GPUs is designed, not built)"}))
        sys.exit(2)
    import torch
    import clot_inputs as ci
    from paper_2304_09180_amd import autotune, clot

    desc = ci.workload(args.workload)
    prec = clot.FP32_MIXED if args.precision == "fp32" else clot.FP64
    tile, tuned = pick_tile([desc], prec, args)
    bricks = pick_bricks([desc], prec, tile, args)
    s = clot.Solver([desc], prec, tile=tile)
    if bricks:
        autotune.apply_bricks(s, bricks)
    xc, xf = ci.noise(desc)
    s.init_state(0, xc, xf)
    ncell = desc["nx"] * desc["ny"] * desc["nz"]
    print(f"# workload {args.workload}: {ncell} cells, dt {desc['dt']:.3e}, shear {desc['shear']:.1f}", file=sys.stderr,
          flush=True)
    for w in range(args.warmup):
        s.step(1)
        print(f"# warmup step {w + 1}/{args.warmup} {s.stats(0)}", file=sys.stderr, flush=True)

    el, probe_ms, probe_n = timed_steps(s, args.steps, args.probe)
    st = s.stats(0)
    print(f"# timed {args.steps} steps: {el * 1e3:.1f} ms {st}", file=sys.stderr, flush=True)
    rxn_us = kernel_us(s, "rxn")
    base_us = {k: kernel_us(s, k) for k in ("tr_asm", "tr_b1")}
    value = ncell * args.steps / el
    bpe = 4 if prec == clot.FP32_MIXED else 8
    nbytes = int(probe_arrays(args.probe, desc["dim"], st) * bpe * ncell)
    roof = None
    if probe_n:
        avg_s = probe_ms / 1e3 / probe_n
        achieved = nbytes / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": args.probe, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(args.workload, args.probe),
                "bytes_per_launch": nbytes, "avg_launch_us": round(avg_s * 1e6, 3), "launches": probe_n}
    if roof is not None:
        ns = 3 if desc["dim"] == 3 else 2
        per_cell = step_arrays(desc["dim"], st, ns) * bpe
        ach = per_cell * ncell / (el / args.steps) / 1e9
        roof["step"] = {"achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_cell_step": round(per_cell, 1),
                        "model": "sum over the step's passes of compulsory bytes x this run's iteration counts"}
    out = {"metric": "cell-timesteps/s", "value": value, "unit": "cell-timesteps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == clot.FP32_MIXED else "f64", "data": "synthetic",
           "config": {"workload": args.workload, "cells": ncell, "dim": desc["dim"], "tile": tile,
                      "grid": [desc["nx"], desc["ny"], desc["nz"]], "dt": desc["dt"], "shear": desc["shear"],
                      "precision": "fp32 fields, fp64 reductions and pressure" if prec == clot.FP32_MIXED else "fp64",
                      "reaction": "plain RK4"},
           "solver": {k: st[k] for k in ("it_mom", "it_p", "it_eta", "it_tr", "refine_p")},
           "rxn_kernel_us": rxn_us,
           "kernel_us": dict(base_us, rxn=rxn_us),
           "roofline": roof}
    if tuned:
        out["autotune"] = {"ms_per_step": tuned["ms_per_step"], "kernel_us": tuned["kernel_us"]}
    if bricks:
        out.setdefault("autotune", {})["bricks"] = {k: bricks[k] for k in (*autotune.BRICK_PROBES, "us")}
    s.close()
    if not args.no_time_scheme:
        out["time_scheme"] = time_scheme_leg(desc, prec, args, xc, xf, tile)
    if not args.no_inhibitor:
        out["inhibitor"] = inhibitor_leg(desc, prec, args, xc, xf)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(desc, prec, args, xc, xf, tile)
    if not args.no_ensemble:
        out["ensemble"] = ensemble_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
