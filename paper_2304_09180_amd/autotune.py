"""Tile autotuner.

The tile (cells owned by one 256-thread block: 256, 512 or 1024, i.e. one, two or
four cells per thread) trades per-block overhead and memory-level parallelism in the
fine-grid stencil and Krylov kernels against the parallelism left on small grids
(the coarse multigrid levels, small channels).  The best size depends on the
dimension, the channel shapes and the precision, so it is measured:

  for each candidate tile, build a context on the workload, run warm-up steps, then
  time whole steps (median of `repeats` runs on the library stream) and the average
  launch of four kernel classes (momentum stencil assembly, transport assembly,
  pressure stencil product, reactions) for the record;
  the fastest median wins, a candidate within 1% of a smaller one loses to it.

Results are cached as JSON keyed by the GPU architecture, the precision and the
multiset of channel shapes.

The LDS-staged finest-level kernels of the momentum preconditioner (a block stages a
brick of 1024 cells and a one-cell halo) take their brick shape per kernel:
`tune_bricks` times each of the three kernels (restriction, prolongation sweep,
sweep) in each of the four shapes on one context (probe average over a few steps),
keeps the fastest per kernel (shape 0 unless another beats it by more than 1%) and
caches the choice under the same key with a "bricks" suffix; `apply_bricks` sets it on
a solver.
"""
from __future__ import annotations

import json
import os
import tempfile
from collections import Counter

import numpy as np

from . import clot

KERNEL_CLASSES = ("mom_asm", "tr_asm", "p_cg_a", "rxn")


def default_cache_path() -> str:
    return os.environ.get("CLOT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "clot", "autotune.json"))


def shape_key(descs) -> str:
    """Multiset of channel shapes, e.g. '2d:128x32x1*17,256x64x1*20'."""
    dims = sorted({int(d["dim"]) for d in descs})
    cnt = Counter(f"{d['nx']}x{d['ny']}x{d['nz']}" for d in descs)
    return "+".join(f"{k}d" for k in dims) + ":" + ",".join(f"{s}*{n}" for s, n in sorted(cnt.items()))


def arch_name() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_key(descs, precision, arch: str) -> str:
    prec = "fp64" if precision == clot.FP64 else "fp32"
    return f"{arch}|{prec}|{shape_key(descs)}"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str, key: str, entry: dict) -> None:
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(times: dict) -> int:
    """Fastest median; a larger tile must beat every smaller one by more than 1%."""
    best = None
    for tile in sorted(times):
        if best is None or times[tile] < 0.99 * times[best]:
            best = tile
    return best


def _measure(descs, precision, tile, steps, warmup, repeats):
    import torch
    s = clot.Solver(descs, precision, tile=tile)
    try:
        for c, d in enumerate(descs):
            n = d["nx"] * d["ny"] * d["nz"]
            nf = s.count(c, "E0")
            # clean initial state (the multiplicative perturbations set to zero)
            s.init_state(c, np.zeros((15, n)), np.zeros((2, nf)))
        for _ in range(warmup):
            s.step(1)
        runs = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.step_async(steps)
            e1.record(s.stream)
            s.sync()
            runs.append(e0.elapsed_time(e1) / steps)
        kernels = {}
        for k in KERNEL_CLASSES:
            s.probe(k)
            s.step(1)
            ms, n = s.probe_read()
            s.probe(None)
            kernels[k] = round(1e3 * ms / n, 3) if n else None
        return float(np.median(runs)), kernels
    finally:
        s.close()


def tune(descs, precision, candidates=clot.TILES, steps=5, warmup=3, repeats=3, cache=None, force=False, log=None):
    """Tile for this workload: from the cache, or measured and stored."""
    path = cache or default_cache_path()
    key = cache_key(descs, precision, arch_name())
    if not force:
        hit = load_cache(path).get(key)
        if hit and hit.get("tile") in candidates:
            return hit
    times, kernels = {}, {}
    for tile in candidates:
        times[tile], kernels[tile] = _measure(descs, precision, tile, steps, warmup, repeats)
        if log:
            log(f"# autotune {key} tile {tile}: {times[tile]:.3f} ms/step {kernels[tile]}")
    best = choose(times)
    entry = {"tile": best, "ms_per_step": {str(t): round(v, 4) for t, v in times.items()},
             "kernel_us": {str(t): v for t, v in kernels.items()}, "steps": steps, "repeats": repeats}
    store_cache(path, key, entry)
    return entry


# each bricked kernel and the probe that times it: the momentum preconditioner's finest
# level, and the pressure hierarchy's LDS-staged coarse-level legs (FP32 contexts)
BRICK_PROBES = {"restrict": "mom_mg_r", "prolong": "mom_mg_p1", "sweep": "mom_mg_p2", "p_down": "p_mg_down",
                "p_up": "p_mg_up"}


def tune_bricks(descs, precision, tile=clot.TILES[0], steps=4, warmup=3, cache=None, force=False, log=None):
    """Brick shape of each LDS-staged kernel for this workload: from the cache, or
    measured (average launch time of the kernel in each shape) and stored.  A kernel the
    workload does not run keeps shape 0."""
    path = cache or default_cache_path()
    key = cache_key(descs, precision, arch_name()) + f"|tile{tile}|bricks"
    if not force:
        hit = load_cache(path).get(key)
        if hit and all(hit.get(k) in range(clot.N_BRICK_SHAPES) for k in BRICK_PROBES):
            return hit
    s = clot.Solver(descs, precision, tile=tile)
    us = {k: {} for k in BRICK_PROBES}
    try:
        for c, d in enumerate(descs):
            n = d["nx"] * d["ny"] * d["nz"]
            s.init_state(c, np.zeros((15, n)), np.zeros((2, s.count(c, "E0"))))
        for _ in range(warmup):
            s.step(1)
        for kernel, probe in BRICK_PROBES.items():
            for shape in range(clot.N_BRICK_SHAPES):
                s.set_brick_shape(kernel, shape)
                s.step(1)
                s.probe(probe)
                s.step(steps)
                ms, nl = s.probe_read()
                s.probe(None)
                us[kernel][shape] = 1e3 * ms / nl if nl else float("inf")
                if log:
                    log(f"# autotune {key} {kernel} shape {shape} {clot.brick_dims(descs[0]['dim'], shape, kernel)}: "
                        f"{us[kernel][shape]:.2f} us over {nl} launches")
                if not nl:      # not run by this workload
                    for q in range(shape + 1, clot.N_BRICK_SHAPES):
                        us[kernel][q] = float("inf")
                    break
            s.set_brick_shape(kernel, 0)
    finally:
        s.close()
    entry = {k: choose(us[k]) for k in BRICK_PROBES}
    entry["us"] = {k: {str(q): round(v, 3) for q, v in us[k].items()} for k in BRICK_PROBES}
    entry["steps"] = steps
    store_cache(path, key, entry)
    return entry


def apply_bricks(solver, entry) -> None:
    """Sets the tuned brick shape of every LDS-staged kernel on a solver."""
    for kernel in BRICK_PROBES:
        solver.set_brick_shape(kernel, int(entry[kernel]))
