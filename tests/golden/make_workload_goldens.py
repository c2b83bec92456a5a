"""Writes the oracle goldens of the full-size workloads (tests/golden/*.npz).

Runs the FP64 CPU oracle (and nothing else: this script imports only `oracle` and the
seeded input module `clot_inputs`) on a workload from its seeded initial state and,
at each checkpoint step, stores for every compared field

  * its full-field l2 norm and sum,
  * its values at a seeded sample of cells: every cell of a band along the injured
    wall (where the coagulation species live) plus uniformly drawn cells,
  * the injury-face fields E0, C0 in full,

so that a GPU run of the same workload for the same steps can be compared with the
oracle cell by cell on the sample and field by field on the norms.

Usage (each run is hours of one core for the big workloads):
  python tests/golden/make_workload_goldens.py channel2d_1024x256 1000
  python tests/golden/make_workload_goldens.py channel3d_256x64x64 20,50,100,200 [--state DIR]
  python tests/golden/make_workload_goldens.py ensemble:0,3,10 500
With --state DIR the oracle's state is also saved at every checkpoint (DIR/<tag>.pkl, a
file this script writes itself) and a run resumes from it when it is there.
"""
from __future__ import annotations

import json
import os
import pickle
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import clot_inputs as ci                      # noqa: E402
from oracle import clot_oracle as oc          # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SPECIES = ["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B", "E2B", "C1", "C2"]
N_RANDOM = 4096


def sample_cells(d: dict, seed: int = 4321) -> np.ndarray:
    """Cell ids (sorted, unique): the band of the first wall layers over the injury patch
    and 8 cells beyond it on every side, plus N_RANDOM uniform draws (or every cell of a
    channel of at most 8192 cells)."""
    nx, ny, nz = d["nx"], d["ny"], d["nz"]
    n = nx * ny * nz
    if n <= 8192:
        return np.arange(n)
    dx, dz = d["Lx"] / nx, d["Lz"] / nz
    i0 = max(int(d["inj_x0"] / dx) - 8, 0)
    i1 = min(int(d["inj_x1"] / dx) + 9, nx)
    layers = 4 if d["dim"] == 2 else 2
    if d["dim"] == 3:
        k0 = max(int(d["inj_z0"] / dz) - 8, 0)
        k1 = min(int(d["inj_z1"] / dz) + 9, nz)
    else:
        k0, k1 = 0, 1
    k, j, i = np.meshgrid(np.arange(k0, k1), np.arange(layers), np.arange(i0, i1), indexing="ij")
    band = (i + nx * (j + ny * k)).ravel()
    rng = np.random.default_rng(seed)
    extra = rng.choice(n, size=N_RANDOM, replace=False)
    return np.unique(np.concatenate([band, extra]))


def write(path: str, d: dict, o: oc.Oracle, idx: np.ndarray, steps: int, wall: float) -> None:
    f = o.fields()
    out = {"idx": idx.astype(np.int64)}
    names = ["UX", "UY"] + (["UZ"] if d["dim"] == 3 else []) + ["P", "ETA"] + SPECIES
    for nm in names:
        v = f[nm]
        out["n_" + nm] = np.array(np.linalg.norm(v))
        out["sum_" + nm] = np.array(v.sum())
        out["s_" + nm] = v[idx]
    for nm in ("E0", "C0"):
        out["f_" + nm] = f[nm]
    meta = dict(desc=d, steps=steps, oracle_seconds=wall, ncell=int(ci.ncell(d)), nsample=int(idx.size),
                made_by="tests/golden/make_workload_goldens.py")
    out["meta"] = np.array(json.dumps(meta))
    np.savez_compressed(path, **out)
    print(f"wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB) after {steps} steps, {wall:.0f} s", flush=True)


def run(tag: str, d: dict, checkpoints: list[int], state_dir: str | None = None) -> None:
    xc, xf = ci.noise(d)
    t0 = time.time()
    spath = os.path.join(state_dir, f"{tag}.pkl") if state_dir else None
    if spath and os.path.exists(spath):
        with open(spath, "rb") as fh:
            o = pickle.load(fh)          # the oracle's own state, written below by this script
        print(f"{tag}: resumed at step {o.n}", flush=True)
    else:
        o = oc.Oracle(d, xc, xf)
    idx = sample_cells(d)
    last = max(checkpoints)
    for s in range(o.n + 1, last + 1):
        o.step()
        if s % 10 == 0:
            print(f"{tag}: step {s}/{last}, {time.time() - t0:.0f} s", flush=True)
        if s in checkpoints:
            write(os.path.join(HERE, f"{tag}_step{s}.npz"), d, o, idx, s, time.time() - t0)
            if spath:
                with open(spath + ".tmp", "wb") as fh:
                    pickle.dump(o, fh)
                os.replace(spath + ".tmp", spath)


def main(argv: list[str]) -> None:
    state_dir = None
    if "--state" in argv:
        i = argv.index("--state")
        state_dir = argv[i + 1]
        os.makedirs(state_dir, exist_ok=True)
        argv = argv[:i] + argv[i + 2:]
    what, cps = argv[1], sorted(int(c) for c in argv[2].split(","))
    if what.startswith("ensemble:"):
        members = [int(m) for m in what.split(":")[1].split(",")]
        descs = ci.ensemble(64)
        for m in members:
            d = descs[m]
            run(f"ensemble64_member{m}_{d['nx']}x{d['ny']}", d, cps, state_dir)
    else:
        run(what, ci.workload(what), cps, state_dir)


if __name__ == "__main__":
    main(sys.argv)
