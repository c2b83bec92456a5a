"""Seeded synthetic workloads for the clotting-step library, its oracle, tests and benchmark.

This module holds no model arithmetic: it only draws random numbers and writes
down workload descriptors (mesh sizes, domain extents, shear rate, injury patch,
time step, step count).  Both the CPU oracle and the GPU library take these
descriptors and the raw normal draws and build their own initial state from them.

Every descriptor is a plain dict with the keys

    dim, nx, ny, nz          mesh (dim=2 => nz=1)
    Lx, Ly, Lz               domain extents in mm (2-D: Lz is the cell depth)
    inj_x0, inj_x1           injury patch on the y=0 wall (x range, mm)
    inj_z0, inj_z1           injury patch z range (2-D: the whole depth)
    shear                    wall shear rate of the inflow, 1/s
    K_y, K_z                 margination amplitudes of the platelet inflow
    dt                       time step, s
    steps                    step count of the workload
    seed                     seed of the species noise

The species noise is drawn as ``numpy.random.default_rng(seed).standard_normal``:
first an array (15, ncell) for the cell species in library field order
(Pmu, Pma, Pba, Pbse, ADP, S1, S2, E1, E2, S1b, S2b, E1b, E2b, C1, C2), cells in
C order (k, j, i), then an array (2, nface) for the injury-face species (E0, C0),
faces x-fastest then z.  Species that start at zero stay zero under the noise.
"""
from __future__ import annotations

import math

import numpy as np

N_CELL_SPECIES = 15
N_FACE_SPECIES = 2

# Channel extents used by every workload: 1 mm long, 0.25 mm high (and wide in 3-D).
LX, LY, LZ3 = 1.0, 0.25, 0.25


def courant_dt(h: float, shear: float, height: float, co: float = 0.75, cap: float = 1e-4) -> float:
    """Fixed time step from a Courant limit: co*h/u_ref with u_ref = shear*height/4.

    u_ref is the centre-line speed of a plane parabolic channel with that wall
    shear; a square duct with the same centre-line wall shear is slower, so the
    bound also holds there.
    """
    return min(cap, co * h / (shear * height / 4.0))


def channel(dim: int, nx: int, ny: int, nz: int = 1, shear: float = 1000.0, dt: float | None = None,
            steps: int = 1, seed: int = 0, inj_frac: float = 0.25, inj_zfrac: float = 0.5,
            K: float | None = None, Lx: float = LX, Ly: float = LY, Lz: float | None = None) -> dict:
    """Descriptor of one straight channel with a centred injury patch on the y=0 wall.

    inj_frac is the patch length as a fraction of Lx; in 3-D the patch is
    inj_zfrac*Lz wide, centred in z.
    """
    if dim == 2:
        nz = 1
        Lz = Ly / ny if Lz is None else Lz
        z0, z1 = 0.0, Lz
        Ky = 330.0 if K is None else K
        Kz = 0.0
    else:
        Lz = LZ3 if Lz is None else Lz
        z0, z1 = 0.5 * Lz * (1 - inj_zfrac), 0.5 * Lz * (1 + inj_zfrac)
        Ky = Kz = (547.0 if K is None else K)
    h = min(Lx / nx, Ly / ny, Lz / nz if dim == 3 else Ly / ny)
    if dt is None:
        dt = courant_dt(h, shear, Ly)
    return dict(dim=dim, nx=nx, ny=ny, nz=nz, Lx=Lx, Ly=Ly, Lz=Lz,
                inj_x0=0.5 * Lx * (1 - inj_frac), inj_x1=0.5 * Lx * (1 + inj_frac),
                inj_z0=z0, inj_z1=z1, shear=float(shear), K_y=Ky, K_z=Kz,
                dt=float(dt), steps=int(steps), seed=int(seed))


def log_uniform_shear(seed: int, lo: float = 100.0, hi: float = 2000.0) -> float:
    """Wall shear rate drawn log-uniformly in [lo, hi] from its own stream of the seed."""
    rng = np.random.default_rng([seed, 1])
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def workload(name: str) -> dict:
    """Named workloads: the five headline configurations plus small parity cases."""
    if name == "channel2d_64x16":          # FP64, 100 steps at 1e-4 s
        return channel(2, 64, 16, shear=1000.0, dt=1e-4, steps=100, seed=0)
    if name == "channel2d_1024x256":       # FP32 mixed, 1000 steps at 1e-5 s (Courant 0.64)
        return channel(2, 1024, 256, shear=1000.0, dt=1e-5, steps=1000, seed=0)
    if name == "channel3d_256x64x64":      # FP32 mixed, 500 steps, shear from the seed
        return channel(3, 256, 64, 64, shear=log_uniform_shear(0), steps=500, seed=0)
    raise KeyError(name)


def ensemble(n: int = 64, steps: int = 500, base_seed: int = 1000) -> list[dict]:
    """Uneven ensemble: member i draws its size, shear and injury length from seed base_seed+i."""
    sizes = [(128, 32), (256, 64), (512, 128)]
    out = []
    for i in range(n):
        rng = np.random.default_rng([base_seed + i, 1])
        nx, ny = sizes[int(rng.integers(0, 3))]
        shear = float(math.exp(rng.uniform(math.log(100.0), math.log(2000.0))))
        frac = float(rng.uniform(0.1, 0.5))
        out.append(channel(2, nx, ny, shear=shear, steps=steps, seed=base_seed + i, inj_frac=frac))
    return out


def ncell(d: dict) -> int:
    return d["nx"] * d["ny"] * d["nz"]


def n_injury_faces(d: dict) -> int:
    """Count of y=0 wall faces whose centre lies inside the patch (x-fastest, then z)."""
    xc = (np.arange(d["nx"]) + 0.5) * (d["Lx"] / d["nx"])
    zc = (np.arange(d["nz"]) + 0.5) * (d["Lz"] / d["nz"])
    nxi = int(np.count_nonzero((xc >= d["inj_x0"]) & (xc <= d["inj_x1"])))
    nzi = int(np.count_nonzero((zc >= d["inj_z0"]) & (zc <= d["inj_z1"]))) if d["dim"] == 3 else 1
    return nxi * nzi


def noise(d: dict) -> tuple[np.ndarray, np.ndarray]:
    """Standard-normal draws for the multiplicative 1% species noise: (15, ncell), (2, nface)."""
    rng = np.random.default_rng(d["seed"])
    cell = rng.standard_normal((N_CELL_SPECIES, ncell(d)))
    face = rng.standard_normal((N_FACE_SPECIES, n_injury_faces(d)))
    return cell, face
