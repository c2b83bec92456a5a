"""GPU checks at the workloads' full sizes, where the FP64 oracle is too slow to run:
properties that hold at any size, the FP32 path against the FP64 path (whose parity
with the oracle the smaller tests establish), and batched against single runs."""
import numpy as np
import pytest

import clot_inputs as ci
from parity_util import compare

pytestmark = pytest.mark.gpu

SPECIES = ["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B", "E2B", "C1", "C2"]


def run(descs, prec, steps, params=None, tile=256, init=True):
    from paper_2304_09180_amd import clot
    s = clot.Solver(descs, prec, params, tile=tile)
    for c, d in enumerate(descs):
        xc, xf = ci.noise(d)
        s.init_state(c, xc, xf)
    s.step(steps)
    out = [s.fields(c) for c in range(len(descs))]
    st = [s.stats(c) for c in range(len(descs))]
    s.close()
    return out, st


def divergence(f, d):
    """Net outflow of every cell from the face fluxes (x-fastest face arrays)."""
    nx, ny, nz = d["nx"], d["ny"], d["nz"]
    fx = f["PHIX"].reshape(nz, ny, nx + 1)
    fy = f["PHIY"].reshape(nz, ny + 1, nx)
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])
    if d["dim"] == 3:
        fz = f["PHIZ"].reshape(nz + 1, ny, nx)
        div = div + (fz[1:] - fz[:-1])
    return div, max(np.abs(fx).max(), np.abs(fy).max())


def check_properties(f, d, div_tol):
    div, scale = divergence(f, d)
    assert np.abs(div).max() <= div_tol * scale, (np.abs(div).max(), scale)
    for n in SPECIES:
        assert np.isfinite(f[n]).all(), n
        # transport and RK4 keep every species non-negative up to round-off of its scale
        assert f[n].min() >= -1e-6 * max(np.abs(f[n]).max(), 1e-30), (n, f[n].min())


def compare_fields(a, b, d, tol):
    """Velocity (as one vector) and the 15 cell species against the tolerance, with
    the near-zero floor of the parity tests; p and eta are reported (p solves a
    Poisson problem, so its relative error carries the Laplacian's conditioning times
    the FP32 rounding of its inputs, while the velocity built from its gradient does
    not)."""
    names = ["UX", "UY"] + (["UZ"] if d["dim"] == 3 else []) + SPECIES
    compare(a, b, tol, names)
    compare(a, b, float("inf"), ["P", "ETA"])


@pytest.mark.parametrize("name,steps", [("channel2d_1024x256", 40), ("channel3d_256x64x64", 10)])
def test_fp32_path_against_fp64_path_at_full_size(name, steps):
    from paper_2304_09180_amd import clot
    d = ci.workload(name)
    f32, s32 = run([d], clot.FP32_MIXED, steps)
    f64, s64 = run([d], clot.FP64, steps)
    print(name, s32[0]["it_mom"], s32[0]["it_p"][:2], s64[0]["it_mom"], s64[0]["it_p"][:2], flush=True)
    assert s32[0]["status"] == "OK" and s64[0]["status"] == "OK"
    check_properties(f64[0], d, 1e-10)
    check_properties(f32[0], d, 1e-5)
    compare_fields(f32[0], f64[0], d, 1e-5)


def test_ensemble_members_match_their_single_runs():
    """Channels share launches but not reductions or convergence: each member of the
    64-channel ensemble (FP32) evolves as it does alone.  Not bit for bit: a batch
    coarsens its pressure multigrid until the largest channel is coarse enough, so a
    smaller member gets more levels (another, equally valid preconditioner) than alone;
    a member of the largest size gets the same hierarchy and must match exactly."""
    from paper_2304_09180_amd import clot
    descs = ci.ensemble(64)
    steps = 4
    batch, st = run(descs, clot.FP32_MIXED, steps)
    assert all(x["status"] == "OK" for x in st), [c for c, x in enumerate(st) if x["status"] != "OK"]
    big = max(ci.ncell(d) for d in descs)
    for c in (0, 7, 21, 38, 63):   # sizes 128x32 .. 512x128 among them
        single, _ = run([descs[c]], clot.FP32_MIXED, steps)
        if ci.ncell(descs[c]) == big:
            for n, v in single[0].items():
                assert np.array_equal(batch[c][n], v), (c, n)
        else:
            compare_fields(batch[c], single[0], descs[c], 1e-5)


def test_surrogate_step_against_plain_step_on_the_duct():
    """The learned reaction step on the 1M-cell duct (plain RK4 as the reference)."""
    from paper_2304_09180_amd import clot, surrogate
    d1 = ci.workload("channel2d_64x16")
    states = surrogate.collect_states([(d1, 100)], log=lambda *a: None)
    tr = surrogate.Trainer(surrogate.sample_rows(states, 100_000), log=lambda *a: None)
    tr.train(epochs=6)
    d = ci.workload("channel3d_256x64x64")
    steps = 10
    plain, _ = run([d], clot.FP32_MIXED, steps)
    s = clot.Solver([d], clot.FP32_MIXED)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    s.set_reaction_mode(clot.SURROGATE, tr.blob(), 1e-3)
    s.step(steps)
    surr = s.fields(0)
    st = s.stats(0)
    s.close()
    print("fallback fraction", st["fallback_frac"], flush=True)
    check_properties(surr, d, 1e-5)
    compare_fields(surr, plain[0], d, 1e-3)
