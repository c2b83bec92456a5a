"""Degenerate and extreme inputs through the C ABI against the FP64 oracle: no flow,
no injury faces, the smallest grids the library accepts, a channel two cells high,
tiny channels batched with ordinary ones, zero steps, and the inputs it must refuse."""
import numpy as np
import pytest

import clot_inputs as ci
from parity_util import compare

pytestmark = pytest.mark.gpu


def run_gpu(descs, prec, steps, **over):
    from paper_2304_09180_amd import clot
    s = clot.Solver(descs, prec, clot.default_params(prec, **over))
    for i, d in enumerate(descs):
        xc, xf = ci.noise(d)
        s.init_state(i, xc, xf)
    s.step(steps)
    out = [s.fields(i) for i in range(len(descs))]
    st = [s.stats(i) for i in range(len(descs))]
    s.close()
    return out, st


def oracle_fields(d, steps, **over):
    from oracle import clot_oracle as oc
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf, oc.Params(**over))
    for _ in range(steps):
        o.step()
    return o.fields()


CASES = {
    "no_flow_2d": ci.channel(2, 24, 8, shear=0.0, dt=1e-3, seed=31),
    "no_flow_3d": ci.channel(3, 12, 6, 5, shear=0.0, dt=1e-3, seed=32),
    "no_injury_faces": ci.channel(2, 32, 8, shear=800.0, dt=1e-4, seed=33, inj_frac=0.0),
    "smallest_2d": ci.channel(2, 2, 2, shear=1000.0, seed=34),
    "smallest_3d": ci.channel(3, 2, 2, 2, shear=1000.0, seed=35),
    "three_by_two": ci.channel(2, 3, 2, shear=1000.0, seed=36),
    "two_cells_high": ci.channel(2, 256, 2, shear=1000.0, dt=1e-4, seed=37, Lx=256 * 0.125),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_degenerate_channel_matches_oracle(name):
    from paper_2304_09180_amd import clot
    d = CASES[name]
    steps = 4
    (g,), (st,) = run_gpu([d], clot.FP64, steps)
    print(name, st, flush=True)
    assert st["status"] == "OK"
    if name == "no_injury_faces":
        assert g["E0"].size == 0 and g["C0"].size == 0
    if name.startswith("no_flow"):
        assert np.abs(g["UX"]).max() == 0.0 and np.abs(g["PHIX"]).max() == 0.0
    compare(g, oracle_fields(d, steps), 1e-10)


def test_fp64_tiny_channels_batched_with_ordinary_ones():
    from paper_2304_09180_amd import clot
    ds = [CASES["smallest_2d"], ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=3), CASES["three_by_two"],
          CASES["no_injury_faces"]]
    gs, sts = run_gpu(ds, clot.FP64, 3)
    for d, g, st in zip(ds, gs, sts):
        assert st["status"] == "OK"
        compare(g, oracle_fields(d, 3), 1e-10)


def test_zero_steps_change_nothing():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=3)
    xc, xf = ci.noise(d)
    s = clot.Solver([d], clot.FP32_MIXED)
    s.init_state(0, xc, xf)
    before = s.fields(0)
    s.step(0)
    after, st = s.fields(0), s.stats(0)
    s.close()
    for name in before:
        assert np.array_equal(before[name], after[name]), name
    assert st["steps"] == 0 and st["t"] == 0.0


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(ny=1), dict(dt=0.0), dict(shear=-1.0), dict(Lx=0.0),
])
def test_invalid_channels_are_refused(bad):
    from paper_2304_09180_amd import clot
    d = dict(ci.channel(2, 8, 4, shear=1000.0, dt=1e-4), **bad)
    with pytest.raises(clot.ClotError):
        clot.Solver([d], clot.FP64)


def test_flat_3d_and_empty_and_oversized_inputs_are_refused():
    from paper_2304_09180_amd import clot
    flat = dict(ci.channel(3, 8, 4, 4, shear=1000.0, dt=1e-4), nz=1)
    with pytest.raises(clot.ClotError):
        clot.Solver([flat], clot.FP64)
    with pytest.raises(clot.ClotError):
        clot.Solver([], clot.FP64)
    huge = ci.channel(3, 2048, 1024, 1025, shear=1000.0, dt=1e-4)     # above 2^31 cells
    with pytest.raises(clot.ClotError):
        clot.Solver([huge], clot.FP64)


@pytest.mark.parametrize("prec_name", ["FP64", "FP32_MIXED"])
def test_stats_continuity_and_non_negativity_agree_with_the_fields(prec_name):
    """clot_stats' div_rel and min_species against the same quantities computed here
    from the fields read back (x-fastest face arrays)."""
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    d = ci.channel(3, 24, 10, 9, shear=800.0, seed=5)
    (g,), (st,) = run_gpu([d], prec, 4)
    nx, ny, nz = d["nx"], d["ny"], d["nz"]
    fx = g["PHIX"].reshape(nz, ny, nx + 1)
    fy = g["PHIY"].reshape(nz, ny + 1, nx)
    fz = g["PHIZ"].reshape(nz + 1, ny, nx)
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :]) + (fz[1:] - fz[:-1])
    big = max(np.abs(fx).max(), np.abs(fy).max(), np.abs(fz).max())
    want_div = np.abs(div).max() / big
    p = clot.default_params(prec)
    scale = {"PMU": p.P_max, "PMA": p.P_max, "PBA": p.P_max, "PBSE": p.P_max, "ADP": p.adp_crit,
             "S1": p.S1_0, "S2": p.S2_0, "E1": p.S1_0, "E2": p.S2_0, "S1B": p.S1_0, "S2B": p.S2_0,
             "E1B": p.S1_0, "E2B": p.S2_0, "C1": p.S2_0, "C2": p.S2_0}
    want_min = min((g[n] / s).min() for n, s in scale.items())
    print(st["div_rel"], want_div, st["min_species"], want_min)
    assert st["div_rel"] == pytest.approx(want_div, rel=1e-3, abs=1e-300)
    assert st["div_rel"] < (1e-10 if prec_name == "FP64" else 1e-5)
    assert st["min_species"] == pytest.approx(want_min, rel=1e-6, abs=1e-300)
