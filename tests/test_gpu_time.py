"""GPU parity of the time integration options (Appendix D discretization table:
Crank-Nicolson psi on every ddt term; the variable step at maxCo) against the FP64
oracle, through the C ABI, plus graph replay and re-initialisation checks."""
import numpy as np
import pytest

import clot_inputs as ci
from parity_util import compare

pytestmark = pytest.mark.gpu

FP32_NAMES = ["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B", "E2B", "C1", "C2",
              "E0", "C0"]


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


def run_oracle(d, steps, **over):
    from oracle import clot_oracle as oc
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf, oc.Params(**over))
    for _ in range(steps):
        o.step()
    return o


def velocity_err(gpu, ref, dim):
    comps = ["UX", "UY"] + (["UZ"] if dim == 3 else [])
    a = np.concatenate([gpu[c] for c in comps])
    b = np.concatenate([ref[c] for c in comps])
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("psi", [0.9, 1.0])
def test_fp64_crank_nicolson_2d(psi):
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=3)
    (g,), (st,) = run_gpu([d], clot.FP64, 6, ddt_psi=psi)
    print(st, flush=True)
    o = run_oracle(d, 6, ddt_psi=psi)
    compare(g, o.fields(), 1e-10)


def test_fp64_crank_nicolson_variable_step_3d():
    """A given step about twice the Courant limit: every step is cut to Courant 0.75."""
    from paper_2304_09180_amd import clot
    d = ci.channel(3, 24, 10, 9, shear=800.0, dt=1.5e-3, seed=5)
    over = dict(ddt_psi=0.9, max_co=0.75)
    (g,), (st,) = run_gpu([d], clot.FP64, 5, **over)
    print(st, flush=True)
    o = run_oracle(d, 5, **over)
    assert o.dt < 0.6 * d["dt"]
    compare(g, o.fields(), 1e-10)
    assert st["t"] == pytest.approx(o.t, rel=1e-12)
    assert st["dt"] == pytest.approx(o.dt, rel=1e-10)


def test_fp64_variable_step_growth_from_a_small_step():
    """Euler with a variable step on a channel whose given step is below the limit:
    the step stays at the given one (the cap), and the clock is n dt."""
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 72, 20, shear=1000.0, dt=5e-5, seed=4)
    (g,), (st,) = run_gpu([d], clot.FP64, 4, max_co=0.75)
    o = run_oracle(d, 4, max_co=0.75)
    compare(g, o.fields(), 1e-10)
    assert st["dt"] == o.dt == d["dt"]
    assert st["t"] == pytest.approx(4 * d["dt"], rel=1e-15)


def test_fp64_uneven_batch_keeps_per_channel_clocks():
    from paper_2304_09180_amd import clot
    ds = [ci.channel(2, 32, 8, shear=300.0, dt=4e-4, seed=11, inj_frac=0.3),
          ci.channel(2, 48, 12, shear=1500.0, dt=4e-4, seed=12, inj_frac=0.15),
          ci.channel(2, 64, 16, shear=700.0, dt=4e-4, seed=13, inj_frac=0.45)]
    over = dict(ddt_psi=0.9, max_co=0.75)
    gs, sts = run_gpu(ds, clot.FP64, 4, **over)
    dts = []
    for d, g, st in zip(ds, gs, sts):
        o = run_oracle(d, 4, **over)
        compare(g, o.fields(), 1e-10)
        assert st["t"] == pytest.approx(o.t, rel=1e-12)
        dts.append(st["dt"])
    assert len(set(dts)) == 3         # each channel at its own limit


@pytest.mark.parametrize("noise,steps", [(False, 30), (True, 6)])
def test_fp32_crank_nicolson_variable_step_2d(noise, steps):
    """FP32 against the FP64 oracle.  The frozen van Leer weights jump where C_D - C_U
    changes sign (r -> +-inf, psi -> 2 or 0); on the 1%-noise initial state some face
    meets neighbours equal to ~1e-9, and where FP32 and FP64 values of C^n fall on
    either side the two take different weights and part by ~Co x noise in a cell.
    Implicit Euler damps that; Crank-Nicolson 0.9 keeps 0.9 of it per step.  So the
    noisy state is compared over 6 steps (its first such split, for this seed, falls
    at step 8) and a smooth state (no noise) over 30."""
    from paper_2304_09180_amd import clot
    from oracle import clot_oracle as oc
    d = ci.channel(2, 72, 20, shear=1000.0, dt=4e-4, seed=4)
    over = dict(ddt_psi=0.9, max_co=0.75)
    xc, xf = ci.noise(d)
    if not noise:
        xc, xf = np.zeros_like(xc), np.zeros_like(xf)
    s = clot.Solver([d], clot.FP32_MIXED, clot.default_params(clot.FP32_MIXED, **over))
    s.init_state(0, xc, xf)
    s.step(steps)
    g, st = s.fields(0), s.stats(0)
    s.close()
    print(st, flush=True)
    o = oc.Oracle(d, xc, xf, oc.Params(**over))
    for _ in range(steps):
        o.step()
    ref = o.fields()
    assert velocity_err(g, ref, 2) < 1e-5
    compare(g, ref, 1e-5, names=FP32_NAMES)
    assert st["t"] == pytest.approx(o.t, rel=1e-5)
    assert st["dt"] == pytest.approx(o.dt, rel=1e-5)


def test_graph_replay_with_variable_step_matches_eager_bitwise():
    """The step and the ddt coefficients live on the device: replays read them there."""
    from paper_2304_09180_amd import clot
    descs = [ci.channel(2, 32, 8, shear=300.0, dt=4e-4, seed=11, inj_frac=0.3),
             ci.channel(2, 64, 16, shear=1500.0, dt=4e-4, seed=13, inj_frac=0.45)]
    prm = clot.default_params(clot.FP32_MIXED, ddt_psi=0.9, max_co=0.75)

    def make():
        s = clot.Solver(descs, clot.FP32_MIXED, prm)
        for c, d in enumerate(descs):
            xc, xf = ci.noise(d)
            s.init_state(c, xc, xf)
        return s
    eager, graph = make(), make()
    graph.set_graph_mode(True, 1.25, 2)
    for step in range(6):
        print(f"step {step}", flush=True)
        eager.step(1)
        graph.step(1)
        for c in range(len(descs)):
            fe, fg = eager.fields(c), graph.fields(c)
            for name in fe:
                assert np.array_equal(fe[name], fg[name]), (step, c, name)
            assert eager.stats(c)["dt"] == graph.stats(c)["dt"]
    assert graph.graph_info()["replays"] == 4
    eager.close()
    graph.close()


def test_reinitialisation_resets_clock_and_history():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, shear=1000.0, dt=4e-4, seed=3)
    prm = clot.default_params(clot.FP64, ddt_psi=0.9, max_co=0.75)
    xc, xf = ci.noise(d)
    s = clot.Solver([d], clot.FP64, prm)
    s.init_state(0, xc, xf)
    s.step(3)
    s.init_state(0, xc, xf)
    s.step(3)
    again, st = s.fields(0), s.stats(0)
    s.close()
    (fresh,), (st2,) = run_gpu([d], clot.FP64, 3, ddt_psi=0.9, max_co=0.75)
    for name in fresh:
        assert np.array_equal(again[name], fresh[name]), name
    assert st["t"] == st2["t"] and st["dt"] == st2["dt"]


def test_time_scheme_parameters_are_checked():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, seed=21)
    for bad in (dict(ddt_psi=-0.1), dict(ddt_psi=1.5), dict(max_co=-1.0), dict(dt_growth=0.5)):
        with pytest.raises(clot.ClotError):
            clot.Solver([d], clot.FP64, clot.default_params(clot.FP64, **bad))


@pytest.mark.parametrize("prec_name,tol", [("FP64", 1e-10), ("FP32_MIXED", 1e-5)])
def test_paper_2d_example_first_steps_match_the_oracle(prec_name, tol):
    """A window of the paper's 2-D thrombosis example (section 4.1; the channel of
    `thrombus2d`: 240 x 60 um, 128 x 32 cells, a 90 um patch, wall shear 1000 1/s, no
    noise, Crank-Nicolson 0.9 and the variable step at Courant 0.75): its first 12 steps
    against the oracle and the clock; FP64 every field, FP32 velocity and species."""
    from oracle import clot_oracle as oc
    from paper_2304_09180_amd import clot, thrombus2d
    d = thrombus2d.channel()
    over = dict(ddt_psi=0.9, max_co=0.75)
    prec = getattr(clot, prec_name)
    s = clot.Solver([d], prec, clot.default_params(prec, **over))
    n = d["nx"] * d["ny"]
    nf = s.count(0, "E0")
    s.init_state(0, np.zeros((15, n)), np.zeros((2, nf)))
    s.step(12)
    g, st = s.fields(0), s.stats(0)
    s.close()
    o = oc.Oracle(d, np.zeros((15, n)), np.zeros((2, nf)), oc.Params(**over))
    for _ in range(12):
        o.step()
    print(prec_name, st, flush=True)
    ref = o.fields()
    if prec == clot.FP64:
        compare(g, ref, tol)
    else:   # the FP32 contract: velocity and species (pressure is reported, not bound)
        compare(g, ref, 1.0, names=["P"])
        assert velocity_err(g, ref, 2) < tol
        compare(g, ref, tol, names=FP32_NAMES)
    assert st["t"] == pytest.approx(o.t, rel=1e-12 if prec == clot.FP64 else 1e-6)
