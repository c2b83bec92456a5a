"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

import clot_inputs as ci
from parity_util import SCALE, VECTOR, compare, rel_l2  # noqa: F401

pytestmark = pytest.mark.gpu


def run_gpu(descs, precision, steps, params=None):
    from paper_2304_09180_amd import clot
    s = clot.Solver(descs, precision, params)
    for i, d in enumerate(descs):
        xc, xf = ci.noise(d)
        s.init_state(i, xc, xf)
    s.step(steps)
    out = [s.fields(i) for i in range(len(descs))]
    st = [s.stats(i) for i in range(len(descs))]
    s.close()
    return out, st


def run_oracle(d, steps):
    from oracle import clot_oracle as oc
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf)
    for _ in range(steps):
        o.step()
    return o.fields()


def velocity_err(gpu, ref, dim):
    comps = ["UX", "UY"] + (["UZ"] if dim == 3 else [])
    a = np.concatenate([gpu[c] for c in comps])
    b = np.concatenate([ref[c] for c in comps])
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("shape", [(40, 12), (72, 20)])
def test_fp64_2d_ragged_few_steps(shape):
    from paper_2304_09180_amd import clot
    d = ci.channel(2, shape[0], shape[1], shear=1000.0, dt=1e-4, steps=5, seed=3)
    (g,), (st,) = run_gpu([d], clot.FP64, 5)
    print(st, flush=True)
    ref = run_oracle(d, 5)
    compare(g, ref, 1e-10)


def test_fp64_3d_ragged_few_steps():
    from paper_2304_09180_amd import clot
    d = ci.channel(3, 24, 10, 9, shear=800.0, steps=4, seed=5)
    (g,), (st,) = run_gpu([d], clot.FP64, 4)
    print(st, flush=True)
    ref = run_oracle(d, 4)
    compare(g, ref, 1e-10)


def test_fp64_channel2d_64x16_100_steps():
    from paper_2304_09180_amd import clot
    d = ci.workload("channel2d_64x16")
    (g,), (st,) = run_gpu([d], clot.FP64, d["steps"])
    print(st, flush=True)
    ref = run_oracle(d, d["steps"])
    assert velocity_err(g, ref, 2) < 1e-10
    compare(g, ref, 1e-10)


def test_fp32_mixed_2d_50_steps():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, steps=50, seed=4)
    (g,), (st,) = run_gpu([d], clot.FP32_MIXED, 50)
    print(st, flush=True)
    ref = run_oracle(d, 50)
    assert velocity_err(g, ref, 2) < 1e-5
    compare(g, ref, 1e-5, names=["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B",
                                 "E2B", "C1", "C2", "E0", "C0"])


def test_fp32_mixed_3d_ragged_20_steps():
    """The FP32 path on a ragged 3-D duct (tiles cut across rows and planes)."""
    from paper_2304_09180_amd import clot
    d = ci.channel(3, 24, 10, 9, shear=800.0, seed=5)
    (g,), (st,) = run_gpu([d], clot.FP32_MIXED, 20)
    print(st, flush=True)
    ref = run_oracle(d, 20)
    assert velocity_err(g, ref, 3) < 1e-5
    compare(g, ref, 1e-5, names=["PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2", "S1B", "S2B", "E1B",
                                 "E2B", "C1", "C2", "E0", "C0"])


def test_fp64_batched_uneven_channels_match_single_runs():
    from paper_2304_09180_amd import clot
    ds = [ci.channel(2, 32, 8, shear=300.0, steps=3, seed=11, inj_frac=0.3),
          ci.channel(2, 48, 12, shear=1500.0, steps=3, seed=12, inj_frac=0.15),
          ci.channel(2, 64, 16, shear=700.0, steps=3, seed=13, inj_frac=0.45)]
    gs, sts = run_gpu(ds, clot.FP64, 3)
    for d, g in zip(ds, gs):
        # each channel keeps its own dt; run the oracle with that channel alone
        ref = run_oracle(d, 3)
        compare(g, ref, 1e-10)


def test_fp64_release_history_pushes_match_oracle():
    """A release-history schedule short enough to push a snapshot every two or three
    steps (dtau = 2.5e-4 s, tau_f = 24 dtau) and a large A_hat, so that sigma and ADP
    carry the trapezoid of several snapshots of different ages."""
    from oracle import clot_oracle as oc
    from paper_2304_09180_amd import clot
    over = dict(dtau=2.5e-4, tau_f=6e-3, A_hat=1e3)
    d = ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=21)
    steps = 12
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf, oc.Params(**over))
    for _ in range(steps):
        o.step()
    ref = o.fields()
    assert np.abs(ref["SIGMA"]).max() > 0.0
    gpu, st = run_gpu([d], clot.FP64, steps, clot.default_params(clot.FP64, **over))
    compare(gpu[0], ref, 1e-10)


def test_release_history_length_is_checked():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, seed=21)
    with pytest.raises(clot.ClotError):
        clot.Solver([d], clot.FP64, clot.default_params(clot.FP64, dtau=0.5))


@pytest.mark.parametrize("prec_name,descs,sweeps", [
    ("FP32_MIXED", [ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=5)], None),
    ("FP32_MIXED", [ci.channel(3, 48, 16, 16, shear=800.0, dt=5e-5, seed=6)], None),
    ("FP64", [ci.channel(2, 40, 12, seed=7), ci.channel(2, 128, 32, shear=400.0, seed=8)], None),
    ("FP32_MIXED", [ci.channel(3, 48, 16, 16, shear=800.0, dt=5e-5, seed=6)], 2),
    ("FP64", [ci.channel(2, 40, 12, seed=7), ci.channel(2, 128, 32, shear=400.0, seed=8)], 3),
    ("FP32_MIXED", [ci.channel(3, 48, 16, 16, shear=800.0, dt=5e-5, seed=6)], 4),
    ("FP64", [ci.channel(2, 40, 12, seed=7), ci.channel(2, 128, 32, shear=400.0, seed=8)], 1),
])
def test_fused_multigrid_tail_is_bitwise_equal_to_separate_launches(prec_name, descs, sweeps):
    """The small levels of the pressure V-cycle in one launch (default) against one
    launch per level and pass (mg_tail = 0), with the automatic sweep count (3 on 3-D
    channels, 2 on 2-D ones) and the others."""
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    over = {} if sweeps is None else {"mg_sweeps": sweeps}
    fused, _ = run_gpu(descs, prec, 6, clot.default_params(prec, **over))
    sep, _ = run_gpu(descs, prec, 6, clot.default_params(prec, mg_tail=0, **over))
    for c in range(len(descs)):
        for name in fused[c]:
            assert np.array_equal(fused[c][name], sep[c][name]), (c, name)


@pytest.mark.parametrize("prec_name,descs,over", [
    ("FP32_MIXED", [ci.channel(3, 96, 32, 32, shear=800.0, dt=5e-5, seed=6)], {}),
    ("FP32_MIXED", [ci.channel(3, 48, 16, 16, shear=800.0, dt=5e-5, seed=6)], {"mg_tail": 0}),
    ("FP32_MIXED", [ci.channel(3, 37, 13, 11, shear=900.0, dt=5e-5, seed=9)], {"mg_sweeps": 2, "mg_tail": 0}),
    ("FP32_MIXED", [ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=5), ci.channel(2, 130, 34, shear=400.0, seed=8)],
     {"mg_tail": 0}),
    ("FP32_MIXED", [ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=5)], {"mg_sweeps": 3, "mg_tail": 0}),
    ("FP32_MIXED", [ci.channel(3, 37, 13, 11, shear=900.0, dt=5e-5, seed=9), ci.channel(2, 130, 34, shear=400.0, seed=8)],
     {"mg_sweeps": 3}),
    ("FP64", [ci.channel(3, 37, 13, 11, shear=900.0, dt=5e-5, seed=9)], {}),
    ("FP64", [ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=5), ci.channel(2, 130, 34, shear=400.0, seed=8)], {}),
])
def test_pressure_bricks_are_bitwise_equal_to_separate_launches(prec_name, descs, over):
    """The brick-ordered legs of the pressure V-cycle (default, mg_brick = 1: the mesh's
    restriction and prolongation, and in FP32 the LDS-staged legs of the coarse levels
    and the mesh's legs in one launch each: the down leg's three sweeps, or two sweeps
    and the restriction; with three, the up leg's prolongation and next sweep) against
    the general separate launches (mg_brick = 0): every cell value is formed by the same
    expression, halo cells included, so the steps agree bit for bit.  In FP32 also checks
    that the staged legs ran (the probes count launches)."""
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    sweeps = over.get("mg_sweeps", 3 if all(d["dim"] == 3 for d in descs) else 2)
    runs = []
    for brick in (1, 0):
        s = clot.Solver(descs, prec, clot.default_params(prec, mg_brick=brick, **over))
        for i, d in enumerate(descs):
            xc, xf = ci.noise(d)
            s.init_state(i, xc, xf)
        s.probe("p_mg_down")
        s.step(2)
        _, n = s.probe_read()
        s.probe("p_mg_mesh_down")
        s.step(2)
        _, n3 = s.probe_read()
        s.probe("p_mg_mesh_up")
        s.step(2)
        _, nu = s.probe_read()
        s.probe(None)
        staged = brick == 1 and prec == clot.FP32_MIXED
        assert (n > 0) == staged, (brick, n)
        assert (n3 > 0) == (staged and sweeps in (2, 3)), (brick, n3)
        assert (nu > 0) == (staged and sweeps == 3), (brick, nu)
        runs.append([s.fields(i) for i in range(len(descs))])
        s.close()
    for c in range(len(descs)):
        for name in runs[0][c]:
            assert np.array_equal(runs[0][c][name], runs[1][c][name]), (c, name)


@pytest.mark.parametrize("descs,steps", [
    ([ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=11)], 5),
    ([ci.channel(3, 24, 10, 9, shear=1000.0, dt=1e-4, seed=12), ci.channel(2, 128, 32, shear=400.0, seed=13)], 4),
])
@pytest.mark.parametrize("sweeps", [1, 3, 4])
def test_fp64_multigrid_sweep_counts_match_oracle(descs, steps, sweeps):
    """The pressure preconditioner with 1, 3 or 4 Jacobi sweeps each way changes only
    the iteration count: the converged step still matches the oracle."""
    from paper_2304_09180_amd import clot
    gpu, st = run_gpu(descs, clot.FP64, steps, clot.default_params(clot.FP64, mg_sweeps=sweeps))
    for c, d in enumerate(descs):
        print(sweeps, c, st[c]["it_p"], flush=True)
        compare(gpu[c], run_oracle(d, steps), 1e-10)


@pytest.mark.parametrize("mom_mg", [0, 1])
@pytest.mark.parametrize("case", ["2d", "3d", "2d_high_D"])
def test_fp64_momentum_preconditioners_match_oracle(case, mom_mg):
    """The momentum predictor with either preconditioner (one multigrid V-cycle per
    BiCGStab direction, or Jacobi) against the oracle; the multigrid solve needs fewer
    iterations.  "2d_high_D": a 256x64 channel at shear 100 s^-1 and dt 1e-4 s, viscous
    diffusion number nu dt/h^2 = 17 (four coarse momentum levels)."""
    from paper_2304_09180_amd import clot
    if case == "2d":
        d, steps = ci.channel(2, 72, 20, shear=1000.0, dt=1e-4, seed=4), 6
    elif case == "3d":
        d, steps = ci.channel(3, 24, 10, 9, shear=800.0, seed=5), 4
    else:
        d, steps = ci.channel(2, 256, 64, shear=100.0, dt=1e-4, seed=6), 3
    (g,), (st,) = run_gpu([d], clot.FP64, steps, clot.default_params(clot.FP64, mom_mg=mom_mg))
    print(case, "mom_mg", mom_mg, "it_mom", st["it_mom"], "res_mom", st["res_mom"], flush=True)
    assert st["status"] == "OK"
    ref = run_oracle(d, steps)
    compare(g, ref, 1e-10)
    if case == "2d_high_D":
        assert st["it_mom"] <= (8 if mom_mg else 400)
        if not mom_mg:
            assert st["it_mom"] > 20
