"""Whole steps replayed as HIP graphs against eager steps, on an uneven batch of
channels (sizes, shear rates and injury lengths drawn as for the ensemble workload)."""
import numpy as np
import pytest

import clot_inputs as ci

pytestmark = pytest.mark.gpu


def _solver(descs, prec):
    from paper_2304_09180_amd import clot
    s = clot.Solver(descs, prec)
    for c, d in enumerate(descs):
        xc, xf = ci.noise(d)
        s.init_state(c, xc, xf)
    return s


def _members(n):
    # the ensemble's draws with every grid a quarter of its size per axis, so that
    # the check runs in seconds
    out = []
    for d in ci.ensemble(n):
        out.append(ci.channel(2, d["nx"] // 4, d["ny"] // 4, shear=d["shear"], seed=d["seed"],
                              inj_frac=(d["inj_x1"] - d["inj_x0"]) / d["Lx"]))
    return out


@pytest.mark.parametrize("prec_name", ["FP32_MIXED", "FP64"])
def test_graph_replay_matches_eager_bitwise(prec_name):
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    descs = _members(5)
    eager = _solver(descs, prec)
    graph = _solver(descs, prec)
    graph.set_graph_mode(True, 1.25, 2)
    for step in range(8):
        print(f"step {step} {prec_name}", flush=True)
        eager.step(1)
        graph.step(1)
        for c in range(len(descs)):
            fe, fg = eager.fields(c), graph.fields(c)
            for name in fe:
                assert np.array_equal(fe[name], fg[name]), (step, c, name)
    info = graph.graph_info()
    print(info)
    assert info["captures"] == 2 and info["replays"] == 6 and info["overflows"] == 0
    for c in range(len(descs)):
        se, sg = eager.stats(c), graph.stats(c)
        assert se["status"] == sg["status"] == "OK"
        for k in ("it_mom", "it_p", "it_eta", "it_tr", "refine_p", "steps"):
            assert se[k] == sg[k], (c, k)
    eager.close()
    graph.close()


def test_graph_budget_overflow_is_reported_and_widened():
    from paper_2304_09180_amd import clot
    descs = _members(3)
    s = _solver(descs, clot.FP32_MIXED)
    s.set_graph_mode(True, 0.0, 1)      # one iteration per solve: certain to fall short
    s.step(3)                           # two calibrating eager steps, then one replay
    info = s.graph_info()
    assert info["replays"] == 1 and info["overflows"] == 1
    assert s.stats(0)["status"] == "W_NOTCONV"
    s.step(1)                           # re-recorded with a wider budget
    assert s.graph_info()["captures"] == 2
    s.set_graph_mode(False)
    s.step(1)
    assert np.isfinite(s.get(0, "UX")).all()
    s.close()


@pytest.mark.parametrize("prec_name", ["FP32_MIXED", "FP64"])
def test_graph_replay_of_3d_channels_matches_eager_bitwise(prec_name):
    """An all-3-D context (three Jacobi sweeps each way in the pressure V-cycle by
    default, weight 6/7): recorded steps equal the eager ones bit for bit."""
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    descs = [ci.channel(3, 24, 10, 9, shear=800.0, dt=1e-4, seed=61),
             ci.channel(3, 40, 12, 12, shear=1200.0, dt=1e-4, seed=62, inj_frac=0.4)]
    eager = _solver(descs, prec)
    graph = _solver(descs, prec)
    graph.set_graph_mode(True, 1.25, 2)
    for step in range(6):
        print(f"step {step} {prec_name}", flush=True)
        eager.step(1)
        graph.step(1)
        for c in range(len(descs)):
            fe, fg = eager.fields(c), graph.fields(c)
            for name in fe:
                assert np.array_equal(fe[name], fg[name]), (step, c, name)
    info = graph.graph_info()
    assert info["replays"] == 4 and info["overflows"] == 0, info
    for c in range(len(descs)):
        assert eager.stats(c)["it_p"] == graph.stats(c)["it_p"]
    eager.close()
    graph.close()
