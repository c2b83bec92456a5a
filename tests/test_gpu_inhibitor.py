"""GPU parity of the inhibitor build (section 3.4's extensibility example: I + E2 -> E2i,
two more transported and reacting species) through the C ABI against the FP64 oracle
run with the same species added.

The seeded start puts thrombin, the inhibitor and the inhibited thrombin into the
channel on both sides (thrombin is absent from the ordinary start), so the new reaction,
the transport of two more scalars, the inhibitor's inlet value and the 9-system batched
transport solve all act within the few steps the oracle affords.  With k_I = 0 the build
must reproduce the base library bit for bit."""
import numpy as np
import pytest

import clot_inputs as ci
from parity_util import compare

pytestmark = pytest.mark.gpu

I_0 = 3.4e-3


def seeded_extra(d, seed, e2i=True):
    """Thrombin, inhibitor and (or not) inhibited thrombin of the start, cells x-fastest."""
    n = d["nx"] * d["ny"] * d["nz"]
    rng = np.random.default_rng(seed)
    out = {"E2": 2e-4 * (1.0 + 0.5 * rng.uniform(-1, 1, n)),
           "I": I_0 * (0.5 + rng.uniform(0, 1, n))}
    if e2i:
        out["E2I"] = 1e-5 * rng.uniform(0, 1, n)
    return out


def run_oracle(d, steps, extra=None, **over):
    from oracle import clot_oracle as oc
    xc, xf = ci.noise(d)
    o = oc.Oracle(d, xc, xf, oc.Params(inhibitor=True, **over))
    by_field = {n.upper(): i for n, i in o.sp.items()}      # field names are upper case
    for name, v in (extra or {}).items():
        o.c[by_field[name]] = v.copy()
    for _ in range(steps):
        o.step()
    return o.fields()


def run_gpu(d, prec, steps, extra=None, inhibitor=True, **over):
    from paper_2304_09180_amd import clot
    s = clot.Solver([d], prec, clot.default_params(prec, **over), inhibitor=inhibitor)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    for name, v in (extra or {}).items():
        s.set(0, name, v)
    s.step(steps)
    g, st = s.fields(0), s.stats(0)
    s.close()
    return g, st


CASES = {
    "2d_ragged": (ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=41), 5),
    "3d_ragged": (ci.channel(3, 24, 10, 9, shear=800.0, seed=42), 4),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_inhibitor_matches_oracle(name):
    from paper_2304_09180_amd import clot
    d, steps = CASES[name]
    # 2-D: E2i starts at zero, so all of it comes from the new reaction; 3-D: a seeded
    # E2i field is transported as well
    extra = seeded_extra(d, 7, e2i=name.startswith("3d"))
    g, st = run_gpu(d, clot.FP64, steps, extra)
    print(name, st, flush=True)
    assert st["status"] == "OK"
    ref = run_oracle(d, steps, extra)
    assert set(ref) >= {"I", "E2I"}
    if "E2I" not in extra:
        assert ref["E2I"].min() >= 0.0 and ref["E2I"].max() > 1e-10
    compare(g, ref, 1e-10)


def test_fp64_inhibitor_fast_rate_matches_oracle():
    """k_I 1e5 times the default: thrombin falls to a fraction of its start within the
    steps, so the coupling of the new pair to the thrombin family is exercised hard."""
    from paper_2304_09180_amd import clot
    d, steps = CASES["2d_ragged"]
    extra = seeded_extra(d, 8)
    g, st = run_gpu(d, clot.FP64, steps, extra, k_I=7.1e5)
    assert st["status"] == "OK"
    ref = run_oracle(d, steps, extra, k_I=7.1e5)
    assert ref["E2"].mean() < 0.7 * extra["E2"].mean()
    compare(g, ref, 1e-10)


def test_fp32_inhibitor_matches_oracle():
    from paper_2304_09180_amd import clot
    d, steps = CASES["2d_ragged"]
    extra = seeded_extra(d, 9)
    g, st = run_gpu(d, clot.FP32_MIXED, steps, extra)
    print(st, flush=True)
    assert st["status"] == "OK"
    compare(g, run_oracle(d, steps, extra), 1e-5)


def test_zero_rate_inhibitor_build_is_the_base_library():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=43)
    for prec in (clot.FP64, clot.FP32_MIXED):
        base, _ = run_gpu(d, prec, 4, inhibitor=False)
        var, st = run_gpu(d, prec, 4, k_I=0.0)
        assert st["status"] == "OK"
        for k, v in base.items():
            assert np.array_equal(v, var[k]), (prec, k, np.abs(v - var[k]).max())
        assert np.allclose(var["I"], I_0, rtol=1e-12 if prec == clot.FP64 else 1e-6, atol=0)
        assert np.abs(var["E2I"]).max() == 0.0


def test_inhibitor_build_refusals_and_base_build_fields():
    from paper_2304_09180_amd import clot
    d = ci.channel(2, 16, 8, shear=1000.0, dt=1e-4, seed=44)
    xc, xf = ci.noise(d)
    s = clot.Solver([d], clot.FP64, inhibitor=True)
    s.init_state(0, xc, xf)
    blob = np.full(s.lib.clot_mlp_nparam() + 28, 0.01, np.float32)   # accepted by the base build
    with pytest.raises(clot.ClotError):       # the learned step covers the base model only
        s.set_reaction_mode(clot.SURROGATE, blob, 1e-3)
    with pytest.raises(clot.ClotError):       # 17 draws per cell are not the interface
        s.init_state(0, np.zeros((17, xc.shape[1])), xf)
    assert s.count(0, "I") == s.count(0, "E2I") == d["nx"] * d["ny"]
    s.close()
    b = clot.Solver([d], clot.FP64)
    b.init_state(0, xc, xf)
    for name in ("I", "E2I"):
        with pytest.raises(clot.ClotError):
            b.get(0, name)
    b.close()


def test_inhibitor_stats_minimum_covers_the_added_species():
    """clot_stats' min_species over all 17 species, each over its scale, against the
    same minimum computed from the fields read back; a negative inhibitor value in the
    start makes the added species the minimum."""
    from paper_2304_09180_amd import clot
    d, _ = CASES["2d_ragged"]
    extra = seeded_extra(d, 10)
    extra["I"][17] = -0.25 * I_0
    g, st = run_gpu(d, clot.FP64, 1, extra)
    p = clot.default_params(clot.FP64)
    scale = {"PMU": p.P_max, "PMA": p.P_max, "PBA": p.P_max, "PBSE": p.P_max, "ADP": p.adp_crit,
             "S1": p.S1_0, "S2": p.S2_0, "E1": p.S1_0, "E2": p.S2_0, "S1B": p.S1_0, "S2B": p.S2_0,
             "E1B": p.S1_0, "E2B": p.S2_0, "C1": p.S2_0, "C2": p.S2_0, "I": p.I_0, "E2I": p.S2_0}
    mins = {n: (g[n] / s).min() for n, s in scale.items()}
    print(st["min_species"], min(mins.items(), key=lambda kv: kv[1]))
    assert min(mins, key=mins.get) == "I"
    assert st["min_species"] == pytest.approx(min(mins.values()), rel=1e-9)


def test_inhibitor_batched_uneven_channels_and_graph_replay():
    """Three uneven channels in one context of the inhibitor build: each equals the
    oracle run alone (FP64), and whole steps replayed as HIP graphs equal the eager
    steps bit for bit (the 9-system transport solve inside the recorded step)."""
    from paper_2304_09180_amd import clot
    descs = [ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=45),
             ci.channel(2, 24, 8, shear=600.0, dt=1e-4, seed=46, inj_frac=0.4),
             ci.channel(3, 12, 6, 5, shear=900.0, dt=1e-4, seed=47)]
    extras = [seeded_extra(d, 50 + c) for c, d in enumerate(descs)]

    def make(prec):
        s = clot.Solver(descs, prec, clot.default_params(prec), inhibitor=True)
        for c, d in enumerate(descs):
            xc, xf = ci.noise(d)
            s.init_state(c, xc, xf)
            for name, v in extras[c].items():
                s.set(c, name, v)
        return s

    s = make(clot.FP64)
    s.step(3)
    for c, d in enumerate(descs):
        assert s.stats(c)["status"] == "OK"
        compare(s.fields(c), run_oracle(d, 3, extras[c]), 1e-10)
    s.close()
    for prec in (clot.FP32_MIXED, clot.FP64):
        eager, graph = make(prec), make(prec)
        graph.set_graph_mode(True, 1.25, 2)
        for step in range(5):
            eager.step(1)
            graph.step(1)
            for c in range(len(descs)):
                fe, fg = eager.fields(c), graph.fields(c)
                for name in fe:
                    assert np.array_equal(fe[name], fg[name]), (prec, step, c, name)
        info = graph.graph_info()
        assert info["captures"] == 2 and info["replays"] == 3 and info["overflows"] == 0, info
        eager.close()
        graph.close()
