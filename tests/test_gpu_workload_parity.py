"""The GPU path against the FP64 oracle at the workloads' full sizes and step counts.

The goldens (tests/golden/<workload>_step<N>.npz) are written by
tests/golden/make_workload_goldens.py, which runs the oracle and nothing else: per
field the full-field norm and the values at a seeded cell sample (the wall band over
the injury, where the coagulation species live, plus uniform draws), and the injury
faces' E0, C0 in full.  The GPU runs the same seeded workload for the same steps:
  * the 1024x256 channel for its 1000 steps and the 1M-cell duct at its checkpoints,
    FP32 mixed, within 1e-5 (velocity as one vector, each of the 15 species);
  * the 64-member ensemble, FP32, one member of each size at steps 100 and 500;
  * the learned reaction step on the duct against the same oracle, within 1e-3 on
    every field.
"""
import glob
import os

import numpy as np
import pytest

import clot_inputs as ci
from parity_util import compare_golden, load_golden

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def goldens(prefix):
    out = []
    for p in glob.glob(os.path.join(GOLD, prefix + "_step*.npz")):
        out.append((int(p.rsplit("_step", 1)[1][:-4]), p))
    return sorted(out)


def run_and_compare(desc, checkpoints, tol, blob=None):
    """Steps one channel through the checkpoints, comparing each with its golden."""
    from paper_2304_09180_amd import clot
    s = clot.Solver([desc], clot.FP32_MIXED)
    xc, xf = ci.noise(desc)
    s.init_state(0, xc, xf)
    if blob is not None:
        s.set_reaction_mode(clot.SURROGATE, blob, 1e-3)
    done, failures = 0, {}
    for n, path in checkpoints:
        s.step(n - done)
        done = n
        meta, g = load_golden(path)
        assert meta["steps"] == n and meta["desc"]["nx"] == desc["nx"]
        st = s.stats(0)
        print(os.path.basename(path), "status", st["status"], "it_mom", st["it_mom"], "it_p", st["it_p"][:3],
              "fallback", st["fallback_frac"], flush=True)
        assert st["status"] == "OK", st
        _, bad = compare_golden(s.fields(0), meta, g, tol)
        if bad:
            failures[n] = bad
    s.close()
    return failures


@pytest.mark.parametrize("name", ["channel2d_1024x256", "channel3d_256x64x64"])
def test_fp32_path_matches_the_oracle_at_full_size(name):
    gs = goldens(name)
    assert gs, f"no oracle golden for {name}"
    failures = run_and_compare(ci.workload(name), gs, 1e-5)
    assert not failures, failures


def test_ensemble_members_match_the_oracle():
    """The whole 64-member ensemble steps together (FP32); one member of each size is
    compared with its own oracle run."""
    from paper_2304_09180_amd import clot
    descs = ci.ensemble(64)
    marks = {}
    for p in glob.glob(os.path.join(GOLD, "ensemble64_member*_step*.npz")):
        base = os.path.basename(p)
        m = int(base.split("member")[1].split("_")[0])
        marks.setdefault(int(base.rsplit("_step", 1)[1][:-4]), []).append((m, p))
    assert marks, "no ensemble goldens"
    sizes = {(descs[m]["nx"], descs[m]["ny"]) for ms in marks.values() for m, _ in ms}
    assert len(sizes) == 3, sizes
    s = clot.Solver(descs, clot.FP32_MIXED)
    for c, d in enumerate(descs):
        xc, xf = ci.noise(d)
        s.init_state(c, xc, xf)
    done, failures = 0, {}
    for n in sorted(marks):
        s.step(n - done)
        done = n
        for m, path in sorted(marks[n]):
            meta, g = load_golden(path)
            assert meta["steps"] == n and meta["desc"]["seed"] == descs[m]["seed"]
            assert s.stats(m)["status"] == "OK"
            print(f"member {m} ({descs[m]['nx']}x{descs[m]['ny']}) step {n}", flush=True)
            _, bad = compare_golden(s.fields(m), meta, g, 1e-5)
            if bad:
                failures[(m, n)] = bad
    s.close()
    assert not failures, failures


def test_learned_reaction_step_matches_the_oracle_on_the_duct():
    """The duct with the surrogate reaction step (trained here on the GPU) against the
    oracle's plain-RK4 run of the same workload: every field within 1e-3."""
    from paper_2304_09180_amd import surrogate
    gs = goldens("channel3d_256x64x64")
    assert gs, "no oracle golden for the duct"
    d1 = ci.workload("channel2d_64x16")
    states = surrogate.collect_states([(d1, 100)], log=lambda *a: None)
    tr = surrogate.Trainer(surrogate.sample_rows(states, 100_000), log=lambda *a: None)
    tr.train(epochs=6)
    failures = run_and_compare(ci.workload("channel3d_256x64x64"), gs, 1e-3, blob=tr.blob())
    assert not failures, failures
