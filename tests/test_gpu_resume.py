"""Checkpoint and resume through the C ABI, and failure reporting forced from the host.

A state saved after k steps and loaded (into the same context or a fresh one) must
continue bit for bit as the saved context does; the state exercised here carries the
Crank-Nicolson history, the variable step, a release history with several snapshots and
the buffer parity.  Failures: non-finite values refused by clot_set_field, a solve that
overflows FP32, and a solve allowed a single iteration."""
import numpy as np
import pytest

import clot_inputs as ci

pytestmark = pytest.mark.gpu

DESCS = [ci.channel(2, 40, 12, shear=1000.0, dt=4e-4, seed=21, inj_frac=0.3),
         ci.channel(2, 64, 16, shear=600.0, dt=4e-4, seed=22, inj_frac=0.45)]
OVER = dict(ddt_psi=0.9, max_co=0.75, dtau=2.5e-4, tau_f=6e-3, A_hat=1e3)


def make(prec_name, graph=False):
    from paper_2304_09180_amd import clot
    prec = getattr(clot, prec_name)
    s = clot.Solver(DESCS, prec, clot.default_params(prec, **OVER))
    for c, d in enumerate(DESCS):
        xc, xf = ci.noise(d)
        s.init_state(c, xc, xf)
    if graph:
        s.set_graph_mode(True, 1.25, 2)
    return s


def snapshot(s):
    return [s.fields(c) for c in range(len(DESCS))], [s.stats(c) for c in range(len(DESCS))]


def same(a, b):
    for c in range(len(DESCS)):
        for name in a[0][c]:
            assert np.array_equal(a[0][c][name], b[0][c][name]), (c, name)
        for k in ("steps", "t", "dt", "it_mom", "it_p", "it_tr"):
            assert a[1][c][k] == b[1][c][k], (c, k)


@pytest.mark.parametrize("prec_name,graph", [("FP32_MIXED", False), ("FP64", False), ("FP32_MIXED", True)])
def test_resume_continues_bit_for_bit(prec_name, graph):
    a = make(prec_name)
    a.step(5)
    blob = a.save_state()
    a.step(5)                       # an odd count: the buffer parity differs from the saved one
    want = snapshot(a)
    assert want[1][0]["steps"] == 10 and np.abs(want[0][0]["SIGMA"]).max() > 0.0
    b = make(prec_name, graph)      # a fresh context, in graph mode or not
    b.step(2)                       # whatever it holds is replaced
    b.load_state(blob)
    b.step(5)
    same(want, snapshot(b))
    a.load_state(blob)              # back into the context that saved it
    a.step(5)
    same(want, snapshot(a))
    a.close()
    b.close()


def test_load_state_refuses_another_layout():
    from paper_2304_09180_amd import clot
    a = make("FP64")
    a.step(1)
    blob = a.save_state()
    other = clot.Solver([DESCS[0]], clot.FP64, clot.default_params(clot.FP64, **OVER))
    with pytest.raises(clot.ClotError):
        other.load_state(blob)
    f32 = make("FP32_MIXED")
    with pytest.raises(clot.ClotError):
        f32.load_state(blob)
    with pytest.raises(clot.ClotError):
        a.load_state(blob[:-1])
    before = a.fields(0)["UX"].copy()
    a.step(1)                       # still usable after the refusals
    assert not np.array_equal(before, a.fields(0)["UX"])
    for s in (a, other, f32):
        s.close()


def test_non_finite_values_are_refused_at_the_boundary():
    from paper_2304_09180_amd import clot
    d = DESCS[0]
    s = clot.Solver([d], clot.FP32_MIXED)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    u = s.get(0, "UX")
    for bad in (np.nan, np.inf):
        v = u.copy()
        v[len(v) // 2] = bad
        with pytest.raises(clot.ClotError):
            s.set(0, "UX", v)
        assert np.array_equal(s.get(0, "UX"), u)
    s.close()


def test_overflow_in_a_solve_is_reported_and_cleared_by_reinitialisation():
    """A finite velocity near the FP32 limit passes the boundary; the FP32 pressure
    solve it drives (p ~ 1e40) overflows, and the step must say so rather than OK (the
    solve stops at the first non-finite sum, so its vector can still read finite)."""
    from paper_2304_09180_amd import clot
    d = DESCS[0]
    s = clot.Solver([d], clot.FP32_MIXED)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    s.step(1)
    assert s.stats(0)["status"] == "OK"
    u = s.get(0, "UX")
    u[len(u) // 2] = 3e38
    s.set(0, "UX", u)
    s.step(1)
    f = s.fields(0)
    nonfinite = [n for n, v in f.items() if not np.isfinite(v).all()]
    print("non-finite fields", nonfinite, s.stats(0)["status"])
    assert s.stats(0)["status"] == "W_NONFINITE"
    s.init_state(0, xc, xf)
    s.step(1)
    assert s.stats(0)["status"] == "OK"
    s.close()


def test_single_iteration_solves_report_not_converged():
    from paper_2304_09180_amd import clot
    d = DESCS[0]
    s = clot.Solver([d], clot.FP64, clot.default_params(clot.FP64, max_iter=1))
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    s.step(1)
    st = s.stats(0)
    print(st)
    assert st["status"] == "W_NOTCONV"
    assert np.isfinite(s.get(0, "UX")).all()
    s.close()
