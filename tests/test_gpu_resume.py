"""Checkpoint and resume through the C ABI, and failure reporting forced from the host.

A state saved after k steps and loaded (into the same context or a fresh one) must
continue bit for bit as the saved context does; the state exercised here carries the
Crank-Nicolson history, the variable step, a release history with several snapshots and
the buffer parity.  Failures: non-finite values refused by clot_set_field, a solve that
overflows FP32 (the call rolled back), and a solve allowed a single iteration; channel
indices outside the context and blobs of channels with other physics are refused."""
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


def test_overflow_in_a_solve_rolls_the_call_back():
    """A finite velocity near the FP32 limit passes the boundary; the FP32 pressure
    solve it drives (p ~ 1e40) overflows.  The step call returns CLOT_ENAN and every
    channel is back at the state of the call's start (the planted velocity included);
    the statistics report the failed step.  Re-initialised, the channel steps with its
    usual iteration counts: the failed solve left no inflated counts behind."""
    from paper_2304_09180_amd import clot
    d = DESCS[0]
    s = clot.Solver([d], clot.FP32_MIXED)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    s.step(1)
    normal = s.stats(0)
    assert normal["status"] == "OK"
    u = s.get(0, "UX")
    u[len(u) // 2] = 3e38
    s.set(0, "UX", u)
    before = s.fields(0)
    with pytest.raises(clot.ClotError, match="ENAN"):
        s.step(2)
    after = s.fields(0)
    for n, v in before.items():
        assert np.array_equal(after[n], v), n
    st = s.stats(0)
    assert st["status"] == "W_NONFINITE" and st["steps"] == 1
    s.init_state(0, xc, xf)
    s.step(1)
    again = s.stats(0)
    print(normal["it_mom"], normal["it_p"][:2], again["it_mom"], again["it_p"][:2], flush=True)
    assert again["status"] == "OK"
    assert again["it_mom"] <= normal["it_mom"] + 2 and max(again["it_p"]) <= max(normal["it_p"]) + 2
    s.close()


def test_asynchronous_window_rolls_back_at_sync():
    """Asynchronous steps share one window: clot_sync finds the non-finite value and
    restores the state of the first asynchronous call; a clean window passes."""
    from paper_2304_09180_amd import clot
    d = DESCS[1]
    s = clot.Solver([d], clot.FP32_MIXED)
    xc, xf = ci.noise(d)
    s.init_state(0, xc, xf)
    s.step_async(2)
    s.step_async(1)
    assert s.sync() == 0
    u = s.get(0, "UX")
    u[5] = 3e38
    s.set(0, "UX", u)
    before = s.fields(0)
    s.step_async(1)
    s.step_async(1)
    with pytest.raises(clot.ClotError, match="ENAN"):
        s.sync()
    after = s.fields(0)
    for n, v in before.items():
        assert np.array_equal(after[n], v), n
    assert s.stats(0)["steps"] == 3
    s.close()


def test_channel_index_outside_the_context_is_refused():
    import ctypes
    from paper_2304_09180_amd import clot
    s = make("FP64")
    lib, ctx = s.lib, s.ctx
    buf = np.zeros(10)
    n = ctypes.c_size_t(0)
    st = clot.Stats()
    xc, xf = ci.noise(DESCS[0])
    for bad in (-1, len(DESCS), 1 << 30):
        assert lib.clot_field_count(ctx, bad, clot.FIELD["UX"], ctypes.byref(n)) == -1
        assert lib.clot_get_field(ctx, bad, clot.FIELD["UX"], buf.ctypes.data, buf.size) == -1
        assert lib.clot_set_field(ctx, bad, clot.FIELD["UX"], buf.ctypes.data, buf.size) == -1
        assert lib.clot_get_stats(ctx, bad, ctypes.byref(st)) == -1
        assert lib.clot_init_state(ctx, bad, xc.ctypes.data, xc.size, xf.ctypes.data, xf.size) == -1
        assert b"outside" in lib.clot_last_error(ctx)
    s.step(1)                       # the context is untouched
    assert s.stats(len(DESCS) - 1)["status"] == "OK"
    s.close()


def test_load_state_refuses_a_channel_with_other_physics():
    """Same grids, but another shear rate or injury patch: the blob's channel tables and
    clocks do not belong to this context."""
    from paper_2304_09180_amd import clot
    a = make("FP64")
    a.step(1)
    blob = a.save_state()
    for change in (dict(shear=700.0), dict(inj_frac=0.2)):
        d0 = dict(DESCS[0])
        d1 = ci.channel(2, d0["nx"], d0["ny"], shear=change.get("shear", d0["shear"]), dt=d0["dt"], seed=21,
                        inj_frac=change.get("inj_frac", 0.3))
        other = clot.Solver([d1, DESCS[1]], clot.FP64, clot.default_params(clot.FP64, **OVER))
        with pytest.raises(clot.ClotError, match="EINVAL"):
            other.load_state(blob)
        other.close()
    a.close()


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
