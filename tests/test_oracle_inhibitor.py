"""CPU pins of the oracle's inhibitor variant (section 3.4: a fluid-phase inhibitor I that
binds thrombin for good, I + E2 -> E2i, rate k_I I E2; the two species are appended to
the 15 and both are transported).

Pins: the reaction step keeps I + E2i and the prothrombin family with E2i exactly; with
only I and E2 present it follows the closed form of second-order A + B -> C kinetics; and
with k_I = 0 the variant is the base model bit for bit, I staying at its inlet value."""
import numpy as np

import clot_inputs as ci
from oracle import clot_oracle as oc
from test_oracle_pins import random_states


def test_inhibitor_reaction_keeps_its_linear_invariants():
    p = oc.Params(inhibitor=True)
    rng = np.random.default_rng(13)
    y14, adp, gam, hadh = random_states(200, rng)
    extra = np.array([rng.uniform(0.2, 1.0, y14.shape[1]) * p.I_0, rng.uniform(0.0, 1e-4, y14.shape[1])])
    y = np.vstack([y14, extra])
    f = lambda v: oc.reaction_rhs(v, adp, gam, hadh, p)
    z = oc.rk4(f, y.copy(), 5e-5, 2)
    R = {n: i for i, n in enumerate(oc.RXN + oc.INHIBITOR_SPECIES)}
    fam = {
        "platelets": ["Pmu", "Pma", "Pba", "Pbse"],
        "X": ["S1", "S1b", "E1", "E1b", "C1", "C2"],
        "II with the inhibited thrombin": ["S2", "S2b", "E2", "E2b", "C1", "C2", "E2i"],
        "inhibitor": ["I", "E2i"],
    }
    for name, members in fam.items():
        a = sum(y[R[s]] for s in members)
        b = sum(z[R[s]] for s in members)
        assert np.allclose(a, b, rtol=1e-14, atol=0), name
    # the inhibitor does act: E2i grows wherever I and E2 meet
    assert np.all(z[R["E2i"]] > y[R["E2i"]])


def test_inhibitor_follows_second_order_kinetics():
    """Only I and E2 present (no platelets, so no binding sites and no activation):
    dI/dt = dE2/dt = -k I E2, whose solution with D = I0 - E2_0 is
    I(t) = D I0 / (I0 - E2_0 exp(-k D t))."""
    p = oc.Params(inhibitor=True, k_I=71.0)      # fast enough to travel far in T
    n = 3
    y = np.zeros((16, n))
    I0 = np.array([3.4e-3, 1.0e-3, 2.0e-4])
    E0 = np.array([1.0e-3, 3.0e-3, 1.5e-4])
    y[14] = I0
    y[7] = E0
    z = np.zeros(n)
    f = lambda v: oc.reaction_rhs(v, z, z, z, p)
    T, steps = 40.0, 4000
    yT = y.copy()
    for _ in range(steps):
        yT = oc.rk4(f, yT, T / steps, 1)
    D = I0 - E0
    I_exact = D * I0 / (I0 - E0 * np.exp(-p.k_I * D * T))
    assert np.allclose(yT[14], I_exact, rtol=1e-9, atol=0)
    assert np.allclose(yT[7], I_exact - D, rtol=1e-8, atol=1e-15)
    assert np.allclose(yT[15], I0 - yT[14], rtol=1e-12, atol=0)
    # the reaction travels far in T (the check is not on a flat start)
    assert np.any(yT[14] < 0.75 * I0)


def test_zero_rate_inhibitor_is_the_base_model():
    desc = ci.channel(2, 40, 12, shear=1000.0, dt=1e-4, seed=3)
    xc, xf = ci.noise(desc)
    base = oc.Oracle(desc, xc, xf)
    var = oc.Oracle(desc, xc, xf, oc.Params(inhibitor=True, k_I=0.0))
    for _ in range(4):
        base.step()
        var.step()
    fb, fv = base.fields(), var.fields()
    for k, v in fb.items():
        assert np.array_equal(v, fv[k]), k
    assert np.allclose(fv["I"], oc.Params().I_0, rtol=1e-12, atol=0)
    assert np.abs(fv["E2I"]).max() == 0.0
