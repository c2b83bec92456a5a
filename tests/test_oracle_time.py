"""CPU pins of the oracle's time integration: the Crank-Nicolson ddt scheme with
off-centring psi and the variable step at a Courant limit (Appendix D, discretization
table and its maxCo statement).

The transport pin is exact: a cosine mode of the zero-gradient diffusion operator
must follow the textbook theta-scheme amplification with theta = 1/(1+psi) after an
implicit-Euler first step, for any sequence of steps.  The momentum pin is exact
too: without pressure correctors the predictor integrates a linear constant-coefficient
system, whose steps must be the theta method in matrix form.  A steady state of the
whole PISO step stays put.
"""
import copy
import dataclasses
import math

import numpy as np
import pytest
import scipy.sparse as sparse
import scipy.sparse.linalg as spla

import clot_inputs as ci
from oracle import clot_oracle as oc


def quiet_oracle(desc, params=None):
    return oc.Oracle(desc, np.zeros((15, ci.ncell(desc))), np.zeros((2, ci.n_injury_faces(desc))), params)


def sp_diag(v, n):
    return sparse.diags(np.full(n, v))


def theta_gain(lam_dt, psi):
    th = 1.0 / (1.0 + psi)
    return (1.0 - (1.0 - th) * lam_dt) / (1.0 + th * lam_dt)


@pytest.mark.parametrize("psi", [0.0, 0.5, 0.9, 1.0])
def test_diffusion_mode_follows_theta_scheme(psi):
    """E1 (zero-gradient on every boundary, no flow, no injury source) carrying the
    cosine mode ky of the wall-normal direction decays by the exact discrete eigenvalue
    lambda = 4 D/dy^2 sin^2(pi ky / 2 ny); its stored derivative is -lambda E1."""
    desc = ci.channel(2, 4, 16, dt=1.0)
    p = oc.Params(ddt_psi=psi)
    o = quiet_oracle(desc, p)
    m = o.m
    for a in range(len(o.phi)):
        o.phi[a][:] = 0.0
    o.u[:] = 0.0
    o.c[:] = 0.0
    o.E0[:] = 0.0
    o.C0[:] = 0.0
    ky = 5
    j = m.yc / m.dy - 0.5
    mode = np.cos(math.pi * ky * (j + 0.5) / m.ny)
    a = 3e-6
    o.c[oc.SP["E1"]] = a * mode
    lam = 4.0 * p.D_chem / m.dy ** 2 * math.sin(math.pi * ky / (2 * m.ny)) ** 2
    for n, dt in enumerate([2.0, 2.0, 1.0, 5.0, 3.0, 2.5, 4.0]):
        o.dt = dt
        o.step(flow=False, react=False)
        a *= 1.0 / (1.0 + lam * dt) if n == 0 else theta_gain(lam * dt, psi)
        assert np.allclose(o.c[oc.SP["E1"]], a * mode, rtol=1e-11, atol=1e-11 * abs(a)), (n, psi)
        assert np.allclose(o.ddt0c["E1"], -lam * a * mode, rtol=1e-9, atol=1e-9 * lam * abs(a))
    # the schemes differ at this lambda dt: a dropped or mis-signed history term shows
    assert lam * 2.0 > 0.3


def stokes_channel(dt):
    """2-D channel of 8x8 square cells at a wall shear of 1/s (Reynolds number ~ 1e-3),
    marched to the discrete steady state of implicit Euler at step dt."""
    H, ny = 0.25, 8
    h = H / ny
    desc = ci.channel(2, 8, ny, shear=1.0, dt=dt, Lx=8 * h)
    o = quiet_oracle(desc, oc.Params(n_corr=8))
    zero = np.zeros(o.m.n)
    for _ in range(int(round(0.2 / dt))):
        o.flow_step(zero)
        o.n += 1
    return o


def bump(x, lo, hi):
    s = np.clip((x - lo) / (hi - lo), 0.0, 1.0)
    return np.sin(math.pi * s) ** 4


def test_crank_nicolson_keeps_the_discrete_steady_state():
    """With a history that vanishes (a steady state) the Crank-Nicolson step at dt has
    the same matrix as implicit Euler at dt/(1+psi), so that Euler steady state stays.
    (A collocated PISO steady state depends on the step through rAU = V/aP.)"""
    psi, dt = 0.9, 1e-3
    o = stokes_channel(dt / (1.0 + psi))
    o.p = dataclasses.replace(o.p, ddt_psi=psi)
    u0 = o.u.copy()
    zero = np.zeros(o.m.n)
    for _ in range(10):
        o.dt = dt
        o.flow_step(zero)
        o.n += 1
    assert np.abs(o.u - u0).max() <= 1e-9 * np.abs(u0).max()


@pytest.mark.parametrize("psi", [0.5, 0.9, 1.0])
def test_momentum_predictor_follows_theta_method(psi):
    """Without pressure correctors the flux, pressure and Darcy term stay fixed, so the
    predictor integrates the linear system V du/dt = -A u + b.  Its steps must be the
    theta method in matrix form, (V/dt + th A) u' = (V/dt - (1-th) A) u + b with
    th = 1/(1+psi), after an implicit-Euler first step, for any step sequence.  A and b
    come from the implicit-Euler system (A = matrix - V/dt, b = rhs - V u/dt)."""
    desc = ci.channel(2, 12, 8, shear=1000.0, dt=1e-4)
    o = quiet_oracle(desc, oc.Params(ddt_psi=psi))
    m = o.m
    o.n_correctors = lambda: 0
    o.u[0] *= 1.0 + 0.3 * bump(m.xc, 0.0, m.nx * m.dx) * bump(m.yc, 0.0, 0.25)
    o.u[1] = 2.0 * bump(m.xc, 0.1, 0.6) * bump(m.yc, 0.05, 0.2)
    alpha = 500.0 * bump(m.xc, 0.3, 0.7)
    S, src = o.momentum_system(alpha)            # n = 0: the implicit-Euler system
    V = m.V
    A = (S.matrix() - sp_diag(V / o.dt, m.n)).tocsc()
    gp = o.grad_p(o.p_)
    b = [src[c] - V * o.u[c] / o.dt - V * gp[c] for c in range(2)]
    u = o.u[:2].copy()
    I = sp_diag(1.0, m.n)
    for n, dt in enumerate([1e-4, 1e-4, 5e-5, 3e-4, 2e-4, 1e-4]):
        o.dt = dt
        o.flow_step(alpha)
        o.n += 1
        th = 1.0 if n == 0 else 1.0 / (1.0 + psi)
        for c in range(2):
            lhs = (V / dt) * I + th * A
            rhs = (V / dt) * u[c] - (1.0 - th) * (A @ u[c]) + b[c]
            u[c] = spla.spsolve(lhs.tocsc(), rhs)
        scale = np.abs(u).max()
        assert np.abs(o.u[:2] - u).max() <= 1e-10 * scale, (n, np.abs(o.u[:2] - u).max() / scale)
    # the stiffest modes here have lambda dt ~ 3 (theta-method gains -0.2 at psi = 1
    # against 0.25 for implicit Euler): the schemes differ visibly
    assert np.abs(A.diagonal()).max() * 3e-4 / V > 2


def cell_courant(o, dt):
    """Largest 0.5 dt sum_f |phi_f| / V, summed face by face here."""
    m = o.m
    tot = np.zeros(m.n)
    for a, (ax, A, d) in enumerate(m.axes):
        f = o.phi[a]
        for cidx in range(m.n):
            k, j, i = np.unravel_index(cidx, m.shape)
            lo = [k, j, i]
            hi = [k, j, i]
            hi[ax] += 1
            tot[cidx] += abs(f[tuple(lo)]) + abs(f[tuple(hi)])
    return 0.5 * dt * tot.max() / m.V


def test_variable_step_holds_the_courant_limit():
    """A channel whose given step runs at Courant ~4: every step, the first included,
    starts from a flux whose Courant number with that step is at most 0.75; the step
    never exceeds the given one, grows by at most 1.2 and the clock is their sum."""
    desc = ci.channel(2, 32, 8, shear=1000.0, dt=1e-3)
    xc, xf = ci.noise(desc)
    o = oc.Oracle(desc, xc, xf, oc.Params(max_co=0.75))
    t, prev = 0.0, None
    limited = 0
    for _ in range(12):
        dt = o.dt
        co = cell_courant(o, dt)
        assert co <= 0.75 * (1 + 1e-12), co
        assert dt <= desc["dt"]
        if prev is not None:
            assert dt <= 1.2 * prev * (1 + 1e-15)
        limited += co > 0.75 * (1 - 1e-9)
        o.step()
        t += dt
        assert o.t == t
        prev = dt
    assert limited >= 10          # the limit binds on this channel


def test_fixed_step_unchanged_by_psi_zero_history():
    """psi = 0 with a fixed step is the implicit-Euler step: the stored derivative is
    never read, so a garbage history changes nothing."""
    desc = ci.workload("channel2d_64x16")
    xc, xf = ci.noise(desc)
    a = oc.Oracle(desc, xc, xf)
    b = oc.Oracle(desc, xc, xf)
    for _ in range(2):
        a.step()
        b.ddt0u[:] = 1e30
        for k in b.ddt0c:
            b.ddt0c[k][:] = 1e30
        b.step()
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
