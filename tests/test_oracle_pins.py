"""CPU pins of the FP64 oracle against closed forms, invariants, limits and printed values.

Each test names the paper passage it follows.  None of them re-types the
oracle's own formula: they check what the mathematics or the paper fixes.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import erf

import clot_inputs as ci
from oracle import clot_oracle as oc

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def quiet_oracle(desc, params=None, inlet_u=None):
    nc = ci.ncell(desc)
    nf = ci.n_injury_faces(desc)
    return oc.Oracle(desc, np.zeros((15, nc)), np.zeros((2, nf)), params, inlet_u=inlet_u)


# ----------------------------------------------------------------------------------------
# Printed values and closed-form constants (Appendix C, Appendix E, section 2)
# ----------------------------------------------------------------------------------------

def test_margination_peak_to_centre_matches_printed_values():
    gold = json.load(open(GOLD))
    p = oc.Params()
    for key, dim in (("margination_2d", 2), ("margination_3d", 3)):
        g = gold[key]
        desc = ci.channel(dim, 8, 200, 8 if dim == 3 else 1, K=g["K"])
        # wall-normal line through the centre (z at mid-depth): R in [0,1) sampled finely
        r = 0.5 * desc["Ly"]
        y = np.linspace(0.0, r, 200001)
        z = np.full_like(y, 0.5 * desc["Lz"])
        c = oc.platelet_inflow(y, z, desc, p)
        ratio = c.max() / c[-1]
        # printed "approximately" value, to the printed digits
        assert abs(ratio - g["peak_to_centre_approx"]) < 0.5 * 10 ** (1 - g["digits_printed"]) + 0.07
        # exact optimum of R^18 (1-R) is at R = 18/19
        exact = 1.0 + g["K"] * (18.0 / 19.0) ** 18 / 19.0
        assert ratio == pytest.approx(exact, rel=1e-8)


def test_margination_mean_is_P0():
    """The normalising C0 makes the cross-section mean of the inflow equal to P_0.

    The bracket is a degree-19 polynomial in R on each half of the channel, so a
    12-point Gauss-Legendre rule per half integrates it exactly.
    """
    p = oc.Params()
    xg, wg = np.polynomial.legendre.leggauss(12)
    for dim in (2, 3):
        desc = ci.channel(dim, 4, 64, 64 if dim == 3 else 1)
        def nodes(L):
            h = 0.5 * L
            pts = np.concatenate([0.5 * h * (xg + 1), h + 0.5 * h * (xg + 1)])
            return pts, np.concatenate([wg, wg]) * 0.5 * h / L
        y, wy = nodes(desc["Ly"])
        if dim == 2:
            mean = np.sum(wy * oc.platelet_inflow(y, np.zeros_like(y), desc, p))
        else:
            z, wz = nodes(desc["Lz"])
            Y, Z = np.meshgrid(y, z, indexing="ij")
            mean = np.sum(np.outer(wy, wz) * oc.platelet_inflow(Y, Z, desc, p))
        assert mean == pytest.approx(p.P_0, rel=1e-13)


def test_printed_unit_conversions_and_viscosity():
    gold = json.load(open(GOLD))
    nu = gold["kinematic_viscosity"]
    assert nu["mu"] / nu["rho"] == pytest.approx(oc.Params().nu, rel=1e-12)
    for a, b in gold["unit_conversion"]["pairs"]:
        # mm^3/nmol = 1e-3 L / 1e-9 mol = 1e6 L/mol ... times 1e-3: clotFOAM column x 1e3 = M^-1 s^-1
        assert b / a == pytest.approx(gold["unit_conversion"]["mm3_per_nmol_per_s_to_per_M_per_s"])
    nc = gold["normal_concentrations"]
    # nmol/mm^3 = 1e-9 mol / 1e-6 L = 1e-3 M = 1e3 uM
    assert nc["S1_nmol_per_mm3"] * 1e3 == pytest.approx(nc["S1_uM"])
    assert nc["S2_nmol_per_mm3"] * 1e3 == pytest.approx(nc["S2_uM"])
    p = oc.Params()
    assert (p.S1_0, p.S2_0) == (nc["S1_nmol_per_mm3"], nc["S2_nmol_per_mm3"])


def test_model_function_special_values():
    p = oc.Params()
    # g(1) = 1 by the choice of g0; g = 0 at and below the threshold
    assert oc.binding_affinity(1.0, p) == pytest.approx(1.0, rel=1e-15)
    assert oc.binding_affinity(p.eta_t, p) == 0.0 and oc.binding_affinity(0.0, p) == 0.0
    # g(eta_t + eta_*) = g0/2
    g0 = (0.4 ** 3 + 0.9 ** 3) / 0.9 ** 3
    assert oc.binding_affinity(0.5, p) == pytest.approx(0.5 * g0, rel=1e-14)
    # Carman-Kozeny at full packing: 1e6 * 0.36 / 0.4^3
    assert oc.carman_kozeny(1.0, p) == pytest.approx(5.625e6, rel=1e-14)
    assert oc.carman_kozeny(0.0, p) == 0.0
    # hindrance: W(0) = tanh(pi), W(1) = 0, W clamps above 1, and W decreases
    assert oc.hindrance(0.0) == pytest.approx(math.tanh(math.pi))
    assert oc.hindrance(1.0) == 0.0 and oc.hindrance(1.7) == 0.0
    th = np.linspace(0, 1, 101)
    assert np.all(np.diff(oc.hindrance(th)) < 0)
    # release bell: fine quadrature over [0, 6] gives erf(3), over [0, inf) gives (1+erf 3)/2 + ...
    a = np.linspace(0.0, 6.0, 600001)
    assert np.trapezoid(oc.release_rate(a), a) == pytest.approx(erf(3.0), rel=1e-10)
    # van Leer: symmetric limiter values
    assert oc.van_leer(np.array([-3.0, 0.0, 1.0]))[:2].tolist() == [0.0, 0.0]
    assert oc.van_leer(np.array([1.0]))[0] == 1.0
    assert oc.van_leer(np.array([1e12]))[0] == pytest.approx(2.0)
    r = np.array([0.3, 2.0, 7.0])
    assert np.allclose(oc.van_leer(r) / r, oc.van_leer(1 / r))   # psi(r)/r = psi(1/r)


def test_parabola_and_duct_profiles():
    shear, r = 1000.0, 0.125
    y = np.array([0.0, r, 2 * r])
    u = oc.parabolic_inflow(y, shear, r)
    assert u[0] == 0.0 and u[2] == 0.0 and u[1] == pytest.approx(shear * r / 2)
    h = 1e-7
    assert (oc.parabolic_inflow(h, shear, r) - oc.parabolic_inflow(0.0, shear, r)) / h == pytest.approx(shear, rel=1e-5)
    a, b = 0.25, 0.25
    # walls are zero, -lap w = 1 in the interior (finite differences), slope matches
    ys = np.array([0.0, a, 0.07, 0.2])
    zs = np.array([0.1, 0.2, 0.0, b])
    assert np.allclose(oc.duct_unit_profile(ys, zs, a, b), 0.0, atol=1e-9)
    hh = 1e-4
    y0, z0 = 0.08, 0.11
    w = lambda yy, zz: oc.duct_unit_profile(np.array([yy]), np.array([zz]), a, b)[0]
    lap = (w(y0 + hh, z0) + w(y0 - hh, z0) + w(y0, z0 + hh) + w(y0, z0 - hh) - 4 * w(y0, z0)) / hh ** 2
    assert lap == pytest.approx(-1.0, rel=1e-4)
    slope = (w(hh, 0.5 * b) - w(0.0, 0.5 * b)) / hh
    assert slope == pytest.approx(oc.duct_wall_slope(a, b), rel=1e-3)
    # very wide duct -> plane Poiseuille in the middle
    wide = oc.duct_unit_profile(np.array([0.06]), np.array([5.0]), a, 10.0)[0]
    assert wide == pytest.approx(0.5 * 0.06 * (a - 0.06), rel=1e-10)
    # square-duct centre value, a classical constant: w_max = 0.0736713... a^2
    assert oc.duct_unit_profile(np.array([a / 2]), np.array([b / 2]), a, b)[0] / a ** 2 == pytest.approx(0.07367135, rel=1e-6)


# ----------------------------------------------------------------------------------------
# Flow: Poiseuille, Brinkman, duct (section 2 eq. NSB, section 3.2 PISO, Appendix C.1)
# ----------------------------------------------------------------------------------------

def run_to_steady(o, alpha, T=0.05):
    """March the flow alone for T seconds: the slowest viscous mode decays like exp(-nu pi^2 T / H^2) ~ 1e-9."""
    for it in range(int(round(T / o.dt))):
        o.flow_step(alpha)


def square_channel(ny, ncol, umax, shear=1000.0, dim=2):
    """Channel of ncol square cells along x at Courant number 0.5."""
    H = 0.25
    h = H / ny
    if dim == 2:
        return ci.channel(2, ncol, ny, shear=shear, dt=0.5 * h / umax, Lx=ncol * h)
    return ci.channel(3, ncol, ny, ny, shear=shear, dt=0.5 * h / umax, Lx=ncol * h)


def outlet_error(o, exact_fn):
    m = o.m
    col = m.idx[:, :, -2].ravel()
    ue = exact_fn(m.yc[col], m.zc[col])
    return np.linalg.norm(o.u[0][col] - ue) / np.linalg.norm(ue)


def observed_orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_poiseuille_second_order_and_pressure_gradient():
    shear, H = 1000.0, 0.25
    errs, grads = [], []
    for ny in (8, 16, 32):
        desc = square_channel(ny, 12, 62.5, shear)
        o = quiet_oracle(desc)
        run_to_steady(o, np.zeros(o.m.n))
        errs.append(outlet_error(o, lambda y, z: oc.parabolic_inflow(y, shear, H / 2)))
        p3 = o.p_.reshape(o.m.shape)
        grads.append((p3[0, ny // 2, -2] - p3[0, ny // 2, -3]) / o.m.dx)
        assert np.abs(o.continuity_residual()).max() < 1e-10 * np.abs(o.phi[0]).max()
    orders = observed_orders(errs)
    assert 1.8 < orders[-1] < 2.3, (errs, orders)
    G = oc.Params().nu * shear / (H / 2)
    assert grads[-1] == pytest.approx(-G, rel=2e-2)
    assert abs(grads[-1] + G) < abs(grads[0] + G)


def brinkman_profile(y, alpha, G, nu, r):
    s = math.sqrt(alpha)
    return (G / (nu * alpha)) * (1.0 - np.cosh(s * (y - r)) / math.cosh(s * r))


@pytest.mark.parametrize("theta0", [0.01, 0.05])
def test_brinkman_second_order(theta0):
    p = oc.Params()
    alpha0 = float(oc.carman_kozeny(theta0, p))
    assert alpha0 == pytest.approx({0.01: 36.656, 0.05: 986.1}[theta0], rel=1e-3)
    H = 0.25
    G = p.nu * 1000.0 / (H / 2)
    errs = []
    for ny in (8, 16, 32):
        desc = square_channel(ny, 12, 62.5)
        m = oc.Mesh(desc)
        col = m.idx[:, :, 0].ravel()
        uin = brinkman_profile(m.yc[col], alpha0, G, p.nu, H / 2)
        o = quiet_oracle(desc, inlet_u=uin)
        o.u[0] = brinkman_profile(m.yc, alpha0, G, p.nu, H / 2)
        o.c[oc.SP["Pbse"]] = theta0 * p.P_max
        alpha = oc.carman_kozeny(o.thetaB(), p)
        run_to_steady(o, alpha)
        errs.append(outlet_error(o, lambda y, z: brinkman_profile(y, alpha0, G, p.nu, H / 2)))
    orders = observed_orders(errs)
    assert 1.8 < orders[-1] < 2.3, (errs, orders)


def test_duct_poiseuille_second_order():
    shear, a = 1000.0, 0.25
    errs = []
    scale = shear / oc.duct_wall_slope(a, a)
    for n in (8, 16, 32):
        desc = square_channel(n, 2, 0.25 * shear * a, shear, dim=3)
        o = quiet_oracle(desc)
        run_to_steady(o, np.zeros(o.m.n), T=0.04)
        errs.append(outlet_error(o, lambda y, z: scale * oc.duct_unit_profile(y, z, a, a)))
        assert np.abs(o.continuity_residual()).max() < 1e-10 * np.abs(o.phi[0]).max()
    orders = observed_orders(errs)
    assert 1.7 < orders[-1] < 2.3, (errs, orders)


# ----------------------------------------------------------------------------------------
# eta: exact discrete eigenmodes of the zero-gradient Helmholtz operator (Appendix A, eq. eta)
# ----------------------------------------------------------------------------------------

def test_eta_cosine_modes_exact():
    p = oc.Params()
    kappa = p.P_diam ** 2
    desc = ci.channel(2, 24, 10, dt=1e-4)
    o = quiet_oracle(desc)
    m = o.m
    for kx, ky in ((0, 0), (3, 0), (0, 2), (5, 4)):
        i = (m.xc / m.dx - 0.5)
        j = (m.yc / m.dy - 0.5)
        th = 0.3 * np.cos(math.pi * kx * (i + 0.5) / m.nx) * np.cos(math.pi * ky * (j + 0.5) / m.ny)
        lam = (2 - 2 * math.cos(math.pi * kx / m.nx)) / m.dx ** 2 + (2 - 2 * math.cos(math.pi * ky / m.ny)) / m.dy ** 2
        eta = o.eta_solve(th)
        assert np.allclose(eta, th / (1 + kappa * lam), rtol=1e-11, atol=1e-14)


# ----------------------------------------------------------------------------------------
# Continuity and conservation (section 3.2 PISO; Appendix D conservative FV transport)
# ----------------------------------------------------------------------------------------

def test_step_keeps_discrete_continuity_and_nonnegativity():
    desc = ci.workload("channel2d_64x16")
    xc, xf = ci.noise(desc)
    o = oc.Oracle(desc, xc, xf)
    for _ in range(10):
        o.step()
        assert np.abs(o.continuity_residual()).max() < 1e-10 * np.abs(o.phi[0]).max()
    scales = {"Pmu": 6.67e7, "Pma": 6.67e7, "Pba": 6.67e7, "Pbse": 6.67e7, "ADP": 2e-3}
    for i, n in enumerate(oc.SPECIES):
        s = scales.get(n, 1.4e-3)
        assert o.c[i].min() >= -1e-14 * s, n
    assert o.E0.min() > 0 and o.C0.min() >= 0


def test_transport_closed_box_conserves_mass():
    """No flow: diffusion and hindered platelet diffusion conserve the total exactly."""
    desc = ci.channel(2, 12, 8, dt=1e-3)
    rng = np.random.default_rng(3)
    o = quiet_oracle(desc)
    for a in range(len(o.phi)):
        o.phi[a][:] = 0.0
    o.C0[:] = 0.0
    o.E0[:] = 0.0
    for n in ("Pmu", "Pma", "ADP", "E2"):
        o.c[oc.SP[n]] = rng.uniform(0.5, 1.5, o.m.n) * (1e6 if n.startswith("P") else 1e-5)
    o.c[oc.SP["Pbse"]] = rng.uniform(0, 0.6, o.m.n) * 6.67e7      # hindrance varies
    thT = o.thetaT()
    for n in ("Pma", "ADP", "E2"):
        before = o.c[oc.SP[n]].sum()
        S = o.transport_system(n, thT)
        after = oc.solve(S.matrix(), S.rhs, False).sum()
        assert after == pytest.approx(before, rel=1e-13)


def test_transport_flow_balance():
    """With flow: change of total = -dt * net boundary outflow evaluated with the new field."""
    desc = ci.workload("channel2d_64x16")
    xc, xf = ci.noise(desc)
    o = oc.Oracle(desc, xc, xf)
    o.step(transport=False, react=False)
    rng = np.random.default_rng(5)
    o.c[oc.SP["ADP"]] = rng.uniform(1e-4, 2e-4, o.m.n)
    o.sigma[:] = 0.0
    S = o.transport_system("ADP", o.thetaT())
    new = oc.solve(S.matrix(), S.rhs, False)
    m = o.m
    lo = m.idx[:, :, 0].ravel()
    hi = m.idx[:, :, -1].ravel()
    out_flux = (o.phi[0][:, :, -1].ravel() * new[hi]).sum() - (o.phi[0][:, :, 0].ravel() * new[lo]).sum()
    lhs = m.V * (new.sum() - o.c[oc.SP["ADP"]].sum()) / o.dt
    assert lhs == pytest.approx(-out_flux, rel=1e-9)


# ----------------------------------------------------------------------------------------
# Reactive wall (Appendix C table; Appendix B eqs. seBound_E0/C0)
# ----------------------------------------------------------------------------------------

def test_robin_wall_equilibrium_and_limits():
    p = oc.Params()
    desc = ci.channel(2, 16, 8, dt=1e-4)
    o = quiet_oracle(desc)
    for a in range(len(o.phi)):
        o.phi[a][:] = 0.0
    # equilibrium: q/k = S1_0 at every injury face -> uniform S1_0 is an exact steady state
    o.C0[:] = p.kC0p * o.E0 * p.S1_0 / p.kC0m
    thT = o.thetaT()
    S = o.transport_system("S1", thT)
    new = oc.solve(S.matrix(), S.rhs, False)
    assert np.allclose(new, p.S1_0, rtol=1e-13)
    # sink sign: with C0 = 0 the wall removes S1 from the injury cells only
    o.C0[:] = 0.0
    S = o.transport_system("S1", thT)
    new = oc.solve(S.matrix(), S.rhs, False)
    assert new[o.m.inj_cells].max() < p.S1_0
    # limits: k -> 0 gives no wall term; k -> inf gives a zero-value wall at distance dy/2
    base = o.transport_system("S1", thT).diag.copy()
    o.E0[:] = 0.0
    d0 = o.transport_system("S1", thT).diag
    o.E0[:] = 1e20
    dinf = o.transport_system("S1", thT).diag
    g = 2 * p.D_chem * o.m.inj_area / o.m.dy
    assert np.allclose((dinf - d0)[o.m.inj_cells], g, rtol=1e-9)
    assert np.all(base[o.m.inj_cells] > d0[o.m.inj_cells])
    # E1 source equals k_cat C0 per unit area
    o.E0[:] = p.E0_0
    o.C0[:] = 3e-9
    S = o.transport_system("E1", thT)
    src = S.rhs - o.m.V * o.c[oc.SP["E1"]] / o.dt
    assert src[o.m.inj_cells] == pytest.approx(o.m.inj_area * p.kC0cat * 3e-9, rel=1e-13)


def test_wall_mass_balance_e0_c0():
    p = oc.Params()
    rng = np.random.default_rng(1)
    y0 = np.array([rng.uniform(1e-7, 2e-7, 50), rng.uniform(0, 1e-8, 50)])
    s1w = rng.uniform(1e-4, 2e-4, 50)
    y = oc.rk4(lambda v: oc.wall_rhs(v, s1w, p), y0, 5e-5, 4)
    assert np.allclose(y.sum(axis=0), y0.sum(axis=0), rtol=1e-15)
    # the linear system has the closed-form solution: relaxation to E0* with rate lambda
    lam = p.kC0p * s1w + p.kC0m + p.kC0cat
    tot = y0.sum(axis=0)
    E0inf = (p.kC0m + p.kC0cat) * tot / lam
    exact = E0inf + (y0[0] - E0inf) * np.exp(-lam * 2e-4)
    assert np.allclose(y[0], exact, rtol=1e-12)


# ----------------------------------------------------------------------------------------
# Reactions (Appendix A and B): invariants and RK4 accuracy
# ----------------------------------------------------------------------------------------

def random_states(n, rng):
    p = oc.Params()
    Pm = p.P_max
    y = np.array([
        rng.uniform(1e5, 1e6, n), rng.uniform(0, 1e6, n), rng.uniform(0, 0.4 * Pm, n), rng.uniform(0, 0.3 * Pm, n),
        rng.uniform(1e-4, 2e-4, n), rng.uniform(1e-3, 2e-3, n), rng.uniform(0, 1e-5, n), rng.uniform(0, 1e-5, n),
        rng.uniform(0, 1e-5, n), rng.uniform(0, 1e-5, n), rng.uniform(0, 1e-6, n), rng.uniform(0, 1e-6, n),
        rng.uniform(0, 1e-7, n), rng.uniform(0, 1e-7, n)])
    adp = rng.uniform(0, 4e-3, n)
    gam = oc.binding_affinity(rng.uniform(0, 1, n), p)
    hadh = (rng.uniform(0, 1, n) < 0.5).astype(float)
    return y, adp, gam, hadh


def test_reaction_linear_invariants_exact():
    p = oc.Params()
    rng = np.random.default_rng(11)
    y, adp, gam, hadh = random_states(200, rng)
    f = lambda v: oc.reaction_rhs(v, adp, gam, hadh, p)
    z = oc.rk4(f, y.copy(), 5e-5, 2)
    R = {n: i for i, n in enumerate(oc.RXN)}
    fam = {
        "platelets": ["Pmu", "Pma", "Pba", "Pbse"],
        "X": ["S1", "S1b", "E1", "E1b", "C1", "C2"],
        "II": ["S2", "S2b", "E2", "E2b", "C1", "C2"],
    }
    for name, members in fam.items():
        a = sum(y[R[s]] for s in members)
        b = sum(z[R[s]] for s in members)
        assert np.allclose(a, b, rtol=1e-14, atol=0), name
    # rhs sums vanish identically
    d = f(y)
    for members in fam.values():
        tot = sum(d[R[s]] for s in members)
        scale = sum(np.abs(d[R[s]]) for s in members) + 1e-300
        assert np.all(np.abs(tot) <= 1e-12 * scale)


def test_reaction_rk4_against_high_accuracy_ode():
    """RK4 error vs DOP853 (rtol 1e-13): fourth order, global error ratio ~16 per halving."""
    p = oc.Params()
    rng = np.random.default_rng(12)
    y, adp, gam, hadh = random_states(6, rng)
    gam = np.full(6, 1.0)             # cohesion at full strength: the fastest rate, 1e4 1/s
    T = 1e-3
    for c in range(6):
        f1 = lambda t, v: oc.reaction_rhs(v, adp[c], gam[c], hadh[c], p)
        ref = solve_ivp(f1, (0, T), y[:, c], method="DOP853", rtol=1e-13, atol=1e-30).y[:, -1]
        errs = []
        # species scales: platelets P_max, the S1 family S1_0, the S2 family S2_0
        scale = np.array([p.P_max] * 4 + [p.S1_0, p.S2_0, p.S1_0, p.S2_0, p.S1_0, p.S2_0, p.S1_0, p.S2_0,
                                          p.S2_0, p.S2_0])
        for nsub in (8, 16, 32):
            z = oc.rk4(lambda v: oc.reaction_rhs(v, adp[c], gam[c], hadh[c], p), y[:, c].copy(), T / nsub, nsub)
            errs.append(np.max(np.abs(z - ref) / scale))
        assert errs[-1] < 1e-8
        ratio = errs[1] / errs[2]
        assert 10 < ratio < 24, (errs, ratio)


# ----------------------------------------------------------------------------------------
# Release source (eq. ADP_source, eq. sigma_disc)
# ----------------------------------------------------------------------------------------

def test_sigma_trapezoid_constant_history_and_single_bell():
    p = oc.Params()
    desc = ci.channel(2, 4, 2, dt=p.dtau)
    o = quiet_oracle(desc)
    th = np.zeros(o.m.n)
    F = 3.0e5                                   # platelets/mm^3/s newly bound
    # constant binding rate: theta rises by F dt / Pmax every step; run past 25 pushes
    for n in range(30):
        o.t = n * o.dt
        o.n = n
        o.sigma_update(th)
        o.thetaB_prev = th.copy()
        th = th + F * o.dt / p.P_max
    ages = np.arange(25) * p.dtau
    w = np.full(25, p.dtau)
    w[0] = w[-1] = 0.5 * p.dtau
    expect = p.A_hat * F * np.sum(w * np.exp(-(ages - 3) ** 2) / math.sqrt(math.pi))
    assert np.allclose(o.sigma, expect, rtol=1e-12)
    # trapezoid of the bell vs the exact window integral erf(3): Euler-Maclaurin end
    # correction h^2/12 (R'(6) - R'(0)) bounds the difference
    h = p.dtau
    dR = lambda a: -2.0 * (a - 3.0) * math.exp(-(a - 3.0) ** 2) / math.sqrt(math.pi)
    em = h * h / 12.0 * abs(dR(6.0) - dR(0.0))
    assert abs(expect / (p.A_hat * F) - erf(3.0)) <= 1.05 * em
    # a single burst of binding gives one bell travelling with age
    o2 = quiet_oracle(desc)
    th = np.zeros(o2.m.n)
    trace = []
    for n in range(20):
        o2.t = n * o2.dt
        o2.n = n
        newth = th + (1e-3 if n == 2 else 0.0)
        o2.sigma_update(newth)
        o2.thetaB_prev = newth.copy()
        th = newth
        trace.append(o2.sigma[0])
    f = p.P_max * 1e-3 / p.dtau
    for n in range(3, 20):
        age = (n - 2) * p.dtau
        wt = 0.5 * p.dtau if n == 2 else p.dtau
        assert trace[n] == pytest.approx(p.A_hat * f * wt * math.exp(-(age - 3) ** 2) / math.sqrt(math.pi), rel=1e-12)
    assert trace[2] == pytest.approx(p.A_hat * f * 0.5 * p.dtau * math.exp(-9) / math.sqrt(math.pi), rel=1e-12)
    assert trace[1] == 0.0


def test_sigma_is_zero_within_short_horizons():
    desc = ci.workload("channel2d_64x16")
    xc, xf = ci.noise(desc)
    o = oc.Oracle(desc, xc, xf)
    for _ in range(3):
        o.step()
    assert not np.any(o.sigma)


# ----------------------------------------------------------------------------------------
# Hindrance interpolation and the limiter (section 3.2, Appendix D)
# ----------------------------------------------------------------------------------------

def test_hindrance_downwind_and_localmax_on_three_cells():
    p = oc.Params()
    desc = ci.channel(2, 3, 1, dt=1e-3, Lx=3e-3, Ly=1e-3)
    o = quiet_oracle(desc)
    m = o.m
    o.phi[0][:] = 2.0e-6        # uniform +x flux
    o.phi[1][:] = 0.0
    th = np.array([0.1, 0.6, 0.3])
    o.c[oc.SP["Pmu"]] = np.array([4e6, 2e6, 1e6])     # monotone: psi frozen from these
    M = o.transport_system("Pmu", th).matrix().toarray()
    A, d = m.axes[0][1], m.axes[0][2]
    # face 0|1: phi > 0, downwind = cell 1 (theta .6), localMax = .6
    Wa01 = math.tanh(math.pi * 0.4)
    Wd01 = math.tanh(math.pi * 0.4)
    # limiter on face 0|1: no far-upwind cell -> upwind, so C_f = C_0
    assert M[0, 1] == pytest.approx(-Wd01 * p.D_P * A / d, rel=1e-14)
    assert M[1, 0] == pytest.approx(-Wa01 * 2e-6 - Wd01 * p.D_P * A / d, rel=1e-14)
    # face 1|2: downwind = cell 2 (theta .3) for advection, localMax = .6 for diffusion
    Wa12 = math.tanh(math.pi * 0.7)
    Wd12 = math.tanh(math.pi * 0.4)
    rr = (2e6 - 4e6) / (1e6 - 2e6)       # r = (C_U - C_UU)/(C_D - C_U) = 2
    psi = (rr + abs(rr)) / (1 + abs(rr))
    assert M[1, 2] == pytest.approx(Wa12 * 2e-6 * psi / 2 - Wd12 * p.D_P * A / d, rel=1e-13)
    assert M[2, 1] == pytest.approx(-Wa12 * 2e-6 * (1 - psi / 2) - Wd12 * p.D_P * A / d, rel=1e-13)
    # constant theta: every coupling of the platelet system scales by W(theta)/W(0)
    o.c[oc.SP["Pmu"]] = np.array([4e6, 2e6, 1e6])
    M0 = o.transport_system("Pmu", np.zeros(3)).matrix().toarray()
    Mc = o.transport_system("Pmu", np.full(3, 0.45)).matrix().toarray()
    off = ~np.eye(3, dtype=bool)
    ratio = math.tanh(math.pi * 0.55) / math.tanh(math.pi)
    assert np.allclose(Mc[off], M0[off] * ratio, rtol=1e-13)


def test_limiter_linear_profile_is_central():
    """On a linear C^n profile r = 1, psi = 1: interior faces use the central average."""
    desc = ci.channel(2, 8, 1, dt=1e-3, Lx=8e-3, Ly=1e-3)
    o = quiet_oracle(desc)
    o.phi[0][:] = 1e-6
    o.phi[1][:] = 0.0
    o.c[oc.SP["E2"]] = 1e-6 * (1.0 + np.arange(8))
    M = o.transport_system("E2", np.zeros(8)).matrix().toarray()
    A, d = o.m.axes[0][1], o.m.axes[0][2]
    D = oc.Params().D_chem
    for i in range(1, 6):       # faces i|i+1 with a far-upwind cell i-1
        assert M[i, i + 1] == pytest.approx(1e-6 * 0.5 - D * A / d, rel=1e-12)


# ----------------------------------------------------------------------------------------
# Momentum convection (section 2, eq. NSB; Appendix D table: Gauss linear div(phi,U))
# ----------------------------------------------------------------------------------------

def _stream_field(Lx, Ly, amp):
    """A divergence-free velocity u = d(psi)/dy, v = -d(psi)/dx from psi = amp sin(ax + .3) sin(by + .2),
    with its closed-form first derivatives; both components satisfy lap f = -(a^2 + b^2) f."""
    a, b = math.pi / Lx, 2.0 * math.pi / Ly

    def psi(x, y):
        return amp * np.sin(a * x + 0.3) * np.sin(b * y + 0.2)

    def fields(x, y):
        sx, cx = np.sin(a * x + 0.3), np.cos(a * x + 0.3)
        sy, cy = np.sin(b * y + 0.2), np.cos(b * y + 0.2)
        u, v = amp * b * sx * cy, -amp * a * cx * sy
        ux, uy = amp * a * b * cx * cy, -amp * b * b * sx * sy
        vx, vy = amp * a * a * sx * sy, -amp * a * b * cx * cy
        return u, v, ux, uy, vx, vy
    return psi, fields, a * a + b * b


def test_momentum_convection_is_central_second_order():
    """The momentum operator applied to a smooth divergence-free field, with face fluxes
    integrated exactly from its stream function, approximates (u.grad)u - nu lap u at
    second order in interior cells (Gauss linear convection of eq. NSB).  Dropping the
    convection leaves an O(1) error; upwind convection an O(h) one; either fails."""
    Lx, Ly = 1.0, 0.5
    psi, fields, k2 = _stream_field(Lx, Ly, 40.0)
    errs = []
    conv_share = []
    for n in (16, 32, 64):
        desc = ci.channel(2, 2 * n, n, dt=1e-3, Lx=Lx, Ly=Ly)
        o = quiet_oracle(desc)
        m = o.m
        xf = np.arange(m.nx + 1) * m.dx
        yf = np.arange(m.ny + 1) * m.dy
        X, Yt = np.meshgrid(xf, yf[1:])
        _, Yb = np.meshgrid(xf, yf[:-1])
        o.phi[0][0] = m.dz * (psi(X, Yt) - psi(X, Yb))          # exact flux through each x face
        Xr, Y = np.meshgrid(xf[1:], yf)
        Xl, _ = np.meshgrid(xf[:-1], yf)
        o.phi[1][0] = -m.dz * (psi(Xr, Y) - psi(Xl, Y))         # and each y face
        u, v, ux, uy, vx, vy = fields(m.xc, m.yc)
        o.u[0], o.u[1] = u, v
        S, src = o.momentum_system(np.zeros(m.n))
        M = S.matrix()
        nu = o.p.nu
        want = (u * ux + v * uy + nu * k2 * u, u * vx + v * vy + nu * k2 * v)
        inner = m.idx[0][1:-1, 1:-1].ravel()
        e = 0.0
        for c in range(2):
            got = (M @ o.u[c] - src[c]) / m.V        # the time terms cancel: u^n is the field itself
            e = max(e, np.abs(got[inner] - want[c][inner]).max() / np.abs(want[c][inner]).max())
        errs.append(e)
        conv_share.append(np.abs(u * ux + v * uy).max() / np.abs(want[0]).max())
    assert min(conv_share) > 0.3          # convection is a large part of what is checked
    orders = observed_orders(errs)
    assert errs[-1] < 6e-3 and min(orders) > 1.8, (errs, orders)


def test_developing_flow_closes_the_momentum_balance():
    """Plug inflow into a 2-D channel at Re = 100, marched to steady state: the x-momentum of
    eq. NSB integrated over the channel balances, to round-off, the momentum carried in and
    out, the pressure force on the inlet and outlet, the viscous force on the inlet face and
    the wall shear.  The profile develops, so the outflow carries 18% more momentum than
    the inflow: without convection the balance would miss by that much."""
    nx, ny, U = 48, 12, 40.0
    p = oc.Params(nu=0.1)
    desc = ci.channel(2, nx, ny, dt=2e-3, Lx=1.0, Ly=0.25)
    o = quiet_oracle(desc, p, inlet_u=np.full(ny, U))
    o.u[0][:] = U
    o.phi[0][:] = o.m.axes[0][1] * U
    for _ in range(80):
        u0 = o.u.copy()
        o.flow_step(np.zeros(o.m.n))
    assert np.abs(o.u - u0).max() < 1e-12 * U            # steady
    m = o.m
    A, d = m.axes[0][1], m.axes[0][2]
    Ay, dy = m.axes[1][1], m.axes[1][2]
    ux = o.u[0].reshape(m.shape)
    P = o.p_.reshape(m.shape)
    flux_in = float(np.sum(o.phi[0][:, :, 0] * U))
    flux_out = float(np.sum(o.phi[0][:, :, -1] * ux[:, :, -1]))     # zero-gradient outlet value
    pressure = float(np.sum(P[:, :, 0]) * A - np.sum(np.full(ny, p.p_out)) * A)
    visc_in = float(np.sum(2.0 * p.nu * A / d * (U - ux[:, :, 0])))  # half-cell gradient at the inlet
    shear = float(np.sum(2.0 * p.nu * Ay / dy * (ux[:, 0, :] + ux[:, -1, :])))
    assert flux_out / flux_in > 1.1
    assert abs(flux_in - flux_out + pressure + visc_in - shear) < 1e-10 * flux_in


# ----------------------------------------------------------------------------------------
# The limiter and hindrance on reversed flow (Appendix D: van Leer, downwind, localMax)
# ----------------------------------------------------------------------------------------

def _mirror(o, axis):
    """Mirror a copy of the oracle's state along a mesh axis ('x', 'y' or 'z'): cell values
    and tangential fluxes move to the image cell/face, normal fluxes also change sign.
    Returns the permutation q with (mirrored field)[q] = field."""
    m = o.m
    nax = {"x": 2, "y": 1, "z": 0}[axis]
    q = np.flip(m.idx, axis=nax).ravel()
    q_inv = np.empty_like(q)
    q_inv[q] = np.arange(q.size)
    flip = lambda a3: np.flip(a3, axis=nax)
    o.c = o.c[:, q]
    for a, (ax, A, d) in enumerate(m.axes):
        f = flip(o.phi[a])
        o.phi[a] = -f if ax == nax else f.copy()
    return q


def _mirrored_system_check(desc, name, axis, rng):
    o = quiet_oracle(desc)
    m = o.m
    p = o.p
    scale = p.P_max if name in ("Pmu", "Pma") else 1e-6
    # C^n with both signs of the slopes, a few platelet values outside [0, P_max]
    c = scale * rng.uniform(0.0, 1.0, m.n)
    if name in ("Pmu", "Pma"):
        c[rng.integers(0, m.n, 3)] = 1.2 * p.P_max
    o.c[o.sp[name]] = c
    for a in range(len(m.axes)):
        o.phi[a] = 1e-5 * rng.standard_normal(o.phi[a].shape)     # fluxes of both signs
    thT = rng.uniform(0.0, 1.1, m.n)
    M = o.transport_system(name, thT).matrix().toarray()
    rhs = o.transport_system(name, thT).rhs
    o2 = quiet_oracle(desc)
    o2.c = o.c.copy()
    o2.phi = [f.copy() for f in o.phi]
    q = _mirror(o2, axis)
    # mirrored state: cell a of the original sits at q_inv[a]; the system must be the image
    q_inv = np.empty_like(q)
    q_inv[q] = np.arange(q.size)
    S2 = o2.transport_system(name, thT[q])
    M2 = S2.matrix().toarray()
    assert np.allclose(M2[np.ix_(q_inv, q_inv)], M, rtol=1e-12, atol=1e-12 * np.abs(M).max())
    assert np.allclose(S2.rhs[q_inv], rhs, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("name", ["E2", "Pma"])
def test_transport_system_is_mirror_symmetric_along_x(name):
    """Reversing the flow along x and mirroring C^n, theta_T and the fluxes gives the mirrored
    matrix (species with zero-gradient inlet and outlet, so the ends swap roles): the
    negative-flux faces take their far-upwind cell at R + 1 as the positive ones take L - 1."""
    rng = np.random.default_rng(11)
    desc = ci.channel(2, 9, 5, dt=1e-3, Lx=9e-3, Ly=5e-3)
    _mirrored_system_check(desc, name, "x", rng)


@pytest.mark.parametrize("name", ["E2", "Pmu", "S2"])
def test_transport_system_is_mirror_symmetric_along_y_and_z(name):
    """The same symmetry across the channel (both walls alike for species without an injury
    term; the inlet profiles are symmetric about the centre line) and, in 3-D, along z."""
    rng = np.random.default_rng(12)
    _mirrored_system_check(ci.channel(2, 6, 9, dt=1e-3, Lx=6e-3, Ly=9e-3, inj_frac=0.0), name, "y", rng)
    d3 = ci.channel(3, 5, 6, 7, dt=1e-3, Lx=5e-3, Ly=6e-3, Lz=7e-3, inj_frac=0.0)
    _mirrored_system_check(d3, name, "y", rng)
    _mirrored_system_check(d3, name, "z", rng)


def test_limiter_linear_profile_is_central_on_reversed_flow():
    """On a linear C^n profile with negative flux, r = 1 again (far-upwind cell R + 1), so the
    faces with a far-upwind cell use the central average."""
    desc = ci.channel(2, 8, 1, dt=1e-3, Lx=8e-3, Ly=1e-3)
    o = quiet_oracle(desc)
    o.phi[0][:] = -1e-6
    o.phi[1][:] = 0.0
    o.c[oc.SP["E2"]] = 1e-6 * (1.0 + np.arange(8))
    M = o.transport_system("E2", np.zeros(8)).matrix().toarray()
    A, d = o.m.axes[0][1], o.m.axes[0][2]
    D = oc.Params().D_chem
    for i in range(0, 6):       # faces i|i+1 with a far-upwind cell i+2
        assert M[i, i + 1] == pytest.approx(-1e-6 * 0.5 - D * A / d, rel=1e-12)
        assert M[i + 1, i] == pytest.approx(1e-6 * 0.5 - D * A / d, rel=1e-12)


@pytest.mark.parametrize("dims", [(2, 8, 4, 1), (3, 4, 4, 4)])
def test_every_assembled_system_is_solved_to_the_dense_direct_solution(monkeypatch, dims):
    """Linear algebra (pin S9): on 8x4 and 4x4x4 channels every system two oracle steps
    assemble (momentum per component, pressure per corrector, eta, the seven transport
    systems) is solved by the Krylov route the oracle takes on large grids (forced here:
    Jacobi CG or BiCGStab to 1e-13) and by a dense direct solve of the same matrix; the
    two agree to 1e-11, and the step goes on with the dense solution."""
    import oracle.clot_oracle as oc
    real = oc.linear_solver
    seen = []

    def both(M, spd, direct_max=oc.DIRECT_MAX):
        krylov = real(M, spd, direct_max=0)
        dense = M.toarray()

        def run(b, x0=None):
            xk = krylov(b, x0)
            xd = np.linalg.solve(dense, b)
            scale = max(float(np.linalg.norm(xd)), 1e-300)
            seen.append((spd, M.shape[0], float(np.linalg.norm(xk - xd)) / scale))
            return xd
        return run

    monkeypatch.setattr(oc, "linear_solver", both)
    dim, nx, ny, nz = dims
    d = ci.channel(dim, nx, ny, nz, shear=1000.0, dt=1e-4, seed=17)
    o = oc.Oracle(d, *ci.noise(d))
    for _ in range(2):
        o.step()
    ncorr = o.n_correctors()
    per_step = dim + ncorr + 1 + 7          # momentum components, correctors, eta, transport
    assert len(seen) == 2 * per_step, (len(seen), per_step)
    assert sum(1 for spd, _, _ in seen if spd) == 2 * (ncorr + 1)
    worst = max(e for _, _, e in seen)
    assert worst <= 1e-11, worst
