"""Plain FP64 CPU oracle of one clotting-model time step (clotFoam, arXiv 2304.09180).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU library:
it assembles every finite-volume system explicitly as a scipy sparse matrix (one
row per cell, one entry per face coupling) and solves it with a sparse direct
factorisation (the momentum and pressure systems up to FLOW_DIRECT_MAX unknowns,
the others up to DIRECT_MAX) or else a Jacobi-preconditioned Krylov solve to a
relative residual of 1e-13.  Everything is float64.

Model (paper section 2, Appendices A-E):
  * Navier-Stokes-Brinkman flow (eq. NSB) with the Carman-Kozeny permeability,
    advanced by one PISO predictor/corrector pass (section 3.2) with the Darcy
    term implicit on the momentum diagonal using the bound fraction of the
    previous step;
  * the virtual substance eta (Appendix A, eq. eta) and the binding affinity g;
  * the ADP release source (eq. ADP_source) by the coarse-tau trapezoid
    (eq. sigma_disc);
  * implicit transport of the mobile platelets (hindered, eq.
    generalPlateletAggregation) and the fluid-phase chemicals with van Leer TVD
    convection, downwind/localMax interpolation of theta_T (Appendix D table),
    the reactive injury-wall conditions (Appendix B, Appendix C table);
  * the reactions by M_rxn sub-steps of classical RK4 (section 3.2 fractional
    step; Appendix A and B right-hand sides; eqs. seBound_E0/C0 on the wall);
  * optionally Crank-Nicolson off-centring of every ddt term and a variable step
    at a Courant limit (Appendix D), and the inhibitor of the extensibility
    example, I + E2 -> E2i (section 3.4).

Where the paper is silent or ambiguous, the reading taken is stated next to the
code that depends on it.

Parity status: every function here is pinned by a CPU test against a closed form,
an invariant, a special case or a printed value of the paper (tests/test_oracle_*).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Sparse LU limits: the momentum and pressure matrices are factorised up to FLOW_DIRECT_MAX
# unknowns (once per step: the velocity components share the momentum matrix and every
# corrector of the step the pressure matrix), the eta and transport systems, which the
# time derivative makes strongly diagonally dominant, up to DIRECT_MAX; larger systems
# take a Jacobi-preconditioned Krylov solve to a relative residual of 1e-13.
FLOW_DIRECT_MAX = 400_000
DIRECT_MAX = 20_000

# Cell species in library field order.
SPECIES = ["Pmu", "Pma", "Pba", "Pbse", "ADP", "S1", "S2", "E1", "E2",
           "S1b", "S2b", "E1b", "E2b", "C1", "C2"]
SP = {n: i for i, n in enumerate(SPECIES)}
# The 14 species integrated by the reaction step (ADP is frozen there).
RXN = ["Pmu", "Pma", "Pba", "Pbse", "S1", "S2", "E1", "E2",
       "S1b", "S2b", "E1b", "E2b", "C1", "C2"]
# The 7 transported scalars (bound species do not move).
TRANSPORTED = ["Pmu", "Pma", "S1", "S2", "E1", "E2", "ADP"]
# The extensibility example (section 3.4): a fluid-phase inhibitor I that binds thrombin
# for good, I + E2 -> E2i.  Both new species are transported and react; they follow the
# 15 species above, whose indices do not change.
INHIBITOR_SPECIES = ["I", "E2i"]


@dataclass
class Params:
    """Model constants of Appendix E (fluid, diffusion, platelet, coagulation tables)."""
    nu: float = 2.62507            # kinematic viscosity mm^2/s
    C_CK: float = 1.0e6            # Carman-Kozeny constant mm^-2
    D_P: float = 2.5e-5            # platelet diffusivity mm^2/s
    D_ADP: float = 5.0e-4
    D_chem: float = 5.0e-5
    P_diam: float = 3.0e-3         # mm
    P_max: float = 6.67e7          # platelets/mm^3
    P_0: float = 2.5e5
    k_adh: float = 3.3212e-8       # mm^3/s
    kcoh_Pmax: float = 1.0e4       # 1/s
    eta_t: float = 0.1
    eta_star: float = 0.4          # reading: eta_star = 0.5 - eta_t
    L_eta_over_Pdiam: float = 2.0
    k_adp: float = 0.34
    adp_crit: float = 2.0e-3
    k_e2: float = 0.5
    e2_crit: float = 1.0e-6
    A_hat: float = 2.0e-8          # nmol ADP per platelet
    tau_f: float = 6.0
    dtau: float = 0.25
    N_A: float = 6.02214076e14
    N1: float = 2700.0
    N2: float = 2000.0
    kC0p: float = 8.95e3
    kC0m: float = 1.0
    kC0cat: float = 1.15
    kC1p: float = 1.03e5
    kC1m: float = 1.0
    kC1cat: float = 30.0
    kC2p: float = 1.73e4
    kC2m: float = 1.0
    kC2cat: float = 0.23
    kS1p: float = 5.7e4
    kS1m: float = 0.17
    kE1p: float = 1.0e4
    kE1m: float = 2.5e-2
    kS2p: float = 1.0e4
    kS2m: float = 5.9
    kE2p: float = 1.0e4
    kE2m: float = 5.9
    S1_0: float = 1.7e-4           # nmol/mm^3
    S2_0: float = 1.4e-3
    E0_0: float = 1.5e-7           # nmol/mm^2
    p_out: float = 0.0
    M_rxn: int = 2
    n_corr: int = 0                # 0: chosen from the viscous diffusion number (see n_correctors)
    marg_m: int = 19
    marg_n: int = 2
    # time integration (Appendix D table): Crank-Nicolson off-centring psi of every ddt
    # term (0 = implicit Euler), and the variable step that holds the largest cell
    # Courant number at max_co (0 = the channel's fixed dt)
    ddt_psi: float = 0.0
    max_co: float = 0.0
    dt_growth: float = 1.2
    # the inhibitor variant (section 3.4 names the reaction, not its constants): an
    # antithrombin-like inlet and initial concentration and association rate
    inhibitor: bool = False
    k_I: float = 7.1               # (nmol/mm^3)^-1 s^-1
    I_0: float = 3.4e-3            # nmol/mm^3


# --------------------------------------------------------------------------------------
# Closed-form model functions
# --------------------------------------------------------------------------------------

def carman_kozeny(thetaB, p: Params):
    """alpha(theta_B) = C_CK (0.6 theta_B)^2 / (1 - 0.6 theta_B)^3 (section 2, below eq. NSB)."""
    s = 0.6 * np.asarray(thetaB, dtype=np.float64)
    return p.C_CK * s * s / (1.0 - s) ** 3


def hindrance(thetaT):
    """W(theta_T) = tanh(pi (1 - theta_T)) (Appendix A); theta_T is clamped to <= 1 inside W."""
    t = np.minimum(np.asarray(thetaT, dtype=np.float64), 1.0)
    return np.tanh(np.pi * (1.0 - t))


def binding_affinity(eta, p: Params):
    """g(eta) = g0 (eta-eta_t)^3 / (eta_*^3 + (eta-eta_t)^3), zero below eta_t (Appendix A).

    g0 = (eta_*^3 + (1-eta_t)^3)/(1-eta_t)^3 makes g(1) = 1.
    """
    e = np.asarray(eta, dtype=np.float64) - p.eta_t
    g0 = (p.eta_star ** 3 + (1.0 - p.eta_t) ** 3) / (1.0 - p.eta_t) ** 3
    e3 = np.where(e > 0.0, e, 0.0) ** 3
    return g0 * e3 / (p.eta_star ** 3 + e3)


def release_rate(a):
    """R(tau) = pi^{-1/2} exp(-(tau-3)^2), the ADP release bell of eq. ADP_source."""
    a = np.asarray(a, dtype=np.float64)
    return np.exp(-(a - 3.0) ** 2) / math.sqrt(math.pi)


def margination_shape(R, K, m, n):
    """1 + K R^{m-1} (1-R)^{n-1}: the un-normalised Eckstein-Belgacem shape (Appendix C.1)."""
    return K * R ** (m - 1) * (1.0 - R) ** (n - 1)


def platelet_inflow(y, z, desc, p: Params):
    """P_mu at the inlet, P_0 c(y) (2-D) or P_0 c(y,z) (3-D) (Appendix C.1, C.2).

    1/C0 is the cross-section mean of the bracket: the integral of R^{m-1}(1-R)^{n-1}
    over [0,1] is the Beta function B(m, n), so 1/C0 = 1 + K B(m,n) per direction.
    """
    m, n = p.marg_m, p.marg_n
    beta = math.gamma(m) * math.gamma(n) / math.gamma(m + n)
    ry = 0.5 * desc["Ly"]
    Ry = np.abs(y - ry) / ry
    bracket = 1.0 + margination_shape(Ry, desc["K_y"], m, n)
    inv_c0 = 1.0 + desc["K_y"] * beta
    if desc["dim"] == 3:
        rz = 0.5 * desc["Lz"]
        Rz = np.abs(z - rz) / rz
        bracket = bracket + margination_shape(Rz, desc["K_z"], m, n)
        inv_c0 += desc["K_z"] * beta
    return p.P_0 * bracket / inv_c0


def parabolic_inflow(y, shear, r):
    """u(y) = -(shear/2r)(y-r)^2 + shear r/2 (eq. parabolicVelocity); wall shear = shear."""
    return -(shear / (2.0 * r)) * (y - r) ** 2 + 0.5 * shear * r


def duct_unit_profile(y, z, a, b, nterms=1000):
    """w solving -lap w = 1 on (0,a)x(0,b), w = 0 on the walls (Fourier series in y).

    w = y(a-y)/2 - sum_{n odd} 4a^2/(pi^3 n^3) cosh(n pi (z-b/2)/a)/cosh(n pi b/(2a)) sin(n pi y/a).
    """
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    w = 0.5 * y * (a - y)
    zz = np.abs(z - 0.5 * b)
    B = 0.5 * b
    for k in range(nterms):
        n = 2 * k + 1
        s = n * math.pi / a
        ratio = (np.exp(s * (zz - B)) + np.exp(-s * (zz + B))) / (1.0 + math.exp(-2.0 * s * B))
        w = w - (4.0 * a * a / (math.pi ** 3 * n ** 3)) * ratio * np.sin(s * y)
    return w


def duct_wall_slope(a, b, nterms=200):
    """dw/dy at the bottom wall centre line (y=0, z=b/2) of duct_unit_profile."""
    s = 0.5 * a
    for k in range(nterms):
        n = 2 * k + 1
        x = n * math.pi * b / (2.0 * a)
        s -= (4.0 * a / (math.pi ** 2 * n ** 2)) * 2.0 * math.exp(-x) / (1.0 + math.exp(-2.0 * x))  # 1/cosh x
    return s


# --------------------------------------------------------------------------------------
# Mesh
# --------------------------------------------------------------------------------------

class Mesh:
    """Uniform structured channel [0,Lx]x[0,Ly](x[0,Lz]); cell id = i + nx (j + ny k).

    x=0 inlet, x=Lx outlet, y=0 and y=Ly walls (and z walls in 3-D).  The injury
    patch is the set of y=0 wall faces whose centre lies in the patch rectangle.
    """

    def __init__(self, desc: dict):
        self.desc = desc
        self.dim = desc["dim"]
        self.nx, self.ny, self.nz = desc["nx"], desc["ny"], desc["nz"]
        self.dx = desc["Lx"] / self.nx
        self.dy = desc["Ly"] / self.ny
        self.dz = desc["Lz"] / self.nz
        self.V = self.dx * self.dy * self.dz
        self.n = self.nx * self.ny * self.nz
        self.shape = (self.nz, self.ny, self.nx)
        self.idx = np.arange(self.n).reshape(self.shape)
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        self.xc = ((i + 0.5) * self.dx).ravel()
        self.yc = ((j + 0.5) * self.dy).ravel()
        self.zc = ((k + 0.5) * self.dz).ravel()
        # axis tuple: (numpy axis in the (nz,ny,nx) view, face area, centre spacing)
        self.axes = [(2, self.dy * self.dz, self.dx), (1, self.dx * self.dz, self.dy)]
        if self.dim == 3:
            self.axes.append((0, self.dx * self.dy, self.dz))
        # injury faces on y=0, x-fastest then z
        xi = (np.arange(self.nx) + 0.5) * self.dx
        zi = (np.arange(self.nz) + 0.5) * self.dz
        inx = (xi >= desc["inj_x0"]) & (xi <= desc["inj_x1"])
        inz = (zi >= desc["inj_z0"]) & (zi <= desc["inj_z1"]) if self.dim == 3 else np.ones(self.nz, bool)
        kk, ii = np.meshgrid(np.nonzero(inz)[0], np.nonzero(inx)[0], indexing="ij")
        self.inj_cells = (ii + self.nx * (0 + self.ny * kk)).ravel()   # j = 0 cells under the faces
        self.inj_area = self.dx * self.dz
        self.nface = self.inj_cells.size

    def face_shape(self, ax):
        s = list(self.shape)
        s[ax] += 1
        return tuple(s)

    def adhesion_mask(self, p: Params):
        """H_adh: 1 in cells over the patch whose centre is within P_diam of y=0.

        If the first cell centre is farther than P_diam from the wall, the
        wall-adjacent layer over the patch is used.
        """
        xin = (self.xc >= self.desc["inj_x0"]) & (self.xc <= self.desc["inj_x1"])
        zin = ((self.zc >= self.desc["inj_z0"]) & (self.zc <= self.desc["inj_z1"])) if self.dim == 3 \
            else np.ones(self.n, bool)
        if 0.5 * self.dy <= p.P_diam:
            near = self.yc <= p.P_diam
        else:
            near = self.yc < self.dy
        return (xin & zin & near).astype(np.float64)


def _pair_slices(ax):
    """Slices of a (nz,ny,nx) cell array giving the L and R cells of interior faces on axis ax."""
    L = [slice(None)] * 3
    R = [slice(None)] * 3
    L[ax] = slice(0, -1)
    R[ax] = slice(1, None)
    return tuple(L), tuple(R)


def _face_interior(ax):
    s = [slice(None)] * 3
    s[ax] = slice(1, -1)
    return tuple(s)


def _face_at(ax, pos):
    s = [slice(None)] * 3
    s[ax] = pos
    return tuple(s)


def _cell_at(ax, pos):
    s = [slice(None)] * 3
    s[ax] = pos
    return tuple(s)


class System:
    """Accumulates one sparse linear system row by row: diagonal, couplings, right-hand side."""

    def __init__(self, n):
        self.n = n
        self.diag = np.zeros(n)
        self.rhs = np.zeros(n)
        self.rows, self.cols, self.vals = [], [], []

    def couple(self, r, c, v):
        self.rows.append(np.asarray(r).ravel())
        self.cols.append(np.asarray(c).ravel())
        self.vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.shape(r)).ravel())

    def offdiag(self):
        if not self.rows:
            return sp.csr_matrix((self.n, self.n))
        return sp.csr_matrix((np.concatenate(self.vals), (np.concatenate(self.rows), np.concatenate(self.cols))),
                             shape=(self.n, self.n))

    def matrix(self):
        return (sp.diags(self.diag) + self.offdiag()).tocsr()


def linear_solver(M, spd, direct_max=DIRECT_MAX):
    """A solve function x = f(b, x0) for M x = b: sparse LU (factorised here, once, for
    any number of right-hand sides) up to direct_max unknowns, else a Jacobi-preconditioned
    CG (spd) or BiCGStab solve to a relative residual of 1e-13, started from x0."""
    n = M.shape[0]
    if n <= direct_max:
        lu = spla.splu(M.tocsc(), permc_spec="MMD_AT_PLUS_A")     # structurally symmetric

        def run(b, x0=None):
            if not np.any(b):
                return np.zeros_like(b)
            return lu.solve(b)
        return run
    d = M.diagonal()
    pre = spla.LinearOperator(M.shape, matvec=lambda v: v / d)
    method = spla.cg if spd else spla.bicgstab

    def run(b, x0=None):
        if not np.any(b):
            return np.zeros_like(b)
        # solved for b/||b||: scipy's breakdown tests are absolute, and a right-hand side
        # as small as a species not yet produced (~1e-20) would trip them at once
        s = float(np.linalg.norm(b))
        x, info = method(M, b / s, x0=None if x0 is None else x0 / s, rtol=1e-13, atol=0.0,
                         maxiter=100000, M=pre)
        if info != 0 and not spd:
            # a BiCGStab breakdown: restarted GMRES, which cannot break down, from where it stopped
            x, info = spla.gmres(M, b / s, x0=x, rtol=1e-13, atol=0.0, restart=100, maxiter=1000, M=pre)
        if info != 0:
            raise RuntimeError(f"oracle Krylov solve did not converge (info={info})")
        return x * s
    return run


def solve(M, b, spd, x0=None):
    """Solve M x = b once (see linear_solver)."""
    return linear_solver(M, spd)(b, x0)


# --------------------------------------------------------------------------------------
# Reaction right-hand sides (Appendix A and B)
# --------------------------------------------------------------------------------------

def reaction_rhs(y, adp, gam, hadh, p: Params):
    """d/dt of the 14 reacting species (RXN order; 16 with the inhibitor, I and E2i last)
    with ADP, g(eta) and H_adh frozen.

    Platelets (Appendix A, eqs. Pmu..Pbse): adhesion k_adh H_adh (Pmax - Pbse),
    activation A1(ADP)+A2(E2) with Hill functions, cohesion kcoh Pmax g(eta).
    Coagulation (Appendix B, reactions reactionFirst..reactionFeedback2) by mass
    action with binding-site totals N1/N_A (Pba+Pbse) and N2/N_A (Pba+Pbse).
    """
    Pmu, Pma, Pba, Pbse, S1, S2, E1, E2, S1b, S2b, E1b, E2b, C1, C2 = y[:14]
    adh = p.k_adh * hadh * (p.P_max - Pbse)
    act = p.k_adp * adp / (p.adp_crit + adp) + p.k_e2 * E2 / (p.e2_crit + E2)
    coh = p.kcoh_Pmax * gam
    B1 = (p.N1 / p.N_A) * (Pba + Pbse) - (S1b + E1b + C1 + C2)
    B2 = (p.N2 / p.N_A) * (Pba + Pbse) - (S2b + E2b + C1 + C2)
    c1f = p.kC1p * S2b * E1b
    c2f = p.kC2p * S1b * E2b
    bS1 = p.kS1p * B1 * S1 - p.kS1m * S1b
    bS2 = p.kS2p * B2 * S2 - p.kS2m * S2b
    bE1 = p.kE1p * B1 * E1 - p.kE1m * E1b
    bE2 = p.kE2p * B2 * E2 - p.kE2m * E2b
    rI = p.k_I * y[14] * E2 if p.inhibitor else 0.0      # I + E2 -> E2i, mass action
    rows = [
        -adh * Pmu - act * Pmu,
        -adh * Pma + act * Pmu - coh * Pma,
        -adh * Pba + coh * Pma,
        adh * (Pmu + Pma + Pba),
        -bS1,
        -bS2,
        -bE1,
        -bE2 - rI,
        bS1 - c2f + p.kC2m * C2,
        bS2 - c1f + p.kC1m * C1,
        bE1 - c1f + (p.kC1m + p.kC1cat) * C1 + p.kC2cat * C2,
        bE2 - c2f + (p.kC2m + p.kC2cat) * C2 + p.kC1cat * C1,
        c1f - (p.kC1m + p.kC1cat) * C1,
        c2f - (p.kC2m + p.kC2cat) * C2,
    ]
    if p.inhibitor:
        rows += [-rI, rI]
    return np.array(rows)


def rk4(f, y, h, nsub):
    """nsub steps of classical fourth-order Runge-Kutta with step h (section 3.2)."""
    for _ in range(nsub):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y


def wall_rhs(E0C0, s1w, p: Params):
    """eqs. seBound_E0 / seBound_C0 with the wall value of S1 frozen."""
    E0, C0 = E0C0
    r = p.kC0p * s1w * E0 - (p.kC0m + p.kC0cat) * C0
    return np.array([-r, r])


def van_leer(r):
    """psi(r) = (r + |r|)/(1 + |r|) (Appendix D: van Leer limiter)."""
    return (r + np.abs(r)) / (1.0 + np.abs(r))


# --------------------------------------------------------------------------------------
# The time stepper
# --------------------------------------------------------------------------------------

class Oracle:
    """State and one-step advance of one channel, in float64.

    Fields: u (3, n) velocity (mm/s; 2-D keeps u_z = 0), p kinematic pressure,
    face fluxes phi[ax] (mm^3/s, positive along +axis), species (15, n),
    E0, C0 per injury face, theta_B of the previous step, the release history
    ring (times and snapshots), sigma, t, n.
    """

    def __init__(self, desc: dict, xi_cell: np.ndarray, xi_face: np.ndarray, params: Params | None = None,
                 inlet_u: np.ndarray | None = None):
        self.p = params or Params()
        self.m = Mesh(desc)
        self.desc = desc
        extra = INHIBITOR_SPECIES if self.p.inhibitor else []
        self.species = SPECIES + extra
        self.sp = {n: i for i, n in enumerate(self.species)}
        self.transported = TRANSPORTED + extra
        self.rxn = RXN + extra
        self.dt = desc["dt"]
        self.dt_max = desc["dt"]
        self._init_state(xi_cell, xi_face, inlet_u)

    # ---- O-init -------------------------------------------------------------------
    def _unit_inflow(self, y, z):
        """Inflow speed profile and the kinematic pressure gradient G = -dp/dx it carries."""
        d, p = self.desc, self.p
        if d["dim"] == 2:
            r = 0.5 * d["Ly"]
            return parabolic_inflow(y, d["shear"], r), p.nu * d["shear"] / r
        scale = d["shear"] / duct_wall_slope(d["Ly"], d["Lz"])
        return scale * duct_unit_profile(y, z, d["Ly"], d["Lz"]), p.nu * scale

    def _init_state(self, xi_cell, xi_face, inlet_u):
        m, p = self.m, self.p
        ucell, G = self._unit_inflow(m.yc, m.zc)
        self.u = np.zeros((3, m.n))
        self.u[0] = ucell
        self.p_ = G * (self.desc["Lx"] - m.xc)
        # inlet face values (the i=0 column shares the cell-centre y, z)
        col = m.idx[:, :, 0].ravel()
        self.u_in = ucell[col].copy() if inlet_u is None else np.asarray(inlet_u, dtype=np.float64)
        self.pmu_in = platelet_inflow(m.yc[col], m.zc[col], self.desc, p)
        self.phi = []
        for (ax, A, d) in m.axes:
            self.phi.append(np.zeros(m.face_shape(ax)))
        # x faces carry the profile (x-face centres share y,z with cell centres)
        u3 = ucell.reshape(m.shape)
        self.phi[0][:, :, :m.nx] = m.axes[0][1] * u3
        self.phi[0][:, :, m.nx] = m.axes[0][1] * u3[:, :, -1]
        if inlet_u is not None:
            self.phi[0][:, :, 0] = m.axes[0][1] * self.u_in.reshape(m.nz, m.ny)
        c = np.zeros((len(self.species), m.n))
        c[SP["Pmu"]] = platelet_inflow(m.yc, m.zc, self.desc, p)
        c[SP["S1"]] = p.S1_0
        c[SP["S2"]] = p.S2_0
        c[:len(SPECIES)] *= 1.0 + 0.01 * xi_cell
        if p.inhibitor:
            c[self.sp["I"]] = p.I_0            # no noise draws for the added species
        self.c = c
        self.E0 = p.E0_0 * (1.0 + 0.01 * xi_face[0])
        self.C0 = np.zeros(m.nface) * (1.0 + 0.01 * xi_face[1])
        self.hadh = m.adhesion_mask(p)
        self.thetaB_prev = self.thetaB()
        self.nhist = int(round(p.tau_f / p.dtau)) + 1
        self.hist_t = np.full(self.nhist, -np.inf)
        self.hist_f = np.zeros((self.nhist, m.n))
        self.sigma = np.zeros(m.n)
        self.eta = np.zeros(m.n)
        self.s1w = np.zeros(m.nface)
        self.t = 0.0
        self.n = 0
        self.dt = self.dt_max
        # stored time derivatives of the fields with a ddt term (Crank-Nicolson history)
        self.ddt0u = np.zeros((3, m.n))
        self.ddt0c = {name: np.zeros(m.n) for name in self.transported}
        if p.max_co > 0.0:
            # a variable step starts at the largest step the initial flux allows
            co = self.courant()
            if co > p.max_co:
                self.dt = p.max_co * self.dt / co
        self.next_push = 0
        self.stats = {}

    # ---- derived (O-0) --------------------------------------------------------------
    def thetaB(self):
        return (self.c[SP["Pba"]] + self.c[SP["Pbse"]]) / self.p.P_max

    def thetaT(self):
        c = self.c
        return (c[SP["Pmu"]] + c[SP["Pma"]] + c[SP["Pba"]] + c[SP["Pbse"]]) / self.p.P_max

    # ---- time scheme -----------------------------------------------------------------
    def ddt_coeffs(self):
        """(k, w) of this step's time derivative of a field f (Appendix D table,
        CrankNicolson psi): ddt f = k (f^{n+1} - f^n)/dt - w D^n, with D^n the stored
        derivative of the previous step, itself updated as D^{n+1} = k (f^{n+1} - f^n)/dt
        - w D^n.  When D^n solves the previous step's equation this is the theta scheme
        with weight 1/(1+psi) on the new and psi/(1+psi) on the old right-hand side
        (psi = 1: trapezoidal Crank-Nicolson, psi = 0: implicit Euler).  The first step
        has no stored derivative and is implicit Euler."""
        psi = self.p.ddt_psi
        if psi == 0.0 or self.n == 0:
            return 1.0, 0.0
        return 1.0 + psi, psi

    def courant(self):
        """Largest cell Courant number 0.5 dt sum_f |phi_f| / V with the current flux."""
        m = self.m
        tot = np.zeros(m.shape)
        for a, (ax, A, d) in enumerate(m.axes):
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[ax] = slice(1, None)
            lo[ax] = slice(0, -1)
            tot += np.abs(self.phi[a][tuple(hi)]) + np.abs(self.phi[a][tuple(lo)])
        return 0.5 * self.dt * float(tot.max()) / m.V

    def next_dt(self):
        """Variable step (Appendix D: the step keeps the Courant number at or below
        maxCo): the step after this one is the largest that holds the largest cell
        Courant number of the current flux at max_co, grows by at most dt_growth per
        step and never exceeds the channel's dt."""
        p = self.p
        co = self.courant()
        cand = min(self.dt_max, p.dt_growth * self.dt)
        if co > 0.0:
            cand = min(cand, p.max_co * self.dt / co)
        return cand

    # ---- helpers ---------------------------------------------------------------------
    def _grad(self, phi_cell, low_value, high_value):
        """Gauss-linear cell gradient: (1/V) sum_f phi_f A n_f with the given boundary face values.

        low_value/high_value(ax, cell_face_slice) return boundary face values.
        """
        m = self.m
        f3 = phi_cell.reshape(m.shape)
        g = np.zeros((3, m.n))
        for comp, (ax, A, d) in enumerate(m.axes):
            fs = np.zeros(m.face_shape(ax))
            L, R = _pair_slices(ax)
            fs[_face_interior(ax)] = 0.5 * (f3[L] + f3[R])
            fs[_face_at(ax, 0)] = low_value(ax, f3[_cell_at(ax, 0)])
            fs[_face_at(ax, -1)] = high_value(ax, f3[_cell_at(ax, -1)])
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[ax] = slice(1, None)
            lo[ax] = slice(0, -1)
            g[comp] = ((fs[tuple(hi)] - fs[tuple(lo)]) / d).ravel()
        return g

    def grad_p(self, pfield):
        """(grad p)_P, Gauss linear; outlet face = p_out, other boundary faces = p_P (zero gradient)."""
        pout = self.p.p_out
        return self._grad(pfield, lambda ax, v: v,
                          lambda ax, v: (np.full_like(v, pout) if ax == 2 else v))

    # ---- O-1 momentum ------------------------------------------------------------------
    def momentum_system(self, alpha):
        """Momentum matrix with the ddt scheme of ddt_coeffs, phi^n convection (Gauss
        linear), nu Laplacian, implicit Darcy nu*alpha*V on the diagonal, and boundary
        terms (Appendix C table).

        Returns (System, src) with src[c] = k V u_c^n/dt + w V D_c^n + boundary sources
        (no pressure)."""
        m, p, dt = self.m, self.p, self.dt
        k, w = self.ddt_coeffs()
        S = System(m.n)
        S.diag += k * m.V / dt + p.nu * alpha * m.V
        src = np.zeros((3, m.n))
        src += k * m.V * self.u / dt + w * m.V * self.ddt0u
        ids = m.idx
        for a, (ax, A, d) in enumerate(m.axes):
            L, R = _pair_slices(ax)
            phi = self.phi[a][_face_interior(ax)]
            dif = p.nu * A / d
            iL, iR = ids[L], ids[R]
            np.add.at(S.diag, iL.ravel(), (0.5 * phi + dif).ravel())
            np.add.at(S.diag, iR.ravel(), (-0.5 * phi + dif).ravel())
            S.couple(iL, iR, 0.5 * phi - dif)
            S.couple(iR, iL, -0.5 * phi - dif)
            lo = ids[_cell_at(ax, 0)].ravel()
            hi = ids[_cell_at(ax, -1)].ravel()
            if ax == 2:      # x: inlet (fixed value) and outlet (zero gradient)
                phi_out_in = -self.phi[a][_face_at(ax, 0)].ravel()
                np.add.at(S.diag, lo, 2.0 * dif)
                src[0][lo] += 2.0 * dif * self.u_in - phi_out_in * self.u_in
                phi_out = self.phi[a][_face_at(ax, -1)].ravel()
                np.add.at(S.diag, hi, phi_out)
            else:            # no-slip walls
                np.add.at(S.diag, lo, 2.0 * dif)
                np.add.at(S.diag, hi, 2.0 * dif)
        return S, src

    # ---- O-2 PISO -------------------------------------------------------------------------
    def n_correctors(self):
        """Pressure corrections per step.  Section 3.2 asks for "multiple" corrections;
        a fixed count is used when set, otherwise it grows with the viscous diffusion
        number nu dt / h_min^2, above which fewer corrections let PISO diverge."""
        if self.p.n_corr > 0:
            return self.p.n_corr
        m = self.m
        h = min(m.dx, m.dy, m.dz if m.dim == 3 else m.dy)
        Dn = self.p.nu * self.dt_max / (h * h)     # the largest step (variable steps never exceed it)
        return 2 if Dn <= 10.0 else 3 if Dn <= 30.0 else 4 if Dn <= 50.0 else 5 if Dn <= 80.0 else 6 if Dn <= 120.0 else 8

    def flow_step(self, alpha):
        """Momentum predictor + n_corr PISO correctors (section 3.2); updates u, p, phi."""
        m, p = self.m, self.p
        ncomp = m.dim
        u_old = self.u.copy()
        k_dt, w_dt = self.ddt_coeffs()
        S, src = self.momentum_system(alpha)
        M = S.matrix()
        Noff = S.offdiag()
        gp = self.grad_p(self.p_)
        mom = linear_solver(M, spd=False, direct_max=FLOW_DIRECT_MAX)   # the components share M
        for c in range(ncomp):
            self.u[c] = mom(src[c] - m.V * gp[c], self.u[c])
        aP = S.diag
        rAU = m.V / aP
        ids = m.idx
        # pressure matrix: sum_f c_f (p_P - p_N) + c_out p_P, c_f = rAU_f A/d; rAU is fixed
        # by the predictor, so every corrector of the step solves with the same matrix
        K = System(m.n)
        r3 = rAU.reshape(m.shape)
        coefs = []
        for a, (ax, A, d) in enumerate(m.axes):
            L, R = _pair_slices(ax)
            cf = 0.5 * (r3[L] + r3[R]) * A / d
            coefs.append(cf)
            iL, iR = ids[L], ids[R]
            np.add.at(K.diag, iL.ravel(), cf.ravel())
            np.add.at(K.diag, iR.ravel(), cf.ravel())
            K.couple(iL, iR, -cf)
            K.couple(iR, iL, -cf)
        Ax, dx = m.axes[0][1], m.axes[0][2]
        out = ids[:, :, -1].ravel()
        c_out = r3[:, :, -1].ravel() * 2.0 * Ax / dx
        np.add.at(K.diag, out, c_out)
        pres = linear_solver(K.matrix(), spd=True, direct_max=FLOW_DIRECT_MAX)
        for _ in range(self.n_correctors()):
            HbyA = np.zeros((3, m.n))
            for c in range(ncomp):
                HbyA[c] = (src[c] - Noff @ self.u[c]) / aP
            # face fluxes of HbyA
            phiH = []
            for a, (ax, A, d) in enumerate(m.axes):
                h3 = HbyA[a].reshape(m.shape)
                f = np.zeros(m.face_shape(ax))
                L, R = _pair_slices(ax)
                f[_face_interior(ax)] = A * 0.5 * (h3[L] + h3[R])
                if ax == 2:
                    f[_face_at(ax, 0)] = A * self.u_in.reshape(m.nz, m.ny)
                    f[_face_at(ax, -1)] = A * h3[_cell_at(ax, -1)]
                phiH.append(f)
            # pressure equation: K p = -div(phiH) + c_out p_out, warm-started from p
            div = np.zeros(m.shape)
            for a, (ax, A, d) in enumerate(m.axes):
                hi = [slice(None)] * 3
                lo = [slice(None)] * 3
                hi[ax] = slice(1, None)
                lo[ax] = slice(0, -1)
                div += phiH[a][tuple(hi)] - phiH[a][tuple(lo)]
            rhs = -div.ravel()
            rhs[out] += c_out * p.p_out
            self.p_ = pres(rhs, self.p_)
            p3 = self.p_.reshape(m.shape)
            for a, (ax, A, d) in enumerate(m.axes):
                L, R = _pair_slices(ax)
                f = phiH[a].copy()
                f[_face_interior(ax)] -= coefs[a] * (p3[R] - p3[L])
                if ax == 2:
                    f[_face_at(ax, -1)] -= c_out.reshape(m.nz, m.ny) * (p.p_out - p3[:, :, -1])
                self.phi[a] = f
            gp = self.grad_p(self.p_)
            for c in range(ncomp):
                self.u[c] = HbyA[c] - rAU * gp[c]
        self.ddt0u = k_dt * (self.u - u_old) / self.dt - w_dt * self.ddt0u
        self.stats["rAU"] = rAU

    def continuity_residual(self):
        """sum_f phi_f (outward) per cell."""
        m = self.m
        div = np.zeros(m.shape)
        for a, (ax, A, d) in enumerate(m.axes):
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[ax] = slice(1, None)
            lo[ax] = slice(0, -1)
            div += self.phi[a][tuple(hi)] - self.phi[a][tuple(lo)]
        return div.ravel()

    # ---- O-3 eta ---------------------------------------------------------------------------
    def eta_solve(self, thetaB):
        """eta - (L_eta^2/4) lap eta = theta_B (Appendix A, eq. eta), zero gradient walls."""
        m, p = self.m, self.p
        kappa = (p.L_eta_over_Pdiam * p.P_diam) ** 2 / 4.0
        S = System(m.n)
        S.diag += m.V
        for a, (ax, A, d) in enumerate(m.axes):
            L, R = _pair_slices(ax)
            iL, iR = m.idx[L], m.idx[R]
            c = kappa * A / d
            np.add.at(S.diag, iL.ravel(), c)
            np.add.at(S.diag, iR.ravel(), c)
            S.couple(iL, iR, -c)
            S.couple(iR, iL, -c)
        return solve(S.matrix(), m.V * thetaB, spd=True, x0=self.eta)

    # ---- O-4 sigma ---------------------------------------------------------------------------
    def sigma_update(self, thetaB):
        """Release-history push and trapezoid of eq. sigma_disc.

        A snapshot Pmax(theta_B^n - theta_B^{n-1})/dt is pushed at n = 0 and at the
        first step whose time reaches each multiple of dtau; sigma is recomputed at
        a push and held in between.  Nodes are the stored snapshots, newest first,
        aged t_n - tau_k; absent ones count as zero.
        """
        p = self.p
        n_now = int(math.floor(self.t / p.dtau + 1e-9))
        if self.n > 0 and n_now < self.next_push:
            return
        self.next_push = n_now + 1
        if self.n == 0:
            f = np.zeros(self.m.n)
        else:
            f = p.P_max * (thetaB - self.thetaB_prev) / self.dt
        self.hist_t = np.roll(self.hist_t, 1)
        self.hist_f = np.roll(self.hist_f, 1, axis=0)
        self.hist_t[0] = self.t
        self.hist_f[0] = f
        ntrap = self.nhist - 1
        sig = np.zeros(self.m.n)
        for k in range(ntrap):
            for kk in (k, k + 1):
                if np.isfinite(self.hist_t[kk]):
                    sig += 0.5 * p.dtau * release_rate(self.t - self.hist_t[kk]) * self.hist_f[kk]
        self.sigma = p.A_hat * sig

    # ---- O-5 transport -------------------------------------------------------------------------
    def transport_system(self, name, thetaT):
        """Implicit upwind-biased TVD transport system of one scalar (Appendix D, App. C table)."""
        m, p, dt = self.m, self.p, self.dt
        k_dt, w_dt = self.ddt_coeffs()
        platelet = name in ("Pmu", "Pma")
        D = p.D_P if platelet else (p.D_ADP if name == "ADP" else p.D_chem)
        Cn = self.c[self.sp[name]]
        C3 = Cn.reshape(m.shape)
        T3 = thetaT.reshape(m.shape)
        S = System(m.n)
        S.diag += k_dt * m.V / dt
        S.rhs = k_dt * m.V * Cn / dt + w_dt * m.V * self.ddt0c[name]
        if name == "ADP":
            S.rhs = S.rhs + m.V * self.sigma
        ids = m.idx
        for a, (ax, A, d) in enumerate(m.axes):
            L, R = _pair_slices(ax)
            phi = self.phi[a][_face_interior(ax)]
            CL, CR = C3[L], C3[R]
            pos = phi >= 0.0
            # upwind, downwind and far-upwind values of C^n
            CU = np.where(pos, CL, CR)
            CD = np.where(pos, CR, CL)
            n_ax = m.shape[ax]
            # far-upwind cell: L-1 for positive flux, R+1 for negative flux
            CUU = np.zeros_like(CU)
            valid = np.zeros(CU.shape, bool)
            if n_ax >= 3:
                sl_lm1 = [slice(None)] * 3
                sl_lm1[ax] = slice(0, -2)
                sl_rp1 = [slice(None)] * 3
                sl_rp1[ax] = slice(2, None)
                inner = [slice(None)] * 3
                inner_p = list(inner)
                inner_p[ax] = slice(1, None)          # faces whose L has a left neighbour
                inner_n = list(inner)
                inner_n[ax] = slice(0, -1)            # faces whose R has a right neighbour
                tmp = np.zeros_like(CU)
                tmp[tuple(inner_p)] = C3[tuple(sl_lm1)]
                vp = np.zeros(CU.shape, bool)
                vp[tuple(inner_p)] = True
                tmn = np.zeros_like(CU)
                tmn[tuple(inner_n)] = C3[tuple(sl_rp1)]
                vn = np.zeros(CU.shape, bool)
                vn[tuple(inner_n)] = True
                CUU = np.where(pos, tmp, tmn)
                valid = np.where(pos, vp, vn)
            den = CD - CU
            ok = valid & (den != 0.0)
            if platelet:
                ok &= (CU >= 0.0) & (CU <= p.P_max) & (CD >= 0.0) & (CD <= p.P_max)
            r = np.where(ok, (CU - CUU) / np.where(den != 0.0, den, 1.0), 0.0)
            psi = np.where(ok, van_leer(r), 0.0)
            wU = 1.0 - 0.5 * psi
            wD = 0.5 * psi
            wL = np.where(pos, wU, wD)
            wR = np.where(pos, wD, wU)
            if platelet:
                Wa = hindrance(np.where(pos, T3[R], T3[L]))       # downwind theta_T
                Wd = hindrance(np.maximum(T3[L], T3[R]))          # localMax theta_T
            else:
                Wa = np.ones_like(phi)
                Wd = np.ones_like(phi)
            dif = Wd * D * A / d
            conv = Wa * phi
            iL, iR = ids[L], ids[R]
            np.add.at(S.diag, iL.ravel(), (conv * wL + dif).ravel())
            np.add.at(S.diag, iR.ravel(), (-conv * wR + dif).ravel())
            S.couple(iL, iR, conv * wR - dif)
            S.couple(iR, iL, -conv * wL - dif)
            if ax == 2:
                lo = ids[:, :, 0].ravel()
                hi = ids[:, :, -1].ravel()
                Wlo = hindrance(thetaT[lo]) if platelet else 1.0
                Whi = hindrance(thetaT[hi]) if platelet else 1.0
                phi_out_in = -self.phi[a][:, :, 0].ravel()
                fixed = {"Pmu": self.pmu_in, "S1": p.S1_0, "S2": p.S2_0, "I": p.I_0}.get(name)
                if fixed is not None:
                    Cb = np.broadcast_to(fixed, lo.shape)
                    g = 2.0 * Wlo * D * A / d
                    np.add.at(S.diag, lo, g * np.ones_like(Cb))
                    S.rhs[lo] += g * Cb - Wlo * phi_out_in * Cb
                else:
                    np.add.at(S.diag, lo, Wlo * phi_out_in)
                phi_out = self.phi[a][:, :, -1].ravel()
                np.add.at(S.diag, hi, Whi * phi_out)
        # reactive injury wall (Appendix C table; normal into the fluid)
        Ai = m.inj_area
        if name == "E1":
            np.add.at(S.rhs, m.inj_cells, Ai * p.kC0cat * self.C0)
        if name == "S1":
            k = p.kC0p * self.E0
            q = p.kC0m * self.C0
            g = p.D_chem / (0.5 * m.dy)
            np.add.at(S.diag, m.inj_cells, Ai * k * g / (g + k))
            np.add.at(S.rhs, m.inj_cells, Ai * q * g / (g + k))
        return S

    def transport(self, thetaT):
        """The 7 transport solves; each species' stored time derivative is that of its
        transport sub-step (from C^n to the transported value; the reactions that follow
        in the fractional step are not part of it)."""
        out = {}
        for name in self.transported:
            S = self.transport_system(name, thetaT)
            out[name] = solve(S.matrix(), S.rhs, spd=False, x0=self.c[self.sp[name]])
        k_dt, w_dt = self.ddt_coeffs()
        for name, v in out.items():
            self.ddt0c[name] = k_dt * (v - self.c[self.sp[name]]) / self.dt - w_dt * self.ddt0c[name]
            self.c[self.sp[name]] = v

    # ---- O-6 reactions ---------------------------------------------------------------------------
    def wall_value_S1(self):
        """S1 on the injury face from the Robin balance g(S1_P - S1_w) = k S1_w - q."""
        p, m = self.p, self.m
        k = p.kC0p * self.E0
        q = p.kC0m * self.C0
        g = p.D_chem / (0.5 * m.dy)
        return (q + g * self.c[SP["S1"]][m.inj_cells]) / (g + k)

    def reactions(self):
        p = self.p
        h = self.dt / p.M_rxn
        # wall first, with the post-transport S1 wall value and E0^n, C0^n
        self.s1w = self.wall_value_S1()
        s1w = self.s1w
        y = rk4(lambda v: wall_rhs(v, s1w, p), np.array([self.E0, self.C0]), h, p.M_rxn)
        self.E0, self.C0 = y[0], y[1]
        gam = binding_affinity(self.eta, p)
        adp = self.c[SP["ADP"]]
        hadh = self.hadh
        ids = [self.sp[s] for s in self.rxn]
        y = rk4(lambda v: reaction_rhs(v, adp, gam, hadh, p), self.c[ids].copy(), h, p.M_rxn)
        self.c[ids] = y

    # ---- one step ---------------------------------------------------------------------------
    def step(self, flow=True, transport=True, react=True):
        thB = self.thetaB()
        thT = self.thetaT()
        if flow:
            self.flow_step(carman_kozeny(thB, self.p))
        self.eta = self.eta_solve(thB)
        self.sigma_update(thB)
        if transport:
            self.transport(thT)
        if react:
            self.reactions()
        self.thetaB_prev = thB
        self.n += 1
        if self.p.max_co > 0.0:
            self.t += self.dt
            self.stats["co"] = self.courant()
            self.dt = self.next_dt()
        else:
            self.t = self.n * self.dt

    def fields(self):
        """Dict of float64 arrays keyed by library field names."""
        out = {"UX": self.u[0].copy(), "UY": self.u[1].copy(), "P": self.p_.copy(),
               "PHIX": self.phi[0].ravel().copy(), "PHIY": self.phi[1].ravel().copy(),
               "E0": self.E0.copy(), "C0": self.C0.copy(), "ETA": self.eta.copy(),
               "SIGMA": self.sigma.copy()}
        if self.m.dim == 3:
            out["UZ"] = self.u[2].copy()
            out["PHIZ"] = self.phi[2].ravel().copy()
        for n in self.species:
            out[n.upper()] = self.c[self.sp[n]].copy()
        return out
