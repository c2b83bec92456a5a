// Per-cell kernels of one clotting time step (gfx950).  Each cites the part of the
// model it computes; the Krylov solves between them live in clot_krylov.h.
#pragma once
#include "clot_krylov.h"

namespace clot {

// theta_B (section 2: bound platelets over P_max) and W(theta_T) (Appendix A).
template <class T>
__global__ __launch_bounds__(NT) void k_derive(Grid G, Fields<T> F, ModelDev M) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        const T pmax = T(M.P_max);
        const T pb = F.spc[PBA][g] + F.spc[PBSE][g];
        const T tt = F.spc[PMU][g] + F.spc[PMA][g] + pb;
        F.thB[g] = pb / pmax;
        F.Wc[g] = hindrance_fn<T>(tt / pmax);
    CLOT_END_CELLS
}

// Momentum predictor matrix diagonal and right-hand sides (section 3.2; Appendix D
// schemes; Appendix C boundary table).  Time derivative k (u' - u)/dt - w D (implicit
// Euler: k = 1, w = 0; Crank-Nicolson psi: k = 1+psi, w = psi with the stored
// derivative D), Gauss-linear convection with the old flux, nu Laplacian, implicit
// Darcy nu alpha(theta_B) V with the Carman-Kozeny alpha, Gauss-linear gradient of the
// old pressure.  With Crank-Nicolson, D is replaced by -(k/dt u + w D); the step's end
// adds k/dt u' (k_ddt_close).
template <class T>
__global__ __launch_bounds__(NT) void k_mom_assemble(Grid G, Fields<T> F, ModelDev M) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int64_t g = P.g;
        const T V = T(C.V), rdt = T(C.rdt), nu = T(M.nu);
        const T kd = T(C.ddtk), kvr = kd * V * rdt;
        const T s = T(0.6) * F.thB[g];
        const T om = T(1) - s;
        const T alpha = T(M.C_CK) * s * s / (om * om * om);
        T aP = kvr + nu * alpha * V;
        T srcx = T(0);
        // x faces: inlet (fixed value) at i = 0, outlet (zero gradient) at i = nx-1
        const T dfx = nu * T(C.gx);
        const T fw = F.phi[0][fx_id(C, P.i, P.j, P.k)];
        const T fe = F.phi[0][fx_id(C, P.i + 1, P.j, P.k)];
        if (P.i > 0) aP += T(-0.5) * fw + dfx;
        else {
            const T ub = F.u_in[C.in0 + P.j + (int64_t)C.ny * P.k];
            aP += T(2) * dfx;
            srcx += T(2) * dfx * ub + fw * ub;     // - (outward flux -fw) * u_b
        }
        if (P.i < C.nx - 1) aP += T(0.5) * fe + dfx;
        else aP += fe;
        // y faces: no-slip walls
        const T dfy = nu * T(C.gy);
        const T fs = F.phi[1][fy_id(C, P.i, P.j, P.k)];
        const T fn = F.phi[1][fy_id(C, P.i, P.j + 1, P.k)];
        aP += (P.j > 0) ? T(-0.5) * fs + dfy : T(2) * dfy;
        aP += (P.j < C.ny - 1) ? T(0.5) * fn + dfy : T(2) * dfy;
        if (C.dim == 3) {
            const T dfz = nu * T(C.gz);
            const T fb = F.phi[2][fz_id(C, P.i, P.j, P.k)];
            const T ff = F.phi[2][fz_id(C, P.i, P.j, P.k + 1)];
            aP += (P.k > 0) ? T(-0.5) * fb + dfz : T(2) * dfz;
            aP += (P.k < C.nz - 1) ? T(0.5) * ff + dfz : T(2) * dfz;
        }
        F.aP[g] = aP;
        F.rAU[g] = T(C.V) / aP;   // fixed for the step: the pressure hierarchy is built from it once
        // Gauss-linear gradient of the old pressure (outlet face p_out, others p_P)
        const double pP = F.p[g];
        const double pw = P.i > 0 ? 0.5 * (F.p[g - 1] + pP) : pP;
        const double pe = P.i < C.nx - 1 ? 0.5 * (F.p[g + 1] + pP) : M.p_out;
        const double ps = P.j > 0 ? 0.5 * (F.p[g - C.nx] + pP) : pP;
        const double pn = P.j < C.ny - 1 ? 0.5 * (F.p[g + C.nx] + pP) : pP;
        const double gx = (pe - pw) / C.dx, gy = (pn - ps) / C.dy;
        T sx = kvr * F.u[0][g] + srcx;
        T sy = kvr * F.u[1][g];
        if (M.psi > 0.0) {
            const T w = T(C.ddtw), kr = kd * rdt;
            const T q0 = F.ddt0u[0][g], q1 = F.ddt0u[1][g];
            sx += w * V * q0;
            sy += w * V * q1;
            F.ddt0u[0][g] = -(kr * F.u[0][g] + w * q0);
            F.ddt0u[1][g] = -(kr * F.u[1][g] + w * q1);
        }
        F.src[0][g] = sx;
        F.src[1][g] = sy;
        F.bm[0][g] = T((double)sx - C.V * gx);
        F.bm[1][g] = T((double)sy - C.V * gy);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            const double pb = P.k > 0 ? 0.5 * (F.p[g - sz] + pP) : pP;
            const double pf = P.k < C.nz - 1 ? 0.5 * (F.p[g + sz] + pP) : pP;
            T sz_ = kvr * F.u[2][g];
            if (M.psi > 0.0) {
                const T w = T(C.ddtw), kr = kd * rdt;
                const T q2 = F.ddt0u[2][g];
                sz_ += w * V * q2;
                F.ddt0u[2][g] = -(kr * F.u[2][g] + w * q2);
            }
            F.src[2][g] = sz_;
            F.bm[2][g] = T((double)sz_ - C.V * (pf - pb) / C.dz);
        } else {
            F.src[2][g] = T(0);
            F.bm[2][g] = T(0);
        }
    CLOT_END_CELLS
}

// PISO: H = src - sum a_N u_N with the latest u; HbyA = H / aP (rAU = V / aP comes
// from the assembly).
template <class T>
__global__ __launch_bounds__(NT) void k_hbya(Grid G, Fields<T> F, MomOp<T> op, const int32_t* mask) {
    CLOT_TILE_PROLOGUE(G)
    if (!mask[chid]) return;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T aP = F.aP[P.g];
        for (int c = 0; c < C.dim; ++c) {
            const T* u = F.u[c];
            const T off = op.offsum(C, P, [&](int64_t g) { return u[g]; });
            F.HbyA[c][P.g] = (F.src[c][P.g] - off) / aP;
        }
        if (C.dim == 2) F.HbyA[2][P.g] = T(0);
    CLOT_END_CELLS
}

// Face flux of HbyA (Gauss linear; inlet: fixed u, walls: 0, outlet: HbyA_P).
template <class T>
__device__ inline double phiH_x(const ChanDev& C, const Fields<T>& F, const Cell& P, int iface) {
    // x-face iface of row (j,k); iface in [0, nx]
    const int64_t row = C.c0 + (int64_t)C.nx * (P.j + (int64_t)C.ny * P.k);
    if (iface == 0) return C.Ax * (double)F.u_in[C.in0 + P.j + (int64_t)C.ny * P.k];
    if (iface == C.nx) return C.Ax * (double)F.HbyA[0][row + C.nx - 1];
    return 0.5 * C.Ax * ((double)F.HbyA[0][row + iface - 1] + (double)F.HbyA[0][row + iface]);
}

// Pressure system: rhs = -sum_f(outward phiHbyA) + c_out p_out, diagonal dP.
template <class T>
__global__ __launch_bounds__(NT) void k_prhs(Grid G, Fields<T> F, ModelDev M, const int32_t* mask) {
    CLOT_TILE_PROLOGUE(G)
    if (!mask[chid]) return;
    PresOp<T, double> op{F.rAU, F.dP};
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int64_t g = P.g;
        double div = phiH_x(C, F, P, P.i + 1) - phiH_x(C, F, P, P.i);
        const double hy = (double)F.HbyA[1][g];
        if (P.j < C.ny - 1) div += 0.5 * C.Ay * (hy + (double)F.HbyA[1][g + C.nx]);
        if (P.j > 0) div -= 0.5 * C.Ay * (hy + (double)F.HbyA[1][g - C.nx]);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            const double hz = (double)F.HbyA[2][g];
            if (P.k < C.nz - 1) div += 0.5 * C.Az * (hz + (double)F.HbyA[2][g + sz]);
            if (P.k > 0) div -= 0.5 * C.Az * (hz + (double)F.HbyA[2][g - sz]);
        }
        double rhs = -div;
        if (P.i == C.nx - 1) rhs += 2.0 * C.gx * (double)F.rAU[g] * M.p_out;
        F.rhs_p[g] = rhs;
        F.dP[g] = T(op.diag_exact(C, P));
    CLOT_END_CELLS
}

// FP64 residual of the pressure system r = rhs - K p; stores r in the inner
// right-hand side (arithmetic type T); partial sums of ||r||^2 and ||rhs||^2.
template <class T>
__global__ __launch_bounds__(NT) void k_pres_resid(Grid G, Fields<T> F, T* rin, T* ein, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5 * 2];
    PresOp<T, double> op{F.rAU, F.dP};
    double acc[2] = {0.0, 0.0};
    const double* p = F.p;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const double kp = op.diag_exact(C, P) * p[P.g] - op.offsum(C, P, [&](int64_t g) { return p[g]; });
        const double b = F.rhs_p[P.g];
        const double r = b - kp;
        rin[P.g] = T(r);
        ein[P.g] = T(0);
        acc[0] += r * r;
        acc[1] += b * b;
    CLOT_END_CELLS
    store_partials<2>(acc, S.part, S.pstride, tile, lds);
}

// Decides on the device whether a channel needs another refinement pass, and the
// inner solve's target: a fraction of this residual, not below the outer goal.  A
// pass that fails to halve the residual ends the refinement: the residual has reached
// the floor the FP64 arithmetic allows (the goal is relative to |b|, which can be
// small next to the terms of A p), and further passes would not change p.
struct EpiPresResid {
    double rtol, rtol_inner;
    int pass;
    int32_t* refmask;
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        double* s = scp(S, ch, 0);
        const double rr = sums[0], bb = sums[1];
        const bool stalled = pass > 0 && rr > 0.25 * s[SC_ORRP];
        s[SC_ORR] = rr;
        s[SC_OBB] = bb;
        s[SC_ORRP] = rr;
        s[SC_PASS] = (double)pass;
        const double target2 = rtol * rtol * bb;
        if (rr <= target2 || bb == 0.0 || !isfinite(rr) || stalled) {
            S.chact[ch] = 0;
            refmask[ch] = 0;
            atomicSub(S.nact, 1);
            s[SC_ACT] = 0.0;
            if (!isfinite(rr)) s[SC_FAIL] = 1.0;
        } else {
            const double inner2 = rtol_inner * rtol_inner * rr;
            s[SC_TOL2] = inner2 > 0.25 * target2 ? inner2 : 0.25 * target2;
            s[SC_ACT] = 1.0;
            s[SC_PASS] = (double)(pass + 1);
            refmask[ch] = 1;
        }
    }
};

// p += e (FP64 accumulation of the inner correction).
template <class T>
__global__ __launch_bounds__(NT) void k_pres_add(Grid G, Fields<T> F, const T* e, const int32_t* chmask) {
    CLOT_TILE_PROLOGUE(G)
    if (!chmask[chid]) return;
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        F.p[g] += (double)e[g];
    CLOT_END_CELLS
}

// PISO flux and velocity correction: phi = phiHbyA - rAU_f (A/d)(p_N - p_P) on the
// faces each cell owns (its low faces, plus the high boundary faces), and
// u = HbyA - rAU (grad p)_P with the Gauss-linear gradient.
template <class T>
__global__ __launch_bounds__(NT) void k_correct(Grid G, Fields<T> F, ModelDev M, const int32_t* mask) {
    CLOT_TILE_PROLOGUE(G)
    if (!mask[chid]) return;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int64_t g = P.g;
        const double* p = F.p;
        const double pP = p[g];
        const double rP = (double)F.rAU[g];
        // x faces
        {
            double f = phiH_x(C, F, P, P.i);
            if (P.i > 0) f -= 0.5 * (rP + (double)F.rAU[g - 1]) * C.gx * (pP - p[g - 1]);
            F.phin[0][fx_id(C, P.i, P.j, P.k)] = T(f);
            if (P.i == C.nx - 1) {
                double fo = phiH_x(C, F, P, C.nx) - rP * 2.0 * C.gx * (M.p_out - pP);
                F.phin[0][fx_id(C, C.nx, P.j, P.k)] = T(fo);
            }
        }
        // y faces (walls carry no flux)
        {
            double f = 0.0;
            if (P.j > 0)
                f = 0.5 * C.Ay * ((double)F.HbyA[1][g - C.nx] + (double)F.HbyA[1][g]) -
                    0.5 * (rP + (double)F.rAU[g - C.nx]) * C.gy * (pP - p[g - C.nx]);
            F.phin[1][fy_id(C, P.i, P.j, P.k)] = T(f);
            if (P.j == C.ny - 1) F.phin[1][fy_id(C, P.i, C.ny, P.k)] = T(0);
        }
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            double f = 0.0;
            if (P.k > 0)
                f = 0.5 * C.Az * ((double)F.HbyA[2][g - sz] + (double)F.HbyA[2][g]) -
                    0.5 * (rP + (double)F.rAU[g - sz]) * C.gz * (pP - p[g - sz]);
            F.phin[2][fz_id(C, P.i, P.j, P.k)] = T(f);
            if (P.k == C.nz - 1) F.phin[2][fz_id(C, P.i, P.j, C.nz)] = T(0);
        }
        // velocity
        const double pw = P.i > 0 ? 0.5 * (p[g - 1] + pP) : pP;
        const double pe = P.i < C.nx - 1 ? 0.5 * (p[g + 1] + pP) : M.p_out;
        const double ps = P.j > 0 ? 0.5 * (p[g - C.nx] + pP) : pP;
        const double pn = P.j < C.ny - 1 ? 0.5 * (p[g + C.nx] + pP) : pP;
        F.u[0][g] = T((double)F.HbyA[0][g] - rP * (pe - pw) / C.dx);
        F.u[1][g] = T((double)F.HbyA[1][g] - rP * (pn - ps) / C.dy);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            const double pb = P.k > 0 ? 0.5 * (p[g - sz] + pP) : pP;
            const double pf = P.k < C.nz - 1 ? 0.5 * (p[g + sz] + pP) : pP;
            F.u[2][g] = T((double)F.HbyA[2][g] - rP * (pf - pb) / C.dz);
        }
    CLOT_END_CELLS
}

// eta right-hand side V theta_B (Appendix A, eq. eta) and its stored diagonal.
template <class T>
__global__ __launch_bounds__(NT) void k_eta_prep(Grid G, Fields<T> F, ModelDev M, T* rhs) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        rhs[P.g] = T(C.V) * F.thB[P.g];
        F.dE[P.g] = EtaOp<T>::diag_of(T(M.kappa_eta), C, P);
    CLOT_END_CELLS
}

// Release history push and trapezoid (section 3.2, eq. sigma_disc): when channel ch
// pushes at this step, hist[slot] = Pmax (theta_B^n - theta_B^{n-1}) / dt (zero at
// the first step) and sigma = sum_k w_k hist[k] with the per-channel weights
// w_k = A_hat * trapezoid weight * R(age_k) computed on the host.
template <class T>
__global__ __launch_bounds__(NT) void k_sigma(Grid G, Fields<T> F, ModelDev M, const double* w, const int32_t* push) {
    CLOT_TILE_PROLOGUE(G)
    const int32_t slot = push[2 * chid];
    if (slot < 0) return;
    const int first = push[2 * chid + 1];
    const double* wc = w + (int64_t)chid * NHIST;
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        const T f = first ? T(0) : T(M.P_max) * (F.thB[g] - F.thB_prev[g]) / T(C.dt);
        F.hist[(int64_t)slot * F.ncell + g] = f;
        double s = 0.0;
        for (int k = 0; k < NHIST; ++k) s += wc[k] * (double)F.hist[(int64_t)k * F.ncell + g];
        F.sigma[g] = T(s);
    CLOT_END_CELLS
}

// Release-history schedule of one channel (section 3.2, eq. for sigma): the time and
// step count, the next snapshot index and the ring of snapshot times.
struct SigState {
    double t;
    int64_t n;
    int64_t next_push;
    int32_t head;      // slot of the newest snapshot (-1: none yet)
    int32_t npushed;
    double hist_t[NHIST];
};

// Decides, per channel, whether this step takes a new snapshot of the release rate
// (every dtau of simulated time, and at the first step), and if so the trapezoid
// weights A_hat w_a exp(-(age_a - 3)^2)/sqrt(pi) of the snapshots (node a = 0 the
// newest, half weight at the two ends).  Then advances the channel clock by one step.
// One thread per channel; push[2c] = slot or -1, push[2c+1] = first-step flag.
__global__ __launch_bounds__(64) void k_sigma_sched(const ChanDev* chans, SigState* sig, int nch, ModelDev M,
                                                    double* w, int32_t* push) {
    for (int c = threadIdx.x; c < nch; c += 64) {
        SigState s = sig[c];
        push[2 * c] = -1;
        push[2 * c + 1] = 0;
        const int64_t m = (int64_t)floor(s.t / M.dtau + 1e-9);
        if (s.n == 0 || m >= s.next_push) {
            s.next_push = m + 1;
            s.head = (s.head + 1) % NHIST;
            s.hist_t[s.head] = s.t;
            s.npushed = s.npushed + 1 < NHIST ? s.npushed + 1 : NHIST;
            push[2 * c] = s.head;
            push[2 * c + 1] = s.n == 0 ? 1 : 0;
            double* wc = w + (int64_t)c * NHIST;
            for (int a = 0; a < NHIST; ++a) {
                const int slot = ((s.head - a) % NHIST + NHIST) % NHIST;
                double v = 0.0;
                if (a < s.npushed) {
                    const double age = s.t - s.hist_t[slot];
                    const double wt = (a == 0 || a == NHIST - 1) ? 0.5 * M.dtau : M.dtau;
                    v = M.A_hat * wt * exp(-(age - 3.0) * (age - 3.0)) / sqrt(3.14159265358979323846);
                }
                wc[slot] = v;
            }
        }
        s.n += 1;
        // fixed step: t = n dt; variable step: the sum of the steps taken
        s.t = M.max_co > 0.0 ? s.t + chans[c].dt : (double)s.n * chans[c].dt;
        sig[c] = s;
    }
}

// Transport assembly (section 3.2, Appendix C table, Appendix D): diagonal and
// right-hand side of the 7 implicit TVD transport systems; initial guess C^n.  The
// time derivative is that of the momentum assembly (k, w and the stored derivative
// of each species' transport sub-step).  With a variable step, each tile also stores
// the largest sum_f |phi_f| of its cells (the new flux) for the next step's Courant
// limit.  Launch: blockIdx.y is the transported species, so a thread makes one pass of
// loads instead of one per species.
template <class T>
__global__ __launch_bounds__(NT) void k_tr_assemble(Grid G, Fields<T> F, TrOp<T> op, ModelDev M) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int64_t g = P.g;
        const T rdt = T(C.rdt);
        const T kd = T(C.ddtk);
        const T Wp = F.Wc[g];
        const bool inj = P.j == 0 && P.i >= C.inj_i0 && P.i < C.inj_i0 + C.inj_ni && P.k >= C.inj_k0 &&
                         P.k < C.inj_k0 + C.inj_nk;
        const int64_t fi = C.inj0 + (P.i - C.inj_i0) + (int64_t)C.inj_ni * (P.k - C.inj_k0);
        const T fin = F.phin[0][fx_id(C, 0, P.j, P.k)];
        const T fout = F.phin[0][fx_id(C, C.nx, P.j, P.k)];
        {
            const int k = (int)blockIdx.y;
            const int sp = tr_species(k);
            const bool plt = k < 2;
            const T* c = op.Cn[k];
            const T D = op.Dk[k];
            const T cn = c[g];
            // diagonal and right-hand side in FP64: each face adds to the diagonal its
            // convective coefficient minus the coupling as stored, so that the row sum is
            // k V/dt + the net outflow coefficient exactly and the starting residual of a
            // field the step leaves unchanged is zero (see TrOp::residual64)
            const double kvr = C.ddtk * C.V * C.rdt;
            double d = kvr;
            double b = kvr * ((double)cn + (double)F.lo[sp][g]);
            if (sp == ADP) b += C.V * (double)F.sigma[g];
            if (M.psi > 0.0) {
                const T w = T(C.ddtw), kr = kd * rdt;
                T* hq = F.ddt0c[k] + g;
                const T q = *hq;
                b += (double)w * C.V * (double)q;
                *hq = -(kr * cn + w * q);
            }
            // couplings of this row, stored for the solver's stencil products
            T* cf = F.trc[k] + g;
            const int64_t n = F.ncell;
            T o[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
            T ad = T(C.gx);
            if (P.i < C.nx - 1) {
                const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g, 1, P.i, C.nx, F.phin[0][fx_id(C, P.i + 1, P.j, P.k)], op.Pmax);
                d += (double)f.conv - (double)f.oLR;
                o[0] = f.oLR;
            }
            if (P.i > 0) {
                const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g - 1, 1, P.i - 1, C.nx, F.phin[0][fx_id(C, P.i, P.j, P.k)], op.Pmax);
                d += -(double)f.conv - (double)f.oRL;
                o[1] = f.oRL;
            }
            ad = T(C.gy);
            if (P.j < C.ny - 1) {
                const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g, C.nx, P.j, C.ny, F.phin[1][fy_id(C, P.i, P.j + 1, P.k)], op.Pmax);
                d += (double)f.conv - (double)f.oLR;
                o[2] = f.oLR;
            }
            if (P.j > 0) {
                const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g - C.nx, C.nx, P.j - 1, C.ny, F.phin[1][fy_id(C, P.i, P.j, P.k)], op.Pmax);
                d += -(double)f.conv - (double)f.oRL;
                o[3] = f.oRL;
            }
            if (C.dim == 3) {
                const int64_t sz = (int64_t)C.nx * C.ny;
                ad = T(C.gz);
                if (P.k < C.nz - 1) {
                    const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g, sz, P.k, C.nz, F.phin[2][fz_id(C, P.i, P.j, P.k + 1)], op.Pmax);
                    d += (double)f.conv - (double)f.oLR;
                    o[4] = f.oLR;
                }
                if (P.k > 0) {
                    const FaceCoef<T> f = tr_face(c, F.Wc, plt, D, ad, g - sz, sz, P.k - 1, C.nz, F.phin[2][fz_id(C, P.i, P.j, P.k)], op.Pmax);
                    d += -(double)f.conv - (double)f.oRL;
                    o[5] = f.oRL;
                }
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) cf[q * n] = o[q];
            const double W = plt ? (double)Wp : 1.0;
            if (P.i == 0) {
                const double fo = -(double)fin;       // outward flux through the inlet face
                const bool fixed = (sp == PMU || sp == S1 || sp == S2 || sp == INH);
                if (fixed) {
                    const double cb = sp == PMU ? (double)F.pmu_in[C.in0 + P.j + (int64_t)C.ny * P.k]
                                    : sp == S1 ? (double)T(M.S1_0) : sp == S2 ? (double)T(M.S2_0) : (double)T(M.I_0);
                    const double gg = 2.0 * W * (double)D * C.gx;
                    d += gg;
                    b += gg * cb - W * fo * cb;
                } else {
                    d += W * fo;
                }
            }
            if (P.i == C.nx - 1) d += W * (double)fout;
            if (inj) {
                const double A = C.dx * C.dz;
                if (sp == E1) b += A * M.kC0cat * (double)F.C0[fi];
                if (sp == S1) {
                    const double kk = M.kC0p * (double)F.E0[fi], qq = M.kC0m * (double)F.C0[fi];
                    const double gg = M.D_chem / (0.5 * C.dy);
                    d += A * kk * gg / (gg + kk);
                    b += A * qq * gg / (gg + kk);
                }
            }
            F.trd[k][g] = T(d);
            F.trd64[k][g] = d;
            F.trb[k][g] = b;
        }
    CLOT_END_CELLS
    if (M.max_co > 0.0 && blockIdx.y == 0) {   // a pass of its own: inside the loop above it doubles the register use
        double co_mx = 0.0;
        CLOT_FOR_CELLS(local)
            const Cell P = cell_at(C, local);
            // face order as the cell Courant number is defined: x, y, z, high + low face
            double sf = fabs((double)F.phin[0][fx_id(C, P.i + 1, P.j, P.k)]) +
                        fabs((double)F.phin[0][fx_id(C, P.i, P.j, P.k)]);
            sf += fabs((double)F.phin[1][fy_id(C, P.i, P.j + 1, P.k)]) +
                  fabs((double)F.phin[1][fy_id(C, P.i, P.j, P.k)]);
            if (C.dim == 3)
                sf += fabs((double)F.phin[2][fz_id(C, P.i, P.j, P.k + 1)]) +
                      fabs((double)F.phin[2][fz_id(C, P.i, P.j, P.k)]);
            co_mx = fmax(co_mx, sf);
        CLOT_END_CELLS
        __shared__ double lds[NT / 64];
        co_mx = block_max(co_mx, lds);
        if (threadIdx.x == 0) F.co_part[tile] = co_mx;
    }
}

// Crank-Nicolson history at the end of the transport sub-step: the assemblies left
// -(k/dt f + w D) in the history; adding k/dt f' leaves D' = k (f' - f)/dt - w D for
// u (final after the correctors) and each transported species (its transport solution).
template <class T>
__global__ __launch_bounds__(NT) void k_ddt_close(Grid G, Fields<T> F) {
    CLOT_TILE_PROLOGUE(G)
    const T kr = T(C.ddtk) * T(C.rdt);
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        for (int c = 0; c < C.dim; ++c) F.ddt0u[c][g] += kr * F.u[c][g];
#pragma unroll
        for (int k = 0; k < NTR; ++k) F.ddt0c[k][g] += kr * F.spc[tr_species(k)][g];
    CLOT_END_CELLS
}

// End of a step, one block per channel, after every kernel that reads the step's dt:
// the Crank-Nicolson coefficients of the steps after the first (k = 1+psi, w = psi),
// and the variable step (Appendix D, maxCo): the largest that holds the largest cell
// Courant number 0.5 dt sum_f |phi_f| / V of the new flux at max_co, at most dt_growth
// times this one and at most the channel's dt.
__global__ __launch_bounds__(256) void k_time_end(ChanDev* chans, const double* co_part, ModelDev M) {
    __shared__ double lds[4];
    const int c = blockIdx.x;
    const int32_t t0 = chans[c].t0, nt = chans[c].nt;
    double mx = 0.0;
    if (M.max_co > 0.0) {
        for (int t = threadIdx.x; t < nt; t += 256) mx = fmax(mx, co_part[t0 + t]);
        mx = block_max<256>(mx, lds);
    }
    if (threadIdx.x == 0) {
        ChanDev& C = chans[c];
        if (M.psi > 0.0) {
            C.ddtk = 1.0 + M.psi;
            C.ddtw = M.psi;
        }
        if (M.max_co > 0.0) {
            const double dt = C.dt;
            const double co = 0.5 * dt * mx / C.V;
            double nd = fmin(C.dtmax, M.dt_growth * dt);
            if (co > 0.0) nd = fmin(nd, M.max_co * dt / co);
            C.dt = nd;
            C.rdt = 1.0 / nd;
        }
    }
}

// Reaction right-hand side (Appendix A platelet equations, Appendix B coagulation
// equations), y in the order Pmu Pma Pba Pbse S1 S2 E1 E2 S1b S2b E1b E2b C1 C2.
// The reaction constants in the arithmetic type, formed once on the host and passed
// as a kernel argument (uniform, so they stay in scalar registers instead of being
// converted from the FP64 model table into vector registers in every thread).
template <class T>
struct RxnK {
    T P_max, k_adh, k_adp, adp_crit, k_e2, e2_crit, kcoh_Pmax, n1, n2;
    T kC1p, kC2p, kS1p, kS1m, kS2p, kS2m, kE1p, kE1m, kE2p, kE2m;
    T kC1m, kC2m, kC1cat, kC2cat, kC1mc, kC2mc, k_I;
    T eta_t, eta_star3, g0;
};
template <class T>
__host__ __device__ inline RxnK<T> rxn_consts(const ModelDev& M) {
    RxnK<T> K;
    K.P_max = T(M.P_max);
    K.k_adh = T(M.k_adh);
    K.k_adp = T(M.k_adp);
    K.adp_crit = T(M.adp_crit);
    K.k_e2 = T(M.k_e2);
    K.e2_crit = T(M.e2_crit);
    K.kcoh_Pmax = T(M.kcoh_Pmax);
    K.n1 = T(M.N1 / M.N_A);
    K.n2 = T(M.N2 / M.N_A);
    K.kC1p = T(M.kC1p);
    K.kC2p = T(M.kC2p);
    K.kS1p = T(M.kS1p);
    K.kS1m = T(M.kS1m);
    K.kS2p = T(M.kS2p);
    K.kS2m = T(M.kS2m);
    K.kE1p = T(M.kE1p);
    K.kE1m = T(M.kE1m);
    K.kE2p = T(M.kE2p);
    K.kE2m = T(M.kE2m);
    K.kC1m = T(M.kC1m);
    K.kC2m = T(M.kC2m);
    K.kC1cat = T(M.kC1cat);
    K.kC2cat = T(M.kC2cat);
    K.kC1mc = T(M.kC1m + M.kC1cat);
    K.kC2mc = T(M.kC2m + M.kC2cat);
    K.k_I = T(M.k_I);
    K.eta_t = T(M.eta_t);
    K.eta_star3 = T(M.eta_star * M.eta_star * M.eta_star);
    K.g0 = T(M.g0);
    return K;
}

template <class T>
__device__ inline void rxn_rhs(const T (&y)[NRX], T adp, T gam, T hadh, const RxnK<T>& K, T (&f)[NRX]) {
    const T adh = K.k_adh * hadh * (K.P_max - y[3]);
    const T act = K.k_adp * adp / (K.adp_crit + adp) + K.k_e2 * y[7] / (K.e2_crit + y[7]);
    const T coh = K.kcoh_Pmax * gam;
    const T bound = y[2] + y[3];
    const T B1 = K.n1 * bound - (y[8] + y[10] + y[12] + y[13]);
    const T B2 = K.n2 * bound - (y[9] + y[11] + y[12] + y[13]);
    const T c1 = K.kC1p * y[9] * y[10];
    const T c2 = K.kC2p * y[8] * y[11];
    const T bS1 = K.kS1p * B1 * y[4] - K.kS1m * y[8];
    const T bS2 = K.kS2p * B2 * y[5] - K.kS2m * y[9];
    const T bE1 = K.kE1p * B1 * y[6] - K.kE1m * y[10];
    const T bE2 = K.kE2p * B2 * y[7] - K.kE2m * y[11];
    f[0] = -(adh + act) * y[0];
    f[1] = -adh * y[1] + act * y[0] - coh * y[1];
    f[2] = -adh * y[2] + coh * y[1];
    f[3] = adh * (y[0] + y[1] + y[2]);
    f[4] = -bS1;
    f[5] = -bS2;
    f[6] = -bE1;
#ifdef CLOT_INHIBITOR
    const T rI = K.k_I * y[14] * y[7];   // I + E2 -> E2i (section 3.4), mass action
    f[7] = -bE2 - rI;
    f[14] = -rI;
    f[15] = rI;
#else
    f[7] = -bE2;
#endif
    f[8] = bS1 - c2 + K.kC2m * y[13];
    f[9] = bS2 - c1 + K.kC1m * y[12];
    f[10] = bE1 - c1 + K.kC1mc * y[12] + K.kC2cat * y[13];
    f[11] = bE2 - c2 + K.kC2mc * y[13] + K.kC1cat * y[12];
    f[12] = c1 - K.kC1mc * y[12];
    f[13] = c2 - K.kC2mc * y[13];
}

template <class T>
__device__ inline T binding_g(T eta, const RxnK<T>& K) {
    const T e = eta - K.eta_t;
    if (!(e > T(0))) return T(0);
    const T e3 = e * e * e;
    return K.g0 * e3 / (K.eta_star3 + e3);
}

// Reactive wall: S1 wall value from the Robin balance with the transported S1,
// then M_rxn RK4 sub-steps of eqs. seBound_E0/C0 per injury face (Appendix B).
template <class T>
__global__ __launch_bounds__(NT) void k_wall_rxn(const ChanDev* chans, const int32_t* f2c, int64_t nfaces, Fields<T> F,
                                                 ModelDev M) {
    const int64_t f = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (f >= nfaces) return;
    const ChanDev& C = chans[f2c[f]];
    const int64_t lf = f - C.inj0;
    const int i = C.inj_i0 + (int)(lf % C.inj_ni);
    const int k = C.inj_k0 + (int)(lf / C.inj_ni);
    const int64_t g = C.c0 + i + (int64_t)C.nx * C.ny * k;
    double E0 = F.E0[f], C0 = F.C0[f];
    const double kk = M.kC0p * E0, qq = M.kC0m * C0;
    const double gg = M.D_chem / (0.5 * C.dy);
    const double s1w = (qq + gg * ((double)F.spc[S1][g] + (double)F.lo[S1][g])) / (gg + kk);
    F.s1w[f] = s1w;
    const double h = C.dt / M.M_rxn;
    const double kf = M.kC0p * s1w, kb = M.kC0m + M.kC0cat;
    for (int m = 0; m < M.M_rxn; ++m) {
        auto rate = [&](double e, double c) { return kf * e - kb * c; };   // d C0/dt = -d E0/dt
        const double r1 = rate(E0, C0);
        const double r2 = rate(E0 - 0.5 * h * r1, C0 + 0.5 * h * r1);
        const double r3 = rate(E0 - 0.5 * h * r2, C0 + 0.5 * h * r2);
        const double r4 = rate(E0 - h * r3, C0 + h * r3);
        const double inc = h / 6.0 * (r1 + 2.0 * r2 + 2.0 * r3 + r4);
        E0 -= inc;
        C0 += inc;
    }
    F.E0[f] = E0;
    F.C0[f] = C0;
}

// The reacting species of a cell in the order of the reaction state vector (Pmu Pma Pba
// Pbse S1 S2 E1 E2 S1b S2b E1b E2b C1 C2, then I and E2i in the inhibitor build).
__host__ __device__ constexpr int rxn_species(int q) {
    return q < 4 ? q : q < 8 ? q + 1 : q < 14 ? q + 1 : q == 14 ? INH : E2I;
}

// M_rxn classical RK4 sub-steps (section 3.2) in increment form: the stages are
// evaluated in T at (state + increment so far), and the increment d is accumulated
// apart from the state, so it keeps its own relative precision however small it is
// next to the state.
// The four stage slopes are summed as they come (k1 + 2 k2 + 2 k3 + k4), so a cell
// holds the state, the increment, one slope, the sum and the stage point.
template <class T>
__device__ inline void rk4_increment(const T (&y)[NRX], T (&d)[NRX], T adp, T gam, T hadh, T h, int nsub,
                                     const RxnK<T>& K) {
#pragma unroll
    for (int q = 0; q < NRX; ++q) d[q] = T(0);
    for (int m = 0; m < nsub; ++m) {
        T k[NRX], acc[NRX], w[NRX];
#pragma unroll
        for (int q = 0; q < NRX; ++q) w[q] = y[q] + d[q];
        rxn_rhs(w, adp, gam, hadh, K, k);
#pragma unroll
        for (int q = 0; q < NRX; ++q) {
            acc[q] = k[q];
            w[q] = (y[q] + d[q]) + T(0.5) * h * k[q];
        }
        rxn_rhs(w, adp, gam, hadh, K, k);
#pragma unroll
        for (int q = 0; q < NRX; ++q) {
            acc[q] += T(2) * k[q];
            w[q] = (y[q] + d[q]) + T(0.5) * h * k[q];
        }
        rxn_rhs(w, adp, gam, hadh, K, k);
#pragma unroll
        for (int q = 0; q < NRX; ++q) {
            acc[q] += T(2) * k[q];
            w[q] = (y[q] + d[q]) + h * k[q];
        }
        rxn_rhs(w, adp, gam, hadh, K, k);
#pragma unroll
        for (int q = 0; q < NRX; ++q) d[q] += h / T(6) * (acc[q] + k[q]);
    }
}

// One cell's reaction step in the field precision: the stages see the stored value plus
// its low part (rounded to T); the new state is (value + low part) + increment, formed
// in FP64 and stored again as value and low part.  A species near the injury grows by
// nearly the same increment step after step, and a state stored in T alone would round
// each of them the same way (a bias of up to half an ulp per step, 1e-5 of the value
// after a thousand FP32 steps); the low part carries that remainder instead.
template <class T>
__device__ inline void rxn_cell(const Fields<T>& F, const ChanDev& C, const Cell& P, int nsub, const RxnK<T>& K) {
    const int64_t g = P.g;
    T y[NRX], d[NRX];
#pragma unroll
    for (int q = 0; q < NRX; ++q) y[q] = T((double)F.spc[rxn_species(q)][g] + (double)F.lo[rxn_species(q)][g]);
    const T adp = F.spc[ADP][g];
    const T gam = binding_g<T>(F.eta[g], K);
    const bool hin = P.j < C.jadh && P.i >= C.inj_i0 && P.i < C.inj_i0 + C.inj_ni && P.k >= C.inj_k0 &&
                     P.k < C.inj_k0 + C.inj_nk;
    rk4_increment<T>(y, d, adp, gam, hin ? T(1) : T(0), T(C.dt / nsub), nsub, K);
#pragma unroll
    for (int q = 0; q < NRX; ++q) {
        const int sp = rxn_species(q);
        const double v = (double)F.spc[sp][g] + (double)F.lo[sp][g] + (double)d[q];
        const T hi = T(v);
        F.spc[sp][g] = hi;
        F.lo[sp][g] = T(v - (double)hi);
    }
}

// Cell reactions: M_rxn RK4 sub-steps with ADP (post transport), g(eta) and H_adh
// frozen, on the species after transport, in place.
template <class T>
__global__ __launch_bounds__(NT) void k_rxn(Grid G, Fields<T> F, int nsub, RxnK<T> K) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        rxn_cell<T>(F, C, cell_at(C, local), nsub, K);
    CLOT_END_CELLS
}

// End of the delta-form transport solve: species = (value + low part) + change, in FP64,
// stored again as value and low part.
template <class T>
__global__ __launch_bounds__(NT) void k_add_change(Grid G, Fields<T> F) {
    CLOT_TILE_PROLOGUE(G)
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
#pragma unroll
        for (int k = 0; k < NTR; ++k) {
            const int sp = tr_species(k);
            const double v = (double)F.spc[sp][g] + (double)F.lo[sp][g] + (double)F.dlt[k][g];
            const T hi = T(v);
            F.spc[sp][g] = hi;
            F.lo[sp][g] = T(v - (double)hi);
        }
    CLOT_END_CELLS
}

// Non-finite scan of the persistent fields after a step call: velocity, pressure,
// every cell species and the injury-face species.  flag = 1 if any value is a NaN or
// an infinity (every writer stores the same value).
template <class T>
__global__ __launch_bounds__(NT) void k_nonfinite_scan(Grid G, Fields<T> F, int64_t ninj, int32_t* flag) {
    CLOT_TILE_PROLOGUE(G)
    bool bad = false;
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        for (int c = 0; c < 3; ++c) bad = bad || !isfinite((double)F.u[c][g]);
        bad = bad || !isfinite(F.p[g]);
        for (int q = 0; q < NSPC; ++q) bad = bad || !isfinite((double)F.spc[q][g]);
    CLOT_END_CELLS
    for (int64_t f = (int64_t)blockIdx.x * NT + threadIdx.x; f < ninj; f += (int64_t)gridDim.x * NT)
        bad = bad || !isfinite((double)F.E0[f]) || !isfinite((double)F.C0[f]);
    if (bad) flag[0] = 1;
}

// Driver bookkeeping kernels (graph-safe replacements for memset and host reads).
// chact = mask, and the active count: zero (a solve's start admits its channels) or, with
// count, the number of channels the mask admits.  One block.
__global__ __launch_bounds__(256) void k_set_active(int32_t* chact, const int32_t* mask, int32_t* nact, int nch,
                                                    int count) {
    for (int c = threadIdx.x; c < nch; c += 256) chact[c] = mask[c];
    if (threadIdx.x == 0) {
        int s = 0;
        if (count)
            for (int c = 0; c < nch; ++c) s += mask[c] != 0;
        *nact = s;
    }
}

// On-demand diagnostics of the current state, per tile: the largest |net outflow| of a
// cell (discrete continuity, section 3.2), the largest face-flux magnitude and the
// smallest species value over its scale (non-negativity).
template <class T>
__global__ __launch_bounds__(NT) void k_diag_tiles(Grid G, Fields<T> F, ModelDev M, double* part) {
    CLOT_TILE_PROLOGUE(G)
    const double sc[NSPC] = {M.P_max, M.P_max, M.P_max, M.P_max, M.adp_crit, M.S1_0, M.S2_0, M.S1_0, M.S2_0,
                             M.S1_0, M.S2_0, M.S1_0, M.S2_0, M.S2_0, M.S2_0
#ifdef CLOT_INHIBITOR
                             , M.I_0, M.S2_0
#endif
    };
    double dmax = 0.0, fmx = 0.0, smin = 1e300;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const double fw = F.phi[0][fx_id(C, P.i, P.j, P.k)], fe = F.phi[0][fx_id(C, P.i + 1, P.j, P.k)];
        const double fs = F.phi[1][fy_id(C, P.i, P.j, P.k)], fn = F.phi[1][fy_id(C, P.i, P.j + 1, P.k)];
        double div = (fe - fw) + (fn - fs);
        double m = fmax(fmax(fabs(fw), fabs(fe)), fmax(fabs(fs), fabs(fn)));
        if (C.dim == 3) {
            const double fb = F.phi[2][fz_id(C, P.i, P.j, P.k)], ff = F.phi[2][fz_id(C, P.i, P.j, P.k + 1)];
            div += ff - fb;
            m = fmax(m, fmax(fabs(fb), fabs(ff)));
        }
        dmax = fmax(dmax, fabs(div));
        fmx = fmax(fmx, m);
#pragma unroll
        for (int q = 0; q < NSPC; ++q) smin = fmin(smin, (double)F.spc[q][P.g] / sc[q]);
    CLOT_END_CELLS
    __shared__ double lds[NT / 64];
    dmax = block_max(dmax, lds);
    fmx = block_max(fmx, lds);
    smin = -block_max(-smin, lds);
    if (threadIdx.x == 0) {
        part[3 * (int64_t)tile] = dmax;
        part[3 * (int64_t)tile + 1] = fmx;
        part[3 * (int64_t)tile + 2] = smin;
    }
}

// The channel's diagnostics from its tiles (one block per channel) into its statistics.
__global__ __launch_bounds__(256) void k_diag_finish(const ChanDev* chans, const double* part, double* stats,
                                                     int nstat, int slot) {
    __shared__ double lds[4];
    const int c = blockIdx.x;
    const int32_t t0 = chans[c].t0, nt = chans[c].nt;
    double d = 0.0, f = 0.0, s = 1e300;
    for (int t = threadIdx.x; t < nt; t += 256) {
        d = fmax(d, part[3 * (int64_t)(t0 + t)]);
        f = fmax(f, part[3 * (int64_t)(t0 + t) + 1]);
        s = fmin(s, part[3 * (int64_t)(t0 + t) + 2]);
    }
    d = block_max<256>(d, lds);
    f = block_max<256>(f, lds);
    s = -block_max<256>(-s, lds);
    if (threadIdx.x == 0) {
        stats[(int64_t)c * nstat + slot] = d;
        stats[(int64_t)c * nstat + slot + 1] = f;
        stats[(int64_t)c * nstat + slot + 2] = s;
    }
}

// Copies Krylov outcomes of the last solve into the per-channel statistics.
// Records one solve's iteration count, residual and failure flag per channel; with
// `mask`, only channels whose mask entry is set took part in the solve.
__global__ void k_record(const double* sc, double* stats, int nstat, int nch, int K, int slot_it, int slot_res,
                         int slot_fail, int add, const int32_t* mask, int slot_sum) {
    for (int c = threadIdx.x; c < nch; c += blockDim.x) {
        if (mask && !mask[c]) continue;
        double it = 0.0, res = 0.0, fail = 0.0, sum = 0.0;
        for (int k = 0; k < K; ++k) {
            const double* s = sc + ((int64_t)c * MAXK + k) * NSC;
            it = fmax(it, s[SC_IT]);
            sum += s[SC_IT];
            if (s[SC_BBS] > 0.0) res = fmax(res, sqrt(s[SC_RR] / s[SC_BBS]));
            fail = fmax(fail, s[SC_FAIL]);
        }
        double* st = stats + (int64_t)c * nstat;
        st[slot_it] = add ? st[slot_it] + it : it;
        if (slot_sum >= 0) st[slot_sum] = add ? st[slot_sum] + sum : sum;   // system-iterations
        if (slot_res >= 0) st[slot_res] = res;
        st[slot_fail] = fmax(st[slot_fail], fail);
    }
}

__global__ void k_record_pass(const double* sc, double* stats, int nstat, int nch, int slot, int slot_res,
                              int slot_fail) {
    for (int c = threadIdx.x; c < nch; c += blockDim.x) {
        const double* s = sc + (int64_t)c * MAXK * NSC;
        stats[(int64_t)c * nstat + slot] = s[SC_PASS];
        if (s[SC_OBB] > 0.0) stats[(int64_t)c * nstat + slot_res] = sqrt(s[SC_ORR] / s[SC_OBB]);
        stats[(int64_t)c * nstat + slot_fail] = fmax(stats[(int64_t)c * nstat + slot_fail], s[SC_FAIL]);
    }
}

// Surrogate fallback fraction per channel.
__global__ void k_record_fallback(const int32_t* fb_chan, const ChanDev* chans, double* stats, int nstat, int nch,
                                  int slot) {
    for (int c = threadIdx.x; c < nch; c += blockDim.x)
        stats[(int64_t)c * nstat + slot] = (double)fb_chan[c] / (double)chans[c].ncell;
}

// After a solve whose iteration count was fixed in advance: every channel still
// active has not converged; flag it as failed and raise the host-visible flag.
__global__ void k_flag_active(const int32_t* chact, double* sc, int nch, int K, int32_t* flag) {
    for (int c = threadIdx.x; c < nch; c += blockDim.x) {
        if (!chact[c]) continue;
        flag[0] = 1;
        for (int k = 0; k < K; ++k) sc[((int64_t)c * MAXK + k) * NSC + SC_FAIL] = 1.0;
    }
}

// Count of channels still iterating and the largest iteration count of a solve.
__global__ void k_solve_info(const double* sc, const int32_t* nact, int nch, int32_t* out) {
    if (threadIdx.x != 0) return;
    int m = 0;
    for (int c = 0; c < nch; ++c) {
        const int it = (int)sc[(int64_t)c * MAXK * NSC + SC_IT];
        m = it > m ? it : m;
    }
    out[0] = *nact;
    out[1] = m;
}

// Small utility kernels (graph-safe replacements for memset).
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <class T>
__global__ void k_copy(T* dst, const T* src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace clot
