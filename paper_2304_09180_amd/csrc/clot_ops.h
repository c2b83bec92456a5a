// Matrix-free finite-volume operators of the clotting step (gfx950).
//
// Each operator gives, for system k at cell P, its diagonal and (A x)_P, where x
// is supplied as a functor xv(global cell) so the Krylov kernels can feed vectors
// that are formed on the fly (p = z + beta p_old, z = r/diag ...) without a pass.
// Coefficients are recomputed from the stored face fluxes, rAU, theta_T hindrance
// and the start-of-step species, so no assembled matrix ever goes to memory.
#pragma once
#include "clot_common.h"

namespace clot {

// Pointers to every field of the context, passed by value.
template <class T>
struct Fields {
    T* u[3];
    double* p;            // kinematic pressure (FP64 in both precisions)
    T* phi[3];            // flux of the previous step (convects the momentum)
    T* phin[3];           // flux written by the PISO correctors
    T* spc[NSPC];         // species (the stored value) ...
    T* lo[NSPC];          // ... and its low part: a species is spc + lo (see the transport and reaction updates)
    T* dlt[NTR];          // the transport solves' unknowns: each species' change over the step
    double* E0;           // injury-face species: FP64 in every precision (each step adds a
    double* C0;           // nearly constant increment, which FP32 rounding would bias)
    double* s1w;
    T* eta;
    T* thB;
    T* thB_prev;
    T* Wc;                // W(theta_T) per cell
    T* sigma;
    T* hist;              // NHIST snapshots, stride ncell
    const T* u_in;
    const T* pmu_in;
    T* aP;
    T* src[3];
    T* bm[3];             // momentum right-hand sides
    T* rAU;
    T* HbyA[3];
    T* dP;                // pressure diagonal
    T* dE;                // eta diagonal
    double* rhs_p;        // pressure right-hand side
    T* trd[NTR];          // transport diagonals (the solver's Jacobi scaling and stencil)
    double* trd64[NTR];   // the same diagonals in FP64, consistent with the stored couplings
    double* trb[NTR];     // transport right-hand sides (FP64)
    T* trc[NTR];      // transport off-diagonal couplings, 6 slots x ncell per species
    T* ddt0u[3];          // Crank-Nicolson history: stored time derivative of u
    T* ddt0c[NTR];        // ... and of each transported species (its transport sub-step)
    double* co_part;      // variable step: per tile, the largest sum_f |phi_f| of its cells
    int64_t ncell;
};

template <class T>
__device__ inline T hindrance_fn(T thT) {
    T t = thT < T(1) ? thT : T(1);
    return tanh(T(3.14159265358979323846) * (T(1) - t));
}

// ---------------------------------------------------------------------------------
// Momentum (implicit Euler, Gauss-linear convection with the old flux, nu Laplacian)
// off-diagonal of the face to neighbour N: (outward flux)/2 - nu A/d.
// ---------------------------------------------------------------------------------
template <class T>
struct MomOp {
    const T* aP;
    const T* phx;
    const T* phy;
    const T* phz;
    T nu;
    __device__ T diag(int, int64_t g) const { return aP[g]; }
    __device__ T floor_scale(int) const { return T(0); }   // no absolute floor
    template <class XV>
    __device__ T offsum(const ChanDev& C, const Cell& P, XV xv) const {
        T s = T(0);
        T d = nu * T(C.gx);
        if (P.i > 0) s += (T(-0.5) * phx[fx_id(C, P.i, P.j, P.k)] - d) * xv(P.g - 1);
        if (P.i < C.nx - 1) s += (T(0.5) * phx[fx_id(C, P.i + 1, P.j, P.k)] - d) * xv(P.g + 1);
        d = nu * T(C.gy);
        if (P.j > 0) s += (T(-0.5) * phy[fy_id(C, P.i, P.j, P.k)] - d) * xv(P.g - C.nx);
        if (P.j < C.ny - 1) s += (T(0.5) * phy[fy_id(C, P.i, P.j + 1, P.k)] - d) * xv(P.g + C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            d = nu * T(C.gz);
            if (P.k > 0) s += (T(-0.5) * phz[fz_id(C, P.i, P.j, P.k)] - d) * xv(P.g - sz);
            if (P.k < C.nz - 1) s += (T(0.5) * phz[fz_id(C, P.i, P.j, P.k + 1)] - d) * xv(P.g + sz);
        }
        return s;
    }
    template <class XV>
    __device__ T apply(int, const ChanDev& C, const Cell& P, XV xv) const {
        return aP[P.g] * xv(P.g) + offsum(C, P, xv);
    }
};

// ---------------------------------------------------------------------------------
// Pressure: sum_f c_f (p_P - p_N) + c_out p_P, c_f = rAU_f A/d, rAU_f linear,
// c_out = rAU_P 2A/dx on the outlet.  A is the arithmetic type.
// ---------------------------------------------------------------------------------
template <class T, class A>
struct PresOp {
    const T* rAU;
    const T* dP;
    __device__ A diag(int, int64_t g) const { return A(dP[g]); }
    template <class XV>
    __device__ A offsum(const ChanDev& C, const Cell& P, XV xv) const {
        const A rP = A(rAU[P.g]);
        A s = A(0);
        A g = A(0.5 * C.gx);
        if (P.i > 0) s += g * (rP + A(rAU[P.g - 1])) * xv(P.g - 1);
        if (P.i < C.nx - 1) s += g * (rP + A(rAU[P.g + 1])) * xv(P.g + 1);
        g = A(0.5 * C.gy);
        if (P.j > 0) s += g * (rP + A(rAU[P.g - C.nx])) * xv(P.g - C.nx);
        if (P.j < C.ny - 1) s += g * (rP + A(rAU[P.g + C.nx])) * xv(P.g + C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            g = A(0.5 * C.gz);
            if (P.k > 0) s += g * (rP + A(rAU[P.g - sz])) * xv(P.g - sz);
            if (P.k < C.nz - 1) s += g * (rP + A(rAU[P.g + sz])) * xv(P.g + sz);
        }
        return s;
    }
    // diagonal recomputed in the arithmetic type
    __device__ A diag_exact(const ChanDev& C, const Cell& P) const {
        const A rP = A(rAU[P.g]);
        A s = A(0);
        A g = A(0.5 * C.gx);
        if (P.i > 0) s += g * (rP + A(rAU[P.g - 1]));
        if (P.i < C.nx - 1) s += g * (rP + A(rAU[P.g + 1]));
        else s += A(2.0 * C.gx) * rP;
        g = A(0.5 * C.gy);
        if (P.j > 0) s += g * (rP + A(rAU[P.g - C.nx]));
        if (P.j < C.ny - 1) s += g * (rP + A(rAU[P.g + C.nx]));
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            g = A(0.5 * C.gz);
            if (P.k > 0) s += g * (rP + A(rAU[P.g - sz]));
            if (P.k < C.nz - 1) s += g * (rP + A(rAU[P.g + sz]));
        }
        return s;
    }
    template <class XV>
    __device__ A apply(int, const ChanDev& C, const Cell& P, XV xv) const {
        return A(dP[P.g]) * xv(P.g) - offsum(C, P, xv);
    }
};

// ---------------------------------------------------------------------------------
// eta: (V + kappa sum A/d) eta_P - kappa sum (A/d) eta_N, zero-gradient walls.
// ---------------------------------------------------------------------------------
template <class T>
struct EtaOp {
    T kappa;
    const T* dE;          // stored diagonal (geometry only)
    __device__ static T diag_of(T kappa, const ChanDev& C, const Cell& P) {
        T gx = kappa * T(C.gx), gy = kappa * T(C.gy), gz = kappa * T(C.gz);
        T d = T(C.V);
        d += gx * T((P.i > 0) + (P.i < C.nx - 1));
        d += gy * T((P.j > 0) + (P.j < C.ny - 1));
        if (C.dim == 3) d += gz * T((P.k > 0) + (P.k < C.nz - 1));
        return d;
    }
    __device__ T diag(int, int64_t g) const { return dE[g]; }
    template <class XV>
    __device__ T apply(int k, const ChanDev& C, const Cell& P, XV xv) const {
        T gx = kappa * T(C.gx), gy = kappa * T(C.gy), gz = kappa * T(C.gz);
        T s = T(0);
        if (P.i > 0) s += gx * xv(P.g - 1);
        if (P.i < C.nx - 1) s += gx * xv(P.g + 1);
        if (P.j > 0) s += gy * xv(P.g - C.nx);
        if (P.j < C.ny - 1) s += gy * xv(P.g + C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            if (P.k > 0) s += gz * xv(P.g - sz);
            if (P.k < C.nz - 1) s += gz * xv(P.g + sz);
        }
        return dE[P.g] * xv(P.g) - s;
    }
};

// ---------------------------------------------------------------------------------
// Transport: face weights of the frozen van Leer TVD interpolation.
// Face between L (low) and R = L + s along an axis; iL is L's index on that axis,
// n the cell count along it.  C_f = wL C_L + wR C_R.
// ---------------------------------------------------------------------------------
template <class T>
__device__ inline void tvd_weights(const T* Cn, int64_t gL, int64_t s, int iL, int n, T phi, bool bounded,
                                   T Pmax, T& wL, T& wR) {
    const bool pos = phi >= T(0);
    const T CL = Cn[gL], CR = Cn[gL + s];
    const T CU = pos ? CL : CR, CD = pos ? CR : CL;
    const bool has_uu = pos ? (iL >= 1) : (iL + 2 <= n - 1);
    T psi = T(0);
    if (has_uu) {
        const T CUU = pos ? Cn[gL - s] : Cn[gL + 2 * s];
        const T den = CD - CU;
        bool ok = den != T(0);
        if (bounded) ok = ok && CU >= T(0) && CU <= Pmax && CD >= T(0) && CD <= Pmax;
        if (ok) {
            const T r = (CU - CUU) / den;
            const T ar = fabs(r);
            psi = (r + ar) / (T(1) + ar);
        }
    }
    const T wU = T(1) - T(0.5) * psi, wD = T(0.5) * psi;
    wL = pos ? wU : wD;
    wR = pos ? wD : wU;
}

// Coefficients of one interior face (L,R): contributions to row L (dL: diagonal,
// oLR: coupling to R) and to row R (dR, oRL).
template <class T>
struct FaceCoef {
    T dL, oLR, dR, oRL;
    T conv;               // the face's convective coefficient W phi (phi positive from L to R)
};

template <class T>
__device__ inline FaceCoef<T> tr_face(const T* Cn, const T* Wc, bool platelet, T D, T A_over_d, int64_t gL, int64_t s,
                                      int iL, int n, T phi, T Pmax) {
    T wL, wR;
    tvd_weights(Cn, gL, s, iL, n, phi, platelet, Pmax, wL, wR);
    T Wa = T(1), Wd = T(1);
    if (platelet) {
        const T WL = Wc[gL], WR = Wc[gL + s];
        Wa = phi >= T(0) ? WR : WL;          // downwind theta_T
        Wd = WL < WR ? WL : WR;              // localMax theta_T (W decreasing)
    }
    const T conv = Wa * phi, dif = Wd * D * A_over_d;
    FaceCoef<T> f;
    f.dL = conv * wL + dif;
    f.oLR = conv * wR - dif;
    f.dR = -conv * wR + dif;
    f.oRL = -conv * wL - dif;
    f.conv = conv;
    return f;
}

template <class T>
__host__ __device__ inline T tr_diffusivity(int k, const ModelDev& M) {
    return k < 2 ? T(M.D_P) : (k == 6 ? T(M.D_ADP) : T(M.D_chem));
}

template <class T>
struct TrOp {
    const T* Cn[NTR];     // start-of-step species, indexed by transported slot
    const T* dg[NTR];     // diagonals
    const T* cf[NTR];     // off-diagonal couplings stored by the assembly: slot s at s*n + g
    int64_t n;            // cells of the context (slot stride)
    T scale[NTR];         // species scales for the absolute floor of the solve's tolerance
    const T* phx;
    const T* phy;
    const T* phz;
    const T* Wc;
    T Dk[NTR];
    T Pmax;
    // Delta form: each solve's unknown is the species' change over the transport step,
    // started at zero from the residual b - A C^n taken in FP64 from an FP64 right-hand
    // side and an FP64 diagonal that the assembly made consistent with the stored
    // couplings (row sum = k V/dt + net outflow coefficient, exactly): a field the step
    // leaves unchanged then starts with a zero residual instead of the FP32 rounding of
    // k V/dt + (face terms), which would otherwise drift it by that rounding every step.
    static constexpr bool kExactResidual = true;
    const double* b64[NTR];
    const double* dg64[NTR];
    const T* Cl[NTR];     // low parts of the start-of-step species
    __device__ double residual64(int k, const ChanDev& C, const Cell& P, double& b) const {
        const T* x = Cn[k];
        const T* xl = Cl[k];
        auto xv = [&](int64_t g) { return (double)x[g] + (double)xl[g]; };
        const T* c = cf[k] + P.g;
        double y = dg64[k][P.g] * xv(P.g);
        if (P.i < C.nx - 1) y += (double)c[0] * xv(P.g + 1);
        if (P.i > 0) y += (double)c[n] * xv(P.g - 1);
        if (P.j < C.ny - 1) y += (double)c[2 * n] * xv(P.g + C.nx);
        if (P.j > 0) y += (double)c[3 * n] * xv(P.g - C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            if (P.k < C.nz - 1) y += (double)c[4 * n] * xv(P.g + sz);
            if (P.k > 0) y += (double)c[5 * n] * xv(P.g - sz);
        }
        b = b64[k][P.g];
        return b - y;
    }
    __device__ T diag(int k, int64_t g) const { return dg[k][g]; }
    __device__ T floor_scale(int k) const { return scale[k]; }
    // The couplings are frozen over the step (TVD weights and hindrance from C^n):
    // the assembly stores them once (row P: to P+x, P-x, P+y, P-y, P+z, P-z).
    template <class XV>
    __device__ T apply(int k, const ChanDev& C, const Cell& P, XV xv) const {
        const T* c = cf[k] + P.g;
        T y = dg[k][P.g] * xv(P.g);
        if (P.i < C.nx - 1) y += c[0] * xv(P.g + 1);
        if (P.i > 0) y += c[n] * xv(P.g - 1);
        if (P.j < C.ny - 1) y += c[2 * n] * xv(P.g + C.nx);
        if (P.j > 0) y += c[3 * n] * xv(P.g - C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            if (P.k < C.nz - 1) y += c[4 * n] * xv(P.g + sz);
            if (P.k > 0) y += c[5 * n] * xv(P.g - sz);
        }
        return y;
    }
};

}  // namespace clot
