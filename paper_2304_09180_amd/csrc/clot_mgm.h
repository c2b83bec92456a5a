// Multigrid preconditioner of the momentum predictor (gfx950).
//
// The predictor's matrix (time derivative, Gauss-linear convection with the old flux,
// nu-Laplacian, Darcy term nu*alpha*V on the diagonal; eq. NSB, section 3.2) is a
// Helmholtz operator with a small skew part: at cell Peclet numbers below one the
// convective couplings are a few per cent of the viscous ones.  Jacobi-preconditioned
// Krylov methods need O(sqrt(1 + 12 D)) iterations for the viscous diffusion number
// D = nu dt / h^2 (33 BiCGStab iterations on a 256x64x64 duct at D = 5.6, about 100 on
// a 512x128 channel at D = 69); one V-cycle of this preconditioner per BiCGStab
// direction brings that to a handful.
//
// Hierarchy: the aggregation levels of the pressure multigrid (each level halves
// every axis with >= 3 cells).  The finest level smooths with the full operator
// (weighted Jacobi on the stored diagonal aP); a coarse level carries the symmetric
// part re-discretised by aggregation: the cell mass k V/dt + nu alpha V summed over
// the aggregate, and the viscous face couplings and Dirichlet (inlet, wall) terms
// summed across each coarse face and halved along a coarsened normal direction (as
// for the pressure operator, this equals the re-discretisation on uniform cells).
// A boundary face coefficient lives in the face array at the boundary position
// (outlet: zero-gradient, no viscous term), so the diagonal of a coarse cell is its
// mass plus its six face coefficients.  A channel's levels are used until the viscous
// part of its diagonal falls below MGM_RATIO times the mass; there two Jacobi sweeps
// from zero stand in for the coarsest solve.
//
// Cycle: V(1,2) — one weighted-Jacobi sweep from zero, formed inside the residual
// restriction, and two sweeps after the prolongation.  All velocity components of a
// channel share every coefficient read; a component (or channel) that has left the
// Krylov solve is skipped.
#pragma once
#include "clot_mg.h"

namespace clot {

constexpr int MGM_K = 3;            // velocity components
constexpr double MGM_RATIO = 2.5;   // coarsest level: viscous part of the diagonal < this x the mass

template <class T>
struct MGVec {
    T* v[MGM_K];
};
template <class T>
struct MGCVec {
    const T* v[MGM_K];
};

// Right-hand side of a V-cycle at the finest level.  FORM 0: the vector b; FORM 1:
// the new BiCGStab direction p = r + beta (p_old - omega v_old); FORM 2: s = r - alpha v
// (alpha, beta, omega: the channel's solve scalars).  A formed right-hand side is also
// written out, for the rest of the cycle and the outer iteration.
template <class T>
struct MGSrc {
    const T* b[MGM_K];
    const T* r[MGM_K];
    const T* p[MGM_K];
    const T* v[MGM_K];
};

template <class T>
__device__ inline T mom_mass(const ChanDev& C, const ModelDev& M, T thB) {
    const T V = T(C.V);
    const T s = T(0.6) * thB;
    const T om = T(1) - s;
    const T alpha = T(M.C_CK) * s * s / (om * om * om);
    return T(C.ddtk) * V * T(C.rdt) + T(M.nu) * alpha * V;
}

// Face coefficient of the finest level along axis ax at face index f (0..n): the
// viscous coupling nu A/d inside, 2 nu A/d on the inlet and the walls, 0 on the outlet.
template <class T>
__device__ inline T mom_face0(const ChanDev& C, T nu, int ax, int f) {
    const int n = ax == 0 ? C.nx : ax == 1 ? C.ny : C.nz;
    const T g = T(ax == 0 ? C.gx : ax == 1 ? C.gy : C.gz);
    if (f > 0 && f < n) return nu * g;
    if (ax == 0 && f == n) return T(0);
    return T(2) * nu * g;
}

// Builds one coarse momentum level from its fine level (FROM0: the mesh itself).
template <class T, bool FROM0>
__global__ __launch_bounds__(NT) void k_mgm_setup(MGPair L, ModelDev M, const T* thB, const T* fmass, const T* fcx,
                                                  const T* fcy, const T* fcz, T* mass, T* dg, T* cx, T* cy, T* cz) {
    CLOT_TILE_PROLOGUE(L.coarse)
    const ChanDev Fc = L.fine.ch[chid];
    const bool ax0 = Fc.nx != C.nx, ax1 = Fc.ny != C.ny, ax2 = Fc.nz != C.nz;
    const T s0 = ax0 ? T(0.5) : T(1), s1 = ax1 ? T(0.5) : T(1), s2 = ax2 ? T(0.5) : T(1);
    const T nu = T(M.nu);
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int i0 = ax0 ? 2 * P.i : P.i, i1 = ax0 ? min(2 * P.i + 1, Fc.nx - 1) : P.i;
        const int j0 = ax1 ? 2 * P.j : P.j, j1 = ax1 ? min(2 * P.j + 1, Fc.ny - 1) : P.j;
        const int k0 = ax2 ? 2 * P.k : P.k, k1 = ax2 ? min(2 * P.k + 1, Fc.nz - 1) : P.k;
        auto fg = [&](int i, int j, int k) { return Fc.c0 + i + (int64_t)Fc.nx * (j + (int64_t)Fc.ny * k); };
        T m = T(0);
        for (int k = k0; k <= k1; ++k)
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i)
                    m += FROM0 ? mom_mass<T>(Fc, M, thB[fg(i, j, k)]) : fmass[fg(i, j, k)];
        // fine coefficients summed across the coarse face at fine face index f of axis ax
        auto across = [&](int ax, int f) -> T {
            T s = T(0);
            if (ax == 0) {
                for (int k = k0; k <= k1; ++k)
                    for (int j = j0; j <= j1; ++j) s += FROM0 ? mom_face0<T>(Fc, nu, 0, f) : fcx[fx_id(Fc, f, j, k)];
            } else if (ax == 1) {
                for (int k = k0; k <= k1; ++k)
                    for (int i = i0; i <= i1; ++i) s += FROM0 ? mom_face0<T>(Fc, nu, 1, f) : fcy[fy_id(Fc, i, f, k)];
            } else {
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i) s += FROM0 ? mom_face0<T>(Fc, nu, 2, f) : fcz[fz_id(Fc, i, j, f)];
            }
            return s;
        };
        const T xl = s0 * across(0, i0), xh = s0 * across(0, i1 + 1);
        const T yl = s1 * across(1, j0), yh = s1 * across(1, j1 + 1);
        T zl = T(0), zh = T(0);
        if (C.dim == 3) {
            zl = s2 * across(2, k0);
            zh = s2 * across(2, k1 + 1);
        }
        cx[fx_id(C, P.i, P.j, P.k)] = xl;
        if (P.i == C.nx - 1) cx[fx_id(C, C.nx, P.j, P.k)] = xh;
        cy[fy_id(C, P.i, P.j, P.k)] = yl;
        if (P.j == C.ny - 1) cy[fy_id(C, P.i, C.ny, P.k)] = yh;
        if (C.dim == 3) {
            cz[fz_id(C, P.i, P.j, P.k)] = zl;
            if (P.k == C.nz - 1) cz[fz_id(C, P.i, P.j, C.nz)] = zh;
        }
        mass[P.g] = m;
        dg[P.g] = m + xl + xh + yl + yh + zl + zh;
    CLOT_END_CELLS
}

// Active components of a channel (k < dim and still iterating).
__device__ inline void mgm_active(const KState& S, int chid, int dim, bool (&act)[MGM_K]) {
#pragma unroll
    for (int k = 0; k < MGM_K; ++k) act[k] = k < dim && scp(S, chid, k)[SC_ACT] != 0.0;
}

// Each channel has its own coarsest momentum level (last[ch], an index of the coarse
// levels), so its cycle does not depend on the other channels of the context.  A
// coarse-level launch of level `level` works for the channels with last > level
// (restriction to the next level, sweeps after its correction) or, with eq, for those
// whose coarsest level it is.  No gate (last = nullptr): every channel.
struct MGGate {
    const int32_t* last;
    int32_t level;
    int32_t eq;
    __device__ bool open(int ch) const { return !last || (eq ? last[ch] == level : last[ch] > level); }
};

// Restriction of the residual of one Jacobi sweep from zero (x = w D^-1 b, ONFLY) or
// of a given x, summed over each aggregate: eight lanes per coarse cell, one per fine
// cell, added by lane shuffles.  FORM 1/2 form the finest right-hand side on the fly
// and write it to bout.  Launch: 8 blocks per coarse tile.
template <class T, class Op, int FORM, bool ONFLY>
__global__ __launch_bounds__(NT) void k_mgm_restrict(MGPair L, Op op, MGSrc<T> src, MGVec<T> bout, MGCVec<T> x,
                                                     MGVec<T> bc, KState S, T w, MGGate gate) {
    constexpr int CPB = NT / 8;
    constexpr int BPT = TILE / CPB;
    const int32_t tile = xcd_tile((int32_t)blockIdx.x / BPT, L.coarse.ntiles);
    const int32_t sub = (int32_t)blockIdx.x % BPT;
    const int32_t chid = L.coarse.t2c[tile];
    if (!S.chact[chid] || !gate.open(chid)) return;
    const ChanDev C = L.coarse.ch[chid];
    const ChanDev Fc = L.fine.ch[chid];
    bool act[MGM_K];
    mgm_active(S, chid, Fc.dim, act);
    double sa[MGM_K] = {}, sb[MGM_K] = {};
#pragma unroll
    for (int k = 0; k < MGM_K; ++k) {
        const double* s = scp(S, chid, k);
        sa[k] = FORM == 1 ? s[SC_BETA] : s[SC_ALPHA];
        sb[k] = s[SC_OMEGA];
    }
    const int64_t local = (int64_t)(tile - C.t0) * TILE + (int64_t)sub * CPB + threadIdx.x / 8;
    const int f = threadIdx.x & 7;
    const bool ax0 = Fc.nx != C.nx, ax1 = Fc.ny != C.ny, ax2 = Fc.nz != C.nz;
    const bool valid = local < C.ncell;
    Cell P{}, Q{};
    bool in = false;
    if (valid) {
        P = cell_at(C, local);
        const int di = f & 1, dj = (f >> 1) & 1, dk = f >> 2;
        const int i = ax0 ? 2 * P.i + di : P.i + 8 * di;
        const int j = ax1 ? 2 * P.j + dj : P.j + 8 * dj;
        const int k = ax2 ? 2 * P.k + dk : P.k + 8 * dk;
        in = (ax0 || di == 0) && (ax1 || dj == 0) && (ax2 || dk == 0) && i < Fc.nx && j < Fc.ny && k < Fc.nz;
        Q.i = i;
        Q.j = j;
        Q.k = k;
        Q.g = Fc.c0 + i + (int64_t)Fc.nx * (j + (int64_t)Fc.ny * k);
    }
#pragma unroll
    for (int k = 0; k < MGM_K; ++k) {
        if (!act[k]) continue;
        const T a = T(sa[k]), om = T(sb[k]);
        const T* b0 = src.b[k];
        const T* r = src.r[k];
        const T* pp = src.p[k];
        const T* vv = src.v[k];
        auto bf = [&](int64_t g) -> T {
            if (FORM == 0) return b0[g];
            if (FORM == 1) return r[g] + a * (pp[g] - om * vv[g]);
            return r[g] - a * vv[g];
        };
        T v = T(0);
        if (in) {
            const T* xk = x.v[k];
            const T bq = bf(Q.g);
            v = bq - op.apply(k, Fc, Q, [&](int64_t g) { return ONFLY ? w * bf(g) / op.diag(k, g) : xk[g]; });
            if (FORM != 0) bout.v[k][Q.g] = bq;
        }
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        if (valid && f == 0) bc.v[k][P.g] = v;
    }
}

// After the prolongation: x1 = w D^-1 b + P xc (the one pre-sweep from zero and the
// injected coarse correction, both formed on the fly), y = x1 + w D^-1 (b - A x1).
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgm_post1(MGPair L, Op op, MGCVec<T> b, MGCVec<T> xc, MGVec<T> y, T w,
                                                  KState S, MGGate gate) {
    CLOT_TILE_PROLOGUE(L.fine)
    if (!S.chact[chid] || !gate.open(chid)) return;
    const ChanDev Cc = L.coarse.ch[chid];
    bool act[MGM_K];
    mgm_active(S, chid, C.dim, act);
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const int64_t gc = coarse_of(C, Cc, P.g);
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) {
            if (!act[k]) continue;
            const T* bk = b.v[k];
            const T* xk = xc.v[k];
            auto x1 = [&](int64_t g) { return w * bk[g] / op.diag(k, g) + xk[coarse_of(C, Cc, g)]; };
            const T ax = op.apply(k, C, P, x1);
            y.v[k][P.g] = w * bk[P.g] / op.diag(k, P.g) + xk[gc] + w * (bk[P.g] - ax) / op.diag(k, P.g);
        }
    CLOT_END_CELLS
}

// One weighted-Jacobi sweep: out = y + w D^-1 (b - A y).
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgm_post2(Grid G, Op op, MGCVec<T> b, MGCVec<T> y, MGVec<T> out, T w,
                                                  KState S, MGGate gate) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid] || !gate.open(chid)) return;
    bool act[MGM_K];
    mgm_active(S, chid, C.dim, act);
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) {
            if (!act[k]) continue;
            const T* yk = y.v[k];
            const T ay = op.apply(k, C, P, [&](int64_t g) { return yk[g]; });
            out.v[k][P.g] = yk[P.g] + w * (b.v[k][P.g] - ay) / op.diag(k, P.g);
        }
    CLOT_END_CELLS
}

// Two weighted-Jacobi sweeps from zero (the coarsest level): x1 = w D^-1 b,
// x = x1 + w D^-1 (b - A x1).
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgm_pre(Grid G, Op op, MGCVec<T> b, MGVec<T> x, T w, KState S, MGGate gate) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid] || !gate.open(chid)) return;
    bool act[MGM_K];
    mgm_active(S, chid, C.dim, act);
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) {
            if (!act[k]) continue;
            const T* bk = b.v[k];
            auto x1 = [&](int64_t g) { return w * bk[g] / op.diag(k, g); };
            const T ax = op.apply(k, C, P, x1);
            x.v[k][P.g] = x1(P.g) + w * (bk[P.g] - ax) / op.diag(k, P.g);
        }
    CLOT_END_CELLS
}

// ---- LDS-staged finest-level kernels ------------------------------------------------
// A block owns a brick of 1024 fine cells, four per thread.  It first forms the value
// its stencil reads (MODE_R, MODE_P: the smoothed x1; MODE_S: the given iterate) at
// every cell of the brick and its one-cell halo exactly once, into LDS (the halo from
// neighbouring bricks' cells, read through L2), then applies the momentum stencil to
// its own cells from LDS.  A bricked launch needs every channel coarsened along every
// axis (aggregates then never straddle bricks).
//
// MODE_R: residual restriction.  x1 = w D^-1 b with b formed per FORM (written to bout);
//   the residuals b - A x1 of each 2x2(x2) aggregate are added in registers and by lane
//   shuffles (a thread's four cells are two aggregate pairs along the slow axis, and the
//   x and (3-D) y partners are lanes l^1 and l^BX) and written to the coarse
//   right-hand side.
// MODE_P: prolongation + sweep.  x1 = w D^-1 b + P xc, out = x1 + w D^-1 (b - A x1).
// MODE_S: one sweep.  out = y + w D^-1 (b - A y).
//
// Brick shapes, chosen per kernel by the tile autotuner (one shape index covers a 3-D
// and a 2-D shape): 3-D BX x BY x BZ with BX <= 32 (the y partner lane stays in the
// wave) and BZ a multiple of 4; 2-D BX x BY.
enum { MGM_MODE_R = 0, MGM_MODE_P = 1, MGM_MODE_S = 2 };
constexpr int MGM_NSHAPE = 4;

struct BrickChan {
    int32_t b0;              // first brick of the channel
    int32_t nbx, nby, nbz;   // bricks along each axis
};
struct BrickGrid {
    const BrickChan* bc;
    const int32_t* b2c;      // brick -> channel
    int32_t nb;              // bricks over all channels
};
template <int DIM, int SHAPE>
struct Brick {
    static constexpr int BX = DIM == 3 ? (SHAPE == 0 ? 32 : SHAPE == 1 ? 16 : SHAPE == 2 ? 32 : 16)
                                       : (SHAPE == 0 ? 64 : SHAPE == 1 ? 128 : SHAPE == 2 ? 32 : 256);
    static constexpr int BY = DIM == 3 ? (SHAPE == 0 ? 8 : SHAPE == 1 ? 16 : SHAPE == 2 ? 4 : 8) : 1024 / BX;
    static constexpr int BZ = DIM == 3 ? 1024 / (BX * BY) : 1;
    static constexpr int EX = BX + 2, EY = BY + 2, EZ = DIM == 3 ? BZ + 2 : 1;
    static constexpr int NE = EX * EY * EZ;
    static_assert(BX * BY * BZ == 1024, "four cells per thread");
    static_assert(DIM == 2 || (BX <= 32 && BZ % 4 == 0), "3-D: y partner in the wave, z pairs in a thread");
    // cell m (0..3) of thread t
    __device__ static void cell(int t, int m, int& lx, int& ly, int& lz) {
        lx = t % BX;
        if (DIM == 3) {
            ly = (t / BX) % BY;
            lz = 4 * (t / (BX * BY)) + m;
        } else {
            constexpr int R = 256 / BX;   // rows a pass of the block covers
            ly = 2 * (t / BX) + (m & 1) + 2 * R * (m >> 1);
            lz = 0;
        }
    }
};
// The brick shape of a channel's dimension, on the host.
inline void brick_dims(int dim, int shape, int& bx, int& by, int& bz) {
    static const int d3[MGM_NSHAPE][3] = {{32, 8, 4}, {16, 16, 4}, {32, 4, 8}, {16, 8, 8}};
    static const int d2[MGM_NSHAPE][2] = {{64, 16}, {128, 8}, {32, 32}, {256, 4}};
    if (dim == 3) {
        bx = d3[shape][0];
        by = d3[shape][1];
        bz = d3[shape][2];
    } else {
        bx = d2[shape][0];
        by = d2[shape][1];
        bz = 1;
    }
}
template <int SHAPE>
struct BrickLds {
    static constexpr int NE = Brick<3, SHAPE>::NE > Brick<2, SHAPE>::NE ? Brick<3, SHAPE>::NE : Brick<2, SHAPE>::NE;
};
constexpr int MGM_BRICK_OWN = 1024;

template <class T, int DIM, int SHAPE, int MODE, int FORM>
__device__ inline void mgm_brick_body(const ChanDev& C, const ChanDev& Cc, int bx, int by, int bz,
                                      const MomOp<T>& op, const MGSrc<T>& src, const MGVec<T>& bout,
                                      const MGCVec<T>& xc, const MGVec<T>& out, const bool (&act)[MGM_K],
                                      const double (&sa)[MGM_K], const double (&sb)[MGM_K], T w,
                                      T (*xs)[BrickLds<SHAPE>::NE], T (*bs)[MGM_BRICK_OWN]) {
    using D = Brick<DIM, SHAPE>;
    const int x0 = bx * D::BX, y0 = by * D::BY, z0 = bz * D::BZ;
    // 1. the stencil's input at every cell of the brick and its halo (zero outside the
    //    channel), and the right-hand side at the own cells
    for (int e = threadIdx.x; e < D::NE; e += NT) {
        const int ex = e % D::EX - 1;
        const int ey = (e / D::EX) % D::EY - 1;
        const int ez = DIM == 3 ? e / (D::EX * D::EY) - 1 : 0;
        const int gi = x0 + ex, gj = y0 + ey, gk = z0 + ez;
        const bool inside = gi >= 0 && gi < C.nx && gj >= 0 && gj < C.ny && gk >= 0 && gk < C.nz;
        const bool own = ex >= 0 && ex < D::BX && ey >= 0 && ey < D::BY && ez >= 0 && ez < D::BZ;
        const int oq = ex + D::BX * (ey + D::BY * ez);
        int64_t g = 0, gc = 0;
        T rd = T(0);
        if (inside) {
            g = C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk);
            rd = w / op.aP[g];
            if (MODE == MGM_MODE_P) gc = Cc.c0 + (gi >> 1) + (int64_t)Cc.nx * ((gj >> 1) + (int64_t)Cc.ny * (gk >> 1));
        }
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) {
            if (!act[k]) continue;
            T b = T(0), x1 = T(0);
            if (inside) {
                if (MODE == MGM_MODE_S) {
                    x1 = xc.v[k][g];                       // the iterate the sweep starts from
                    if (own) b = src.b[k][g];
                } else {
                    if (MODE == MGM_MODE_P || FORM == 0) b = src.b[k][g];
                    else if (FORM == 1) b = src.r[k][g] + T(sa[k]) * (src.p[k][g] - T(sb[k]) * src.v[k][g]);
                    else b = src.r[k][g] - T(sa[k]) * src.v[k][g];
                    x1 = rd * b;
                    if (MODE == MGM_MODE_P) x1 += xc.v[k][gc];
                }
                if (own) {
                    bs[k][oq] = b;
                    if (MODE == MGM_MODE_R && FORM != 0) bout.v[k][g] = b;
                }
            }
            xs[k][e] = x1;
        }
    }
    __syncthreads();
    // 2. stencil on the own cells
    const int t = threadIdx.x;
    T res[4][MGM_K];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        int lx, ly, lz;
        D::cell(t, m, lx, ly, lz);
        const int gi = x0 + lx, gj = y0 + ly, gk = z0 + lz;
        const bool inside = gi < C.nx && gj < C.ny && gk < C.nz;
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) res[m][k] = T(0);
        if (!inside) continue;
        const int64_t g = C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk);
        const int e = (lx + 1) + D::EX * ((ly + 1) + D::EY * (DIM == 3 ? lz + 1 : 0));
        const int oq = lx + D::BX * (ly + D::BY * lz);
        // the momentum operator's coefficients (MomOp), in its order: x-, x+, y-, y+, z-, z+
        const T nu = op.nu;
        T cxm = T(0), cxp = T(0), cym = T(0), cyp = T(0), czm = T(0), czp = T(0);
        T d = nu * T(C.gx);
        if (gi > 0) cxm = T(-0.5) * op.phx[fx_id(C, gi, gj, gk)] - d;
        if (gi < C.nx - 1) cxp = T(0.5) * op.phx[fx_id(C, gi + 1, gj, gk)] - d;
        d = nu * T(C.gy);
        if (gj > 0) cym = T(-0.5) * op.phy[fy_id(C, gi, gj, gk)] - d;
        if (gj < C.ny - 1) cyp = T(0.5) * op.phy[fy_id(C, gi, gj + 1, gk)] - d;
        if (DIM == 3) {
            d = nu * T(C.gz);
            if (gk > 0) czm = T(-0.5) * op.phz[fz_id(C, gi, gj, gk)] - d;
            if (gk < C.nz - 1) czp = T(0.5) * op.phz[fz_id(C, gi, gj, gk + 1)] - d;
        }
        const T aP = op.aP[g];
        constexpr int SY = D::EX, SZ = D::EX * D::EY;
#pragma unroll
        for (int k = 0; k < MGM_K; ++k) {
            if (!act[k]) continue;
            const T* x = xs[k];
            T s = T(0);
            if (gi > 0) s += cxm * x[e - 1];
            if (gi < C.nx - 1) s += cxp * x[e + 1];
            if (gj > 0) s += cym * x[e - SY];
            if (gj < C.ny - 1) s += cyp * x[e + SY];
            if (DIM == 3) {
                if (gk > 0) s += czm * x[e - SZ];
                if (gk < C.nz - 1) s += czp * x[e + SZ];
            }
            const T r = bs[k][oq] - (aP * x[e] + s);
            if (MODE == MGM_MODE_R) res[m][k] = r;
            else out.v[k][g] = x[e] + w * r / aP;
        }
    }
    if (MODE == MGM_MODE_R) {
        // aggregates: cells m = 0,1 and 2,3 of a thread, then the x pair (lane ^ 1) and,
        // in 3-D, the y pair (lane ^ BX)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int lx, ly, lz;
            D::cell(t, 2 * h, lx, ly, lz);
#pragma unroll
            for (int k = 0; k < MGM_K; ++k) {
                if (!act[k]) continue;
                T v = res[2 * h][k] + res[2 * h + 1][k];
                v += __shfl_xor(v, 1, 64);
                if (DIM == 3) v += __shfl_xor(v, D::BX, 64);
                const int ci = (x0 + lx) >> 1, cj = (y0 + ly) >> 1, ck = (z0 + lz) >> 1;
                const bool lead = (lx & 1) == 0 && (DIM == 2 || (ly & 1) == 0);
                if (lead && ci < Cc.nx && cj < Cc.ny && ck < Cc.nz)
                    out.v[k][Cc.c0 + ci + (int64_t)Cc.nx * (cj + (int64_t)Cc.ny * ck)] = v;
            }
        }
    }
}

template <class T, int MODE, int FORM, int SHAPE>
__global__ __launch_bounds__(NT) void k_mgm_brick(BrickGrid BG, MGPair L, MomOp<T> op, MGSrc<T> src, MGVec<T> bout,
                                                  MGCVec<T> xc, MGVec<T> out, KState S, T w) {
    const int32_t b = xcd_tile((int32_t)blockIdx.x, BG.nb);
    const int32_t chid = BG.b2c[b];
    if (!S.chact[chid]) return;
    const ChanDev C = L.fine.ch[chid];
    const ChanDev Cc = L.coarse.ch[chid];
    const BrickChan B = BG.bc[chid];
    const int lb = b - B.b0;
    const int bx = lb % B.nbx, by = (lb / B.nbx) % B.nby, bz = lb / (B.nbx * B.nby);
    bool act[MGM_K];
    mgm_active(S, chid, C.dim, act);
    double sa[MGM_K], sb[MGM_K];
#pragma unroll
    for (int k = 0; k < MGM_K; ++k) {
        const double* s = scp(S, chid, k);
        sa[k] = FORM == 1 ? s[SC_BETA] : s[SC_ALPHA];
        sb[k] = s[SC_OMEGA];
    }
    __shared__ T xs[MGM_K][BrickLds<SHAPE>::NE];
    __shared__ T bs[MGM_K][MGM_BRICK_OWN];
    if (C.dim == 3)
        mgm_brick_body<T, 3, SHAPE, MODE, FORM>(C, Cc, bx, by, bz, op, src, bout, xc, out, act, sa, sb, w, xs, bs);
    else
        mgm_brick_body<T, 2, SHAPE, MODE, FORM>(C, Cc, bx, by, bz, op, src, bout, xc, out, act, sa, sb, w, xs, bs);
}

// ---- BiCGStab with the V-cycle as right preconditioner ------------------------------
// y = M^-1 p and z = M^-1 s come from the V-cycles; the phases apply A to them.

// v = A y; rhat . v
// One component per grid row (blockIdx.y), as the Jacobi BiCGStab's phases.
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_pbicg_1(Grid G, Op op, KVec<T, K> V, MGCVec<T> y, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    if (scp(S, chid, k)[SC_ACT] == 0.0) {
        zero_partials_at<1>(S, tile, k);
        return;
    }
    __shared__ double lds[5];
    double acc[1] = {0.0};
    const T* yk = y.v[k];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T vn = op.apply(k, C, P, [&](int64_t g) { return yk[g]; });
        V.v[par ^ 1][k][P.g] = vn;
        acc[0] += (double)V.rh[k][P.g] * (double)vn;
    CLOT_END_CELLS
    store_partials_at<1>(acc, S, tile, k, lds);
}

// t = A z; t.s, t.t
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_pbicg_2(Grid G, Op op, KVec<T, K> V, MGCVec<T> z, MGCVec<T> s, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    if (scp(S, chid, k)[SC_ACT] == 0.0) {
        zero_partials_at<2>(S, tile, 2 * k);
        return;
    }
    __shared__ double lds[5 * 2];
    double acc[2] = {0.0, 0.0};
    const T* zk = z.v[k];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T t = op.apply(k, C, P, [&](int64_t g) { return zk[g]; });
        V.t[k][P.g] = t;
        const T sv = s.v[k][P.g];
        acc[0] += (double)t * (double)sv;
        acc[1] += (double)t * (double)t;
    CLOT_END_CELLS
    store_partials_at<2>(acc, S, tile, 2 * k, lds);
}

// x += alpha y + omega z; r = s - omega t; rhat.r, r.r
template <class T, int K>
__global__ __launch_bounds__(NT) void k_pbicg_3(Grid G, KVec<T, K> V, MGCVec<T> y, MGCVec<T> z, MGCVec<T> s,
                                                KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    const double* sc = scp(S, chid, k);
    if (sc[SC_ACT] == 0.0) {
        zero_partials_at<2>(S, tile, 2 * k);
        return;
    }
    __shared__ double lds[5 * 2];
    double acc[2] = {0.0, 0.0};
    const T a = (T)sc[SC_ALPHA], om = (T)sc[SC_OMEGA];
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        const T sv = s.v[k][g];
        V.x[k][g] += a * y.v[k][g] + om * z.v[k][g];
        const T r = sv - om * V.t[k][g];
        V.r[k][g] = r;
        acc[0] += (double)V.rh[k][g] * (double)r;
        acc[1] += (double)r * (double)r;
    CLOT_END_CELLS
    store_partials_at<2>(acc, S, tile, 2 * k, lds);
}

}  // namespace clot
