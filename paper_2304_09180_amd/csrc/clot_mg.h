// Geometric multigrid preconditioner for the pressure system (gfx950).
//
// Hierarchy: each level halves every axis that still has >= 3 cells (ceil(n/2)),
// per channel, until the channel has <= MG_COARSE cells.  The coarse operator is
// the aggregation (piecewise-constant) Galerkin product with every coupling normal
// to a coarsened axis scaled by 1/2, which reproduces the re-discretised Laplacian
// on uniform cells and keeps the operator SPD.  A V-cycle is two weighted-Jacobi
// sweeps down, residual restriction by summation (eight lanes per aggregate), the
// exact inverse on the coarsest level (a dense matrix built once per pressure
// solve), prolongation by injection fused into the first of two Jacobi sweeps up:
// a symmetric preconditioner for CG.
#pragma once
#include "clot_krylov.h"

namespace clot {

constexpr int MG_COARSE = 64;       // max cells on a channel's coarsest level
constexpr int MG_MAXLEV = 14;

// Face-coefficient operator of a coarse level: y = d x - sum_f c_f x_N.
template <class T>
struct CoefOp {
    const T* dg;
    const T* cx;
    const T* cy;
    const T* cz;
    __device__ T diag(int, int64_t g) const { return dg[g]; }
    template <class XV>
    __device__ T offsum(const ChanDev& C, const Cell& P, XV xv) const {
        T s = T(0);
        if (P.i > 0) s += cx[fx_id(C, P.i, P.j, P.k)] * xv(P.g - 1);
        if (P.i < C.nx - 1) s += cx[fx_id(C, P.i + 1, P.j, P.k)] * xv(P.g + 1);
        if (P.j > 0) s += cy[fy_id(C, P.i, P.j, P.k)] * xv(P.g - C.nx);
        if (P.j < C.ny - 1) s += cy[fy_id(C, P.i, P.j + 1, P.k)] * xv(P.g + C.nx);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            if (P.k > 0) s += cz[fz_id(C, P.i, P.j, P.k)] * xv(P.g - sz);
            if (P.k < C.nz - 1) s += cz[fz_id(C, P.i, P.j, P.k + 1)] * xv(P.g + sz);
        }
        return s;
    }
    template <class XV>
    __device__ T apply(int, const ChanDev& C, const Cell& P, XV xv) const {
        return dg[P.g] * xv(P.g) - offsum(C, P, xv);
    }
};

// Face coefficient of the fine level, for building the next one.
template <class T>
struct FineCoefPres {      // level 0: c_f = (rAU_L + rAU_R)/2 * A/d, outlet 2 A/dx rAU_P
    const T* rAU;
    __device__ T face(const ChanDev& C, int ax, int64_t gL, int64_t gR) const {
        const double a = ax == 0 ? C.gx : ax == 1 ? C.gy : C.gz;
        return T(0.5 * a) * (rAU[gL] + rAU[gR]);
    }
    __device__ T outlet(const ChanDev& C, int64_t g) const { return T(2.0 * C.gx) * rAU[g]; }
};

template <class T>
struct FineCoefLevel {     // coarse level as the fine side of the next one
    const T* cx;
    const T* cy;
    const T* cz;
    const T* cout;
    // face between fine cells gL, gR along ax, where gR is the high neighbour; i,j,k of gR
    __device__ T face_at(const ChanDev& C, int ax, int i, int j, int k) const {
        return ax == 0 ? cx[fx_id(C, i, j, k)] : ax == 1 ? cy[fy_id(C, i, j, k)] : cz[fz_id(C, i, j, k)];
    }
};

struct MGPair {
    Grid fine;
    Grid coarse;
};

// Build one coarse level from its fine level: face coefficients (low faces of each
// coarse cell plus the high boundary faces), outlet coefficient and diagonal.
template <class T, bool FROM_PRES>
__global__ __launch_bounds__(NT) void k_mg_setup(MGPair L, FineCoefPres<T> fp, FineCoefLevel<T> fl, T* cx, T* cy, T* cz,
                                                 T* cout, T* dg) {
    CLOT_TILE_PROLOGUE(L.coarse)
    const ChanDev Fc = L.fine.ch[chid];
    const bool ax0 = Fc.nx != C.nx, ax1 = Fc.ny != C.ny, ax2 = Fc.nz != C.nz;
    const T s0 = ax0 ? T(0.5) : T(1), s1 = ax1 ? T(0.5) : T(1), s2 = ax2 ? T(0.5) : T(1);
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        // fine index ranges of this aggregate
        const int i0 = ax0 ? 2 * P.i : P.i, i1 = ax0 ? min(2 * P.i + 1, Fc.nx - 1) : P.i;
        const int j0 = ax1 ? 2 * P.j : P.j, j1 = ax1 ? min(2 * P.j + 1, Fc.ny - 1) : P.j;
        const int k0 = ax2 ? 2 * P.k : P.k, k1 = ax2 ? min(2 * P.k + 1, Fc.nz - 1) : P.k;
        auto fg = [&](int i, int j, int k) { return Fc.c0 + i + (int64_t)Fc.nx * (j + (int64_t)Fc.ny * k); };
        // sum of fine couplings across the coarse face on the low (lo=true) or high side of axis ax
        auto across = [&](int ax, bool lo) -> T {
            T s = T(0);
            if (ax == 0) {
                const int fi = lo ? i0 : i1 + 1;        // fine face index along x (between fi-1 and fi)
                if (fi <= 0 || fi >= Fc.nx) return T(0);
                for (int k = k0; k <= k1; ++k)
                    for (int j = j0; j <= j1; ++j)
                        s += FROM_PRES ? fp.face(Fc, 0, fg(fi - 1, j, k), fg(fi, j, k)) : fl.face_at(Fc, 0, fi, j, k);
            } else if (ax == 1) {
                const int fj = lo ? j0 : j1 + 1;
                if (fj <= 0 || fj >= Fc.ny) return T(0);
                for (int k = k0; k <= k1; ++k)
                    for (int i = i0; i <= i1; ++i)
                        s += FROM_PRES ? fp.face(Fc, 1, fg(i, fj - 1, k), fg(i, fj, k)) : fl.face_at(Fc, 1, i, fj, k);
            } else {
                const int fk = lo ? k0 : k1 + 1;
                if (fk <= 0 || fk >= Fc.nz) return T(0);
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i)
                        s += FROM_PRES ? fp.face(Fc, 2, fg(i, j, fk - 1), fg(i, j, fk)) : fl.face_at(Fc, 2, i, j, fk);
            }
            return s;
        };
        const T xl = s0 * across(0, true), xh = s0 * across(0, false);
        const T yl = s1 * across(1, true), yh = s1 * across(1, false);
        T zl = T(0), zh = T(0);
        if (C.dim == 3) {
            zl = s2 * across(2, true);
            zh = s2 * across(2, false);
        }
        T co = T(0);
        if (i1 == Fc.nx - 1) {
            for (int k = k0; k <= k1; ++k)
                for (int j = j0; j <= j1; ++j)
                    co += FROM_PRES ? fp.outlet(Fc, fg(Fc.nx - 1, j, k)) : fl.cout[fg(Fc.nx - 1, j, k)];
            co *= s0;
        }
        cx[fx_id(C, P.i, P.j, P.k)] = xl;
        if (P.i == C.nx - 1) cx[fx_id(C, C.nx, P.j, P.k)] = T(0);
        cy[fy_id(C, P.i, P.j, P.k)] = yl;
        if (P.j == C.ny - 1) cy[fy_id(C, P.i, C.ny, P.k)] = T(0);
        if (C.dim == 3) {
            cz[fz_id(C, P.i, P.j, P.k)] = zl;
            if (P.k == C.nz - 1) cz[fz_id(C, P.i, P.j, C.nz)] = T(0);
        }
        cout[P.g] = co;
        dg[P.g] = xl + xh + yl + yh + zl + zh + co;
    CLOT_END_CELLS
}

// Two weighted-Jacobi sweeps from zero: x1 = w D^-1 b, x = x1 + w D^-1 (b - A x1).
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mg_pre(Grid G, Op op, const T* b, T* x, T w, const int32_t* chact) {
    CLOT_TILE_PROLOGUE(G)
    if (!chact[chid]) return;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto x1 = [&](int64_t g) { return w * b[g] / op.diag(0, g); };
        const T ax = op.apply(0, C, P, x1);
        x[P.g] = x1(P.g) + w * (b[P.g] - ax) / op.diag(0, P.g);
    CLOT_END_CELLS
}

// Restriction by summation of the fine residual over each aggregate (with ONFLY
// the smoothed x is the single sweep from zero, w D^-1 b, formed where it is read).  Eight lanes
// share a coarse cell (one per fine cell of the 2x2x2 aggregate), so the fine
// stencils are evaluated in parallel; the eight values are added by lane shuffles.
// Launch: 8 blocks per coarse tile (32 coarse cells per block).
template <class T, class Op, bool ONFLY>
__global__ __launch_bounds__(NT) void k_mg_restrict(MGPair L, Op op, const T* b, const T* x, T* bc,
                                                    const int32_t* chact, T w) {
    constexpr int CPB = NT / 8;                      // coarse cells per block
    constexpr int BPT = TILE / CPB;                  // blocks per coarse tile
    const int32_t tile = xcd_tile((int32_t)blockIdx.x / BPT, L.coarse.ntiles);
    const int32_t sub = (int32_t)blockIdx.x % BPT;
    const int32_t chid = L.coarse.t2c[tile];
    if (!chact[chid]) return;
    const ChanDev C = L.coarse.ch[chid];
    const ChanDev Fc = L.fine.ch[chid];
    const int64_t local = (int64_t)(tile - C.t0) * TILE + (int64_t)sub * CPB + threadIdx.x / 8;
    const int f = threadIdx.x & 7;
    const bool ax0 = Fc.nx != C.nx, ax1 = Fc.ny != C.ny, ax2 = Fc.nz != C.nz;
    T v = T(0);
    bool valid = local < C.ncell;
    Cell P;
    if (valid) {
        P = cell_at(C, local);
        const int di = f & 1, dj = (f >> 1) & 1, dk = f >> 2;
        const int i = ax0 ? 2 * P.i + di : P.i + 8 * di;     // offsets on uncoarsened axes are invalid
        const int j = ax1 ? 2 * P.j + dj : P.j + 8 * dj;
        const int k = ax2 ? 2 * P.k + dk : P.k + 8 * dk;
        const bool in = (ax0 || di == 0) && (ax1 || dj == 0) && (ax2 || dk == 0) && i < Fc.nx && j < Fc.ny &&
                        k < Fc.nz;
        if (in) {
            Cell Q;
            Q.i = i;
            Q.j = j;
            Q.k = k;
            Q.g = Fc.c0 + i + (int64_t)Fc.nx * (j + (int64_t)Fc.ny * k);
            v = b[Q.g] - op.apply(0, Fc, Q, [&](int64_t g) { return ONFLY ? w * b[g] / op.diag(0, g) : x[g]; });
        }
    }
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    if (valid && f == 0) bc[P.g] = v;
}

// Coarse cell of fine cell g (injection prolongation).
__device__ inline int64_t coarse_of(const ChanDev& Fc, const ChanDev& Cc, int64_t g) {
    const Cell Q = cell_at(Fc, g - Fc.c0);
    const int i = Fc.nx != Cc.nx ? Q.i >> 1 : Q.i;
    const int j = Fc.ny != Cc.ny ? Q.j >> 1 : Q.j;
    const int k = Fc.nz != Cc.nz ? Q.k >> 1 : Q.k;
    return Cc.c0 + i + (int64_t)Cc.nx * (j + (int64_t)Cc.ny * k);
}

// x1 = x + P xc (formed on the fly), then one Jacobi sweep into y.
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mg_post1(MGPair L, Op op, const T* b, const T* x, const T* xc, T* y, T w,
                                                 const int32_t* chact) {
    CLOT_TILE_PROLOGUE(L.fine)
    if (!chact[chid]) return;
    const ChanDev Cc = L.coarse.ch[chid];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto x1 = [&](int64_t g) { return x[g] + xc[coarse_of(C, Cc, g)]; };
        const T ax = op.apply(0, C, P, x1);
        y[P.g] = x1(P.g) + w * (b[P.g] - ax) / op.diag(0, P.g);
    CLOT_END_CELLS
}

// Final Jacobi sweep x = y + w D^-1 (b - A y); on the finest level it also forms
// r.z for the outer CG (DOT = true) and finishes beta on the device.
template <class T, class Op, bool DOT>
__global__ __launch_bounds__(NT) void k_mg_post2(Grid G, Op op, const T* b, const T* y, T* x, T w, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5];
    double acc[1] = {0.0};
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T ay = op.apply(0, C, P, [&](int64_t g) { return y[g]; });
        const T z = y[P.g] + w * (b[P.g] - ay) / op.diag(0, P.g);
        x[P.g] = z;
        if (DOT) acc[0] += (double)b[P.g] * (double)z;
    CLOT_END_CELLS
    if (DOT) store_partials<1>(acc, S.part, S.pstride, tile, lds);
}

// One post-smoothing sweep with the prolonged correction (the single-sweep cycle):
// x1 = w D^-1 b + P xc (formed on the fly), z = x1 + w D^-1 (b - A x1); on the
// finest level also r.z for the outer CG.
template <class T, class Op, bool DOT>
__global__ __launch_bounds__(NT) void k_mg_post_one(MGPair L, Op op, const T* b, const T* xc, T* z, T w, KState S) {
    CLOT_TILE_PROLOGUE(L.fine)
    if (!S.chact[chid]) return;
    const ChanDev Cc = L.coarse.ch[chid];
    __shared__ double lds[5];
    double acc[1] = {0.0};
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto x1 = [&](int64_t g) { return w * b[g] / op.diag(0, g) + xc[coarse_of(C, Cc, g)]; };
        const T ax = op.apply(0, C, P, x1);
        const T zz = x1(P.g) + w * (b[P.g] - ax) / op.diag(0, P.g);
        z[P.g] = zz;
        if (DOT) acc[0] += (double)b[P.g] * (double)zz;
    CLOT_END_CELLS
    if (DOT) store_partials<1>(acc, S.part, S.pstride, tile, lds);
}

struct EpiMgDot {   // r.z of the new preconditioned residual -> beta
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        double* s = scp(S, ch, 0);
        if (s[SC_ACT] == 0.0) return;
        const double rz = sums[0];
        s[SC_BETA] = s[SC_IT] > 0.0 && s[SC_RZ] != 0.0 ? rz / s[SC_RZ] : 0.0;
        s[SC_RZ] = rz;
    }
};

// Coarsest level, set-up: one 64-thread block per channel builds the dense matrix
// of its (<= MG_COARSE) cells and inverts it in place by Gauss-Jordan elimination
// in FP64 (SPD, so no pivoting).  inv holds MG_COARSE^2 doubles per channel.
template <class T>
__global__ __launch_bounds__(MG_COARSE) void k_mg_coarse_setup(Grid G, CoefOp<T> op, double* inv, int nch) {
    const int chid = blockIdx.x;
    if (chid >= nch) return;
    const ChanDev C = G.ch[chid];
    const int n = (int)C.ncell;
    const int t = threadIdx.x;
    __shared__ double a[MG_COARSE][MG_COARSE + 1];
    for (int j = 0; j < MG_COARSE; ++j) a[t][j] = (t == j) ? 1.0 : 0.0;
    if (t < n) {
        const Cell P = cell_at(C, t);
        a[t][t] = (double)op.dg[P.g];
        // off-diagonals: -c_f at each neighbour (probe the operator with unit vectors)
        auto put = [&](int64_t gn, T cf) { a[t][gn - C.c0] = -(double)cf; };
        if (P.i > 0) put(P.g - 1, op.cx[fx_id(C, P.i, P.j, P.k)]);
        if (P.i < C.nx - 1) put(P.g + 1, op.cx[fx_id(C, P.i + 1, P.j, P.k)]);
        if (P.j > 0) put(P.g - C.nx, op.cy[fy_id(C, P.i, P.j, P.k)]);
        if (P.j < C.ny - 1) put(P.g + C.nx, op.cy[fy_id(C, P.i, P.j + 1, P.k)]);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            if (P.k > 0) put(P.g - sz, op.cz[fz_id(C, P.i, P.j, P.k)]);
            if (P.k < C.nz - 1) put(P.g + sz, op.cz[fz_id(C, P.i, P.j, P.k + 1)]);
        }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = a[k][k];
        __syncthreads();
        if (t < n) a[k][t] = (t == k ? 1.0 : a[k][t]) / piv;
        __syncthreads();
        if (t < n && t != k) {
            const double f = a[t][k];
            for (int j = 0; j < n; ++j) a[t][j] = (j == k ? 0.0 : a[t][j]) - f * a[k][j];
        }
        __syncthreads();
    }
    double* out = inv + (int64_t)chid * MG_COARSE * MG_COARSE;
    for (int j = 0; j < MG_COARSE; ++j) out[t * MG_COARSE + j] = (t < n && j < n) ? a[t][j] : 0.0;
}

// Coarsest level, solve: x = A^-1 b per channel.
template <class T>
__global__ __launch_bounds__(MG_COARSE) void k_mg_coarse(Grid G, const double* inv, const T* b, T* x,
                                                         const int32_t* chact, int nch) {
    const int chid = blockIdx.x;
    if (chid >= nch || !chact[chid]) return;
    const ChanDev C = G.ch[chid];
    const int n = (int)C.ncell;
    const int t = threadIdx.x;
    __shared__ double bs[MG_COARSE];
    bs[t] = t < n ? (double)b[C.c0 + t] : 0.0;
    __syncthreads();
    if (t >= n) return;
    const double* row = inv + ((int64_t)chid * MG_COARSE + t) * MG_COARSE;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += row[j] * bs[j];
    x[C.c0 + t] = T(s);
}

// ------------------------------------------------------------------------------------
// The small end of the hierarchy in one launch: for the levels whose every channel
// has at most a few thousand cells (the separate launches of those levels cost more
// than their work), one 1024-thread block per channel runs the rest of the V-cycle
// in LDS: it reads its channel's plan (the levels' geometry and LDS layout, built on
// the host at set-up), loads the levels' coefficients and the restricted residual once, does
// the pre-smoothing and restriction down to the coarsest level, the dense solve, the
// prolongation and post-smoothing back up, with block barriers between the passes,
// and writes back the correction of the first tail level.  Every cell update is the
// expression of the separate kernels above (the eight-value restriction sum in the
// same pairwise order), so the result is the same bit for bit.
// ------------------------------------------------------------------------------------
constexpr int MG_TAIL_BS = 1024;

template <class T>
struct MGTailLevel {   // a tail level's arrays (the channels' geometry comes from TailPlan)
    T *x, *y, *b, *dg, *cx, *cy, *cz, *cout;
};
template <class T>
struct MGTail {
    MGTailLevel<T> L[MG_MAXLEV];
    int n;      // levels in the tail; the last is the coarsest
};

// Element counts of one channel's level arrays held in LDS: b, x, y, dg (cells) and
// the three face-coefficient arrays; the coarsest level keeps b and x only.
__host__ __device__ inline int64_t tail_align(int64_t e, int bytes) {
    const int64_t q = 16 / bytes;   // keep every array 16-byte aligned
    return (e + q - 1) / q * q;
}
__host__ __device__ inline int64_t tail_level_elems(int dim, int nx, int ny, int nz, bool coarsest, int bytes) {
    const int64_t n = (int64_t)nx * ny * nz;
    if (coarsest) return 2 * tail_align(n, bytes);
    const int64_t fx = (int64_t)(nx + 1) * ny * nz, fy = (int64_t)nx * (ny + 1) * nz;
    const int64_t fz = dim == 3 ? (int64_t)nx * ny * (nz + 1) : 0;
    return 4 * tail_align(n, bytes) + tail_align(fx, bytes) + tail_align(fy, bytes) + tail_align(fz, bytes);
}

// One tail level as the block sees it: the channel's level table with zero offsets
// (the arrays are the block's own) and the element offsets of its LDS arrays.
struct TailLds {
    ChanDev C;
    int32_t ob, ox, oy, odg, ocx, ocy, ocz;
    int32_t nfx, nfy, nfz;
};

// One array copied into the tail's LDS: n elements from src to lds[dst].
template <class T>
struct TailSeg {
    const T* src;
    int32_t dst, n;
};
constexpr int MG_TAIL_SEGS = 4 * MG_MAXLEV + 1;

// The tail's set-up for one channel, built on the host when the context is created
// (geometry only, no addresses, so a saved workspace carries it unchanged): each
// level's table with zero offsets and the LDS offsets of its arrays, and the arrays to
// copy in as (level, array, first element, LDS offset, count).  The block reads it in
// one round of loads instead of walking the levels' channel tables from one thread.
enum { TAIL_DG = 0, TAIL_CX = 1, TAIL_CY = 2, TAIL_CZ = 3, TAIL_B = 4 };
struct TailSegRef {
    int64_t off;
    int32_t lvl, kind, dst, n;
};
struct TailPlan {
    TailLds lv[MG_MAXLEV];
    TailSegRef seg[MG_TAIL_SEGS];
    int32_t start[MG_TAIL_SEGS + 1];
    int32_t nseg, nl;
    int64_t out0;   // the channel's first cell on the first tail level (the write-back)
};
static_assert(sizeof(TailPlan) % 4 == 0, "copied as 32-bit words");

// lc[l]: this channel's table on tail level l (l < nl, the last the coarsest).
inline void tail_plan_build(TailPlan& P, int nl, const ChanDev* lc, int bytes) {
    P = TailPlan{};
    P.nl = nl;
    int64_t o = 0;
    for (int l = 0; l < nl; ++l) {
        TailLds& v = P.lv[l];
        v.C = lc[l];
        v.C.c0 = 0;
        v.C.fx0 = 0;
        v.C.fy0 = 0;
        v.C.fz0 = 0;
        const int64_t n = v.C.ncell;
        v.ob = (int32_t)o;
        o += tail_align(n, bytes);
        v.ox = (int32_t)o;
        o += tail_align(n, bytes);
        v.oy = v.odg = v.ocx = v.ocy = v.ocz = 0;
        v.nfx = (v.C.nx + 1) * v.C.ny * v.C.nz;
        v.nfy = v.C.nx * (v.C.ny + 1) * v.C.nz;
        v.nfz = v.C.dim == 3 ? v.C.nx * v.C.ny * (v.C.nz + 1) : 0;
        if (l + 1 == nl) break;
        v.oy = (int32_t)o;
        o += tail_align(n, bytes);
        v.odg = (int32_t)o;
        o += tail_align(n, bytes);
        v.ocx = (int32_t)o;
        o += tail_align(v.nfx, bytes);
        v.ocy = (int32_t)o;
        o += tail_align(v.nfy, bytes);
        v.ocz = (int32_t)o;
        o += tail_align(v.nfz, bytes);
    }
    int ns = 0;
    int32_t e = 0;
    auto add = [&](int lvl, int kind, int64_t off, int32_t dst, int32_t n) {
        if (n <= 0) return;
        P.seg[ns] = TailSegRef{off, lvl, kind, dst, n};
        P.start[ns] = e;
        e += n;
        ++ns;
    };
    for (int l = 0; l + 1 < nl; ++l) {
        const ChanDev& C = lc[l];
        const TailLds& v = P.lv[l];
        add(l, TAIL_DG, C.c0, v.odg, (int32_t)C.ncell);
        add(l, TAIL_CX, C.fx0, v.ocx, v.nfx);
        add(l, TAIL_CY, C.fy0, v.ocy, v.nfy);
        add(l, TAIL_CZ, C.fz0, v.ocz, v.nfz);
    }
    add(0, TAIL_B, lc[0].c0, P.lv[0].ob, (int32_t)lc[0].ncell);
    P.start[ns] = e;
    P.nseg = ns;
    P.out0 = lc[0].c0;
}

// All the segments in one pass over their concatenation: each thread issues the loads
// of up to U elements, whatever arrays they fall in, before it stores any of them, so
// that the latencies of the arrays overlap instead of adding up array by array.
template <class T>
__device__ inline void tail_copy_in(T* lds, const TailSeg<T>* seg, const int32_t* start, int nseg) {
    constexpr int U = 16;
    const int32_t tot = start[nseg];
    for (int32_t e0 = threadIdx.x; e0 < tot; e0 += U * MG_TAIL_BS) {
        T v[U];
        int32_t d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = e0 + u * MG_TAIL_BS;
            d[u] = -1;
            v[u] = T(0);
            if (e < tot) {
                int s = 0;
                while (e >= start[s + 1]) ++s;
                const int32_t q = e - start[s];
                v[u] = seg[s].src[q];
                d[u] = seg[s].dst + q;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (d[u] >= 0) lds[d[u]] = v[u];
    }
}

template <class T>
__global__ __launch_bounds__(MG_TAIL_BS) void k_mg_tail(MGTail<T> tl, const TailPlan* plans, T w, const double* inv,
                                                        const int32_t* chact, int sweeps) {
    const int chid = blockIdx.x;
    if (!chact[chid]) return;
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T* const lds = reinterpret_cast<T*>(tail_lds);
    // the channel's plan, copied in by the whole block, then each segment's address
    __shared__ TailPlan pl;
    __shared__ TailSeg<T> seg[MG_TAIL_SEGS];
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(plans + chid);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&pl);
        for (int q = threadIdx.x; q < (int)(sizeof(TailPlan) / 4); q += MG_TAIL_BS) dst[q] = src[q];
    }
    __syncthreads();
    if ((int)threadIdx.x < pl.nseg) {
        const TailSegRef& r = pl.seg[threadIdx.x];
        const MGTailLevel<T>& L = tl.L[r.lvl];
        const T* base = r.kind == TAIL_DG ? L.dg : r.kind == TAIL_CX ? L.cx : r.kind == TAIL_CY ? L.cy
                      : r.kind == TAIL_CZ ? L.cz : L.b;
        seg[threadIdx.x] = TailSeg<T>{base + r.off, r.dst, r.n};
    }
    __syncthreads();
    const TailLds* const tv = pl.lv;
    const int nl = tl.n;
    tail_copy_in(lds, seg, pl.start, pl.nseg);
    __syncthreads();
    // down: `sweeps` Jacobi sweeps (from zero) and the residual restriction per level
    for (int l = 0; l + 1 < nl; ++l) {
        const TailLds& v = tv[l];
        const ChanDev& C = v.C;
        const CoefOp<T> op{lds + v.odg, lds + v.ocx, lds + v.ocy, lds + v.ocz};
        const T* b = lds + v.ob;
        T* x = lds + v.ox;
        T* y = lds + v.oy;
        // first sweep from zero, stored (the same value the separate kernel forms at
        // each neighbour), then the others alternating between x and y so that the last
        // lands in x
        T* cur = sweeps % 2 == 0 ? y : x;
        for (int64_t g = threadIdx.x; g < C.ncell; g += MG_TAIL_BS) cur[g] = w * b[g] / op.diag(0, g);
        __syncthreads();
        for (int k = 1; k < sweeps; ++k) {
            T* nxt = cur == x ? y : x;
            for (int64_t local = threadIdx.x; local < C.ncell; local += MG_TAIL_BS) {
                const Cell P = cell_at(C, local);
                const T ac = op.apply(0, C, P, [&](int64_t g) { return cur[g]; });
                nxt[P.g] = cur[P.g] + w * (b[P.g] - ac) / op.diag(0, P.g);
            }
            __syncthreads();
            cur = nxt;
        }
        const ChanDev& Cc = tv[l + 1].C;
        T* bc = lds + tv[l + 1].ob;
        const bool ax0 = C.nx != Cc.nx, ax1 = C.ny != Cc.ny, ax2 = C.nz != Cc.nz;
        for (int64_t local = threadIdx.x; local < Cc.ncell; local += MG_TAIL_BS) {
            const Cell P = cell_at(Cc, local);
            T r[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int di = f & 1, dj = (f >> 1) & 1, dk = f >> 2;
                const int i = ax0 ? 2 * P.i + di : P.i + 8 * di;
                const int j = ax1 ? 2 * P.j + dj : P.j + 8 * dj;
                const int k = ax2 ? 2 * P.k + dk : P.k + 8 * dk;
                const bool in = (ax0 || di == 0) && (ax1 || dj == 0) && (ax2 || dk == 0) && i < C.nx && j < C.ny &&
                                k < C.nz;
                r[f] = T(0);
                if (in) {
                    Cell Q;
                    Q.i = i;
                    Q.j = j;
                    Q.k = k;
                    Q.g = i + (int64_t)C.nx * (j + (int64_t)C.ny * k);
                    r[f] = b[Q.g] - op.apply(0, C, Q, [&](int64_t g) { return x[g]; });
                }
            }
            // the butterfly order of the shuffle reduction: pairs, then pairs of pairs
            const T s01 = r[0] + r[1], s23 = r[2] + r[3], s45 = r[4] + r[5], s67 = r[6] + r[7];
            bc[P.g] = (s01 + s23) + (s45 + s67);
        }
        __syncthreads();
    }
    // coarsest level: x = A^-1 b (dense inverse, FP64 accumulation)
    {
        const TailLds& v = tv[nl - 1];
        const int n = (int)v.C.ncell;
        __shared__ double bs[MG_COARSE];
        if (threadIdx.x < MG_COARSE) bs[threadIdx.x] = (int)threadIdx.x < n ? (double)lds[v.ob + threadIdx.x] : 0.0;
        __syncthreads();
        if ((int)threadIdx.x < n) {
            const double* row = inv + ((int64_t)chid * MG_COARSE + threadIdx.x) * MG_COARSE;
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += row[j] * bs[j];
            lds[v.ox + threadIdx.x] = T(s);
        }
        __syncthreads();
    }
    // up: prolongation by injection fused into the first sweep, then the second sweep
    for (int l = nl - 2; l >= 0; --l) {
        const TailLds& v = tv[l];
        const ChanDev& C = v.C;
        const ChanDev& Cc = tv[l + 1].C;
        // the finished correction of the level below: x after an even number of sweeps, y
        // after an odd one (the coarsest level's is x, from the dense solve)
        const T* xc = lds + ((l + 1 == nl - 1 || sweeps % 2 == 0) ? tv[l + 1].ox : tv[l + 1].oy);
        const CoefOp<T> op{lds + v.odg, lds + v.ocx, lds + v.ocy, lds + v.ocz};
        const T* b = lds + v.ob;
        T* x = lds + v.ox;
        T* y = lds + v.oy;
        // prolongation by injection, in place, then the sweeps alternating x -> y -> x ...
        for (int64_t g = threadIdx.x; g < C.ncell; g += MG_TAIL_BS) x[g] = x[g] + xc[coarse_of(C, Cc, g)];
        __syncthreads();
        T* cur = x;
        for (int k = 0; k < sweeps; ++k) {
            T* nxt = cur == x ? y : x;
            for (int64_t local = threadIdx.x; local < C.ncell; local += MG_TAIL_BS) {
                const Cell P = cell_at(C, local);
                const T ac = op.apply(0, C, P, [&](int64_t g) { return cur[g]; });
                nxt[P.g] = cur[P.g] + w * (b[P.g] - ac) / op.diag(0, P.g);
            }
            __syncthreads();
            cur = nxt;
        }
    }
    // the first tail level's correction, for the prolongation of the level above
    const int32_t o0 = (nl == 1 || sweeps % 2 == 0) ? tv[0].ox : tv[0].oy;
    for (int64_t q = threadIdx.x; q < tv[0].C.ncell; q += MG_TAIL_BS) tl.L[0].x[pl.out0 + q] = lds[o0 + q];
}

// ------------------------------------------------------------------------------------
// CG driven by the V-cycle: z is stored by the preconditioner.
// ------------------------------------------------------------------------------------

// r = b - A x; rr, bb.  (z and rz come from the first V-cycle.)
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgcg_init(Grid G, Op op, KVec<T, 1> V, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5 * 2];
    double acc[2] = {0.0, 0.0};
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T* x = V.x[0];
        const T ax = op.apply(0, C, P, [&](int64_t g) { return x[g]; });
        const T b = V.b[0][P.g];
        const T r = b - ax;
        V.r[0][P.g] = r;
        V.p[0][0][P.g] = T(0);
        acc[0] += (double)b * (double)b;
        acc[1] += (double)r * (double)r;
    CLOT_END_CELLS
    store_partials<2>(acc, S.part, S.pstride, tile, lds);
}

struct EpiMgcgInit {
    static constexpr bool kInit = true;
    double rtol;
    int tol_mode;
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        double* s = scp(S, ch, 0);
        s[SC_BB] = sums[0];
        s[SC_BBS] = sums[0];
        s[SC_RR] = sums[1];
        s[SC_RR0] = sums[1];
        if (tol_mode == 0) s[SC_TOL2] = rtol * rtol * sums[0];
        s[SC_BETA] = 0.0;
        s[SC_RZ] = 0.0;
        s[SC_IT] = 0.0;
        s[SC_FAIL] = 0.0;
        const bool act = s[SC_BB] > 0.0 && s[SC_RR] > s[SC_TOL2];
        s[SC_ACT] = act ? 1.0 : 0.0;
        S.chact[ch] = act;
        if (act) atomicAdd(S.nact, 1);
    }
};

// p_new = z + beta p_old (own cell and neighbours), q = A p_new, alpha = rz/(p.q)
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgcg_a(Grid G, Op op, KVec<T, 1> V, const T* z, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5];
    double acc[1] = {0.0};
    const double* s0 = scp(S, chid, 0);
    const T bk = (T)s0[SC_BETA];
    const T* po = V.p[par][0];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T q = op.apply(0, C, P, [&](int64_t g) { return z[g] + bk * po[g]; });
        const T pn = z[P.g] + bk * po[P.g];
        V.p[par ^ 1][0][P.g] = pn;
        V.t[0][P.g] = q;
        acc[0] += (double)pn * (double)q;
    CLOT_END_CELLS
    store_partials<1>(acc, S.part, S.pstride, tile, lds);
}

// x += alpha p; r -= alpha q; rr; convergence (the next z comes from the V-cycle).
template <class T, class Op>
__global__ __launch_bounds__(NT) void k_mgcg_b(Grid G, Op op, KVec<T, 1> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5];
    double acc[1] = {0.0};
    const T a = (T)scp(S, chid, 0)[SC_ALPHA];
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        V.x[0][g] += a * V.p[par ^ 1][0][g];
        const T r = V.r[0][g] - a * V.t[0][g];
        V.r[0][g] = r;
        acc[0] += (double)r * (double)r;
    CLOT_END_CELLS
    store_partials<1>(acc, S.part, S.pstride, tile, lds);
}

struct EpiMgcgB {   // convergence of the MG-preconditioned CG
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        double* s = scp(S, ch, 0);
        if (s[SC_ACT] == 0.0) return;
        s[SC_RR] = sums[0];
        s[SC_IT] += 1.0;
        bool stop = false;
        if (s[SC_RR] <= s[SC_TOL2]) {
            s[SC_ACT] = 0.0;
            stop = true;
        } else if (s[SC_IT] >= S.maxit || !isfinite(s[SC_RR])) {
            s[SC_ACT] = 0.0;
            s[SC_FAIL] = 1.0;
            stop = true;
        }
        if (stop) {
            S.chact[ch] = 0;
            atomicSub(S.nact, 1);
        }
    }
};

}  // namespace clot
