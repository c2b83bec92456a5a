// Pressure multigrid legs in bricks (gfx950): the LDS-staged multi-sweep legs of the
// coarse levels (FP32 contexts), and, at the end of the file, the mesh's restriction and
// prolongation sweep for meshes that every channel coarsens along every axis (both
// precisions) and the mesh's legs in LDS-staged launches (FP32 contexts).
//
// Above the fused tail, each coarse level's legs are six separate launches (first two
// sweeps, the other sweeps, restriction; prolongation sweep, the other sweeps), each
// bound by launch latency rather than by its few thousand to a hundred thousand cells.
// A brick kernel does one whole leg of one level in one launch.  A 1024-thread block
// owns a brick of 1024 cells and stages the brick with an H-cell halo in LDS: the
// right-hand side, the level's diagonal and face coefficients and the leg's starting
// iterate.  It then runs the leg's H stencil stages from LDS; each stage covers a region
// one cell narrower than the one before, so the last covers exactly the own cells.  The
// halo cells are computed redundantly by the neighbouring bricks, with the expressions
// of the separate kernels, so every value is the same bit for bit.
//
//   DOWN: x1 = w D^-1 b (in the halo too), H-1 sweeps, then the residual b - A x_H of
//         the own cells summed over each 2x2(x2) aggregate (in the pairwise order of the
//         separate restriction) into the coarse right-hand side; x_H is stored for the
//         up leg.  H = sweeps each way.
//   UP:   x1 = x + P xc (injection), then H sweeps; the last is stored.
//
// A level is bricked only when every channel is coarsened along every axis there
// (aggregates never straddle bricks, whose origins are even).  On the mesh the whole
// leg loses: the staged arrays leave room for one block per CU and the three-cell halo
// triples the work, against separate launches that are already wide.  Only the mesh's
// legs are staged there with a two-cell halo and five arrays (k_mg_mesh_leg: the down
// leg's sweeps, with the restriction when there are two; the up leg's prolongation and
// the sweep after it).
#pragma once
#include "clot_mgm.h"

namespace clot {

enum { MGB_DOWN = 0, MGB_UP = 1 };
constexpr int MGB_BS = 1024;

// Brick shapes, chosen per leg by the tile autotuner (one shape index covers a 3-D and a
// 2-D shape; every dimension even, so aggregates never straddle bricks): 3-D 16x8x8,
// 32x8x4, 8x8x16, 16x16x4; 2-D 64x16, 128x8, 32x32, 256x4.
constexpr int MGB_NSHAPE = 4;
__host__ __device__ constexpr int pb_dim(int dim, int shape, int axis) {
    return dim == 3 ? (shape == 0 ? (axis == 0 ? 16 : 8)
                       : shape == 1 ? (axis == 0 ? 32 : axis == 1 ? 8 : 4)
                       : shape == 2 ? (axis == 2 ? 16 : 8)
                                    : (axis == 2 ? 4 : 16))
                    : (axis == 2 ? 1
                       : shape == 0 ? (axis == 0 ? 64 : 16)
                       : shape == 1 ? (axis == 0 ? 128 : 8)
                       : shape == 2 ? 32
                                    : (axis == 0 ? 256 : 4));
}
template <int DIM, int H, int SHAPE>
struct PBrick {
    static constexpr int BX = pb_dim(DIM, SHAPE, 0), BY = pb_dim(DIM, SHAPE, 1), BZ = pb_dim(DIM, SHAPE, 2);
    static constexpr int EX = BX + 2 * H, EY = BY + 2 * H, EZ = DIM == 3 ? BZ + 2 * H : 1;
    static constexpr int NE = EX * EY * EZ;
    static_assert(BX * BY * BZ == MGB_BS, "one own cell per thread");
    static_assert(BX % 2 == 0 && BY % 2 == 0 && (DIM == 2 || BZ % 2 == 0), "whole aggregates");
};
inline void pbrick_dims(int dim, int shape, int& bx, int& by, int& bz) {
    bx = pb_dim(dim, shape, 0);
    by = pb_dim(dim, shape, 1);
    bz = pb_dim(dim, shape, 2);
}
// LDS elements per array (the larger of the shape's 2-D and 3-D bricks) and the bytes
// of the seven arrays: b, the diagonal, two iterates, the three face-coefficient arrays.
__host__ __device__ constexpr int mgb_ne(int h, int shape) {
    return (pb_dim(3, shape, 0) + 2 * h) * (pb_dim(3, shape, 1) + 2 * h) * (pb_dim(3, shape, 2) + 2 * h) >
                   (pb_dim(2, shape, 0) + 2 * h) * (pb_dim(2, shape, 1) + 2 * h)
               ? (pb_dim(3, shape, 0) + 2 * h) * (pb_dim(3, shape, 1) + 2 * h) * (pb_dim(3, shape, 2) + 2 * h)
               : (pb_dim(2, shape, 0) + 2 * h) * (pb_dim(2, shape, 1) + 2 * h);
}
__host__ __device__ constexpr size_t mgb_lds_bytes(int h, int shape, size_t tsize) {
    return 7 * (size_t)mgb_ne(h, shape) * tsize;
}

template <class T, int MODE, int H, int SHAPE, int DIM>
__device__ inline void mgb_body(const ChanDev& C, const ChanDev& Cc, int bx, int by, int bz, const CoefOp<T>& op,
                                const T* b, const T* xin, const T* xc, T* xout, T* bc, T w, T* sm) {
    using D = PBrick<DIM, H, SHAPE>;
    constexpr int NE = mgb_ne(H, SHAPE);
    T* const sb = sm;
    T* const sd = sm + NE;
    T* s0 = sm + 2 * NE;
    T* s1 = sm + 3 * NE;
    T* const sa = sm + 4 * NE;     // cx
    T* const sy = sm + 5 * NE;     // cy
    T* const sz = sm + 6 * NE;     // cz
    const int ox = bx * D::BX - H, oy = by * D::BY - H, oz = DIM == 3 ? bz * D::BZ - H : 0;
    // 1. stage the brick and its halo; the leg's first iterate, pointwise
    for (int e = threadIdx.x; e < D::NE; e += MGB_BS) {
        const int ex = e % D::EX, ey = (e / D::EX) % D::EY, ez = DIM == 3 ? e / (D::EX * D::EY) : 0;
        const int gi = ox + ex, gj = oy + ey, gk = oz + ez;
        const bool in = gi >= 0 && gi < C.nx && gj >= 0 && gj < C.ny && gk >= 0 && gk < C.nz;
        T vb = T(0), vd = T(1), va = T(0), vy = T(0), vz = T(0), vx = T(0);
        if (in) {
            const int64_t g = C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk);
            vb = b[g];
            vd = op.dg[g];
            va = op.cx[fx_id(C, gi, gj, gk)];
            vy = op.cy[fy_id(C, gi, gj, gk)];
            if (DIM == 3) vz = op.cz[fz_id(C, gi, gj, gk)];
            if (MODE == MGB_DOWN)
                vx = w * vb / vd;
            else
                vx = xin[g] + xc[Cc.c0 + (gi >> 1) + (int64_t)Cc.nx * ((gj >> 1) + (int64_t)Cc.ny * (gk >> 1))];
        }
        sb[e] = vb;
        sd[e] = vd;
        sa[e] = va;
        sy[e] = vy;
        if (DIM == 3) sz[e] = vz;
        s0[e] = vx;
    }
    __syncthreads();
    // 2. the stencil stages, each on a region one cell narrower than the last
    constexpr int SY = D::EX, SZ = D::EX * D::EY;
#pragma unroll
    for (int s = 1; s <= H; ++s) {
        const int m = H - s;
        const int RX = D::BX + 2 * m, RY = D::BY + 2 * m, RZ = DIM == 3 ? D::BZ + 2 * m : 1;
        const int NR = RX * RY * RZ;
        const bool last = s == H;
        for (int q = threadIdx.x; q < NR; q += MGB_BS) {
            const int ex = q % RX + s, ey = (q / RX) % RY + s, ez = DIM == 3 ? q / (RX * RY) + s : 0;
            const int gi = ox + ex, gj = oy + ey, gk = oz + ez;
            if (gi < 0 || gi >= C.nx || gj < 0 || gj >= C.ny || gk < 0 || gk >= C.nz) continue;
            const int e = ex + SY * (ey + D::EY * ez);
            // CoefOp's stencil, in its order: x-, x+, y-, y+, z-, z+
            const T* x = s0;
            T sacc = T(0);
            if (gi > 0) sacc += sa[e] * x[e - 1];
            if (gi < C.nx - 1) sacc += sa[e + 1] * x[e + 1];
            if (gj > 0) sacc += sy[e] * x[e - SY];
            if (gj < C.ny - 1) sacc += sy[e + SY] * x[e + SY];
            if (DIM == 3) {
                if (gk > 0) sacc += sz[e] * x[e - SZ];
                if (gk < C.nz - 1) sacc += sz[e + SZ] * x[e + SZ];
            }
            const T ax = sd[e] * x[e] - sacc;
            if (MODE == MGB_DOWN && last) {
                s1[e] = sb[e] - ax;     // residual of the own cell
            } else {
                const T z = x[e] + w * (sb[e] - ax) / sd[e];
                s1[e] = z;
                if (last) xout[C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk)] = z;
            }
        }
        __syncthreads();
        if (!(MODE == MGB_DOWN && last)) {
            T* t = s0;
            s0 = s1;
            s1 = t;
        }
    }
    if (MODE == MGB_DOWN) {
        // s0: x_H, s1: the own cells' residuals.  The iterate for the up leg, then the
        // aggregate sums ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111)).
        {
            const int q = threadIdx.x;
            const int lx = q % D::BX, ly = (q / D::BX) % D::BY, lz = DIM == 3 ? q / (D::BX * D::BY) : 0;
            const int gi = ox + H + lx, gj = oy + H + ly, gk = oz + (DIM == 3 ? H : 0) + lz;
            if (gi < C.nx && gj < C.ny && gk < C.nz)
                xout[C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk)] =
                    s0[(lx + H) + SY * ((ly + H) + D::EY * (DIM == 3 ? lz + H : 0))];
        }
        constexpr int AX = D::BX / 2, AY = D::BY / 2, AZ = DIM == 3 ? D::BZ / 2 : 1;
        for (int a = threadIdx.x; a < AX * AY * AZ; a += MGB_BS) {
            const int ax = a % AX, ay = (a / AX) % AY, az = a / (AX * AY);
            T r[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int di = f & 1, dj = (f >> 1) & 1, dk = f >> 2;
                const int lx = 2 * ax + di, ly = 2 * ay + dj, lz = DIM == 3 ? 2 * az + dk : 0;
                const int gi = ox + H + lx, gj = oy + H + ly, gk = oz + (DIM == 3 ? H : 0) + lz;
                const bool in = (DIM == 3 || dk == 0) && gi < C.nx && gj < C.ny && gk < C.nz;
                r[f] = in ? s1[(lx + H) + SY * ((ly + H) + D::EY * (DIM == 3 ? lz + H : 0))] : T(0);
            }
            const T s01 = r[0] + r[1], s23 = r[2] + r[3], s45 = r[4] + r[5], s67 = r[6] + r[7];
            const int ci = (ox + H) / 2 + ax, cj = (oy + H) / 2 + ay, ck = DIM == 3 ? (oz + H) / 2 + az : 0;
            if (ci < Cc.nx && cj < Cc.ny && ck < Cc.nz)
                bc[Cc.c0 + ci + (int64_t)Cc.nx * (cj + (int64_t)Cc.ny * ck)] = (s01 + s23) + (s45 + s67);
        }
    }
}

template <class T, int MODE, int H, int SHAPE>
__global__ __launch_bounds__(MGB_BS) void k_mg_brick(BrickGrid BG, MGPair L, CoefOp<T> op, const T* b, const T* xin,
                                                     const T* xc, T* xout, T* bc, T w, const int32_t* chact) {
    const int32_t bk = xcd_tile((int32_t)blockIdx.x, BG.nb);
    const int32_t chid = BG.b2c[bk];
    if (!chact[chid]) return;
    const ChanDev C = L.fine.ch[chid];
    const ChanDev Cc = L.coarse.ch[chid];
    const BrickChan B = BG.bc[chid];
    const int lb = bk - B.b0;
    const int bx = lb % B.nbx, by = (lb / B.nbx) % B.nby, bz = lb / (B.nbx * B.nby);
    extern __shared__ __align__(16) unsigned char mgb_lds[];
    T* const sm = reinterpret_cast<T*>(mgb_lds);
    if (C.dim == 3)
        mgb_body<T, MODE, H, SHAPE, 3>(C, Cc, bx, by, bz, op, b, xin, xc, xout, bc, w, sm);
    else
        mgb_body<T, MODE, H, SHAPE, 2>(C, Cc, bx, by, bz, op, b, xin, xc, xout, bc, w, sm);
}

}  // namespace clot

// ---- The mesh's leg ends, for a mesh that every channel coarsens along every axis -----
namespace clot {

// Residual restriction of the mesh: r = b - A x at every mesh cell, summed over each
// 2x2(x2) aggregate into the coarse right-hand side.  The block walks a brick in the
// momentum bricks' shape 0 (3-D 32x8x4, 2-D 64x16), so its loads run along x rows: a
// thread's four cells are two aggregate pairs along the slow axis, the x partner is
// lane l^1 and, in 3-D, the y partner lane l^32.  The sums are those of k_mg_restrict in
// its order ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111)), the
// missing z half of a 2-D aggregate adding (0 + 0) + (0 + 0) as there.
template <class T, int DIM>
__device__ inline void mg_restrict_mesh_body(const ChanDev& C, const ChanDev& Cc, int bx, int by, int bz,
                                             const PresOp<T, T>& op, const T* b, const T* x, T* bc) {
    using D = Brick<DIM, 0>;
    const int x0 = bx * D::BX, y0 = by * D::BY, z0 = bz * D::BZ;
    const int t = threadIdx.x;
    T r[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        int lx, ly, lz;
        D::cell(t, m, lx, ly, lz);
        Cell P;
        P.i = x0 + lx;
        P.j = y0 + ly;
        P.k = z0 + lz;
        r[m] = T(0);
        if (P.i < C.nx && P.j < C.ny && P.k < C.nz) {
            P.g = C.c0 + P.i + (int64_t)C.nx * (P.j + (int64_t)C.ny * P.k);
            r[m] = b[P.g] - op.apply(0, C, P, [&](int64_t g) { return x[g]; });
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        T s;
        if (DIM == 3) {
            T a0 = r[2 * h], a1 = r[2 * h + 1];     // dk = 0, 1
            a0 += __shfl_xor(a0, 1, 64);
            a1 += __shfl_xor(a1, 1, 64);
            a0 += __shfl_xor(a0, 32, 64);
            a1 += __shfl_xor(a1, 32, 64);
            s = a0 + a1;
        } else {
            T a0 = r[2 * h], a1 = r[2 * h + 1];     // dj = 0, 1
            a0 += __shfl_xor(a0, 1, 64);
            a1 += __shfl_xor(a1, 1, 64);
            s = (a0 + a1) + (T(0) + T(0));
        }
        int lx, ly, lz;
        D::cell(t, 2 * h, lx, ly, lz);
        const int gi = x0 + lx, gj = y0 + ly, gk = z0 + lz;
        const bool lead = (lx & 1) == 0 && (DIM == 2 || (ly & 1) == 0);
        if (lead && gi < C.nx && gj < C.ny && gk < C.nz)
            bc[Cc.c0 + (gi >> 1) + (int64_t)Cc.nx * ((gj >> 1) + (int64_t)Cc.ny * (gk >> 1))] = s;
    }
}

template <class T>
__global__ __launch_bounds__(NT) void k_mg_restrict_mesh(BrickGrid BG, MGPair L, PresOp<T, T> op, const T* b,
                                                         const T* x, T* bc, const int32_t* chact) {
    const int32_t bk = xcd_tile((int32_t)blockIdx.x, BG.nb);
    const int32_t chid = BG.b2c[bk];
    if (!chact[chid]) return;
    const ChanDev C = L.fine.ch[chid];
    const ChanDev Cc = L.coarse.ch[chid];
    const BrickChan B = BG.bc[chid];
    const int lb = bk - B.b0;
    const int bx = lb % B.nbx, by = (lb / B.nbx) % B.nby, bz = lb / (B.nbx * B.nby);
    if (C.dim == 3)
        mg_restrict_mesh_body<T, 3>(C, Cc, bx, by, bz, op, b, x, bc);
    else
        mg_restrict_mesh_body<T, 2>(C, Cc, bx, by, bz, op, b, x, bc);
}

// Legs of the mesh's V-cycle in one launch each, in three forms:
//   MESH_DOWN3: three sweeps from zero (k_mg_pre's two and one k_mg_post2; the residual
//     restriction stays a launch of its own, since a third halo cell would cost more
//     than it saves);
//   MESH_DOWN2R: two sweeps from zero and the residual summed over each aggregate
//     (k_mg_pre and k_mg_restrict_mesh);
//   MESH_UP2: the prolonged iterate x + P xc and two sweeps (k_mg_post1_mesh and one
//     k_mg_post2; the last sweep, which also forms r.z, stays a launch of its own, so
//     that r.z is summed in the same order).
// The last two need a mesh that every channel coarsens along every axis.  A
// 1024-thread block stages a brick of shape 0 with a two-cell halo in LDS (rAU, the
// diagonal, b and two iterates; 58 KB in FP32 in 3-D, 27 KB in 2-D): the first iterate
// in the whole halo, pointwise (w D^-1 b, or x + P xc with the coarse cell by halving),
// the next on the brick and a one-cell ring, then the last (or the residual) on the
// brick.  PresOp's stencil in its order, each value the separate kernels' expression,
// the aggregate sums in the separate restriction's pairwise order.
enum { MESH_DOWN3 = 0, MESH_DOWN2R = 1, MESH_UP2 = 2 };
template <class T, int DIM, int MODE>
__device__ inline void mesh_leg_body(const ChanDev& C, const ChanDev& Cc, int bx, int by, int bz,
                                     const PresOp<T, T>& op, const T* b, const T* xin, const T* xc, T* xout, T* bc,
                                     T w, T* sm) {
    constexpr bool RESTRICT = MODE == MESH_DOWN2R;
    constexpr int H = 2;
    using D = PBrick<DIM, H, 0>;
    constexpr int NE = D::NE;
    T* const sb = sm;
    T* const sd = sm + NE;
    T* const sa = sm + 2 * NE;     // rAU
    T* s0 = sm + 3 * NE;
    T* s1 = sm + 4 * NE;
    const int ox = bx * D::BX - H, oy = by * D::BY - H, oz = DIM == 3 ? bz * D::BZ - H : 0;
    for (int e = threadIdx.x; e < D::NE; e += MGB_BS) {
        const int ex = e % D::EX, ey = (e / D::EX) % D::EY, ez = DIM == 3 ? e / (D::EX * D::EY) : 0;
        const int gi = ox + ex, gj = oy + ey, gk = oz + ez;
        const bool in = gi >= 0 && gi < C.nx && gj >= 0 && gj < C.ny && gk >= 0 && gk < C.nz;
        T vb = T(0), vd = T(1), va = T(0), vx = T(0);
        if (in) {
            const int64_t g = C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk);
            vb = b[g];
            vd = op.dP[g];
            va = op.rAU[g];
            if (MODE == MESH_UP2)
                vx = xin[g] + xc[Cc.c0 + (gi >> 1) + (int64_t)Cc.nx * ((gj >> 1) + (int64_t)Cc.ny * (gk >> 1))];
            else
                vx = w * vb / vd;
        }
        sb[e] = vb;
        sd[e] = vd;
        sa[e] = va;
        s0[e] = vx;
    }
    __syncthreads();
    constexpr int SY = D::EX, SZ = D::EX * D::EY;
    const T gxh = T(0.5 * C.gx), gyh = T(0.5 * C.gy), gzh = T(0.5 * C.gz);
#pragma unroll
    for (int s = 1; s <= H; ++s) {
        const int m = H - s;
        const bool resid = RESTRICT && s == H;
        const int RX = D::BX + 2 * m, RY = D::BY + 2 * m, RZ = DIM == 3 ? D::BZ + 2 * m : 1;
        const int NR = RX * RY * RZ;
        for (int q = threadIdx.x; q < NR; q += MGB_BS) {
            const int ex = q % RX + s, ey = (q / RX) % RY + s, ez = DIM == 3 ? q / (RX * RY) + s : 0;
            const int gi = ox + ex, gj = oy + ey, gk = oz + ez;
            if (gi < 0 || gi >= C.nx || gj < 0 || gj >= C.ny || gk < 0 || gk >= C.nz) continue;
            const int e = ex + SY * (ey + D::EY * ez);
            const T* x = s0;
            const T rP = sa[e];
            T sacc = T(0);
            if (gi > 0) sacc += gxh * (rP + sa[e - 1]) * x[e - 1];
            if (gi < C.nx - 1) sacc += gxh * (rP + sa[e + 1]) * x[e + 1];
            if (gj > 0) sacc += gyh * (rP + sa[e - SY]) * x[e - SY];
            if (gj < C.ny - 1) sacc += gyh * (rP + sa[e + SY]) * x[e + SY];
            if (DIM == 3) {
                if (gk > 0) sacc += gzh * (rP + sa[e - SZ]) * x[e - SZ];
                if (gk < C.nz - 1) sacc += gzh * (rP + sa[e + SZ]) * x[e + SZ];
            }
            const T ax = sd[e] * x[e] - sacc;
            if (resid) {
                s1[e] = sb[e] - ax;
            } else {
                const T z = x[e] + w * (sb[e] - ax) / sd[e];
                s1[e] = z;
                if (s == H) xout[C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk)] = z;
            }
        }
        __syncthreads();
        if (!resid) {
            T* t = s0;
            s0 = s1;
            s1 = t;
        }
    }
    if (RESTRICT) {
        // s0: x2, s1: the own cells' residuals.  x2 for the up leg, then the aggregate
        // sums ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111)).
        {
            const int q = threadIdx.x;
            const int lx = q % D::BX, ly = (q / D::BX) % D::BY, lz = DIM == 3 ? q / (D::BX * D::BY) : 0;
            const int gi = ox + H + lx, gj = oy + H + ly, gk = oz + (DIM == 3 ? H : 0) + lz;
            if (gi < C.nx && gj < C.ny && gk < C.nz)
                xout[C.c0 + gi + (int64_t)C.nx * (gj + (int64_t)C.ny * gk)] =
                    s0[(lx + H) + SY * ((ly + H) + D::EY * (DIM == 3 ? lz + H : 0))];
        }
        constexpr int AX = D::BX / 2, AY = D::BY / 2, AZ = DIM == 3 ? D::BZ / 2 : 1;
        for (int a = threadIdx.x; a < AX * AY * AZ; a += MGB_BS) {
            const int ax = a % AX, ay = (a / AX) % AY, az = a / (AX * AY);
            T r[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int di = f & 1, dj = (f >> 1) & 1, dk = f >> 2;
                const int lx = 2 * ax + di, ly = 2 * ay + dj, lz = DIM == 3 ? 2 * az + dk : 0;
                const int gi = ox + H + lx, gj = oy + H + ly, gk = oz + (DIM == 3 ? H : 0) + lz;
                const bool in = (DIM == 3 || dk == 0) && gi < C.nx && gj < C.ny && gk < C.nz;
                r[f] = in ? s1[(lx + H) + SY * ((ly + H) + D::EY * (DIM == 3 ? lz + H : 0))] : T(0);
            }
            const T s01 = r[0] + r[1], s23 = r[2] + r[3], s45 = r[4] + r[5], s67 = r[6] + r[7];
            const int ci = (ox + H) / 2 + ax, cj = (oy + H) / 2 + ay, ck = DIM == 3 ? (oz + H) / 2 + az : 0;
            if (ci < Cc.nx && cj < Cc.ny && ck < Cc.nz)
                bc[Cc.c0 + ci + (int64_t)Cc.nx * (cj + (int64_t)Cc.ny * ck)] = (s01 + s23) + (s45 + s67);
        }
    }
}

template <class T, int MODE>
__global__ __launch_bounds__(MGB_BS) void k_mg_mesh_leg(BrickGrid BG, MGPair L, PresOp<T, T> op, const T* b,
                                                        const T* xin, const T* xc, T* xout, T* bc, T w,
                                                        const int32_t* chact) {
    const int32_t bk = xcd_tile((int32_t)blockIdx.x, BG.nb);
    const int32_t chid = BG.b2c[bk];
    if (!chact[chid]) return;
    const ChanDev C = L.fine.ch[chid];
    const ChanDev Cc = MODE == MESH_DOWN3 ? C : L.coarse.ch[chid];
    const BrickChan B = BG.bc[chid];
    const int lb = bk - B.b0;
    const int bx = lb % B.nbx, by = (lb / B.nbx) % B.nby, bz = lb / (B.nbx * B.nby);
    extern __shared__ __align__(16) unsigned char mgb_lds[];
    T* const sm = reinterpret_cast<T*>(mgb_lds);
    if (C.dim == 3)
        mesh_leg_body<T, 3, MODE>(C, Cc, bx, by, bz, op, b, xin, xc, xout, bc, w, sm);
    else
        mesh_leg_body<T, 2, MODE>(C, Cc, bx, by, bz, op, b, xin, xc, xout, bc, w, sm);
}
// dynamic LDS of k_mg_mesh_leg: five arrays of the larger brick among the dimensions present
constexpr size_t mesh_leg_lds_bytes(bool any3d, size_t tsize) {
    return 5 * (size_t)(any3d ? PBrick<3, 2, 0>::NE : PBrick<2, 2, 0>::NE) * tsize;
}

// Prolongation and the first up sweep on the mesh: x1 = x + P xc, y = x1 + w D^-1 (b -
// A x1).  k_mg_post1's expressions (PresOp's stencil in its order), with each
// neighbour's coarse cell taken from its indices by halving instead of by division.
template <class T>
__global__ __launch_bounds__(NT) void k_mg_post1_mesh(MGPair L, PresOp<T, T> op, const T* b, const T* x, const T* xc,
                                                      T* y, T w, const int32_t* chact) {
    CLOT_TILE_PROLOGUE(L.fine)
    if (!chact[chid]) return;
    const ChanDev Cc = L.coarse.ch[chid];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto x1 = [&](int64_t g, int i, int j, int k) {
            return x[g] + xc[Cc.c0 + (i >> 1) + (int64_t)Cc.nx * ((j >> 1) + (int64_t)Cc.ny * (k >> 1))];
        };
        const T* rAU = op.rAU;
        const T rP = rAU[P.g];
        T s = T(0);
        T gf = T(0.5 * C.gx);
        if (P.i > 0) s += gf * (rP + rAU[P.g - 1]) * x1(P.g - 1, P.i - 1, P.j, P.k);
        if (P.i < C.nx - 1) s += gf * (rP + rAU[P.g + 1]) * x1(P.g + 1, P.i + 1, P.j, P.k);
        gf = T(0.5 * C.gy);
        if (P.j > 0) s += gf * (rP + rAU[P.g - C.nx]) * x1(P.g - C.nx, P.i, P.j - 1, P.k);
        if (P.j < C.ny - 1) s += gf * (rP + rAU[P.g + C.nx]) * x1(P.g + C.nx, P.i, P.j + 1, P.k);
        if (C.dim == 3) {
            const int64_t sz = (int64_t)C.nx * C.ny;
            gf = T(0.5 * C.gz);
            if (P.k > 0) s += gf * (rP + rAU[P.g - sz]) * x1(P.g - sz, P.i, P.j, P.k - 1);
            if (P.k < C.nz - 1) s += gf * (rP + rAU[P.g + sz]) * x1(P.g + sz, P.i, P.j, P.k + 1);
        }
        const T xp = x1(P.g, P.i, P.j, P.k);
        const T ax = op.dP[P.g] * xp - s;
        y[P.g] = xp + w * (b[P.g] - ax) / op.dP[P.g];
    CLOT_END_CELLS
}

}  // namespace clot
