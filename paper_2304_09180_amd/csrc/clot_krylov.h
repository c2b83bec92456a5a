// Batched, per-channel Krylov solvers as phase kernels (gfx950).
//
// K independent systems per channel share one launch.  Every dot product is an
// FP64 per-tile partial; a small finishing launch (one block per channel) adds a
// channel's partials in tile order and runs the scalar epilogue of the phase:
// the recurrence scalars (alpha, beta, omega) and the convergence decision stay on
// the device and the host never reads a scalar to continue.  A channel whose
// systems have all converged stops doing work (its blocks return at entry) and
// decrements the global active count that the host polls between chunks.
//
// Jacobi-preconditioned CG (SPD: eta) and BiCGStab (momentum, transport).  The
// preconditioned direction vectors are formed on the fly from r, p and v at each
// stencil point, so each iteration costs two (CG) or three (BiCGStab) passes.
#pragma once
#include "clot_ops.h"

#include <type_traits>
#include <utility>

namespace clot {

// Per (channel, system) scalar slots.
enum {
    SC_BB = 0, SC_RR, SC_RZ, SC_RHO, SC_ALPHA, SC_OMEGA, SC_BETA, SC_IT, SC_ACT, SC_TOL2, SC_RR0, SC_PQ,
    SC_TS, SC_TT, SC_FAIL, SC_PASS,
    SC_ORR, SC_OBB, SC_ORRP,  // pressure refinement: outer r.r, b.b, r.r of the previous pass
    SC_BBS                    // squared norm the reported relative residual is taken against
};

struct KState {
    double* sc;          // [nch][MAXK][NSC]
    int32_t* chact;      // [nch] 1 while any system of the channel iterates
    int32_t* nact;       // global count of active channels
    double* part;        // [ntiles][NV]
    uint32_t* tick;      // [nch] arrival tickets of a split finishing launch (0 between launches)
    double* fin;         // [nch][FIN_MAXNV] its per-component totals
    int32_t* nanflag;    // set to 1 when a NaN or infinity reaches any reduction
    int32_t maxit;
    int32_t sc_ch0;      // channel whose slots sc starts at (0: the whole table)
    int32_t pstride;     // partials: part[q*pstride + tile]
};

__device__ inline double* scp(const KState& S, int ch, int k) {
    return S.sc + ((int64_t)(ch - S.sc_ch0) * MAXK + k) * NSC;
}

template <class T, int K>
struct KVec {
    T* x[K];
    const T* b[K];
    T* r[K];
    T* rh[K];
    T* p[2][K];
    T* v[2][K];
    T* t[K];
};

#define CLOT_TILE_PROLOGUE(G)                                     \
    const int32_t tile = xcd_tile((int32_t)blockIdx.x, G.ntiles); \
    const int32_t chid = G.t2c[tile];                             \
    const ChanDev C = G.ch[chid];                                 \
    const int64_t tbase = (int64_t)(tile - C.t0) * TILE;

#define CLOT_FOR_CELLS(local)                                        \
    for (int q_ = 0; q_ < CPT; ++q_) {                               \
        const int64_t local = tbase + (int64_t)q_ * NT + threadIdx.x; \
        if (local >= C.ncell) break;

#define CLOT_END_CELLS }

// Epilogue traits.  An initialising epilogue (static member kInit) admits a channel to
// the solve and adds it to the active count; in every later phase the channel is
// already counted.  An epilogue with a refmask member also keeps the channel in a
// further refinement pass.
template <class E, class = void>
struct epi_is_init : std::false_type {};
template <class E>
struct epi_is_init<E, std::void_t<decltype(E::kInit)>> : std::true_type {};
// An operator with kExactResidual forms the starting residual itself, in FP64.
template <class O, class = void>
struct op_exact_residual : std::false_type {};
template <class O>
struct op_exact_residual<O, std::void_t<decltype(O::kExactResidual)>> : std::true_type {};
template <class E, class = void>
struct epi_has_refmask : std::false_type {};
template <class E>
struct epi_has_refmask<E, std::void_t<decltype(std::declval<E>().refmask)>> : std::true_type {};

// Sums the tile partials of each active channel (fixed order) and runs the phase
// epilogue in thread 0.  1024-thread blocks, blockIdx.x the channel.  A reduction of
// more than three values is spread over several blocks per channel (blockIdx.y, two
// components each: one CU's read rate bounds a block, 14 values took 13.9 us in one):
// each block writes its totals, and the last to arrive (a ticket per channel; the
// fence costs little here, the kernel writing only those totals) runs the epilogue on
// all of them.  Each component is summed in the same order either way (a thread's
// tiles in increasing order, then the block's waves), so the totals are the same.
constexpr int FIN_BS = 1024;
constexpr int FIN_MAXNV = 32;
template <int NV>
struct FinSplit {
    static constexpr int CPG = NV <= 3 ? NV : 2;            // components per block
    static constexpr int G = (NV + CPG - 1) / CPG;          // blocks per channel
};

// The epilogue of one channel in thread 0, on its scalar slots staged in LDS (scl), or,
// when a NaN or infinity reached the sums, the channel's failure.
template <int NV, class Epi>
__device__ inline void finish_epilogue(const KState& S, const Epi& epi, int chid, const double (&acc)[NV],
                                       double* scl) {
    KState SL = S;
    SL.sc = scl;
    SL.sc_ch0 = chid;
    bool finite = true;
#pragma unroll
    for (int q = 0; q < NV; ++q) finite = finite && isfinite(acc[q]);
    if (finite) {
        epi(acc, SL, chid);
    } else {
        // a NaN or infinity reached the reductions: the channel's systems stop,
        // marked failed (2), and the channel leaves the solve (and the active
        // count, unless this phase would have admitted it) and any further
        // refinement pass
        for (int k = 0; k < MAXK; ++k) {
            double* s = scp(SL, chid, k);
            s[SC_FAIL] = 2.0;
            s[SC_ACT] = 0.0;
        }
        S.chact[chid] = 0;
        if (!epi_is_init<Epi>::value) atomicSub(S.nact, 1);
        if constexpr (epi_has_refmask<Epi>::value) epi.refmask[chid] = 0;
        if (S.nanflag) S.nanflag[0] = 1;
    }
}

template <int NV, class Epi>
__global__ __launch_bounds__(FIN_BS) void k_finish(const ChanDev* chans, KState S, Epi epi) {
    using FS = FinSplit<NV>;
    constexpr int CPG = FS::CPG;
    const int chid = blockIdx.x;
    if (!S.chact[chid]) return;
    const int32_t t0 = chans[chid].t0, nt = chans[chid].nt;
    const int q0 = FS::G > 1 ? (int)blockIdx.y * CPG : 0;
    __shared__ double lds[CPG * (FIN_BS / 64 + 1)];
    // the channel's scalar slots, staged in LDS by all threads so that the epilogue
    // (one thread, system after system) does not wait on memory for each of them
    __shared__ double scl[MAXK * NSC];
    double* scg = S.sc + (int64_t)chid * MAXK * NSC;
    if (FS::G == 1)
        for (int q = threadIdx.x; q < MAXK * NSC; q += FIN_BS) scl[q] = scg[q];
    double acc[CPG];
#pragma unroll
    for (int q = 0; q < CPG; ++q) acc[q] = 0.0;
    // U tiles per thread in flight at once
    constexpr int U = 4;
    for (int tb = threadIdx.x; tb < nt; tb += U * FIN_BS) {
        double v[U][CPG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = tb + u * FIN_BS;
#pragma unroll
            for (int q = 0; q < CPG; ++q)
                v[u][q] = (t < nt && q0 + q < NV) ? S.part[(int64_t)(q0 + q) * S.pstride + t0 + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < CPG; ++q) acc[q] += v[u][q];
    }
    block_sum<CPG, FIN_BS>(acc, lds);   // its barriers also publish scl
    if (FS::G == 1) {
        if (threadIdx.x == 0) {
            double all[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) all[q] = acc[q];
            finish_epilogue<NV>(S, epi, chid, all, scl);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < MAXK * NSC; q += FIN_BS) scg[q] = scl[q];
        return;
    }
    __shared__ int last;
    if (threadIdx.x == 0) {
        double* tot = S.fin + (int64_t)chid * FIN_MAXNV;
#pragma unroll
        for (int q = 0; q < CPG; ++q)
            if (q0 + q < NV) tot[q0 + q] = acc[q];
        __threadfence();
        const unsigned tk = atomicAdd(&S.tick[chid], 1u);
        last = tk == (unsigned)(FS::G - 1);
        if (last) {
            S.tick[chid] = 0u;
            __threadfence();
        }
    }
    __syncthreads();
    if (!last) return;
    for (int q = threadIdx.x; q < MAXK * NSC; q += FIN_BS) scl[q] = scg[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        const double* tot = S.fin + (int64_t)chid * FIN_MAXNV;
        double all[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) all[q] = __hip_atomic_load(tot + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        finish_epilogue<NV>(S, epi, chid, all, scl);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < MAXK * NSC; q += FIN_BS) scg[q] = scl[q];
}

// ---- epilogues ---------------------------------------------------------------------
// tol_mode 0: tolerance rtol^2 ||b||^2; 1: tolerance already in SC_TOL2.
template <int K>
struct EpiCgInit {
    static constexpr bool kInit = true;
    double rtol;
    int tol_mode;
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        int any = 0;
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            s[SC_RZ] = sums[3 * k];
            s[SC_BB] = sums[3 * k + 1];
            s[SC_BBS] = sums[3 * k + 1];
            s[SC_RR] = sums[3 * k + 2];
            s[SC_RR0] = sums[3 * k + 2];
            if (tol_mode == 0) s[SC_TOL2] = rtol * rtol * sums[3 * k + 1];
            s[SC_BETA] = 0.0;
            s[SC_IT] = 0.0;
            s[SC_FAIL] = 0.0;
            const bool act = s[SC_BB] > 0.0 && s[SC_RR] > s[SC_TOL2];
            s[SC_ACT] = act ? 1.0 : 0.0;
            any |= act;
        }
        S.chact[ch] = any;
        if (any) atomicAdd(S.nact, 1);
    }
};

template <int K>
struct EpiCgA {   // alpha = rz / (p.q)
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            if (s[SC_ACT] == 0.0) continue;
            s[SC_PQ] = sums[k];
            if (!(sums[k] > 0.0) || !isfinite(sums[k])) {
                s[SC_ALPHA] = 0.0;
                s[SC_ACT] = 0.0;
                s[SC_FAIL] = 1.0;
            } else {
                s[SC_ALPHA] = s[SC_RZ] / sums[k];
            }
        }
    }
};

template <int K>
struct EpiCgB {   // beta, convergence
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        int any = 0;
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            if (s[SC_ACT] != 0.0) {
                const double rz = sums[2 * k];
                s[SC_BETA] = s[SC_RZ] != 0.0 ? rz / s[SC_RZ] : 0.0;
                s[SC_RZ] = rz;
                s[SC_RR] = sums[2 * k + 1];
                s[SC_IT] += 1.0;
                if (s[SC_RR] <= s[SC_TOL2]) s[SC_ACT] = 0.0;
                else if (s[SC_IT] >= S.maxit || !isfinite(s[SC_RR])) {
                    s[SC_ACT] = 0.0;
                    s[SC_FAIL] = 1.0;
                }
            }
            any |= s[SC_ACT] != 0.0;
        }
        if (!any) {
            S.chact[ch] = 0;
            atomicSub(S.nact, 1);
        }
    }
};

// Tolerance: |r|^2 <= max(rtol^2 |b|^2, floor).  In FP32 the floor is what a change
// of 1e-30 of the field's scale in every cell would leave (sum of (1e-30 s d_ii)^2,
// and at least 1e-34 per cell): a species not yet produced (1e-33 of its scale, say)
// has nothing to converge at that level, and its iterates would otherwise reach the
// FP32 denormal range, where BiCGStab's recurrences break down.  Real but small fields
// (an enzyme at 1e-8 of its scale) lie far above it.  FP64 has no floor.
template <int K>
struct EpiBicgInit {
    static constexpr bool kInit = true;
    double rtol;
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        int any = 0;
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            s[SC_BB] = sums[3 * k];
            s[SC_RR] = sums[3 * k + 1];
            s[SC_RR0] = sums[3 * k + 1];
            s[SC_RHO] = sums[3 * k + 1];       // rhat . r with rhat = r
            const double rel2 = rtol * rtol * sums[3 * k];
            s[SC_TOL2] = rel2 > sums[3 * k + 2] ? rel2 : sums[3 * k + 2];
            // a floored system reports its residual against the norm its floor stands for
            s[SC_BBS] = (rel2 >= sums[3 * k + 2] || rtol <= 0.0) ? sums[3 * k] : sums[3 * k + 2] / (rtol * rtol);
            s[SC_ALPHA] = 1.0;
            s[SC_OMEGA] = 1.0;
            s[SC_BETA] = 0.0;
            s[SC_IT] = 0.0;
            s[SC_FAIL] = 0.0;
            const bool act = s[SC_BB] > 0.0 && s[SC_RR] > s[SC_TOL2];
            s[SC_ACT] = act ? 1.0 : 0.0;
            any |= act;
        }
        S.chact[ch] = any;
        if (any) atomicAdd(S.nact, 1);
    }
};

template <int K>
struct EpiBicg1 {   // alpha = rho / (rhat . v)
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            if (s[SC_ACT] == 0.0) continue;
            if (sums[k] == 0.0 || !isfinite(sums[k])) {
                s[SC_ACT] = 0.0;
                s[SC_FAIL] = 1.0;
                s[SC_ALPHA] = 0.0;
            } else {
                s[SC_ALPHA] = s[SC_RHO] / sums[k];
            }
        }
    }
};

template <int K>
struct EpiBicg2 {   // omega = (t.s)/(t.t)
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            if (s[SC_ACT] == 0.0) continue;
            s[SC_TS] = sums[2 * k];
            s[SC_TT] = sums[2 * k + 1];
            s[SC_OMEGA] = sums[2 * k + 1] > 0.0 ? sums[2 * k] / sums[2 * k + 1] : 0.0;
        }
    }
};

template <int K>
struct EpiBicg3 {   // rho_new, beta, convergence
    __device__ void operator()(const double* sums, const KState& S, int ch) const {
        int any = 0;
        for (int k = 0; k < K; ++k) {
            double* s = scp(S, ch, k);
            if (s[SC_ACT] != 0.0) {
                const double rho = sums[2 * k];
                s[SC_RR] = sums[2 * k + 1];
                s[SC_IT] += 1.0;
                const double om = s[SC_OMEGA];
                if (s[SC_RR] <= s[SC_TOL2]) {
                    s[SC_ACT] = 0.0;
                } else if (s[SC_IT] >= S.maxit || !isfinite(s[SC_RR]) || om == 0.0 || rho == 0.0) {
                    s[SC_ACT] = 0.0;
                    s[SC_FAIL] = 1.0;
                } else {
                    s[SC_BETA] = (rho / s[SC_RHO]) * (s[SC_ALPHA] / om);
                    s[SC_RHO] = rho;
                }
            }
            any |= s[SC_ACT] != 0.0;
        }
        if (!any) {
            S.chact[ch] = 0;
            atomicSub(S.nact, 1);
        }
    }
};

// ---- Jacobi PCG ---------------------------------------------------------------------
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_cg_init(Grid G, Op op, KVec<T, K> V, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5 * 3 * K];
    double acc[3 * K];
#pragma unroll
    for (int q = 0; q < 3 * K; ++q) acc[q] = 0.0;
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T* x = V.x[k];
            const T ax = op.apply(k, C, P, [&](int64_t g) { return x[g]; });
            const T b = V.b[k][P.g];
            const T r = b - ax;
            const T z = r / op.diag(k, P.g);
            V.r[k][P.g] = r;
            V.p[0][k][P.g] = z;
            acc[3 * k + 0] += (double)r * (double)z;
            acc[3 * k + 1] += (double)b * (double)b;
            acc[3 * k + 2] += (double)r * (double)r;
        }
    CLOT_END_CELLS
    store_partials<3 * K>(acc, S.part, S.pstride, tile, lds);
}

// q = A p_new with p_new = z + beta p_old formed on the fly.
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_cg_a(Grid G, Op op, KVec<T, K> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5 * K];
    double acc[K];
    double beta[K];
    bool act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0;
        const double* s = scp(S, chid, k);
        beta[k] = s[SC_BETA];
        act[k] = s[SC_ACT] != 0.0;
    }
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!act[k]) continue;
            const T* r = V.r[k];
            const T* po = V.p[par][k];
            const T bk = (T)beta[k];
            const T q = op.apply(k, C, P, [&](int64_t g) { return r[g] / op.diag(k, g) + bk * po[g]; });
            const T pn = r[P.g] / op.diag(k, P.g) + bk * po[P.g];
            V.p[par ^ 1][k][P.g] = pn;
            V.t[k][P.g] = q;
            acc[k] += (double)pn * (double)q;
        }
    CLOT_END_CELLS
    store_partials<K>(acc, S.part, S.pstride, tile, lds);
}

// x += alpha p; r -= alpha q; r.z and r.r.
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_cg_b(Grid G, Op op, KVec<T, K> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    __shared__ double lds[5 * 2 * K];
    double acc[2 * K];
    double alpha[K];
    bool act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[2 * k] = acc[2 * k + 1] = 0.0;
        const double* s = scp(S, chid, k);
        alpha[k] = s[SC_ALPHA];
        act[k] = s[SC_ACT] != 0.0;
    }
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!act[k]) continue;
            const T a = (T)alpha[k];
            V.x[k][g] += a * V.p[par ^ 1][k][g];
            const T r = V.r[k][g] - a * V.t[k][g];
            V.r[k][g] = r;
            const T z = r / op.diag(k, g);
            acc[2 * k] += (double)r * (double)z;
            acc[2 * k + 1] += (double)r * (double)r;
        }
    CLOT_END_CELLS
    store_partials<2 * K>(acc, S.part, S.pstride, tile, lds);
}

// ---- BiCGStab ----------------------------------------------------------------------
// With the Jacobi preconditioner D (k_bicg_1/2/3) the solve keeps the preconditioned
// vectors instead of dividing at every stencil point: V.r holds z = D^-1 r, V.p the
// preconditioned direction D^-1 p and V.v the scaled product D^-1 v, with
//   D^-1 p' = z + beta (D^-1 p - omega D^-1 v),  v' = A (D^-1 p'),
//   D^-1 s  = z - alpha D^-1 v',                   s = D (D^-1 s),  t = A (D^-1 s),
//   x += alpha D^-1 p' + omega D^-1 s,             r = s - omega t,  z = D^-1 r:
// right-preconditioned BiCGStab with one division per cell and phase.  V.rh holds the
// unscaled shadow residual, and every reduction takes the unscaled vectors.  SCALED
// selects that form of the start (z in V.r); without it V.r holds r (the multigrid-
// preconditioned momentum solve).
// One system per grid row: blockIdx.y is the system k, so a thread's loads are those
// of one system and a converged system's blocks only zero their partials.  The
// partials of system k are components NV k .. NV k + NV - 1 of the phase's sums.
template <int NV>
__device__ inline void store_partials_at(double (&v)[NV], const KState& S, int32_t tile, int q0, double* lds) {
    block_sum<NV>(v, lds);
#pragma unroll
    for (int q = 0; q < NV; ++q)
        if (threadIdx.x == q) S.part[(int64_t)(q0 + q) * S.pstride + tile] = v[q];
}
template <int NV>
__device__ inline void zero_partials_at(const KState& S, int32_t tile, int q0) {
    if (threadIdx.x < NV) S.part[(int64_t)(q0 + threadIdx.x) * S.pstride + tile] = 0.0;
}

template <class T, int K, class Op, bool SCALED = false>
__global__ __launch_bounds__(NT) void k_bicg_init(Grid G, Op op, KVec<T, K> V, KState S) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    __shared__ double lds[5 * 3];
    double acc[3] = {0.0, 0.0, 0.0};
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        const T* x = V.x[k];
        double bd;
        T r;
        if constexpr (op_exact_residual<Op>::value) {
            // delta form: the unknown is the change, starting at zero
            r = T(op.residual64(k, C, P, bd));
            V.x[k][P.g] = T(0);
        } else {
            const T ax = op.apply(k, C, P, [&](int64_t g) { return x[g]; });
            const T b = V.b[k][P.g];
            bd = (double)b;
            r = b - ax;
        }
        V.r[k][P.g] = SCALED ? r / op.diag(k, P.g) : r;
        V.rh[k][P.g] = r;
        V.p[0][k][P.g] = T(0);
        V.v[0][k][P.g] = T(0);
        acc[0] += bd * bd;
        acc[1] += (double)r * (double)r;
        // FP32: 1e-30 of the scale, and no residual below 1e-34 (the normal range
        // ends at 1.2e-38); FP64: no floor
        double f = 0.0;
        if (sizeof(T) == 4) {
            f = 1e-30 * (double)op.floor_scale(k) * (double)op.diag(k, P.g);
            f = f > 1e-34 ? f : 1e-34;
        }
        acc[2] += f * f;
    CLOT_END_CELLS
    store_partials_at<3>(acc, S, tile, 3 * k, lds);
}

// D^-1 p_new = z + beta (D^-1 p_old - omega D^-1 v_old); v_new = A D^-1 p_new;
// stores D^-1 p_new and D^-1 v_new; rhat.v_new
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_bicg_1(Grid G, Op op, KVec<T, K> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    const double* sk = scp(S, chid, k);
    if (sk[SC_ACT] == 0.0) {
        zero_partials_at<1>(S, tile, k);
        return;
    }
    __shared__ double lds[5];
    double acc[1] = {0.0};
    const T bk = (T)sk[SC_BETA], om = (T)sk[SC_OMEGA];
    const T* z = V.r[k];
    const T* po = V.p[par][k];
    const T* wo = V.v[par][k];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto pn = [&](int64_t g) { return z[g] + bk * (po[g] - om * wo[g]); };
        const T vn = op.apply(k, C, P, pn);
        V.p[par ^ 1][k][P.g] = pn(P.g);
        V.v[par ^ 1][k][P.g] = vn / op.diag(k, P.g);
        acc[0] += (double)V.rh[k][P.g] * (double)vn;
    CLOT_END_CELLS
    store_partials_at<1>(acc, S, tile, k, lds);
}

// D^-1 s = z - alpha D^-1 v; t = A D^-1 s; t.s, t.t with s = D (D^-1 s)
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_bicg_2(Grid G, Op op, KVec<T, K> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    const double* sk = scp(S, chid, k);
    if (sk[SC_ACT] == 0.0) {
        zero_partials_at<2>(S, tile, 2 * k);
        return;
    }
    __shared__ double lds[5 * 2];
    double acc[2] = {0.0, 0.0};
    const T a = (T)sk[SC_ALPHA];
    const T* z = V.r[k];
    const T* wn = V.v[par ^ 1][k];
    CLOT_FOR_CELLS(local)
        const Cell P = cell_at(C, local);
        auto sh = [&](int64_t g) { return z[g] - a * wn[g]; };
        const T t = op.apply(k, C, P, sh);
        const T sv = op.diag(k, P.g) * sh(P.g);
        V.t[k][P.g] = t;
        acc[0] += (double)t * (double)sv;
        acc[1] += (double)t * (double)t;
    CLOT_END_CELLS
    store_partials_at<2>(acc, S, tile, 2 * k, lds);
}

// x += alpha D^-1 p + omega D^-1 s; r = s - omega t; z = D^-1 r; rhat.r, r.r
template <class T, int K, class Op>
__global__ __launch_bounds__(NT) void k_bicg_3(Grid G, Op op, KVec<T, K> V, KState S, int par) {
    CLOT_TILE_PROLOGUE(G)
    if (!S.chact[chid]) return;
    const int k = (int)blockIdx.y;
    const double* sk = scp(S, chid, k);
    if (sk[SC_ACT] == 0.0) {
        zero_partials_at<2>(S, tile, 2 * k);
        return;
    }
    __shared__ double lds[5 * 2];
    double acc[2] = {0.0, 0.0};
    const T a = (T)sk[SC_ALPHA], om = (T)sk[SC_OMEGA];
    CLOT_FOR_CELLS(local)
        const int64_t g = C.c0 + local;
        const T d = op.diag(k, g);
        const T sh = V.r[k][g] - a * V.v[par ^ 1][k][g];
        V.x[k][g] += a * V.p[par ^ 1][k][g] + om * sh;
        const T r = d * sh - om * V.t[k][g];
        V.r[k][g] = r / d;
        acc[0] += (double)V.rh[k][g] * (double)r;
        acc[1] += (double)r * (double)r;
    CLOT_END_CELLS
    store_partials_at<2>(acc, S, tile, 2 * k, lds);
}

}  // namespace clot
