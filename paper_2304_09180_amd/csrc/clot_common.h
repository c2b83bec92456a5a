// Shared device-side definitions of the clotting-step library (gfx950).
//
// Layout: every channel's cells are contiguous in the global SoA arrays, x fastest
// (cell id i + nx*(j + ny*k)).  All launches run over a flattened tile space: a
// tile is TILE consecutive cells of one channel; a 256-thread block owns one tile.
// Blocks are remapped so that consecutive tiles run on the same XCD (the hardware
// deals blocks round-robin over the 8 XCDs, each with its own L2), which keeps the
// j±1 and k±1 stencil rows of a tile in the L2 that has just read them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clot {

constexpr int NT = 256;           // threads per block (4 wavefronts of 64)
#ifndef CLOT_CPT
#define CLOT_CPT 1
#endif
constexpr int CPT = CLOT_CPT;     // cells per thread (a build option: 1, 2 or 4)
constexpr int TILE = NT * CPT;    // cells per tile
constexpr int NXCD = 8;
#ifdef CLOT_INHIBITOR
// The extensibility example (section 3.4): an inhibitor I that binds thrombin for good,
// I + E2 -> E2i; both new species follow the 15, are transported and react.
constexpr int NSPC = 17;          // cell species
constexpr int NTR = 9;            // transported species
constexpr int NRX = 16;           // reacting species
constexpr int MAXK = 9;           // max systems in one batched Krylov solve
#else
constexpr int NSPC = 15;          // cell species
constexpr int NTR = 7;            // transported species
constexpr int NRX = 14;           // reacting species
constexpr int MAXK = 8;           // max systems in one batched Krylov solve
#endif
constexpr int NSPC_DRAWN = 15;    // species with initial-noise draws (the added ones have none)
constexpr int NHIST = 25;         // release-history nodes (tau_f/dtau + 1)
constexpr int NSC = 64;           // per-channel scalar slots

// Cell species slots (library field order).
enum { PMU = 0, PMA, PBA, PBSE, ADP, S1, S2, E1, E2, S1B, S2B, E1B, E2B, C1, C2, INH, E2I };
// Transported species, solve order (the inhibitor variant adds I and E2i last).
__host__ __device__ constexpr int tr_species(int k) {
    return k == 0 ? PMU : k == 1 ? PMA : k == 2 ? S1 : k == 3 ? S2 : k == 4 ? E1 : k == 5 ? E2 : k == 6 ? ADP
         : k == 7 ? INH : E2I;
}

struct ChanDev {
    int32_t dim, nx, ny, nz;
    int64_t c0, ncell;            // first cell, cell count
    int64_t fx0, fy0, fz0;        // first x/y/z face
    int64_t in0;                  // first inflow face (ny*nz of them)
    int64_t inj0;                 // first injury face
    int32_t ninj, inj_i0, inj_ni, inj_k0, inj_nk;
    int32_t jadh;                 // adhesion layers (cells j < jadh over the patch)
    int32_t t0, nt;               // tile range
    uint32_t mnx, lnx, mny, lny;  // magic multipliers/shifts for division by nx and ny
    double dx, dy, dz, V, Ax, Ay, Az;
    double dt;                    // this step (rewritten on the device by a variable step)
    double gx, gy, gz, rdt;       // Ax/dx, Ay/dy, Az/dz, 1/dt
    double ddtk, ddtw;            // this step's ddt coefficients k, w (k (f'-f)/dt - w D)
    double dtmax;                 // the channel's given step: the largest a variable step takes
};

// Round-up magic-number division of 32-bit unsigned n by a fixed d (host computes m, l).
__host__ inline void fastdiv_magic(uint32_t d, uint32_t& m, uint32_t& l) {
    l = 0;
    while ((1ull << l) < d) ++l;
    m = (uint32_t)((((unsigned __int128)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
}
__device__ inline uint32_t fastdiv(uint32_t n, uint32_t m, uint32_t l) {
    if (l == 0) return n;
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> 1)) >> (l - 1);
}

// Model constants on the device (same names as clot_params).
struct ModelDev {
    double nu, C_CK, D_P, D_ADP, D_chem, P_diam, P_max, P_0, k_adh, kcoh_Pmax;
    double eta_t, eta_star, kappa_eta, k_adp, adp_crit, k_e2, e2_crit;
    double A_hat, tau_f, dtau, N_A, N1, N2;
    double kC0p, kC0m, kC0cat, kC1p, kC1m, kC1cat, kC2p, kC2m, kC2cat;
    double kS1p, kS1m, kE1p, kE1m, kS2p, kS2m, kE2p, kE2m;
    double S1_0, S2_0, E0_0, p_out;
    double g0;
    int32_t M_rxn;
    double psi, max_co, dt_growth;   // time scheme: Crank-Nicolson off-centring, variable step
    double k_I, I_0;                 // inhibitor variant: association rate, inlet value
};

// Launch-wide tables.
struct Grid {
    const ChanDev* ch;            // per channel
    const int32_t* t2c;           // tile -> channel
    int32_t ntiles;
};

__device__ inline int32_t xcd_tile(int32_t b, int32_t nb) {
    int32_t q = nb / NXCD, r = nb % NXCD;
    int32_t x = b % NXCD, i = b / NXCD;
    return x * q + (x < r ? x : r) + i;
}

struct Cell {
    int64_t g;      // global cell id
    int32_t i, j, k;
};

__device__ inline Cell cell_at(const ChanDev& c, int64_t local) {
    Cell p;
    p.g = c.c0 + local;
    const uint32_t loc = (uint32_t)local;
    const uint32_t r = fastdiv(loc, c.mnx, c.lnx);
    p.i = (int32_t)(loc - r * (uint32_t)c.nx);
    const uint32_t k = fastdiv(r, c.mny, c.lny);
    p.j = (int32_t)(r - k * (uint32_t)c.ny);
    p.k = (int32_t)k;
    return p;
}

__device__ inline int64_t fx_id(const ChanDev& c, int i, int j, int k) {
    return c.fx0 + i + (int64_t)(c.nx + 1) * (j + (int64_t)c.ny * k);
}
__device__ inline int64_t fy_id(const ChanDev& c, int i, int j, int k) {
    return c.fy0 + i + (int64_t)c.nx * (j + (int64_t)(c.ny + 1) * k);
}
__device__ inline int64_t fz_id(const ChanDev& c, int i, int j, int k) {
    return c.fz0 + i + (int64_t)c.nx * (j + (int64_t)c.ny * k);
}

// ---------------------------------------------------------------------------------
// Block reductions and the per-channel "last tile finishes the sum" pattern.
// Partial sums land in part[tile*NV + v]; the block that finishes last in its
// channel (an atomic ticket per channel) adds the channel's partials in tile order,
// so the result is deterministic, then runs the caller's scalar epilogue.
// ---------------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-wide sums of NV values; lds holds NV*(BS/64 + 1) doubles.
template <int NV, int BS = NT>
__device__ inline void block_sum(double (&v)[NV], double* lds) {
    constexpr int NW = BS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) lds[q * NW + w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += lds[threadIdx.x * NW + ww];
        lds[NV * NW + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = lds[NV * NW + q];
}

// Block-wide maximum of v, returned to every thread; lds holds BS/64 doubles.
template <int BS = NT>
__device__ inline double block_max(double v, double* lds) {
    constexpr int NW = BS / 64;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = lds[0];
    for (int w = 1; w < NW; ++w) m = fmax(m, lds[w]);
    __syncthreads();
    return m;
}

// Writes the block's totals of v[] as the tile partials part[q*stride + tile]
// (component-major, so the finishing launch reads each component's partials as one
// contiguous run).  The per-channel totals are finished by k_finish (clot_krylov.h):
// a separate small launch, so no block needs a device-wide fence (on a multi-XCD part
// each such fence writes back the whole L2) and the summation order is fixed.
template <int NV>
__device__ inline void store_partials(double (&v)[NV], double* part, int32_t stride, int32_t tile, double* lds) {
    block_sum<NV>(v, lds);
#pragma unroll
    for (int q = 0; q < NV; ++q)
        if (threadIdx.x == q) part[(int64_t)q * stride + tile] = v[q];
}

}  // namespace clot
