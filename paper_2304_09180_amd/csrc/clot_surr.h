// Learned reaction step (gfx950).
//
// The surrogate predicts the reaction increment of one transport step Dt as the
// explicit-midpoint increment f = Dt R(y + Dt R(y)/2) (two right-hand sides) times a
// learned relative correction:
//     Delta_i = f_i (1 + clamp(sc_i c_i, -1/2, 1/2)),   c = MLP(features),
// with sc_i the RMS over the training set of (Delta_RK4 - f)_i / |f_i| (the RK4
// increment's relative departure from f), so the network output is O(1), a cell at
// a fixed point stays exact, and a poor network can move an increment by at most
// half of itself.  Features (32), signed-log scaled: slog(y_i/s_i) for the 14
// species, slog(f_i/(s_i sf_i)) with sf_i the RMS of f/s, ADP/ADP*, g(eta), H_adh,
// log10(Dt)+5.  The same device function builds the
// features for training and inference.  A cell is accepted when its midpoint defect
// relative to the increment,
//     max_i |Delta_i - Dt R_i(y + Delta/2)| / (|Delta_i| + 1e-5 |y_i| + 1e-6 s_i),
// is below the residual tolerance; otherwise it is queued for the plain RK4 step (so a
// zero tolerance sends every cell to the plain integrator).  The exact increment's
// defect is O(Dt^3), so the test bounds the error of each increment by a fraction of
// the increment: summed over steps, the error of a field stays that fraction of its
// change.  Measured against the species' size or scale instead, a slowly changing
// species (|Delta| << |y|, or thrombin three decades under S2_0) would pass with its
// increment wrong by tens of percent.  The floor terms, about a hundred units in the
// last place of the stored value and a millionth of the scale, keep cells where a
// species barely changes from failing on rounding.
#pragma once
#include "clot_mlp.h"
#include "clot_step.h"

namespace clot {

struct SurrTables {
    float s[MLP_NSP];      // species scales
    float sf[MLP_NSP];     // RMS of Dt R / s over the training set
    float sc[MLP_NSP];     // RMS of the relative corrections over the training set
    float inv_s[MLP_NSP];  // 1/s
    float inv_f[MLP_NSP];  // 1/(s sf)
    float fl[MLP_NSP];     // floor of the defect's denominator, 1e-6 s
};

__host__ __device__ inline void species_scales(const ModelDev& M, float (&s)[MLP_NSP]) {
    // Pmu Pma Pba Pbse S1 S2 E1 E2 S1b S2b E1b E2b C1 C2
    const float pm = (float)M.P_max, a = (float)M.S1_0, b = (float)M.S2_0;
    const float v[MLP_NSP] = {pm, pm, pm, pm, a, b, a, b, a, b, a, b, b, b};
    for (int i = 0; i < MLP_NSP; ++i) s[i] = v[i];
}

// Fills the species scales and the reciprocals from sf and sc.
inline void surr_tables_finish(const ModelDev& M, SurrTables& tb) {
    species_scales(M, tb.s);
    for (int i = 0; i < MLP_NSP; ++i) {
        tb.inv_s[i] = 1.f / tb.s[i];
        tb.inv_f[i] = 1.f / (tb.s[i] * tb.sf[i]);
        tb.fl[i] = 1e-6f * tb.s[i];
    }
}

#ifndef CLOT_INHIBITOR   // the network covers the 14 reacting species of the base model
// Signed logarithm of a scaled value: |v| in [1e-12, 1] maps onto [0, 1], zero below
// 1e-12 (single precision: the feature is rounded to bf16 afterwards).
__device__ inline float slog(float v) {
    const float a = fabsf(v);
    if (!(a > 1e-12f)) return 0.f;
    const float m = fmaf(__log2f(a), 0.025085832972f, 1.f);   // (log10|v| + 12)/12
    return copysignf(m, v);
}

template <class T>
__device__ inline void surr_features(const T (&y)[NRX], T adp, T gam, T hadh, T dt, const RxnK<T>& K,
                                     const SurrTables& tb, float (&x)[MLP_IN], T (&f)[NRX]) {
    T k1[NRX], ym[NRX];
    rxn_rhs(y, adp, gam, hadh, K, k1);
#pragma unroll
    for (int i = 0; i < NRX; ++i) ym[i] = y[i] + T(0.5) * dt * k1[i];
    rxn_rhs(ym, adp, gam, hadh, K, f);
#pragma unroll
    for (int i = 0; i < NRX; ++i) {
        f[i] *= dt;
        x[i] = slog((float)y[i] * tb.inv_s[i]);
        x[NRX + i] = slog((float)f[i] * tb.inv_f[i]);
    }
    x[28] = (float)(adp / K.adp_crit);
    x[29] = (float)gam;
    x[30] = (float)hadh;
    x[31] = fmaf(__log2f((float)dt), 0.30102999566f, 5.f);   // log10(Dt) + 5
}

// Whether every species' midpoint defect, relative to the increment, is below tol (one
// right-hand-side evaluation; compared as |defect| < tol * den, so a NaN fails).
template <class T>
__device__ inline bool surr_accept(const T (&y)[NRX], const T (&inc)[NRX], T adp, T gam, T hadh, T dt,
                                   const RxnK<T>& K, const SurrTables& tb, float tol) {
    T ym[NRX], fm[NRX];
#pragma unroll
    for (int i = 0; i < NRX; ++i) ym[i] = y[i] + T(0.5) * inc[i];
    rxn_rhs(ym, adp, gam, hadh, K, fm);
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NRX; ++i) {
        const float den = fabsf((float)inc[i]) + 1e-5f * fabsf((float)y[i]) + tb.fl[i];
        ok = ok && (float)fabs(inc[i] - dt * fm[i]) < tol * den;
    }
    return ok;
}

// The learned step works on the stored values (FP32 in the mixed path) and leaves no low parts.
template <class T>
__device__ inline void load_rxn_state(const Fields<T>& F, int64_t g, T (&y)[NRX]) {
#pragma unroll
    for (int q = 0; q < NRX; ++q) y[q] = F.spc[rxn_species(q)][g];
}

template <class T>
__device__ inline void store_rxn_state(const Fields<T>& F, int64_t g, const T (&y)[NRX]) {
#pragma unroll
    for (int q = 0; q < NRX; ++q) {
        F.spc[rxn_species(q)][g] = y[q];
        F.lo[rxn_species(q)][g] = T(0);
    }
}

template <class T>
__device__ inline bool adhesion_cell(const ChanDev& C, const Cell& P) {
    return P.j < C.jadh && P.i >= C.inj_i0 && P.i < C.inj_i0 + C.inj_ni && P.k >= C.inj_k0 &&
           P.k < C.inj_k0 + C.inj_nk;
}

// Surrogate reaction step.  One lane per cell does the per-cell work; the wave then
// runs the MLP on MFMA over its four groups of 16 cells, inputs and outputs passing
// through a per-wave LDS tile.  Rejected cells are appended to a list.
constexpr int SURR_XLD = 36;   // bf16 row stride of the input tile (conflict-free B reads)
constexpr int SURR_OLD = 17;   // float row stride of the output tile
constexpr int SURR_WAVE_BYTES = 64 * SURR_XLD * 2;
static_assert(64 * SURR_OLD * 4 <= SURR_WAVE_BYTES, "output tile fits the input tile");

template <class T>
__global__ __launch_bounds__(256) void k_rxn_surr(Grid G, Fields<T> F, RxnK<T> K, MLPWeights w, SurrTables tb,
                                                  float tol, int32_t* fb_list, int32_t* fb_count, int32_t* fb_chan) {
    CLOT_TILE_PROLOGUE(G)
    __shared__ __align__(16) unsigned char tileb[4][SURR_WAVE_BYTES];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint16_t* sX = reinterpret_cast<uint16_t*>(tileb[wv]);
    float* sO = reinterpret_cast<float*>(tileb[wv]);
    const int rq = 4 * (l >> 4);
    MLPRegs R;
    R.load(w);
    for (int sub = 0; sub < TILE / 256; ++sub) {   // 256 cells per pass
        const int64_t local = tbase + sub * 256 + threadIdx.x;
        const bool own = local < C.ncell;
        T y[NRX], f[NRX];
        T adp = T(0), gam = T(0), hadh = T(0);
        const T dt = T(C.dt);
        int64_t g = 0;
        {
            float x[MLP_IN];
            if (own) {
                const Cell P = cell_at(C, local);
                g = P.g;
                load_rxn_state(F, g, y);
                adp = F.spc[ADP][g];
                gam = binding_g<T>(F.eta[g], K);
                hadh = adhesion_cell<T>(C, P) ? T(1) : T(0);
                surr_features(y, adp, gam, hadh, dt, K, tb, x, f);
            } else {
#pragma unroll
                for (int i = 0; i < MLP_IN; ++i) x[i] = 0.f;
            }
#pragma unroll
            for (int i = 0; i < MLP_IN; i += 4)
                *reinterpret_cast<bf16x4*>(sX + l * SURR_XLD + i) = pack4_bf16(x[i], x[i + 1], x[i + 2], x[i + 3]);
        }
        __builtin_amdgcn_wave_barrier();   // the tile is the wave's own: its lanes' LDS ops stay in order
        bf16x4 xb[4][2];
#pragma unroll
        for (int grp = 0; grp < 4; ++grp)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) xb[grp][kb] = load_b_cm(sX, SURR_XLD, 16 * kb, 16 * grp);
        __builtin_amdgcn_wave_barrier();   // the output tile overwrites the input tile
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            bf16x4 h1[4], h2[4];
            const f32x4 o = mlp_chain16(R, w, xb[grp], h1, h2);
            float* q = sO + (16 * grp + (l & 15)) * SURR_OLD + rq;
            q[0] = o[0];
            q[1] = o[1];
            q[2] = o[2];
            q[3] = o[3];
        }
        __builtin_amdgcn_wave_barrier();
        if (own) {
            T inc[NRX];
#pragma unroll
            for (int i = 0; i < NRX; ++i) {
                float r = tb.sc[i] * sO[l * SURR_OLD + i];
                r = r > 0.5f ? 0.5f : (r < -0.5f ? -0.5f : r);
                inc[i] = f[i] * (T(1) + T(r));
            }
            if (surr_accept(y, inc, adp, gam, hadh, dt, K, tb, tol)) {
#pragma unroll
                for (int i = 0; i < NRX; ++i) y[i] += inc[i];
                store_rxn_state(F, g, y);
            } else {
                const int32_t slot = atomicAdd(fb_count, 1);
                fb_list[slot] = (int32_t)g;
                atomicAdd(&fb_chan[chid], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();   // the next pass rewrites the tile
    }
}

// Plain RK4 reaction step (as k_rxn) for the listed cells.
template <class T>
__global__ __launch_bounds__(NT) void k_rxn_list(const ChanDev* chans, int nch, Fields<T> F, int nsub, RxnK<T> K,
                                                 const int32_t* fb_list, const int32_t* fb_count) {
    const int32_t nfb = *fb_count;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < nfb; q += (int64_t)gridDim.x * NT) {
    const int64_t g = fb_list[q];
    // find the channel of cell g (channels are few; binary search over c0)
    int lo = 0, hi = nch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chans[mid].c0 <= g) lo = mid;
        else hi = mid - 1;
    }
    const ChanDev C = chans[lo];
    rxn_cell<T>(F, C, cell_at(C, g - C.c0), nsub, K);   // exactly the plain step's cell update
    }
}

// ---------------------------------------------------------------------------------
// Batch kernels on arbitrary states (training data).  A state row has 18 doubles:
// 14 species (RXN order), ADP, eta, H_adh, Dt.
// ---------------------------------------------------------------------------------
constexpr int SURR_ROW = 18;

__device__ inline void unpack_row(const double* r, const RxnK<double>& K, double (&y)[NRX], double& adp, double& gam,
                                  double& hadh, double& dt) {
#pragma unroll
    for (int i = 0; i < NRX; ++i) y[i] = r[i];
    adp = r[14];
    gam = binding_g<double>(r[15], K);
    hadh = r[16];
    dt = r[17];
}

// Plain RK4 increments (M_rxn sub-steps, FP64) of each state.
__global__ __launch_bounds__(NT) void k_rxn_batch(const double* rows, int64_t n, int nsub, RxnK<double> K, double* inc) {
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (q >= n) return;
    double y[NRX], adp, gam, hadh, dt;
    unpack_row(rows + q * SURR_ROW, K, y, adp, gam, hadh, dt);
    double y0[NRX];
#pragma unroll
    for (int i = 0; i < NRX; ++i) y0[i] = y[i];
    const double h = dt / nsub;
    for (int m = 0; m < nsub; ++m) {
        double k1[NRX], k2[NRX], k3[NRX], k4[NRX], w[NRX];
        rxn_rhs(y, adp, gam, hadh, K, k1);
        for (int i = 0; i < NRX; ++i) w[i] = y[i] + 0.5 * h * k1[i];
        rxn_rhs(w, adp, gam, hadh, K, k2);
        for (int i = 0; i < NRX; ++i) w[i] = y[i] + 0.5 * h * k2[i];
        rxn_rhs(w, adp, gam, hadh, K, k3);
        for (int i = 0; i < NRX; ++i) w[i] = y[i] + h * k3[i];
        rxn_rhs(w, adp, gam, hadh, K, k4);
        for (int i = 0; i < NRX; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    for (int i = 0; i < NRX; ++i) inc[q * NRX + i] = y[i] - y0[i];
}

// Training set: bf16 features [n][32] and f32 targets [n][16]: relative corrections
// (Delta_RK4 - f)/|f| clamped to [-1/2, 1/2] (the range the step applies), in units
// of sc_i, and zero where |f_i| <= 1e-12 s_i (negligible rates, where the relative
// correction is noise); outputs 14..15 zero.  With stats != NULL it instead
// accumulates per-block sums (42 per block): the squares of f/s, the squares of the
// clamped relative corrections, and the count of rows with non-negligible f.
__global__ __launch_bounds__(NT) void k_surr_dataset(const double* rows, const double* inc, int64_t n, RxnK<double> K,
                                                     SurrTables tb, uint16_t* x, float* t, double* stats) {
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
    __shared__ double lds[42 * (NT / 64 + 1)];
    double acc[42];
#pragma unroll
    for (int i = 0; i < 42; ++i) acc[i] = 0.0;
    if (q < n) {
        double y[NRX], adp, gam, hadh, dt, f[NRX];
        unpack_row(rows + q * SURR_ROW, K, y, adp, gam, hadh, dt);
        float xf[MLP_IN];
        surr_features<double>(y, adp, gam, hadh, dt, K, tb, xf, f);
        for (int i = 0; i < NRX; ++i) {
            const bool live = fabs(f[i]) > 1e-12 * tb.s[i];
            double rel = live ? (inc[q * NRX + i] - f[i]) / fabs(f[i]) : 0.0;
            rel = rel > 0.5 ? 0.5 : (rel < -0.5 ? -0.5 : rel);
            if (stats) {
                const double fs = f[i] / tb.s[i];
                acc[i] = fs * fs;
                acc[NRX + i] = rel * rel;
                acc[2 * NRX + i] = live ? 1.0 : 0.0;
            } else {
                t[q * MLP_OUT + i] = (float)(rel / tb.sc[i]);
            }
        }
        if (!stats) {
            t[q * MLP_OUT + 14] = 0.f;
            t[q * MLP_OUT + 15] = 0.f;
            for (int i = 0; i < MLP_IN; i += 4)
                *reinterpret_cast<bf16x4*>(x + q * MLP_IN + i) = pack4_bf16(xf[i], xf[i + 1], xf[i + 2], xf[i + 3]);
        }
    }
    if (stats) {
        block_sum<42>(acc, lds);
        if (threadIdx.x == 0)
            for (int i = 0; i < 42; ++i) stats[(int64_t)blockIdx.x * 42 + i] = acc[i];
    }
}

#endif  // CLOT_INHIBITOR

}  // namespace clot
