// Host side of the clotting-step library: C ABI, workspace layout, step plan and
// the Krylov drivers.  Kernels are in clot_step.h / clot_krylov.h / clot_ops.h.
#include "../../include/clot.h"
#include "clot_step.h"
#include "clot_mg.h"
#include "clot_mgm.h"
#include "clot_mgb.h"
#include "clot_surr.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace clot;

namespace {

constexpr int NPOOL = 7 + 7 * NTR;   // Krylov vector pool (CG scratch + one BiCGStab set per transported species)
constexpr int NPART = 3 * MAXK;      // max partial sums per tile
constexpr int NSTAT = 40;            // per-channel statistics slots
constexpr int MAXCORR = 8;
enum { ST_MOM = 0, ST_ETA = 1, ST_TR = 2, ST_P = 3 /* +corr */, ST_REF = 12 /* +corr */, ST_RESM = 21, ST_RESP = 22,
       ST_RESE = 23, ST_REST = 24, ST_FAIL = 25, ST_FALLBACK = 26, ST_DIAG = 27 /* div, |phi| max, min species */,
       ST_SYSIT_TR = 30 };

struct Carver {
    char* base;
    size_t off = 0;
    template <class X>
    X* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        X* p = base ? reinterpret_cast<X*>(base + off) : nullptr;
        off += n * sizeof(X);
        return p;
    }
};

const double PI = 3.14159265358979323846;

// Rectangular duct (0,a)x(0,b): w with -lap w = 1, w = 0 on the walls, as the
// plane-Poiseuille part minus its Fourier-series wall correction in y.
double duct_w(double y, double z, double a, double b) {
    double w = 0.5 * y * (a - y);
    const double zz = std::fabs(z - 0.5 * b), B = 0.5 * b;
    for (int n = 1; n < 4000; n += 2) {
        const double s = n * PI / a;
        const double e1 = std::exp(s * (zz - B)), e2 = std::exp(-s * (zz + B));
        const double term = 4.0 * a * a / (PI * PI * PI * n * (double)n * n) * (e1 + e2) / (1.0 + std::exp(-2.0 * s * B)) *
                            std::sin(s * y);
        w -= term;
        if (e1 < 1e-18 && n > 50) break;
    }
    return w;
}
double duct_slope(double a, double b) {   // dw/dy at (0, b/2)
    double s = 0.5 * a;
    for (int n = 1; n < 400; n += 2) s -= 4.0 * a / (PI * PI * n * (double)n) / std::cosh(n * PI * b / (2.0 * a));
    return s;
}

struct ChanHost {
    clot_channel d;
    int64_t c0, ncell, fx0, fy0, fz0, nfx, nfy, nfz, in0, inj0;
    int32_t ninj, inj_i0, inj_ni, inj_k0, inj_nk, jadh, t0, nt, ncorr;
    double dx, dy, dz;
    int64_t n = 0;           // steps taken (the clock itself lives on the device)
};

}  // namespace

struct clot_ctx {
    clot_precision prec;
    int32_t nchan = 0;
    std::string err;
    virtual ~clot_ctx() {}
    virtual clot_status init_state(int ch, const double* xc, size_t nc, const double* xf, size_t nf) = 0;
    virtual clot_status count(int ch, clot_field f, size_t* n) const = 0;
    virtual clot_status set(int ch, clot_field f, const double* h, size_t n) = 0;
    virtual clot_status get(int ch, clot_field f, double* h, size_t n) = 0;
    virtual clot_status step(int nsteps, bool wait) = 0;
    virtual clot_status sync() = 0;
    virtual clot_status stats(int ch, clot_stats* s) const = 0;
    virtual clot_status probe(int id) = 0;
    virtual clot_status set_rxn(clot_rxn_mode mode, const void* blob, size_t nb, double tol) = 0;
    virtual clot_status probe_read(double* ms, int64_t* n) = 0;
    virtual clot_status set_graph(int on, double scale, int pad) = 0;
    virtual clot_status set_brick(int kernel, int shape) = 0;
    virtual clot_status graph_info(int64_t* info) = 0;
    virtual clot_status state_size(size_t* bytes) const = 0;
    virtual clot_status save_state(void* host, size_t bytes) = 0;
    virtual clot_status load_state(const void* host, size_t bytes) = 0;
};

namespace {

// Launch, bracketed by probe events when this phase is the one being timed.
// A probed launch carries its start and stop events in the dispatch itself, so the
// interval between them is the kernel's execution, as a profiler records it.
template <typename F, typename... Args>
static inline void probed_launch(hipEvent_t e0, hipEvent_t e1, F kernel, dim3 grid, dim3 block, uint32_t shmem,
                                 hipStream_t stream, Args... args) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, e0, e1, 0u, args...);
}

#define CLOT_LAUNCH(id, ...)                                                     \
    do {                                                                         \
        const bool pr_ = (id) == probe_id && !capturing && ev_used + 2 <= (int)evs.size(); \
        if (pr_) {                                                               \
            probed_launch(evs[ev_used], evs[ev_used + 1], __VA_ARGS__);          \
            ev_used += 2;                                                        \
        } else {                                                                 \
            hipLaunchKernelGGL(__VA_ARGS__);                                     \
        }                                                                        \
    } while (0)

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            err = std::string(#x) + ": " + hipGetErrorString(e_);                       \
            return CLOT_EHIP;                                                           \
        }                                                                               \
    } while (0)

template <class T>
struct Ctx : clot_ctx {
    std::vector<ChanHost> ch;
    clot_params prm;
    ModelDev M;
    hipStream_t st;
    int64_t N = 0, NFX = 0, NFY = 0, NFZ = 0, NIN = 0, NINJ = 0;
    int32_t ntiles = 0;
    int maxcorr = 2;
    // device tables
    ChanDev* d_ch = nullptr;
    std::vector<ChanDev> hch;   // host copy of the channel table as uploaded (clock reset)
    char* ws_base = nullptr;    // the caller's workspace (every device array of the context)
    size_t ws_bytes = 0;
    int32_t* d_t2c = nullptr;
    int32_t* d_f2c = nullptr;
    Fields<T> F{};
    T* pool[NPOOL];
    T* u_in = nullptr;
    T* pmu_in = nullptr;
    KState S{};
    int32_t* refmask = nullptr;
    int32_t* allmask = nullptr;
    int32_t* corrmask = nullptr;      // [MAXCORR][nch]
    double* sigw = nullptr;           // [nch][NHIST]
    int32_t* push = nullptr;          // [nch][2]
    double* dstats = nullptr;         // [nch][NSTAT]
    int32_t* h_nact = nullptr;        // pinned: [0] active channels; [4..5] eta solve info
    // the concurrent eta solve
    KState Se{};
    T* eta_v[5] = {};                 // right-hand side, r, p (two), t
    int32_t* eta_info = nullptr;      // device: [channels still iterating, largest iteration count]
    hipStream_t st2 = nullptr;
    hipEvent_t ev_derive = nullptr, ev_eta = nullptr, ev_info = nullptr, ev_asm = nullptr, ev_mg = nullptr;
    int eta_budget = 32;
    int fixed_iters = 0;
    SigState* sig = nullptr;          // [nch] release-history schedule
    int last_it[8] = {8, 8, 8, 8, 8, 8, 8, 8};
    // Graph replay.  Slots: 0 momentum, 1..3 pressure (corrector 1, 2, later), 4 eta,
    // 5 transport; slot 6 counts pressure refinement passes.
    bool graph_on = false, capturing = false;
    double g_scale = 1.1;
    int g_pad = 1;
    int calib_left = 0;
    int it_max[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int budget[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int it_pmax[3][12] = {};          // pressure: per corrector slot and refinement pass
    int pbudget[3][12] = {};
    hipStream_t cst = nullptr;        // capture stream
    // one recorded step per parity, as a chain of graphs of at most about SEG_NODES
    // kernel nodes each (recording is cut between Krylov iterations)
    std::vector<hipGraphExec_t> gseg[2];
    static constexpr size_t SEG_NODES = 1500;
    std::vector<hipGraphExec_t>* cap_out = nullptr;
    clot_status seg_err = CLOT_OK;
    int parity = 0;                   // buffer-rotation parity of the next step
    int32_t* gflag = nullptr;         // device: a fixed-budget solve ended unconverged
    int64_t g_replays = 0, g_captures = 0, g_overflows = 0, g_nodes = 0, g_segs = 0;
    // multigrid hierarchy of the pressure preconditioner (level 0 = the mesh)
    struct Level {
        std::vector<ChanDev> ch;
        std::vector<int32_t> t2c;
        ChanDev* d_ch = nullptr;
        int32_t* d_t2c = nullptr;
        int32_t ntiles = 0;
        int64_t N = 0, NFX = 0, NFY = 0, NFZ = 0;
        T *x = nullptr, *y = nullptr, *b = nullptr, *dg = nullptr, *cx = nullptr, *cy = nullptr, *cz = nullptr,
          *cout = nullptr;
        // the momentum preconditioner's operator on this level (boundary face slots hold
        // the Dirichlet terms) and its V-cycle vectors, one per velocity component
        T *mmass = nullptr, *mdg = nullptr, *mcx = nullptr, *mcy = nullptr, *mcz = nullptr;
        T *mb[MGM_K] = {}, *mx[MGM_K] = {}, *my[MGM_K] = {};
        Grid grid() const { return Grid{d_ch, d_t2c, ntiles}; }
        CoefOp<T> mom_op() const { return CoefOp<T>{mdg, mcx, mcy, mcz}; }
    };
    std::vector<Level> lev;
    T mg_w = T(0.8);         // weighted-Jacobi smoothing weight (set with the channels)
    int mg_t0 = -1;          // first level run by the fused tail launch (-1: none)
    size_t mg_tail_lds = 0;  // its dynamic LDS bytes
    TailPlan* d_tplan = nullptr;   // per channel: the fused tail's set-up (clot_mg.h)
    std::vector<TailPlan> h_tplan;  // its host copy (kept until the upload completes)
    T* mg_y0 = nullptr;      // level-0 smoother scratch
    T* mg_z0 = nullptr;      // preconditioned residual z = M r
    double* mg_inv = nullptr;  // per-channel inverse of the coarsest-level matrix
    int mgm_nc = 0;          // coarse levels of the momentum preconditioner (0: Jacobi BiCGStab)
    std::vector<int32_t> h_mgm_last;   // per channel: its coarsest momentum level
    int32_t* d_mgm_last = nullptr;
    // LDS-staged finest-level momentum kernels: the bricks of every channel (when every
    // channel is coarsened along every axis), one table per brick shape; each bricked
    // kernel has its own shape (the tile autotuner's choice, clot_set_brick_shape)
    std::vector<BrickChan> h_brick[MGM_NSHAPE];
    std::vector<int32_t> h_b2c[MGM_NSHAPE];
    BrickChan* d_brick[MGM_NSHAPE] = {};
    int32_t* d_b2c[MGM_NSHAPE] = {};
    int brick_shape[CLOT_NBRICK_KERNELS] = {};   // per bricked kernel (clot_brick_kernel)
    BrickGrid bricks(int s) const { return BrickGrid{d_brick[s], d_b2c[s], (int32_t)h_b2c[s].size()}; }
    bool bricked() const { return !h_b2c[0].empty(); }
    // LDS-staged legs of the pressure V-cycle's coarse levels (clot_mgb.h).  Table j >= 1:
    // lev[j - 1], whose restriction reaches lev[j]; empty where some channel is not
    // coarsened along every axis there (table 0, the mesh, stays empty).  The tables
    // depend on the geometry only; mgb_use (mg_brick, FP32, 2 or 3 sweeps) decides
    // whether they are used.
    // One set of tables per brick shape.
    std::vector<BrickChan> h_pbr[MGB_NSHAPE][MG_MAXLEV];
    std::vector<int32_t> h_pb2c[MGB_NSHAPE][MG_MAXLEV];
    BrickChan* d_pbr[MGB_NSHAPE][MG_MAXLEV] = {};
    int32_t* d_pb2c[MGB_NSHAPE][MG_MAXLEV] = {};
    bool mgb_use = false;
    // The mesh's restriction in bricks of shape 0 (k_mg_restrict_mesh) and its
    // prolongation by halving (k_mg_post1_mesh): when every channel is coarsened along
    // every axis from the mesh to lev[0] (the table) and mg_brick is set
    std::vector<BrickChan> h_rbr;
    std::vector<int32_t> h_rb2c;
    BrickChan* d_rbr = nullptr;
    int32_t* d_rb2c = nullptr;
    bool mesh_on = false;
    bool mesh_halves() const { return mesh_on && !h_rb2c.empty(); }
    // The mesh's legs in LDS-staged launches (k_mg_mesh_leg), bricks of the pressure shape
    // 0, in FP32 contexts with mg_brick set: the down leg's three sweeps (mesh_down_n = 3),
    // or two sweeps and the restriction where every channel is coarsened along every axis
    // (2); with three sweeps on such a mesh also the up leg's prolongation and the sweep
    // after it (mesh_up2).
    std::vector<BrickChan> h_p3br;
    std::vector<int32_t> h_p3b2c;
    BrickChan* d_p3br = nullptr;
    int32_t* d_p3b2c = nullptr;
    int mesh_down_n = 0;
    bool mesh_up2 = false;
    bool mesh_down_3d = false;   // some channel is 3-D (the larger LDS brick)
    bool mesh_down() const { return !h_p3b2c.empty(); }
    size_t mesh_down_lds() const { return mesh_leg_lds_bytes(mesh_down_3d, sizeof(T)); }
    BrickGrid pbricks(int q, int j) const { return BrickGrid{d_pbr[q][j], d_pb2c[q][j], (int32_t)h_pb2c[q][j].size()}; }
    bool pbricked(int j) const { return mgb_use && !h_pb2c[0][j].empty(); }
    // reaction surrogate
    clot_rxn_mode rxn_mode = CLOT_RXN_PLAIN;
    float surr_tol = 1e-3f;
    SurrTables surr_tb{};
    uint16_t* mlp_wb = nullptr;
    float* mlp_wf = nullptr;
    int32_t* fb_list = nullptr;
    int32_t* fb_count = nullptr;
    int32_t* fb_chan = nullptr;
    int probe_id = 0;
    std::vector<hipEvent_t> evs;
    int ev_used = 0;
    double probe_ms = 0.0;
    int64_t probe_n = 0;
    bool nonconv = false;
    // rollback: a step call that meets a non-finite value restores the state of its start
    char* snap = nullptr;             // device copy of the persistent state
    size_t state_bytes = 0;           // the persistent state: the workspace's first bytes
    int32_t* nanflag = nullptr;       // device: [0] a reduction met a NaN or infinity, [1] the state scan did
    bool snap_valid = false;          // a copy of the current call window's start exists
    int snap_parity = 0;
    Fields<T> snap_F{};
    std::vector<int64_t> snap_n;
    Grid grid() const { return Grid{d_ch, d_t2c, ntiles}; }
    ~Ctx() override {
        drop_graphs();
        if (st2) (void)hipStreamSynchronize(st2);
        if (ev_derive) (void)hipEventDestroy(ev_derive);
        if (ev_eta) (void)hipEventDestroy(ev_eta);
        if (ev_info) (void)hipEventDestroy(ev_info);
        if (ev_asm) (void)hipEventDestroy(ev_asm);
        if (ev_mg) (void)hipEventDestroy(ev_mg);
        if (st2) (void)hipStreamDestroy(st2);
        if (cst) (void)hipStreamDestroy(cst);
        if (h_nact) (void)hipHostFree(h_nact);
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    }
    void probe_collect() {
        for (int i = 0; i + 1 < ev_used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, evs[i], evs[i + 1]) == hipSuccess) {
                probe_ms += ms;
                probe_n += 1;
            }
        }
        ev_used = 0;
    }
    clot_status probe(int id) override {
        HIPCHK(hipStreamSynchronize(st));
        if (st2) HIPCHK(hipStreamSynchronize(st2));
        probe_collect();
        if (id < 0 || id >= CLOT_PROBE_NKERNELS) {
            err = "unknown probe kernel";
            return CLOT_EINVAL;
        }
        if (id && evs.empty()) {
            evs.resize(2048);
            for (auto& e : evs) HIPCHK(hipEventCreate(&e));
        }
        probe_id = id;
        probe_ms = 0.0;
        probe_n = 0;
        return CLOT_OK;
    }
    clot_status set_rxn(clot_rxn_mode mode, const void* blob, size_t nb, double tol) override {
        drop_graphs();   // the recorded step holds the reaction kernel and its tables
        if (mode == CLOT_RXN_PLAIN) {
            rxn_mode = mode;
            return CLOT_OK;
        }
#ifdef CLOT_INHIBITOR
        err = "set_reaction_mode: the learned reaction step covers the base model's 14 reacting species only";
        return CLOT_EINVAL;
#endif
        if (mode != CLOT_RXN_SURROGATE || !blob || nb != (MLP_NPARAM + 2 * MLP_NSP) * sizeof(float) || !(tol >= 0.0)) {
            err = "set_reaction_mode: expected a float32 blob of MLP parameters + 28 scales and tol >= 0";
            return CLOT_EINVAL;
        }
        const float* f = (const float*)blob;
        std::vector<uint16_t> wb(MLP_NPARAM);
        for (int q = 0; q < MLP_NPARAM; ++q) {
            if (!std::isfinite(f[q])) {
                err = "set_reaction_mode: non-finite weight";
                return CLOT_EINVAL;
            }
            wb[q] = f2bf(f[q]);
        }
        for (int i = 0; i < MLP_NSP; ++i) {
            surr_tb.sf[i] = f[MLP_NPARAM + i];
            surr_tb.sc[i] = f[MLP_NPARAM + MLP_NSP + i];
            if (!(surr_tb.sf[i] > 0.f) || !(surr_tb.sc[i] > 0.f)) {
                err = "set_reaction_mode: scales must be positive";
                return CLOT_EINVAL;
            }
        }
        surr_tables_finish(M, surr_tb);
        HIPCHK(hipMemcpyAsync(mlp_wf, f, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(mlp_wb, wb.data(), MLP_NPARAM * sizeof(uint16_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        rxn_mode = mode;
        surr_tol = (float)tol;
        return CLOT_OK;
    }

    clot_status probe_read(double* ms, int64_t* n) override {
        HIPCHK(hipStreamSynchronize(st));
        if (st2) HIPCHK(hipStreamSynchronize(st2));
        probe_collect();
        *ms = probe_ms;
        *n = probe_n;
        return CLOT_OK;
    }

    // ---------------------------------------------------------------------------
    size_t layout(char* base) {
        Carver cv{base};
        const int nch = (int)ch.size();
        // the persistent state first (what a step reads from the previous one: fields,
        // clocks, histories, and the constant tables), one contiguous range that a step
        // call copies aside and restores if it meets a non-finite value
        d_ch = cv.take<ChanDev>(nch);
        d_t2c = cv.take<int32_t>(ntiles);
        d_f2c = cv.take<int32_t>(std::max<int64_t>(NINJ, 1));
        for (int c = 0; c < 3; ++c) F.u[c] = cv.take<T>(N);
        F.p = cv.take<double>(N);
        F.phi[0] = cv.take<T>(NFX);
        F.phi[1] = cv.take<T>(NFY);
        F.phi[2] = cv.take<T>(std::max<int64_t>(NFZ, 1));
        F.phin[0] = cv.take<T>(NFX);
        F.phin[1] = cv.take<T>(NFY);
        F.phin[2] = cv.take<T>(std::max<int64_t>(NFZ, 1));
        for (int s = 0; s < NSPC; ++s) F.spc[s] = cv.take<T>(N);
        for (int q = 0; q < NSPC; ++q) F.lo[q] = cv.take<T>(N);
        const int64_t ni = std::max<int64_t>(NINJ, 1);
        F.E0 = cv.take<double>(ni);
        F.C0 = cv.take<double>(ni);
        F.s1w = cv.take<double>(ni);
        F.eta = cv.take<T>(N);
        F.thB = cv.take<T>(N);
        F.thB_prev = cv.take<T>(N);
        F.sigma = cv.take<T>(N);
        F.hist = cv.take<T>((size_t)N * NHIST);
        u_in = cv.take<T>(NIN);
        pmu_in = cv.take<T>(NIN);
        F.u_in = u_in;
        F.pmu_in = pmu_in;
        for (int c = 0; c < 3; ++c) F.ddt0u[c] = cv.take<T>(N);
        for (int k = 0; k < NTR; ++k) F.ddt0c[k] = cv.take<T>(N);
        allmask = cv.take<int32_t>(nch);
        corrmask = cv.take<int32_t>((size_t)MAXCORR * nch);
        sig = cv.take<SigState>(nch);
        state_bytes = (cv.off + 255) & ~size_t(255);
        // per-step scratch
        for (int k = 0; k < NTR; ++k) F.dlt[k] = cv.take<T>(N);
        F.Wc = cv.take<T>(N);
        F.aP = cv.take<T>(N);
        for (int c = 0; c < 3; ++c) F.src[c] = cv.take<T>(N);
        for (int c = 0; c < 3; ++c) F.bm[c] = cv.take<T>(N);
        F.rAU = cv.take<T>(N);
        for (int c = 0; c < 3; ++c) F.HbyA[c] = cv.take<T>(N);
        F.dP = cv.take<T>(N);
        F.dE = cv.take<T>(N);
        F.rhs_p = cv.take<double>(N);
        for (int k = 0; k < NTR; ++k) F.trd[k] = cv.take<T>(N);
        for (int k = 0; k < NTR; ++k) F.trd64[k] = cv.take<double>(N);
        for (int k = 0; k < NTR; ++k) F.trb[k] = cv.take<double>(N);
        for (int k = 0; k < NTR; ++k) F.trc[k] = cv.take<T>((size_t)6 * N);
        F.co_part = cv.take<double>(ntiles);
        for (int q = 0; q < NPOOL; ++q) pool[q] = cv.take<T>(N);
        F.ncell = N;
        S.maxit = prm.max_iter;
        S.sc = cv.take<double>((size_t)nch * MAXK * NSC);
        S.chact = cv.take<int32_t>(nch);
        S.nact = cv.take<int32_t>(1);
        S.part = cv.take<double>((size_t)ntiles * NPART);
        S.pstride = ntiles;
        S.tick = cv.take<uint32_t>(nch);
        S.fin = cv.take<double>((size_t)nch * FIN_MAXNV);
        refmask = cv.take<int32_t>(nch);
        sigw = cv.take<double>((size_t)nch * NHIST);
        push = cv.take<int32_t>((size_t)nch * 2);
        dstats = cv.take<double>((size_t)nch * NSTAT);
        gflag = cv.take<int32_t>(1);
        nanflag = cv.take<int32_t>(2);
        S.nanflag = nanflag;
        Se.maxit = prm.max_iter;
        Se.sc = cv.take<double>((size_t)nch * MAXK * NSC);
        Se.chact = cv.take<int32_t>(nch);
        Se.nact = cv.take<int32_t>(1);
        Se.part = cv.take<double>((size_t)ntiles * NPART);
        Se.pstride = ntiles;
        Se.nanflag = nanflag;
        Se.tick = cv.take<uint32_t>(nch);
        Se.fin = cv.take<double>((size_t)nch * FIN_MAXNV);
        for (int q = 0; q < 5; ++q) eta_v[q] = cv.take<T>(N);
        eta_info = cv.take<int32_t>(2);
        mg_y0 = cv.take<T>(N);
        mg_z0 = cv.take<T>(N);
        mg_inv = cv.take<double>((size_t)nch * MG_COARSE * MG_COARSE);
        mlp_wb = cv.take<uint16_t>(MLP_NPARAM);
        mlp_wf = cv.take<float>(MLP_NPARAM);
        fb_list = cv.take<int32_t>(N);
        fb_count = cv.take<int32_t>(1);
        fb_chan = cv.take<int32_t>(nch);
        for (Level& L : lev) {
            L.d_ch = cv.take<ChanDev>(nch);
            L.d_t2c = cv.take<int32_t>(std::max(L.ntiles, 1));
            L.x = cv.take<T>(L.N);
            L.y = cv.take<T>(L.N);
            L.b = cv.take<T>(L.N);
            L.dg = cv.take<T>(L.N);
            L.cout = cv.take<T>(L.N);
            L.cx = cv.take<T>(L.NFX);
            L.cy = cv.take<T>(L.NFY);
            L.cz = cv.take<T>(L.NFZ);
        }
        d_mgm_last = cv.take<int32_t>(nch);
        d_tplan = cv.take<TailPlan>(nch);
        for (int q = 0; q < MGB_NSHAPE; ++q)
            for (int j = 0; j < MG_MAXLEV; ++j) {
                d_pbr[q][j] = cv.take<BrickChan>(std::max<size_t>(h_pbr[q][j].size(), 1));
                d_pb2c[q][j] = cv.take<int32_t>(std::max<size_t>(h_pb2c[q][j].size(), 1));
            }
        d_rbr = cv.take<BrickChan>(std::max<size_t>(h_rbr.size(), 1));
        d_rb2c = cv.take<int32_t>(std::max<size_t>(h_rb2c.size(), 1));
        d_p3br = cv.take<BrickChan>(std::max<size_t>(h_p3br.size(), 1));
        d_p3b2c = cv.take<int32_t>(std::max<size_t>(h_p3b2c.size(), 1));
        for (int q = 0; q < MGM_NSHAPE; ++q) {
            d_brick[q] = cv.take<BrickChan>(std::max<size_t>(h_brick[q].size(), 1));
            d_b2c[q] = cv.take<int32_t>(std::max<size_t>(h_b2c[q].size(), 1));
        }
        for (int l = 0; l < mgm_nc; ++l) {
            Level& L = lev[l];
            L.mmass = cv.take<T>(L.N);
            L.mdg = cv.take<T>(L.N);
            L.mcx = cv.take<T>(L.NFX);
            L.mcy = cv.take<T>(L.NFY);
            L.mcz = cv.take<T>(L.NFZ);
            for (int k = 0; k < MGM_K; ++k) {
                L.mb[k] = cv.take<T>(L.N);
                L.mx[k] = cv.take<T>(L.N);
                L.my[k] = cv.take<T>(L.N);
            }
        }
        snap = cv.take<char>(state_bytes);
        return cv.off + 256;
    }

    // ---------------------------------------------------------------------------
    clot_status setup(const clot_channel* cs, int nch, const clot_params* p) {
        prm = *p;
        // the release history holds tau_f/dtau + 1 snapshots in a ring of fixed length
        if (!(prm.dtau > 0) || !(prm.tau_f > 0) || std::fabs(prm.tau_f / prm.dtau - (NHIST - 1)) > 1e-9 * (NHIST - 1)) {
            err = "params: tau_f/dtau must equal " + std::to_string(NHIST - 1) + " (release history of " +
                  std::to_string(NHIST) + " snapshots)";
            return CLOT_EINVAL;
        }
        ch.resize(nch);
        int64_t c0 = 0, fx = 0, fy = 0, fz = 0, in = 0, inj = 0;
        int32_t t0 = 0;
        for (int i = 0; i < nch; ++i) {
            ChanHost& h = ch[i];
            h.d = cs[i];
            const clot_channel& d = cs[i];
            if (!(d.dim == 2 || d.dim == 3) || d.nx < 2 || d.ny < 2 || d.nz < 1 || (d.dim == 2 && d.nz != 1) ||
                (d.dim == 3 && d.nz < 2) || !(d.Lx > 0) || !(d.Ly > 0) || !(d.Lz > 0) || !(d.dt > 0) || !(d.shear >= 0)) {
                err = "channel " + std::to_string(i) + ": invalid dimensions, extents or time step";
                return CLOT_EINVAL;
            }
            if ((int64_t)d.nx * d.ny * d.nz > (int64_t)1 << 31) {
                err = "channel too large";
                return CLOT_EINVAL;
            }
            h.dx = d.Lx / d.nx;
            h.dy = d.Ly / d.ny;
            h.dz = d.Lz / d.nz;
            h.ncell = (int64_t)d.nx * d.ny * d.nz;
            h.c0 = c0;
            c0 += h.ncell;
            h.nfx = (int64_t)(d.nx + 1) * d.ny * d.nz;
            h.nfy = (int64_t)d.nx * (d.ny + 1) * d.nz;
            h.nfz = d.dim == 3 ? (int64_t)d.nx * d.ny * (d.nz + 1) : 0;
            h.fx0 = fx;
            h.fy0 = fy;
            h.fz0 = fz;
            fx += h.nfx;
            fy += h.nfy;
            fz += h.nfz;
            h.in0 = in;
            in += (int64_t)d.ny * d.nz;
            // injury patch: face centres inside [x0,x1] x [z0,z1] on y = 0
            int i0 = -1, i1 = -1, k0 = -1, k1 = -1;
            for (int ii = 0; ii < d.nx; ++ii) {
                const double xc = (ii + 0.5) * h.dx;
                if (xc >= d.inj_x0 && xc <= d.inj_x1) {
                    if (i0 < 0) i0 = ii;
                    i1 = ii;
                }
            }
            if (d.dim == 3) {
                for (int kk = 0; kk < d.nz; ++kk) {
                    const double zc = (kk + 0.5) * h.dz;
                    if (zc >= d.inj_z0 && zc <= d.inj_z1) {
                        if (k0 < 0) k0 = kk;
                        k1 = kk;
                    }
                }
            } else {
                k0 = 0;
                k1 = 0;
            }
            if (i0 < 0 || k0 < 0) {
                h.inj_i0 = 0;
                h.inj_ni = 0;
                h.inj_k0 = 0;
                h.inj_nk = 0;
            } else {
                h.inj_i0 = i0;
                h.inj_ni = i1 - i0 + 1;
                h.inj_k0 = k0;
                h.inj_nk = k1 - k0 + 1;
            }
            h.ninj = h.inj_ni * h.inj_nk;
            h.inj0 = inj;
            inj += h.ninj;
            // adhesion layers: cell centres within P_diam of the wall, else the first layer
            int ja = 0;
            for (int jj = 0; jj < d.ny; ++jj)
                if ((jj + 0.5) * h.dy <= p->P_diam) ja = jj + 1;
            h.jadh = ja > 0 ? ja : 1;
            h.nt = (int32_t)((h.ncell + TILE - 1) / TILE);
            h.t0 = t0;
            t0 += h.nt;
            // PISO corrections: fixed, or chosen from the viscous diffusion number
            const double hmin = std::min(h.dx, std::min(h.dy, d.dim == 3 ? h.dz : h.dy));
            const double Dn = p->nu * d.dt / (hmin * hmin);
            h.ncorr = p->n_corr > 0 ? p->n_corr
                                    : (Dn <= 10.0 ? 2 : Dn <= 30.0 ? 3 : Dn <= 50.0 ? 4 : Dn <= 80.0 ? 5 : Dn <= 120.0 ? 6 : 8);
            if (h.ncorr > MAXCORR) h.ncorr = MAXCORR;
            maxcorr = std::max(maxcorr, h.ncorr);
        }
        N = c0;
        NFX = fx;
        NFY = fy;
        NFZ = fz;
        NIN = in;
        NINJ = inj;
        ntiles = t0;
        build_levels();
        if (!lev.empty())
            for (const ChanDev& c : lev.back().ch)
                if (c.ncell > MG_COARSE) {
                    err = "channel too long for the pressure multigrid hierarchy";
                    return CLOT_EINVAL;
                }
        // Jacobi smoothing weight of the pressure V-cycle: for the 7-point Laplacian omega =
        // 6/7 shrinks every error mode with a component above half the grid frequency to at
        // most 5/7 per sweep, the best a single weight does; for the 5-point one omega = 4/5
        // (at most 3/5).  A context with a 2-D channel keeps 4/5.
        bool all3d = true;
        for (const ChanHost& h : ch) all3d = all3d && h.d.dim == 3;
        mg_w = T(all3d ? 6.0 / 7.0 : 0.8);
        // momentum preconditioner: each channel's coarse levels run until the viscous part
        // of its diagonal (nu dt sum_ax 2/h_ax^2 of the mass V/dt; Darcy and Crank-Nicolson
        // only add mass) is below MGM_RATIO times the mass (a CPU model of the cycle: 4
        // BiCGStab iterations on the duct and 2 on a 512x128 channel at D = 69 whether the
        // coarsest level's ratio is 0.5 or 8; each level dropped saves three launches per
        // cycle).  The context keeps as many levels as its deepest channel needs.
        mgm_nc = 0;
        h_mgm_last.assign(nch, 0);
        if (p->mom_mg && !lev.empty()) {
            for (int i = 0; i < nch; ++i) {
                const clot_channel& d = ch[i].d;
                int l = 0;
                for (; l + 1 < (int)lev.size(); ++l) {
                    const ChanDev& c = lev[l].ch[i];
                    const double hx = d.Lx / c.nx, hy = d.Ly / c.ny, hz = d.Lz / c.nz;
                    double v = 2.0 / (hx * hx) + 2.0 / (hy * hy);
                    if (c.dim == 3) v += 2.0 / (hz * hz);
                    if (p->nu * d.dt * v < MGM_RATIO) break;
                }
                h_mgm_last[i] = l;
                mgm_nc = std::max(mgm_nc, l + 1);
            }
        }
        for (int q = 0; q < MGM_NSHAPE; ++q) {
            h_brick[q].clear();
            h_b2c[q].clear();
        }
        if (mgm_nc > 0) {
            bool ok = true;
            for (const ChanHost& h : ch) ok = ok && h.d.nx >= 3 && h.d.ny >= 3 && (h.d.dim == 2 || h.d.nz >= 3);
            for (int q = 0; ok && q < MGM_NSHAPE; ++q)
                for (int i = 0; i < nch; ++i) {
                    const clot_channel& d = ch[i].d;
                    int bx, by, bz;
                    brick_dims(d.dim, q, bx, by, bz);
                    BrickChan b{(int32_t)h_b2c[q].size(), (d.nx + bx - 1) / bx, (d.ny + by - 1) / by,
                                (d.nz + bz - 1) / bz};
                    for (int t = 0; t < b.nbx * b.nby * b.nbz; ++t) h_b2c[q].push_back(i);
                    h_brick[q].push_back(b);
                }
        }
        // sweeps each way, automatic: a third sweep saves a third of the CG iterations on
        // 3-D channels (13 -> 9 per corrector on the 1M-cell duct, 7% of the step), while on
        // 2-D channels the iterations it saves cost about what the sweep adds
        if (prm.mg_sweeps == 0) prm.mg_sweeps = all3d ? 3 : 2;
        // fused launch for the trailing levels whose channels all fit the cell threshold
        // and, with every level's arrays, the LDS of one block
        mg_t0 = -1;
        mg_tail_lds = 0;
        if (p->mg_tail > 0 && !lev.empty()) {
            int dev = 0, lds_max = 65536;
            if (hipGetDevice(&dev) == hipSuccess)
                (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
            // less the kernel's static LDS (level table, coarse right-hand side) and a margin
            const int64_t limit =
                (int64_t)lds_max - (int64_t)(sizeof(TailPlan) + MG_TAIL_SEGS * sizeof(TailSeg<T>)) - 1024;
            const int nl = (int)lev.size();
            auto bytes_from = [&](int t) {
                int64_t worst = 0;
                for (int i = 0; i < nch; ++i) {
                    int64_t e = 0;
                    for (int l = t; l < nl; ++l) {
                        const ChanDev& c = lev[l].ch[i];
                        e += tail_level_elems(c.dim, c.nx, c.ny, c.nz, l == nl - 1, (int)sizeof(T));
                    }
                    worst = std::max(worst, e * (int64_t)sizeof(T));
                }
                return worst;
            };
            int t = nl;
            while (t > 0) {
                int64_t mx = 0;
                for (const ChanDev& c : lev[t - 1].ch) mx = std::max(mx, c.ncell);
                if (mx > p->mg_tail || bytes_from(t - 1) > limit) break;
                --t;
            }
            if (t < nl) {
                mg_t0 = t;
                mg_tail_lds = (size_t)bytes_from(t);
            }
        }
        // LDS-staged legs of the coarse levels: a table per level that every channel
        // coarsens along every axis
        {
            const int nl = (int)lev.size();
            for (int q = 0; q < MGB_NSHAPE; ++q)
                for (int j = 0; j < MG_MAXLEV; ++j) {
                    h_pbr[q][j].clear();
                    h_pb2c[q][j].clear();
                }
            for (int j = 1; j < nl && j < MG_MAXLEV; ++j) {
                bool ok = true;
                for (int i = 0; ok && i < nch; ++i) {
                    const ChanDev& c = lev[j].ch[i];
                    const ChanDev& f = lev[j - 1].ch[i];
                    ok = c.nx != f.nx && c.ny != f.ny && (c.dim == 2 || c.nz != f.nz);
                }
                if (!ok) continue;
                for (int q = 0; q < MGB_NSHAPE; ++q)
                    for (int i = 0; i < nch; ++i) {
                        const int dim = lev[j].ch[i].dim;
                        const int fx = lev[j - 1].ch[i].nx, fy = lev[j - 1].ch[i].ny, fz = lev[j - 1].ch[i].nz;
                        int bx, by, bz;
                        pbrick_dims(dim, q, bx, by, bz);
                        BrickChan b{(int32_t)h_pb2c[q][j].size(), (fx + bx - 1) / bx, (fy + by - 1) / by,
                                    (fz + bz - 1) / bz};
                        for (int t = 0; t < b.nbx * b.nby * b.nbz; ++t) h_pb2c[q][j].push_back(i);
                        h_pbr[q][j].push_back(b);
                    }
            }
            mgb_use = p->mg_brick != 0 && sizeof(T) == 4 && (prm.mg_sweeps == 2 || prm.mg_sweeps == 3);
            mesh_on = p->mg_brick != 0;
            h_rbr.clear();
            h_rb2c.clear();
            bool ok = nl > 0;
            for (int i = 0; ok && i < nch; ++i) {
                const ChanDev& c = lev[0].ch[i];
                ok = c.nx != ch[i].d.nx && c.ny != ch[i].d.ny && (c.dim == 2 || c.nz != ch[i].d.nz);
            }
            for (int i = 0; ok && i < nch; ++i) {
                const clot_channel& d = ch[i].d;
                int bx, by, bz;
                brick_dims(d.dim, 0, bx, by, bz);
                BrickChan b{(int32_t)h_rb2c.size(), (d.nx + bx - 1) / bx, (d.ny + by - 1) / by, (d.nz + bz - 1) / bz};
                for (int t = 0; t < b.nbx * b.nby * b.nbz; ++t) h_rb2c.push_back(i);
                h_rbr.push_back(b);
            }
            h_p3br.clear();
            h_p3b2c.clear();
            mesh_down_n = 0;
            if (p->mg_brick != 0 && sizeof(T) == 4 && nl > 0)
                mesh_down_n = prm.mg_sweeps == 3 ? 3 : (prm.mg_sweeps == 2 && !h_rb2c.empty() ? 2 : 0);
            mesh_up2 = mesh_down_n == 3 && !h_rb2c.empty();
            mesh_down_3d = false;
            if (mesh_down_n > 0)
                for (int i = 0; i < nch; ++i) {
                    mesh_down_3d = mesh_down_3d || ch[i].d.dim == 3;
                    const clot_channel& d = ch[i].d;
                    int bx, by, bz;
                    pbrick_dims(d.dim, 0, bx, by, bz);
                    BrickChan b{(int32_t)h_p3b2c.size(), (d.nx + bx - 1) / bx, (d.ny + by - 1) / by,
                                (d.nz + bz - 1) / bz};
                    for (int t = 0; t < b.nbx * b.nby * b.nbz; ++t) h_p3b2c.push_back(i);
                    h_p3br.push_back(b);
                }
        }
        const clot_params& q = *p;
        M = ModelDev{q.nu, q.C_CK, q.D_P, q.D_ADP, q.D_chem, q.P_diam, q.P_max, q.P_0, q.k_adh, q.kcoh_Pmax,
                     q.eta_t, q.eta_star, 0.0, q.k_adp, q.adp_crit, q.k_e2, q.e2_crit,
                     q.A_hat, q.tau_f, q.dtau, q.N_A, q.N1, q.N2,
                     q.kC0p, q.kC0m, q.kC0cat, q.kC1p, q.kC1m, q.kC1cat, q.kC2p, q.kC2m, q.kC2cat,
                     q.kS1p, q.kS1m, q.kE1p, q.kE1m, q.kS2p, q.kS2m, q.kE2p, q.kE2m,
                     q.S1_0, q.S2_0, q.E0_0, q.p_out, 0.0, q.M_rxn};
        const double Le = q.L_eta_over_Pdiam * q.P_diam;
        M.kappa_eta = Le * Le / 4.0;
        M.g0 = (std::pow(q.eta_star, 3) + std::pow(1.0 - q.eta_t, 3)) / std::pow(1.0 - q.eta_t, 3);
        M.psi = q.ddt_psi;
        M.max_co = q.max_co;
        M.dt_growth = q.dt_growth;
        M.k_I = q.k_I;
        M.I_0 = q.I_0;
        return CLOT_OK;
    }

    // Dynamic LDS limits of the kernels that use more than the default: a device call,
    // so it runs at clot_create, not in setup (which the workspace query runs without one).
    clot_status lds_limits() {
        bool set = true;
        auto attr = [&](const void* f, size_t bytes) {
            if (bytes > 65536)
                set = set && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
        };
        if (mg_t0 >= 0) attr(reinterpret_cast<const void*>(&k_mg_tail<T>), mg_tail_lds);
        if (mesh_down()) {
            attr(reinterpret_cast<const void*>(&k_mg_mesh_leg<T, MESH_DOWN3>), mesh_down_lds());
            attr(reinterpret_cast<const void*>(&k_mg_mesh_leg<T, MESH_DOWN2R>), mesh_down_lds());
            attr(reinterpret_cast<const void*>(&k_mg_mesh_leg<T, MESH_UP2>), mesh_down_lds());
        }
        if (mgb_use) {
            const int h = prm.mg_sweeps;
            auto both = [&](const void* down, const void* up, int q) {
                attr(down, mgb_lds_bytes(h, q, sizeof(T)));
                attr(up, mgb_lds_bytes(h, q, sizeof(T)));
            };
#define CLOT_MGB_ATTR(H, Q)                                                          \
    both(reinterpret_cast<const void*>(&k_mg_brick<T, MGB_DOWN, H, Q>),              \
         reinterpret_cast<const void*>(&k_mg_brick<T, MGB_UP, H, Q>), Q)
            if (h == 3) {
                CLOT_MGB_ATTR(3, 0);
                CLOT_MGB_ATTR(3, 1);
                CLOT_MGB_ATTR(3, 2);
                CLOT_MGB_ATTR(3, 3);
            } else {
                CLOT_MGB_ATTR(2, 0);
                CLOT_MGB_ATTR(2, 1);
                CLOT_MGB_ATTR(2, 2);
                CLOT_MGB_ATTR(2, 3);
            }
#undef CLOT_MGB_ATTR
        }
        if (!set) {
            err = "cannot raise the dynamic LDS limit of the multigrid kernels";
            return CLOT_EHIP;
        }
        return CLOT_OK;
    }

    // Level dims: halve every axis with >= 3 cells until the largest channel has
    // <= MG_COARSE cells; smaller channels keep halving (down to 2 per axis).
    void build_levels() {
        const int nch = (int)ch.size();
        lev.clear();
        std::vector<std::array<int, 3>> dims(nch);
        for (int i = 0; i < nch; ++i) dims[i] = {ch[i].d.nx, ch[i].d.ny, ch[i].d.nz};
        auto ncells = [&](const std::array<int, 3>& d) { return (int64_t)d[0] * d[1] * d[2]; };
        for (int l = 1; l < MG_MAXLEV; ++l) {
            bool all_small = true;
            for (int i = 0; i < nch; ++i) all_small &= ncells(dims[i]) <= MG_COARSE;
            if (all_small) break;
            for (int i = 0; i < nch; ++i)
                for (int a = 0; a < 3; ++a)
                    if (dims[i][a] >= 3) dims[i][a] = (dims[i][a] + 1) / 2;
            Level L;
            int64_t c0 = 0, fx = 0, fy = 0, fz = 0;
            int32_t t0 = 0;
            for (int i = 0; i < nch; ++i) {
                ChanDev c{};
                c.dim = ch[i].d.dim;
                c.nx = dims[i][0];
                c.ny = dims[i][1];
                c.nz = dims[i][2];
                c.ncell = ncells(dims[i]);
                c.c0 = c0;
                c0 += c.ncell;
                c.fx0 = fx;
                c.fy0 = fy;
                c.fz0 = fz;
                fx += (int64_t)(c.nx + 1) * c.ny * c.nz;
                fy += (int64_t)c.nx * (c.ny + 1) * c.nz;
                fz += c.dim == 3 ? (int64_t)c.nx * c.ny * (c.nz + 1) : 0;
                c.nt = (int32_t)((c.ncell + TILE - 1) / TILE);
                c.t0 = t0;
                t0 += c.nt;
                fastdiv_magic((uint32_t)c.nx, c.mnx, c.lnx);
                fastdiv_magic((uint32_t)c.ny, c.mny, c.lny);
                for (int t = 0; t < c.nt; ++t) L.t2c.push_back(i);
                L.ch.push_back(c);
            }
            L.N = c0;
            L.NFX = fx;
            L.NFY = fy;
            L.NFZ = std::max<int64_t>(fz, 1);
            L.ntiles = t0;
            lev.push_back(L);
        }
    }

    clot_status upload_tables() {
        const int nch = (int)ch.size();
        std::vector<ChanDev> dv(nch);
        std::vector<int32_t> t2c(ntiles), f2c(std::max<int64_t>(NINJ, 1), 0);
        for (int i = 0; i < nch; ++i) {
            const ChanHost& h = ch[i];
            ChanDev& c = dv[i];
            c.dim = h.d.dim;
            c.nx = h.d.nx;
            c.ny = h.d.ny;
            c.nz = h.d.nz;
            c.c0 = h.c0;
            c.ncell = h.ncell;
            c.fx0 = h.fx0;
            c.fy0 = h.fy0;
            c.fz0 = h.fz0;
            c.in0 = h.in0;
            c.inj0 = h.inj0;
            c.ninj = h.ninj;
            c.inj_i0 = h.inj_i0;
            c.inj_ni = h.inj_ni;
            c.inj_k0 = h.inj_k0;
            c.inj_nk = h.inj_nk;
            c.jadh = h.jadh;
            c.t0 = h.t0;
            c.nt = h.nt;
            fastdiv_magic((uint32_t)c.nx, c.mnx, c.lnx);
            fastdiv_magic((uint32_t)c.ny, c.mny, c.lny);
            c.dx = h.dx;
            c.dy = h.dy;
            c.dz = h.dz;
            c.V = h.dx * h.dy * h.dz;
            c.Ax = h.dy * h.dz;
            c.Ay = h.dx * h.dz;
            c.Az = h.dx * h.dy;
            c.dt = h.d.dt;
            c.gx = c.Ax / c.dx;
            c.gy = c.Ay / c.dy;
            c.gz = c.Az / c.dz;
            c.rdt = 1.0 / c.dt;
            c.ddtk = 1.0;
            c.ddtw = 0.0;
            c.dtmax = h.d.dt;
            for (int t = 0; t < h.nt; ++t) t2c[h.t0 + t] = i;
            for (int f = 0; f < h.ninj; ++f) f2c[h.inj0 + f] = i;
        }
        HIPCHK(hipMemcpyAsync(d_ch, dv.data(), nch * sizeof(ChanDev), hipMemcpyHostToDevice, st));
        hch = dv;
        for (Level& L : lev) {
            HIPCHK(hipMemcpyAsync(L.d_ch, L.ch.data(), nch * sizeof(ChanDev), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(L.d_t2c, L.t2c.data(), L.t2c.size() * 4, hipMemcpyHostToDevice, st));
        }
        HIPCHK(hipMemcpyAsync(d_t2c, t2c.data(), t2c.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d_mgm_last, h_mgm_last.data(), nch * 4, hipMemcpyHostToDevice, st));
        if (mg_t0 >= 0) {
            const int nl = (int)lev.size();
            h_tplan.assign(nch, TailPlan{});
            std::vector<ChanDev> lc(nl - mg_t0);
            for (int i = 0; i < nch; ++i) {
                for (int l = mg_t0; l < nl; ++l) lc[l - mg_t0] = lev[l].ch[i];
                tail_plan_build(h_tplan[i], nl - mg_t0, lc.data(), (int)sizeof(T));
            }
            HIPCHK(hipMemcpyAsync(d_tplan, h_tplan.data(), nch * sizeof(TailPlan), hipMemcpyHostToDevice, st));
        }
        if (!h_rb2c.empty()) {
            HIPCHK(hipMemcpyAsync(d_rbr, h_rbr.data(), h_rbr.size() * sizeof(BrickChan), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(d_rb2c, h_rb2c.data(), h_rb2c.size() * 4, hipMemcpyHostToDevice, st));
        }
        if (mesh_down()) {
            HIPCHK(hipMemcpyAsync(d_p3br, h_p3br.data(), h_p3br.size() * sizeof(BrickChan), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(d_p3b2c, h_p3b2c.data(), h_p3b2c.size() * 4, hipMemcpyHostToDevice, st));
        }
        for (int q = 0; q < MGB_NSHAPE; ++q)
            for (int j = 0; j < MG_MAXLEV; ++j)
                if (!h_pb2c[q][j].empty()) {
                    HIPCHK(hipMemcpyAsync(d_pbr[q][j], h_pbr[q][j].data(), h_pbr[q][j].size() * sizeof(BrickChan),
                                          hipMemcpyHostToDevice, st));
                    HIPCHK(hipMemcpyAsync(d_pb2c[q][j], h_pb2c[q][j].data(), h_pb2c[q][j].size() * 4,
                                          hipMemcpyHostToDevice, st));
                }
        for (int q = 0; q < MGM_NSHAPE; ++q)
            if (!h_b2c[q].empty()) {
                HIPCHK(hipMemcpyAsync(d_brick[q], h_brick[q].data(), h_brick[q].size() * sizeof(BrickChan),
                                      hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(d_b2c[q], h_b2c[q].data(), h_b2c[q].size() * 4, hipMemcpyHostToDevice, st));
            }
        HIPCHK(hipMemcpyAsync(d_f2c, f2c.data(), f2c.size() * 4, hipMemcpyHostToDevice, st));
        std::vector<int32_t> ones(nch, 1), cm((size_t)MAXCORR * nch, 0);
        for (int k = 0; k < MAXCORR; ++k)
            for (int i = 0; i < nch; ++i) cm[(size_t)k * nch + i] = k < ch[i].ncorr ? 1 : 0;
        HIPCHK(hipMemcpyAsync(allmask, ones.data(), nch * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(corrmask, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, st));
        std::vector<SigState> sv(nch, fresh_sig());
        HIPCHK(hipMemcpyAsync(sig, sv.data(), nch * sizeof(SigState), hipMemcpyHostToDevice, st));
        fill(gflag, 0, 1);
        clot_status r = upload_inflow();
        if (r) return r;
        std::vector<uint32_t> z(nch, 0);
        HIPCHK(hipMemcpy(S.tick, z.data(), nch * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(Se.tick, z.data(), nch * 4, hipMemcpyHostToDevice));
        std::vector<double> zs((size_t)nch * NSTAT, 0.0);
        HIPCHK(hipMemcpy(dstats, zs.data(), zs.size() * 8, hipMemcpyHostToDevice));
        return CLOT_OK;
    }

    // inflow profiles of every channel (Appendix C.1 / C.2), from the host descriptors
    // and this context's parameters
    clot_status upload_inflow() {
        const int nch = (int)ch.size();
        std::vector<T> ui(NIN), pi(NIN);
        for (int i = 0; i < nch; ++i) {
            const ChanHost& h = ch[i];
            for (int k = 0; k < h.d.nz; ++k)
                for (int j = 0; j < h.d.ny; ++j) {
                    const double y = (j + 0.5) * h.dy, z = (k + 0.5) * h.dz;
                    ui[h.in0 + j + (int64_t)h.d.ny * k] = T(inflow_u(h, y, z));
                    pi[h.in0 + j + (int64_t)h.d.ny * k] = T(inflow_pmu(h, y, z));
                }
        }
        HIPCHK(hipMemcpyAsync(u_in, ui.data(), NIN * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(pmu_in, pi.data(), NIN * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return CLOT_OK;
    }

    // inflow speed (eq. parabolicVelocity in 2-D; duct Poiseuille in 3-D) and its
    // Poiseuille pressure gradient magnitude
    double inflow_u(const ChanHost& h, double y, double z) const {
        const double g = h.d.shear;
        if (h.d.dim == 2) {
            const double r = 0.5 * h.d.Ly;
            return -(g / (2.0 * r)) * (y - r) * (y - r) + 0.5 * g * r;
        }
        return g / duct_slope(h.d.Ly, h.d.Lz) * duct_w(y, z, h.d.Ly, h.d.Lz);
    }
    double inflow_dpdx(const ChanHost& h) const {
        if (h.d.dim == 2) return prm.nu * h.d.shear / (0.5 * h.d.Ly);
        return prm.nu * h.d.shear / duct_slope(h.d.Ly, h.d.Lz);
    }
    // margination (Appendix C.1, C.2): P0 [1 + K R^{m-1}(1-R)^{n-1} (+ z term)] / (1 + K B(m,n) (+ ...))
    double inflow_pmu(const ChanHost& h, double y, double z) const {
        const int m = prm.marg_m, n = prm.marg_n;
        const double beta = std::exp(std::lgamma((double)m) + std::lgamma((double)n) - std::lgamma((double)(m + n)));
        const double ry = 0.5 * h.d.Ly;
        const double Ry = std::fabs(y - ry) / ry;
        double br = 1.0 + h.d.K_y * std::pow(Ry, m - 1) * std::pow(1.0 - Ry, n - 1);
        double norm = 1.0 + h.d.K_y * beta;
        if (h.d.dim == 3) {
            const double rz = 0.5 * h.d.Lz;
            const double Rz = std::fabs(z - rz) / rz;
            br += h.d.K_z * std::pow(Rz, m - 1) * std::pow(1.0 - Rz, n - 1);
            norm += h.d.K_z * beta;
        }
        return prm.P_0 * br / norm;
    }

    // ---------------------------------------------------------------------------
    clot_status upload(T* dst, const std::vector<double>& src) {
        std::vector<T> tmp(src.begin(), src.end());
        HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return CLOT_OK;
    }

    clot_status init_state(int c, const double* xc, size_t nc, const double* xf, size_t nf) override {
        snap_valid = false;
        ChanHost& h = ch[c];
        const int64_t n = h.ncell;
        if (nc != (size_t)(NSPC_DRAWN * n) || nf != (size_t)(2 * h.ninj) || (!xc && nc) || (!xf && nf)) {
            err = "init_state: expected 15*ncell cell draws and 2*nface face draws";
            return CLOT_EINVAL;
        }
        std::vector<double> u(n), zero(n, 0.0), pr(n);
        const double G = inflow_dpdx(h);
        for (int k = 0; k < h.d.nz; ++k)
            for (int j = 0; j < h.d.ny; ++j) {
                const double y = (j + 0.5) * h.dy, z = (k + 0.5) * h.dz;
                const double uu = inflow_u(h, y, z);
                for (int i = 0; i < h.d.nx; ++i) {
                    const int64_t g = i + (int64_t)h.d.nx * (j + (int64_t)h.d.ny * k);
                    u[g] = uu;
                    pr[g] = G * (h.d.Lx - (i + 0.5) * h.dx);
                }
            }
        clot_status s;
        if ((s = upload(F.u[0] + h.c0, u))) return s;
        if ((s = upload(F.u[1] + h.c0, zero))) return s;
        if ((s = upload(F.u[2] + h.c0, zero))) return s;
        HIPCHK(hipMemcpy(F.p + h.c0, pr.data(), n * 8, hipMemcpyHostToDevice));
        // fluxes: x faces carry the profile, the others none
        std::vector<double> fxv(h.nfx), fyv(h.nfy, 0.0), fzv(h.nfz, 0.0);
        const double Ax = h.dy * h.dz;
        for (int k = 0; k < h.d.nz; ++k)
            for (int j = 0; j < h.d.ny; ++j) {
                const double uu = inflow_u(h, (j + 0.5) * h.dy, (k + 0.5) * h.dz);
                for (int i = 0; i <= h.d.nx; ++i) fxv[i + (int64_t)(h.d.nx + 1) * (j + (int64_t)h.d.ny * k)] = Ax * uu;
            }
        if ((s = upload(F.phi[0] + h.fx0, fxv))) return s;
        if ((s = upload(F.phi[1] + h.fy0, fyv))) return s;
        if (h.nfz && (s = upload(F.phi[2] + h.fz0, fzv))) return s;
        // species with 1% multiplicative noise; the inhibitor variant's I starts at its
        // inlet value and E2i at zero, neither with a draw
        for (int sp = 0; sp < NSPC; ++sp) {
            std::vector<double> v(n, sp == INH ? prm.I_0 : 0.0);
            if (sp >= NSPC_DRAWN) {
                if ((s = upload(F.spc[sp] + h.c0, v))) return s;
                continue;
            }
            for (int k = 0; k < h.d.nz; ++k)
                for (int j = 0; j < h.d.ny; ++j) {
                    const double y = (j + 0.5) * h.dy, z = (k + 0.5) * h.dz;
                    const double base = sp == PMU ? inflow_pmu(h, y, z) : sp == S1 ? prm.S1_0 : sp == S2 ? prm.S2_0 : 0.0;
                    for (int i = 0; i < h.d.nx; ++i) {
                        const int64_t g = i + (int64_t)h.d.nx * (j + (int64_t)h.d.ny * k);
                        v[g] = base * (1.0 + 0.01 * xc[(size_t)sp * n + g]);
                    }
                }
            if ((s = upload(F.spc[sp] + h.c0, v))) return s;
        }
        std::vector<double> e0(h.ninj), c0(h.ninj, 0.0);
        for (int f = 0; f < h.ninj; ++f) {
            e0[f] = prm.E0_0 * (1.0 + 0.01 * xf[f]);
            c0[f] = 0.0 * (1.0 + 0.01 * xf[h.ninj + f]);
        }
        if (h.ninj) {
            HIPCHK(hipMemcpy(F.E0 + h.inj0, e0.data(), h.ninj * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(F.C0 + h.inj0, c0.data(), h.ninj * sizeof(double), hipMemcpyHostToDevice));
        }
        for (int q = 0; q < NSPC; ++q)
            if ((s = upload(F.lo[q] + h.c0, zero))) return s;
        if ((s = upload(F.eta + h.c0, zero))) return s;
        if ((s = upload(F.sigma + h.c0, zero))) return s;
        for (int q = 0; q < NHIST; ++q)
            if ((s = upload(F.hist + (int64_t)q * N + h.c0, zero))) return s;
        // theta_B of the "previous" step = current
        std::vector<double> thb(n, 0.0);
        if ((s = upload(F.thB_prev + h.c0, thb))) return s;
        h.n = 0;
        {   // statistics (and the failure status they carry) start afresh
            const std::vector<double> zs(NSTAT, 0.0);
            HIPCHK(hipMemcpy(dstats + (size_t)c * NSTAT, zs.data(), NSTAT * 8, hipMemcpyHostToDevice));
        }
        // the clock: the channel's step, or with a variable step the largest the initial
        // flux allows (cell Courant number 0.5 dt sum_f |phi_f| / V, x faces only carry
        // flux); implicit Euler first; no time-derivative history
        {
            ChanDev cd = hch[c];
            cd.dt = h.d.dt;
            if (prm.max_co > 0.0) {
                double mx = 0.0;
                for (int64_t r = 0; r < (int64_t)h.d.ny * h.d.nz; ++r)
                    for (int i = 0; i < h.d.nx; ++i) {
                        const double* f = fxv.data() + (int64_t)(h.d.nx + 1) * r + i;
                        mx = std::max(mx, (std::fabs(f[1]) + std::fabs(f[0])) + 0.0);
                    }
                const double co = 0.5 * cd.dt * mx / cd.V;
                if (co > prm.max_co) cd.dt = prm.max_co * cd.dt / co;
            }
            cd.rdt = 1.0 / cd.dt;
            cd.ddtk = 1.0;
            cd.ddtw = 0.0;
            hch[c] = cd;
            HIPCHK(hipMemcpyAsync(d_ch + c, &hch[c], sizeof(ChanDev), hipMemcpyHostToDevice, st));
            for (int q = 0; q < 3; ++q)
                if ((s = upload(F.ddt0u[q] + h.c0, zero))) return s;
            for (int k = 0; k < NTR; ++k)
                if ((s = upload(F.ddt0c[k] + h.c0, zero))) return s;
        }
        const SigState s0 = fresh_sig();
        HIPCHK(hipMemcpyAsync(sig + c, &s0, sizeof(SigState), hipMemcpyHostToDevice, st));
        // thB_prev must equal theta_B of the initial state: compute it on the device
        hipLaunchKernelGGL(k_derive<T>, dim3(ntiles), dim3(NT), 0, st, grid(), F, M);
        HIPCHK(hipGetLastError());
        const int64_t cnt = h.ncell;
        hipLaunchKernelGGL(k_copy<T>, dim3((cnt + 255) / 256), dim3(256), 0, st, F.thB_prev + h.c0, F.thB + h.c0, cnt);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return CLOT_OK;
    }

    // ---------------------------------------------------------------------------
    struct FieldRef {
        void* ptr;
        int64_t n;
        bool dbl;
        bool ro;
    };
    FieldRef ref(int c, clot_field f) const {
        const ChanHost& h = ch[c];
        const int64_t n = h.ncell;
        switch (f) {
            case CLOT_UX: return {F.u[0] + h.c0, n, false, false};
            case CLOT_UY: return {F.u[1] + h.c0, n, false, false};
            case CLOT_UZ: return {F.u[2] + h.c0, h.d.dim == 3 ? n : 0, false, false};
            case CLOT_P: return {F.p + h.c0, n, true, false};
            case CLOT_PHIX: return {F.phi[0] + h.fx0, h.nfx, false, false};
            case CLOT_PHIY: return {F.phi[1] + h.fy0, h.nfy, false, false};
            case CLOT_PHIZ: return {F.phi[2] + h.fz0, h.nfz, false, false};
            case CLOT_E0: return {F.E0 + h.inj0, h.ninj, true, false};
            case CLOT_C0: return {F.C0 + h.inj0, h.ninj, true, false};
            case CLOT_ETA: return {F.eta + h.c0, n, false, true};
            case CLOT_THETAB: return {F.thB_prev + h.c0, n, false, true};
            case CLOT_SIGMA: return {F.sigma + h.c0, n, false, true};
            case CLOT_HADH: return {nullptr, n, false, true};
#ifdef CLOT_INHIBITOR
            case CLOT_I: return {F.spc[INH] + h.c0, n, false, false};
            case CLOT_E2I: return {F.spc[E2I] + h.c0, n, false, false};
#endif
            default:
                if (f >= CLOT_PMU && f <= CLOT_C2) return {F.spc[f - CLOT_PMU] + h.c0, n, false, false};
        }
        return {nullptr, 0, false, true};
    }

    // The species index of a cell-species field, or -1.
    static int species_of(clot_field f) {
        if (f >= CLOT_PMU && f <= CLOT_C2) return (int)f - (int)CLOT_PMU;
#ifdef CLOT_INHIBITOR
        if (f == CLOT_I) return INH;
        if (f == CLOT_E2I) return E2I;
#endif
        return -1;
    }
    static bool unknown(const FieldRef& r, clot_field f) {
        return !r.ptr && r.n == 0 && f != CLOT_UZ && f != CLOT_PHIZ && f != CLOT_HADH;
    }
    clot_status count(int c, clot_field f, size_t* n) const override {
        FieldRef r = ref(c, f);
        if (unknown(r, f)) {
            const_cast<Ctx*>(this)->err = "unknown field (or one of another build)";
            return CLOT_EINVAL;
        }
        *n = (size_t)r.n;
        return CLOT_OK;
    }

    clot_status set(int c, clot_field f, const double* h, size_t n) override {
        FieldRef r = ref(c, f);
        if (unknown(r, f)) {
            err = "unknown field (or one of another build)";
            return CLOT_EINVAL;
        }
        if (r.ro) {
            err = "field is read only";
            return CLOT_EINVAL;
        }
        if ((int64_t)n != r.n || (!h && n)) {
            err = "set_field: size mismatch";
            return CLOT_EINVAL;
        }
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(h[i])) {
                err = "set_field: non-finite value";
                return CLOT_ENAN;
            }
        snap_valid = false;   // a state changed between steps starts a new call window
        if (r.dbl) {
            HIPCHK(hipMemcpyAsync(r.ptr, h, n * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            return CLOT_OK;
        }
        std::vector<double> v(h, h + n);
        const int bq = species_of(f);
        if (bq >= 0) {   // stored value + low part, so the field is set to full precision
            std::vector<T> hi(n);
            std::vector<double> rem(n);
            for (size_t i = 0; i < n; ++i) {
                hi[i] = T(h[i]);
                rem[i] = h[i] - (double)hi[i];
            }
            HIPCHK(hipMemcpyAsync(r.ptr, hi.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
            clot_status rs = upload(F.lo[bq] + ch[c].c0, rem);
            if (rs) return rs;
            HIPCHK(hipStreamSynchronize(st));
            return CLOT_OK;
        }
        return upload((T*)r.ptr, v);
    }

    clot_status get(int c, clot_field f, double* h, size_t n) override {
        FieldRef r = ref(c, f);
        if (unknown(r, f)) {
            err = "unknown field (or one of another build)";
            return CLOT_EINVAL;
        }
        if ((int64_t)n != r.n || (!h && n)) {
            err = "get_field: size mismatch";
            return CLOT_EINVAL;
        }
        if (f == CLOT_HADH) {   // adhesion mask: cells j < jadh over the injury patch
            const ChanHost& q = ch[c];
            for (int k = 0; k < q.d.nz; ++k)
                for (int j = 0; j < q.d.ny; ++j)
                    for (int i = 0; i < q.d.nx; ++i)
                        h[i + (int64_t)q.d.nx * (j + (int64_t)q.d.ny * k)] =
                            (j < q.jadh && i >= q.inj_i0 && i < q.inj_i0 + q.inj_ni && k >= q.inj_k0 &&
                             k < q.inj_k0 + q.inj_nk) ? 1.0 : 0.0;
            return CLOT_OK;
        }
        HIPCHK(hipStreamSynchronize(st));
        if (r.dbl) {
            HIPCHK(hipMemcpy(h, r.ptr, n * 8, hipMemcpyDeviceToHost));
            return CLOT_OK;
        }
        std::vector<T> tmp(n);
        HIPCHK(hipMemcpy(tmp.data(), r.ptr, n * sizeof(T), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i) h[i] = (double)tmp[i];
        const int bq = species_of(f);
        if (bq >= 0) {   // stored value + low part
            HIPCHK(hipMemcpy(tmp.data(), F.lo[bq] + ch[c].c0, n * sizeof(T), hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i) h[i] += (double)tmp[i];
        }
        return CLOT_OK;
    }

    // ---------------------------------------------------------------------------
    // Krylov drivers
    int32_t poll() {
        (void)hipMemcpyAsync(h_nact, S.nact, 4, hipMemcpyDeviceToHost, st);
        (void)hipStreamSynchronize(st);
        if (ev_used) probe_collect();
        return *h_nact;
    }
    void fill(int32_t* p, int32_t v, int64_t n) {
        hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    }
    // chact = mask with the active count zero (count = false: the solve's start admits its
    // channels) or the mask's count (count = true).
    void set_active(const int32_t* mask, bool count = false) {
        hipLaunchKernelGGL(k_set_active, dim3(1), dim3(256), 0, st, S.chact, mask, S.nact, (int)ch.size(),
                           count ? 1 : 0);
    }

    // The iterations of one solve.  Eagerly: chunks of iterations, polling the count of
    // active channels in between.  Under graph capture: exactly the slot's budget, then
    // every channel still active is flagged as unconverged.
    template <int K, class Body>
    int iterate(int slot, int keep, int next_chunk, int gbudget, Body&& body, int par0 = 0, int done = 0) {
        int it = 0, par = par0;
        if (fixed_iters > 0) {   // a solve on the side stream: no polls, no failure flag
            for (; it < fixed_iters; ++it, par ^= 1) body(par);
            return it;
        }
        if (capturing) {
            for (; it < gbudget; ++it, par ^= 1) {
                body(par);
                seg_point();
            }
            hipLaunchKernelGGL(k_flag_active, dim3(1), dim3(64), 0, st, S.chact, S.sc, (int)ch.size(), K, gflag);
            return it;
        }
        int chunk = std::max(2, last_it[slot]);
        while (it + done < prm.max_iter) {
            for (int c = 0; c < chunk && it + done < prm.max_iter; ++c, ++it, par ^= 1) body(par);
            if (poll() == 0) break;
            chunk = next_chunk;
        }
        last_it[slot] = std::max(keep, it - keep);
        it_max[slot] = std::max(it_max[slot], it);
        return it;
    }

    template <class Op, int K>
    int run_cg(const Op& op, KVec<T, K> V, double rtol, int tol_mode, const int32_t* mask, int slot, int pa, int pb) {
        set_active(mask);
        hipLaunchKernelGGL((k_cg_init<T, K, Op>), dim3(ntiles), dim3(NT), 0, st, grid(), op, V, S);
        finish<3 * K>(EpiCgInit<K>{rtol, tol_mode});
        return cg_iterations<Op, K>(op, V, slot, pa, pb, 0, 0);
    }
    // CG iterations of a started solve (par0: parity of the next iteration's vectors,
    // done: iterations already taken)
    template <class Op, int K>
    int cg_iterations(const Op& op, KVec<T, K> V, int slot, int pa, int pb, int par0, int done) {
        return iterate<K>(slot, 2, 4, budget[slot], [&](int par) {
            CLOT_LAUNCH(pa, (k_cg_a<T, K, Op>), dim3(ntiles), dim3(NT), 0, st, grid(), op, V, S, par);
            finish<K>(EpiCgA<K>{});
            CLOT_LAUNCH(pb, (k_cg_b<T, K, Op>), dim3(ntiles), dim3(NT), 0, st, grid(), op, V, S, par);
            finish<2 * K>(EpiCgB<K>{});
        }, par0, done);
    }

    // ---------------------------------------------------------------------------
    // The eta solve depends only on theta_B of the step's start: eagerly it runs on a
    // second stream, concurrently with the flow and transport solves, for a fixed
    // number of iterations (converged channels skip the rest); the main stream joins
    // it before the transport solve, whose first poll also brings back the count of
    // channels still iterating, and a solve that needs more iterations finishes on
    // the main stream with the usual polls.
    KVec<T, 1> eta_vecs() {
        KVec<T, 1> V{};
        V.x[0] = F.eta;
        V.b[0] = eta_v[0];
        V.r[0] = eta_v[1];
        V.rh[0] = eta_v[1];
        V.p[0][0] = eta_v[2];
        V.p[1][0] = eta_v[3];
        V.v[0][0] = eta_v[2];
        V.v[1][0] = eta_v[3];
        V.t[0] = eta_v[4];
        return V;
    }
    EtaOp<T> eta_op() const { return EtaOp<T>{T(M.kappa_eta), F.dE}; }
    void eta_start() {
        hipLaunchKernelGGL(k_eta_prep<T>, dim3(ntiles), dim3(NT), 0, st, grid(), F, M, eta_v[0]);
        EtaOp<T> eop = eta_op();
        KVec<T, 1> V = eta_vecs();
        set_active(allmask);
        hipLaunchKernelGGL((k_cg_init<T, 1, EtaOp<T>>), dim3(ntiles), dim3(NT), 0, st, grid(), eop, V, S);
        finish<3>(EpiCgInit<1>{prm.rtol_s, 0});
    }
    void side_swap() {
        std::swap(S, Se);
        std::swap(st, st2);
    }
    clot_status eta_side_launch() {
        if (!st2) {
            HIPCHK(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&ev_derive, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&ev_eta, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&ev_info, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&ev_asm, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&ev_mg, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(ev_derive, st));
        HIPCHK(hipStreamWaitEvent(st2, ev_derive, 0));
        side_swap();
        eta_start();
        fixed_iters = eta_budget;
        cg_iterations<EtaOp<T>, 1>(eta_op(), eta_vecs(), 4, CLOT_PROBE_ETA_CG_A, CLOT_PROBE_ETA_CG_B, 0, 0);
        fixed_iters = 0;
        hipLaunchKernelGGL(k_solve_info, dim3(1), dim3(64), 0, st, S.sc, S.nact, (int)ch.size(), eta_info);
        side_swap();
        HIPCHK(hipEventRecord(ev_eta, st2));
        return CLOT_OK;
    }
    clot_status eta_side_join() {
        HIPCHK(hipStreamWaitEvent(st, ev_eta, 0));
        HIPCHK(hipMemcpyAsync(h_nact + 4, eta_info, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(ev_info, st));
        return CLOT_OK;
    }
    // after a poll of the main stream: finish the eta solve if its budget fell short
    clot_status eta_side_finish() {
        HIPCHK(hipEventSynchronize(ev_info));   // already complete after the transport solve's polls
        const int32_t still = h_nact[4], its = h_nact[5];
        int total = its;
        if (still > 0) {
            std::swap(S, Se);
            total = eta_budget + cg_iterations<EtaOp<T>, 1>(eta_op(), eta_vecs(), 4, CLOT_PROBE_ETA_CG_A,
                                                            CLOT_PROBE_ETA_CG_B, eta_budget & 1, eta_budget);
            std::swap(S, Se);
            eta_budget = std::min(prm.max_iter, 2 * eta_budget);
        } else {
            eta_budget = std::min(prm.max_iter, std::max(8, (int)std::ceil(1.25 * its) + 4));
        }
        it_max[4] = std::max(it_max[4], total);   // for graph budgets
        hipLaunchKernelGGL(k_record, dim3(1), dim3(64), 0, st, Se.sc, dstats, NSTAT, (int)ch.size(), 1, (int)ST_ETA,
                           (int)ST_RESE, (int)ST_FAIL, 0, (const int32_t*)nullptr, -1);
        return CLOT_OK;
    }

    template <class Op, int K>
    int run_bicg(const Op& op, KVec<T, K> V, double rtol, const int32_t* mask, int slot, int p1) {
        set_active(mask);
        hipLaunchKernelGGL((k_bicg_init<T, K, Op, true>), dim3(ntiles, K), dim3(NT), 0, st, grid(), op, V, S);
        finish<3 * K>(EpiBicgInit<K>{rtol});
        // past the first chunk, one iteration per poll: an iteration run after every
        // channel has converged costs more launches than the poll it saves
        return iterate<K>(slot, 1, 1, budget[slot], [&](int par) {
            CLOT_LAUNCH(p1, (k_bicg_1<T, K, Op>), dim3(ntiles, K), dim3(NT), 0, st, grid(), op, V, S, par);
            finish<K>(EpiBicg1<K>{});
            CLOT_LAUNCH(p1 + 1, (k_bicg_2<T, K, Op>), dim3(ntiles, K), dim3(NT), 0, st, grid(), op, V, S, par);
            finish<2 * K>(EpiBicg2<K>{});
            CLOT_LAUNCH(p1 + 2, (k_bicg_3<T, K, Op>), dim3(ntiles, K), dim3(NT), 0, st, grid(), op, V, S, par);
            finish<2 * K>(EpiBicg3<K>{});
        });
    }

    template <int NV, class E>
    void finish(const E& e) {
        hipLaunchKernelGGL((k_finish<NV, E>), dim3((int)ch.size(), FinSplit<NV>::G), dim3(FIN_BS), 0, st, d_ch, S, e);
    }

    // Pressure preconditioner setup: coarse operators from the current rAU.
    void mg_setup() {
        FineCoefPres<T> fp{F.rAU};
        for (size_t l = 0; l < lev.size(); ++l) {
            Level& L = lev[l];
            MGPair pr{l == 0 ? grid() : lev[l - 1].grid(), L.grid()};
            if (l == 0) {
                FineCoefLevel<T> fl{nullptr, nullptr, nullptr, nullptr};
                hipLaunchKernelGGL((k_mg_setup<T, true>), dim3(L.ntiles), dim3(NT), 0, st, pr, fp, fl, L.cx, L.cy, L.cz,
                                   L.cout, L.dg);
            } else {
                const Level& Fl = lev[l - 1];
                FineCoefLevel<T> fl{Fl.cx, Fl.cy, Fl.cz, Fl.cout};
                hipLaunchKernelGGL((k_mg_setup<T, false>), dim3(L.ntiles), dim3(NT), 0, st, pr, fp, fl, L.cx, L.cy,
                                   L.cz, L.cout, L.dg);
            }
        }
        if (!lev.empty()) {
            Level& Lc = lev.back();
            CoefOp<T> op{Lc.dg, Lc.cx, Lc.cy, Lc.cz};
            hipLaunchKernelGGL(k_mg_coarse_setup<T>, dim3((int)ch.size()), dim3(MG_COARSE), 0, st, Lc.grid(), op, mg_inv,
                               (int)ch.size());
        }
    }

    // z = M r on level 0 (V-cycle); the last kernel also forms r.z and beta.
    void vcycle(const T* r) {
        const int nl = (int)lev.size();
        PresOp<T, T> p0{F.rAU, F.dP};
        const int32_t* act = S.chact;
        if (nl == 0) {   // mesh already coarse: two Jacobi sweeps
            hipLaunchKernelGGL((k_mg_pre<T, PresOp<T, T>>), dim3(ntiles), dim3(NT), 0, st, grid(), p0, r, mg_y0, mg_w, act);
            hipLaunchKernelGGL((k_mg_post2<T, PresOp<T, T>, true>), dim3(ntiles), dim3(NT), 0, st, grid(), p0, r, mg_y0,
                               mg_z0, mg_w, S);
            finish<1>(EpiMgDot{});
            return;
        }
        const int t0 = mg_t0 >= 0 ? mg_t0 : nl - 1;   // levels from t0 on: fused launch or coarse solve
        auto tail_or_coarse = [&]() {
            if (mg_t0 >= 0) {
                MGTail<T> tl{};
                tl.n = nl - t0;
                for (int l = t0; l < nl; ++l) {
                    Level& L = lev[l];
                    tl.L[l - t0] = MGTailLevel<T>{L.x, L.y, L.b, L.dg, L.cx, L.cy, L.cz, L.cout};
                }
                hipLaunchKernelGGL(k_mg_tail<T>, dim3((int)ch.size()), dim3(MG_TAIL_BS), mg_tail_lds, st, tl,
                                   (const TailPlan*)d_tplan, mg_w, mg_inv,
                                   act, (int)prm.mg_sweeps);
            } else {
                Level& Lc = lev[nl - 1];
                hipLaunchKernelGGL(k_mg_coarse<T>, dim3((int)ch.size()), dim3(MG_COARSE), 0, st, Lc.grid(), mg_inv, Lc.b,
                                   Lc.x, act, (int)ch.size());
            }
        };
        if (prm.mg_sweeps == 1) {
            // one sweep each way: the pre-sweep from zero is formed inside the restriction
            hipLaunchKernelGGL((k_mg_restrict<T, PresOp<T, T>, true>), dim3(lev[0].ntiles * (TILE / (NT / 8))), dim3(NT),
                               0, st, MGPair{grid(), lev[0].grid()}, p0, r, (const T*)nullptr, lev[0].b, act, mg_w);
            for (int l = 0; l < t0; ++l) {
                Level& L = lev[l];
                CoefOp<T> op{L.dg, L.cx, L.cy, L.cz};
                hipLaunchKernelGGL((k_mg_restrict<T, CoefOp<T>, true>), dim3(lev[l + 1].ntiles * (TILE / (NT / 8))),
                                   dim3(NT), 0, st, MGPair{L.grid(), lev[l + 1].grid()}, op, L.b, (const T*)nullptr,
                                   lev[l + 1].b, act, mg_w);
            }
            tail_or_coarse();
            for (int l = t0 - 1; l >= 0; --l) {
                Level& L = lev[l];
                CoefOp<T> op{L.dg, L.cx, L.cy, L.cz};
                hipLaunchKernelGGL((k_mg_post_one<T, CoefOp<T>, false>), dim3(L.ntiles), dim3(NT), 0, st,
                                   MGPair{L.grid(), lev[l + 1].grid()}, op, L.b, lev[l + 1].x, L.x, mg_w, S);
            }
            CLOT_LAUNCH(CLOT_PROBE_P_MG_POST, (k_mg_post_one<T, PresOp<T, T>, true>), dim3(ntiles), dim3(NT), 0, st,
                        MGPair{grid(), lev[0].grid()}, p0, r, lev[0].x, mg_z0, mg_w, S);
            finish<1>(EpiMgDot{});
            return;
        }
        // n >= 2 sweeps each way on a level with buffers X (where its result must end) and
        // Y: k_mg_pre forms the first two from zero in X, further ones alternate X -> Y ->
        // X ...; the restriction reads the last.  Up: the prolonged correction enters the
        // first sweep (k_mg_post1, into the buffer the pre-smoothing did not end in), the
        // others alternate and the last lands in X (on the finest level it also forms r.z).
        const int ns = prm.mg_sweeps;
        auto down = [&](auto op, const T* b, T* X, T* Y, const Grid& g, int nt) -> T* {
            hipLaunchKernelGGL((k_mg_pre<T, decltype(op)>), dim3(nt), dim3(NT), 0, st, g, op, b, X, mg_w, act);
            T* cur = X;
            for (int k = 2; k < ns; ++k) {
                T* nxt = cur == X ? Y : X;
                hipLaunchKernelGGL((k_mg_post2<T, decltype(op), false>), dim3(nt), dim3(NT), 0, st, g, op, b,
                                   (const T*)cur, nxt, mg_w, S);
                cur = nxt;
            }
            return cur;
        };
        // the up-sweeps after k_mg_post1 (which wrote `cur`); the last one into X
        auto up_rest = [&](auto op, const T* b, T* X, T* Y, T* cur, const Grid& g, int nt, bool finest) {
            for (int k = 1; k < ns; ++k) {
                T* nxt = cur == X ? Y : X;
                if (finest && k + 1 == ns)
                    CLOT_LAUNCH(CLOT_PROBE_P_MG_POST, (k_mg_post2<T, decltype(op), true>), dim3(nt), dim3(NT), 0, st, g,
                                op, b, (const T*)cur, nxt, mg_w, S);
                else
                    hipLaunchKernelGGL((k_mg_post2<T, decltype(op), false>), dim3(nt), dim3(NT), 0, st, g, op, b,
                                       (const T*)cur, nxt, mg_w, S);
                cur = nxt;
            }
        };
        // down (a bricked level leaves its smoothed iterate in Y for its up leg; the mesh's
        // fused leg ends where the separate launches do, three sweeps in Y and two in X,
        // except before a fused up leg, which needs its input apart from its output: X)
        T* s0 = nullptr;
        const BrickGrid mdg{d_p3br, d_p3b2c, (int32_t)h_p3b2c.size()};
        const MGPair m0{grid(), lev[0].grid()};
        if (mesh_down_n == 3) {
            s0 = mesh_up2 ? mg_z0 : mg_y0;
            CLOT_LAUNCH(CLOT_PROBE_P_MG_MESH_DOWN, (k_mg_mesh_leg<T, MESH_DOWN3>), dim3((unsigned)h_p3b2c.size()),
                        dim3(MGB_BS), mesh_down_lds(), st, mdg, m0, p0, r, (const T*)nullptr, (const T*)nullptr, s0,
                        (T*)nullptr, mg_w, act);
        } else if (mesh_down_n == 2) {
            s0 = mg_z0;
            CLOT_LAUNCH(CLOT_PROBE_P_MG_MESH_DOWN, (k_mg_mesh_leg<T, MESH_DOWN2R>), dim3((unsigned)h_p3b2c.size()),
                        dim3(MGB_BS), mesh_down_lds(), st, mdg, m0, p0, r, (const T*)nullptr, (const T*)nullptr, s0,
                        lev[0].b, mg_w, act);
        } else {
            s0 = down(p0, r, mg_z0, mg_y0, grid(), (int)ntiles);
        }
        if (mesh_down_n != 2) {   // (the two-sweep fused leg restricts too)
            if (mesh_halves())
                hipLaunchKernelGGL(k_mg_restrict_mesh<T>, dim3((unsigned)h_rb2c.size()), dim3(NT), 0, st,
                                   BrickGrid{d_rbr, d_rb2c, (int32_t)h_rb2c.size()}, MGPair{grid(), lev[0].grid()}, p0,
                                   r, (const T*)s0, lev[0].b, act);
            else
                hipLaunchKernelGGL((k_mg_restrict<T, PresOp<T, T>, false>), dim3(lev[0].ntiles * (TILE / (NT / 8))),
                                   dim3(NT), 0, st, MGPair{grid(), lev[0].grid()}, p0, r, (const T*)s0, lev[0].b, act,
                                   mg_w);
        }
        T* pre_end[MG_MAXLEV];
        for (int l = 0; l < t0; ++l) {
            Level& L = lev[l];
            CoefOp<T> op{L.dg, L.cx, L.cy, L.cz};
            if (pbricked(l + 1)) {
                mgb_launch<MGB_DOWN>(l + 1, CLOT_PROBE_P_MG_DOWN, MGPair{L.grid(), lev[l + 1].grid()}, op, L.b, nullptr,
                                     nullptr, L.y, lev[l + 1].b);
                pre_end[l] = L.y;
                continue;
            }
            pre_end[l] = down(op, (const T*)L.b, L.x, L.y, L.grid(), (int)L.ntiles);
            hipLaunchKernelGGL((k_mg_restrict<T, CoefOp<T>, false>), dim3(lev[l + 1].ntiles * (TILE / (NT / 8))), dim3(NT),
                               0, st, MGPair{L.grid(), lev[l + 1].grid()}, op, L.b, (const T*)pre_end[l], lev[l + 1].b,
                               act, mg_w);
        }
        tail_or_coarse();
        // up
        for (int l = t0 - 1; l >= 0; --l) {
            Level& L = lev[l];
            CoefOp<T> op{L.dg, L.cx, L.cy, L.cz};
            if (pbricked(l + 1)) {
                mgb_launch<MGB_UP>(l + 1, CLOT_PROBE_P_MG_UP, MGPair{L.grid(), lev[l + 1].grid()}, op, L.b, pre_end[l],
                                   lev[l + 1].x, L.x, nullptr);
                continue;
            }
            T* o1 = pre_end[l] == L.x ? L.y : L.x;
            hipLaunchKernelGGL((k_mg_post1<T, CoefOp<T>>), dim3(L.ntiles), dim3(NT), 0, st, MGPair{L.grid(), lev[l + 1].grid()},
                               op, L.b, (const T*)pre_end[l], lev[l + 1].x, o1, mg_w, act);
            up_rest(op, (const T*)L.b, L.x, L.y, o1, L.grid(), (int)L.ntiles, false);
        }
        if (mesh_up2) {
            // prolongation and the first two up sweeps in one launch (X -> Y), then the last
            // sweep with r.z (Y -> X)
            CLOT_LAUNCH(CLOT_PROBE_P_MG_MESH_UP, (k_mg_mesh_leg<T, MESH_UP2>), dim3((unsigned)h_p3b2c.size()),
                        dim3(MGB_BS), mesh_down_lds(), st, BrickGrid{d_p3br, d_p3b2c, (int32_t)h_p3b2c.size()},
                        MGPair{grid(), lev[0].grid()}, p0, r, (const T*)s0, (const T*)lev[0].x, mg_y0, (T*)nullptr,
                        mg_w, act);
            CLOT_LAUNCH(CLOT_PROBE_P_MG_POST, (k_mg_post2<T, PresOp<T, T>, true>), dim3(ntiles), dim3(NT), 0, st, grid(),
                        p0, r, (const T*)mg_y0, mg_z0, mg_w, S);
            finish<1>(EpiMgDot{});
            return;
        }
        T* o1 = s0 == mg_z0 ? mg_y0 : mg_z0;
        if (mesh_halves())
            hipLaunchKernelGGL(k_mg_post1_mesh<T>, dim3(ntiles), dim3(NT), 0, st, MGPair{grid(), lev[0].grid()}, p0, r,
                               (const T*)s0, lev[0].x, o1, mg_w, act);
        else
            hipLaunchKernelGGL((k_mg_post1<T, PresOp<T, T>>), dim3(ntiles), dim3(NT), 0, st, MGPair{grid(), lev[0].grid()},
                               p0, r, (const T*)s0, lev[0].x, o1, mg_w, act);
        up_rest(p0, r, mg_z0, mg_y0, o1, grid(), (int)ntiles, true);
        finish<1>(EpiMgDot{});
    }

    // One LDS-staged leg of the pressure V-cycle on the coarse level of brick table j, in
    // the brick shape chosen for that leg.
    template <int MODE>
    void mgb_launch(int j, int probe, const MGPair& pr, const CoefOp<T>& op, const T* b, const T* xin, const T* xc,
                    T* xout, T* bc) {
        const int q = brick_shape[MODE == MGB_DOWN ? CLOT_BRICK_P_DOWN : CLOT_BRICK_P_UP];
        const dim3 gd((unsigned)h_pb2c[q][j].size());
        const int h = prm.mg_sweeps;
        const size_t lds = mgb_lds_bytes(h, q, sizeof(T));
        const BrickGrid bg = pbricks(q, j);
        const int32_t* act = S.chact;
#define CLOT_MGB(H, Q)                                                                                              \
    CLOT_LAUNCH(probe, (k_mg_brick<T, MODE, H, Q>), gd, dim3(MGB_BS), lds, st, bg, pr, op, b, xin, xc, xout, bc, mg_w, \
                act)
        switch (h * 4 + q) {
            case 8: CLOT_MGB(2, 0); break;
            case 9: CLOT_MGB(2, 1); break;
            case 10: CLOT_MGB(2, 2); break;
            case 11: CLOT_MGB(2, 3); break;
            case 12: CLOT_MGB(3, 0); break;
            case 13: CLOT_MGB(3, 1); break;
            case 14: CLOT_MGB(3, 2); break;
            default: CLOT_MGB(3, 3); break;
        }
#undef CLOT_MGB
    }

    // Multigrid-preconditioned CG on the pressure correction.
    int run_mgcg(KVec<T, 1> V, double rtol, int tol_mode, const int32_t* mask, int slot, int pass) {
        PresOp<T, T> pop{F.rAU, F.dP};
        set_active(mask);
        hipLaunchKernelGGL((k_mgcg_init<T, PresOp<T, T>>), dim3(ntiles), dim3(NT), 0, st, grid(), pop, V, S);
        finish<2>(EpiMgcgInit{rtol, tol_mode});
        vcycle(V.r[0]);
        const int ps = std::min(pass, 11);
        const int it = iterate<1>(slot, 1, 2, pbudget[slot - 1][ps], [&](int par) {
            CLOT_LAUNCH(CLOT_PROBE_P_CG_A, (k_mgcg_a<T, PresOp<T, T>>), dim3(ntiles), dim3(NT), 0, st, grid(), pop, V,
                        mg_z0, S, par);
            finish<1>(EpiCgA<1>{});
            CLOT_LAUNCH(CLOT_PROBE_P_CG_B, (k_mgcg_b<T, PresOp<T, T>>), dim3(ntiles), dim3(NT), 0, st, grid(), pop, V,
                        S, par);
            finish<1>(EpiMgcgB{});
            vcycle(V.r[0]);
        });
        if (!capturing) it_pmax[slot - 1][ps] = std::max(it_pmax[slot - 1][ps], it);
        return it;
    }

    // ---- momentum predictor: BiCGStab preconditioned by a V-cycle (clot_mgm.h) ----
    // Coarse operators of the momentum preconditioner: from the mesh's mass (theta_B,
    // the channel's dt) and viscous couplings, then level by level.
    void mgm_setup() {
        for (int l = 0; l < mgm_nc; ++l) {
            Level& L = lev[l];
            if (l == 0)
                hipLaunchKernelGGL((k_mgm_setup<T, true>), dim3(L.ntiles), dim3(NT), 0, st, MGPair{grid(), L.grid()}, M,
                                   (const T*)F.thB, (const T*)nullptr, (const T*)nullptr, (const T*)nullptr,
                                   (const T*)nullptr, L.mmass, L.mdg, L.mcx, L.mcy, L.mcz);
            else {
                const Level& Fl = lev[l - 1];
                hipLaunchKernelGGL((k_mgm_setup<T, false>), dim3(L.ntiles), dim3(NT), 0, st,
                                   MGPair{Fl.grid(), L.grid()}, M, (const T*)nullptr, (const T*)Fl.mmass,
                                   (const T*)Fl.mcx, (const T*)Fl.mcy, (const T*)Fl.mcz, L.mmass, L.mdg, L.mcx, L.mcy,
                                   L.mcz);
            }
        }
    }
    static MGCVec<T> cv3(T* const (&v)[MGM_K]) { return MGCVec<T>{{v[0], v[1], v[2]}}; }
    static MGVec<T> mv3(T* const (&v)[MGM_K]) { return MGVec<T>{{v[0], v[1], v[2]}}; }
    // scratch vectors of the momentum solve (the transport solve's, unused until then):
    // 0..2 y = M^-1 p, 3..5 z = M^-1 s, 6..8 s, 9..11 and 12..14 finest-level sweeps
    T* const (&mgm_vec(int q) const)[MGM_K] { return *reinterpret_cast<T* const(*)[MGM_K]>(pool + 7 + 7 * 3 + 3 * q); }

    // A bricked finest-level momentum kernel in the shape chosen for it.
    template <int MODE, int FORM>
    void brick_launch(int probe, const MomOp<T>& mop, const MGSrc<T>& src, const MGVec<T>& bout, const MGCVec<T>& xc,
                      const MGVec<T>& out) {
        const int kid = MODE == MGM_MODE_R ? 0 : MODE == MGM_MODE_P ? 1 : 2;
        const int q = brick_shape[kid];
        const MGPair pr{grid(), lev[0].grid()};
        const dim3 gd((unsigned)h_b2c[q].size());
        switch (q) {
            case 0:
                CLOT_LAUNCH(probe, (k_mgm_brick<T, MODE, FORM, 0>), gd, dim3(NT), 0, st, bricks(0), pr, mop, src, bout,
                            xc, out, S, mg_w);
                break;
            case 1:
                CLOT_LAUNCH(probe, (k_mgm_brick<T, MODE, FORM, 1>), gd, dim3(NT), 0, st, bricks(1), pr, mop, src, bout,
                            xc, out, S, mg_w);
                break;
            case 2:
                CLOT_LAUNCH(probe, (k_mgm_brick<T, MODE, FORM, 2>), gd, dim3(NT), 0, st, bricks(2), pr, mop, src, bout,
                            xc, out, S, mg_w);
                break;
            default:
                CLOT_LAUNCH(probe, (k_mgm_brick<T, MODE, FORM, 3>), gd, dim3(NT), 0, st, bricks(3), pr, mop, src, bout,
                            xc, out, S, mg_w);
                break;
        }
    }

    // out = M^-1 b (one V(1,2) cycle) for the active components; FORM (clot_mgm.h) says
    // how the finest right-hand side is formed; a formed one is written to bout.
    template <int FORM>
    void vcycle_mom(const MomOp<T>& mop, const MGSrc<T>& src, T* const (&bout)[MGM_K], T* const (&out)[MGM_K]) {
        const int nc = mgm_nc;
        const unsigned rb = TILE / (NT / 8);   // restriction blocks per coarse tile
        const MGCVec<T> none{};
        const bool brick = bricked();
        if (brick)
            brick_launch<MGM_MODE_R, FORM>(CLOT_PROBE_MOM_MG_R, mop, src, mv3(bout), none, mv3(lev[0].mb));
        else
            CLOT_LAUNCH(CLOT_PROBE_MOM_MG_R, (k_mgm_restrict<T, MomOp<T>, FORM, true>), dim3(lev[0].ntiles * rb),
                        dim3(NT), 0, st, MGPair{grid(), lev[0].grid()}, mop, src, mv3(bout), none, mv3(lev[0].mb), S,
                        mg_w, MGGate{});
        // a channel's coarsest level: two Jacobi sweeps from zero (the mass dominates there)
        auto coarsest = [&](int l) {
            bool any = false;
            for (int32_t q : h_mgm_last) any = any || q == l;
            if (!any) return;
            Level& L = lev[l];
            hipLaunchKernelGGL((k_mgm_pre<T, CoefOp<T>>), dim3(L.ntiles), dim3(NT), 0, st, L.grid(), L.mom_op(),
                               cv3(L.mb), mv3(L.mx), mg_w, S, MGGate{d_mgm_last, l, 1});
        };
        for (int l = 0; l + 1 < nc; ++l) {
            Level& L = lev[l];
            coarsest(l);
            MGSrc<T> sl{};
            for (int k = 0; k < MGM_K; ++k) sl.b[k] = L.mb[k];
            hipLaunchKernelGGL((k_mgm_restrict<T, CoefOp<T>, 0, true>), dim3(lev[l + 1].ntiles * rb), dim3(NT), 0, st,
                               MGPair{L.grid(), lev[l + 1].grid()}, L.mom_op(), sl, MGVec<T>{}, none,
                               mv3(lev[l + 1].mb), S, mg_w, MGGate{d_mgm_last, l, 0});
        }
        coarsest(nc - 1);
        for (int l = nc - 2; l >= 0; --l) {
            Level& L = lev[l];
            const MGGate up{d_mgm_last, l, 0};
            hipLaunchKernelGGL((k_mgm_post1<T, CoefOp<T>>), dim3(L.ntiles), dim3(NT), 0, st,
                               MGPair{L.grid(), lev[l + 1].grid()}, L.mom_op(), cv3(L.mb), cv3(lev[l + 1].mx),
                               mv3(L.my), mg_w, S, up);
            hipLaunchKernelGGL((k_mgm_post2<T, CoefOp<T>>), dim3(L.ntiles), dim3(NT), 0, st, L.grid(), L.mom_op(),
                               cv3(L.mb), cv3(L.my), mv3(L.mx), mg_w, S, up);
        }
        const MGCVec<T> bf = FORM == 0 ? MGCVec<T>{{src.b[0], src.b[1], src.b[2]}} : cv3(bout);
        if (brick) {
            MGSrc<T> sb{};
            for (int k = 0; k < MGM_K; ++k) sb.b[k] = bf.v[k];
            brick_launch<MGM_MODE_P, 0>(CLOT_PROBE_MOM_MG_P1, mop, sb, MGVec<T>{}, cv3(lev[0].mx), mv3(mgm_vec(3)));
            brick_launch<MGM_MODE_S, 0>(CLOT_PROBE_MOM_MG_P2, mop, sb, MGVec<T>{}, cv3(mgm_vec(3)), mv3(out));
        } else {
            CLOT_LAUNCH(CLOT_PROBE_MOM_MG_P1, (k_mgm_post1<T, MomOp<T>>), dim3(ntiles), dim3(NT), 0, st,
                        MGPair{grid(), lev[0].grid()}, mop, bf, cv3(lev[0].mx), mv3(mgm_vec(3)), mg_w, S, MGGate{});
            CLOT_LAUNCH(CLOT_PROBE_MOM_MG_P2, (k_mgm_post2<T, MomOp<T>>), dim3(ntiles), dim3(NT), 0, st, grid(), mop,
                        bf, cv3(mgm_vec(3)), mv3(out), mg_w, S, MGGate{});
        }
    }

    // BiCGStab on the momentum system with one V-cycle per direction (right
    // preconditioning): y = M^-1 p, v = A y, s = r - alpha v, z = M^-1 s, t = A z,
    // x += alpha y + omega z, r = s - omega t; the recurrence scalars are those of the
    // Jacobi-preconditioned solve.
    int run_mom_mg(const MomOp<T>& mop, KVec<T, 3> V, double rtol) {
        set_active(allmask);
        hipLaunchKernelGGL((k_bicg_init<T, 3, MomOp<T>>), dim3(ntiles, 3), dim3(NT), 0, st, grid(), mop, V, S);
        finish<9>(EpiBicgInit<3>{rtol});
        T* const (&Y)[MGM_K] = mgm_vec(0);
        T* const (&Z)[MGM_K] = mgm_vec(1);
        T* const (&Sv)[MGM_K] = mgm_vec(2);
        // one iteration per poll past the first chunk, as in run_bicg
        return iterate<3>(0, 1, 1, budget[0], [&](int par) {
            MGSrc<T> s1{};
            for (int k = 0; k < MGM_K; ++k) {
                s1.r[k] = V.r[k];
                s1.p[k] = V.p[par][k];
                s1.v[k] = V.v[par][k];
            }
            T* pn[MGM_K] = {V.p[par ^ 1][0], V.p[par ^ 1][1], V.p[par ^ 1][2]};
            vcycle_mom<1>(mop, s1, pn, Y);
            CLOT_LAUNCH(CLOT_PROBE_MOM_B1, (k_pbicg_1<T, 3, MomOp<T>>), dim3(ntiles, 3), dim3(NT), 0, st, grid(), mop, V,
                        cv3(Y), S, par);
            finish<3>(EpiBicg1<3>{});
            MGSrc<T> s2{};
            for (int k = 0; k < MGM_K; ++k) {
                s2.r[k] = V.r[k];
                s2.v[k] = V.v[par ^ 1][k];
            }
            vcycle_mom<2>(mop, s2, Sv, Z);
            CLOT_LAUNCH(CLOT_PROBE_MOM_B2, (k_pbicg_2<T, 3, MomOp<T>>), dim3(ntiles, 3), dim3(NT), 0, st, grid(), mop, V,
                        cv3(Z), cv3(Sv), S);
            finish<6>(EpiBicg2<3>{});
            CLOT_LAUNCH(CLOT_PROBE_MOM_B3, (k_pbicg_3<T, 3>), dim3(ntiles, 3), dim3(NT), 0, st, grid(), V, cv3(Y), cv3(Z),
                        cv3(Sv), S);
            finish<6>(EpiBicg3<3>{});
        });
    }

    template <int K>
    KVec<T, K> bicg_vecs(int first) {
        KVec<T, K> V{};
        for (int k = 0; k < K; ++k) {
            T** b = pool + 7 + 7 * (first + k);
            V.r[k] = b[0];
            V.rh[k] = b[1];
            V.p[0][k] = b[2];
            V.p[1][k] = b[3];
            V.v[0][k] = b[4];
            V.v[1][k] = b[5];
            V.t[k] = b[6];
        }
        return V;
    }
    KVec<T, 1> cg_vecs(T* x, const T* b) {
        KVec<T, 1> V{};
        V.x[0] = x;
        V.b[0] = b;
        V.r[0] = pool[1];
        V.rh[0] = pool[1];
        V.p[0][0] = pool[2];
        V.p[1][0] = pool[3];
        V.v[0][0] = pool[2];
        V.v[1][0] = pool[3];
        V.t[0] = pool[4];
        return V;
    }

    void record(int slot_it, int slot_res, int K, bool add, const int32_t* mask = nullptr, int slot_sum = -1) {
        hipLaunchKernelGGL(k_record, dim3(1), dim3(64), 0, st, S.sc, dstats, NSTAT, (int)ch.size(), K, slot_it, slot_res,
                           (int)ST_FAIL, add ? 1 : 0, mask, slot_sum);
    }

    // ---------------------------------------------------------------------------
    clot_status one_step() {
        const Grid G = grid();
        const dim3 gb(ntiles), tb(NT);
        const int nch = (int)ch.size();
        // O-0 derived coefficients
        hipLaunchKernelGGL(k_derive<T>, gb, tb, 0, st, G, F, M);
        // O-3 eta (needs only theta_B): on the side stream when not recording a graph
        const bool eta_side = !capturing;
        if (eta_side) {
            const clot_status r = eta_side_launch();
            if (r < 0) return r;
        }
        // O-1 momentum predictor
        CLOT_LAUNCH(CLOT_PROBE_MOM_ASM, k_mom_assemble<T>, gb, tb, 0, st, G, F, M);
        mgm_setup();
        // the pressure preconditioner depends only on rAU: built once per step, on the
        // side stream (behind eta) while the momentum predictor is solved
        if (eta_side) {
            HIPCHK(hipEventRecord(ev_asm, st));
            HIPCHK(hipStreamWaitEvent(st2, ev_asm, 0));
            std::swap(st, st2);
            mg_setup();
            std::swap(st, st2);
            HIPCHK(hipEventRecord(ev_mg, st2));
        } else {
            mg_setup();
        }
        MomOp<T> mop{F.aP, F.phi[0], F.phi[1], F.phi[2], T(prm.nu)};
        {
            KVec<T, 3> V = bicg_vecs<3>(0);
            for (int c = 0; c < 3; ++c) {
                V.x[c] = F.u[c];
                V.b[c] = F.bm[c];
            }
            if (mgm_nc > 0) run_mom_mg(mop, V, prm.rtol_s);
            else run_bicg<MomOp<T>, 3>(mop, V, prm.rtol_s, allmask, 0, CLOT_PROBE_MOM_B1);
            record(ST_MOM, ST_RESM, 3, false);
        }
        // O-2 PISO correctors
        for (int k = 0; k < maxcorr; ++k) {
            const int32_t* cm = corrmask + (size_t)k * nch;
            CLOT_LAUNCH(CLOT_PROBE_HBYA, k_hbya<T>, gb, tb, 0, st, G, F, mop, cm);
            CLOT_LAUNCH(CLOT_PROBE_PRHS, k_prhs<T>, gb, tb, 0, st, G, F, M, cm);
            if (k == 0 && eta_side) HIPCHK(hipStreamWaitEvent(st, ev_mg, 0));
            // FP64 iterative refinement around a T-precision MG-PCG
            set_active(cm, true);    // with the count of active channels for the residual kernel
            T* e = pool[5];
            T* rin = pool[0];
            PresOp<T, T> pop{F.rAU, F.dP};
            const int npass = capturing ? budget[6] : 12;
            for (int pass = 0; pass < npass; ++pass) {
                CLOT_LAUNCH(CLOT_PROBE_P_RESID, k_pres_resid<T>, gb, tb, 0, st, G, F, rin, e, S);
                finish<2>(EpiPresResid{prm.rtol_p, prec == CLOT_FP64 ? 0.0 : prm.rtol_inner, pass, refmask});
                if (!capturing) {
                    it_max[6] = std::max(it_max[6], pass);
                    if (poll() == 0) break;
                }
                KVec<T, 1> V = cg_vecs(e, rin);
                run_mgcg(V, 0.0, 1, refmask, 1 + std::min(k, 2), pass);
                record(ST_P + std::min(k, MAXCORR - 1), ST_RESP, 1, pass > 0, refmask);
                hipLaunchKernelGGL(k_pres_add<T>, gb, tb, 0, st, G, F, e, refmask);
                set_active(refmask, true);
            }
            if (capturing) {   // a channel still needing refinement after the last pass
                CLOT_LAUNCH(CLOT_PROBE_P_RESID, k_pres_resid<T>, gb, tb, 0, st, G, F, rin, e, S);
                finish<2>(EpiPresResid{prm.rtol_p, prec == CLOT_FP64 ? 0.0 : prm.rtol_inner, npass, refmask});
                hipLaunchKernelGGL(k_flag_active, dim3(1), dim3(64), 0, st, refmask, S.sc, nch, 1, gflag);
            }
            hipLaunchKernelGGL(k_record_pass, dim3(1), dim3(64), 0, st, S.sc, dstats, NSTAT, nch,
                               ST_REF + std::min(k, MAXCORR - 1), ST_RESP, (int)ST_FAIL);
            CLOT_LAUNCH(CLOT_PROBE_CORRECT, k_correct<T>, gb, tb, 0, st, G, F, M, cm);
        }
        // O-3 eta
        if (!eta_side) {
            eta_start();
            cg_iterations<EtaOp<T>, 1>(eta_op(), eta_vecs(), 4, CLOT_PROBE_ETA_CG_A, CLOT_PROBE_ETA_CG_B, 0, 0);
            record(ST_ETA, ST_RESE, 1, false);
        }
        // O-4 sigma
        hipLaunchKernelGGL(k_sigma_sched, dim3(1), dim3(64), 0, st, d_ch, sig, nch, M, sigw, push);
        hipLaunchKernelGGL(k_sigma<T>, gb, tb, 0, st, G, F, M, sigw, push);
        // O-5 transport
        TrOp<T> top;
        for (int k = 0; k < NTR; ++k) {
            top.Cn[k] = F.spc[tr_species(k)];
            top.dg[k] = F.trd[k];
            top.dg64[k] = F.trd64[k];
            top.b64[k] = F.trb[k];
            top.Cl[k] = F.lo[tr_species(k)];
            top.cf[k] = F.trc[k];
            const int sp = tr_species(k);
            top.scale[k] = T(sp == PMU || sp == PMA ? M.P_max
                             : sp == S1 || sp == E1 ? M.S1_0
                             : sp == S2 || sp == E2 || sp == E2I ? M.S2_0
                             : sp == INH ? M.I_0 : M.adp_crit);
            top.Dk[k] = tr_diffusivity<T>(k, M);
        }
        top.phx = F.phin[0];
        top.phy = F.phin[1];
        top.phz = F.phin[2];
        top.Wc = F.Wc;
        top.Pmax = T(M.P_max);
        top.n = N;
        CLOT_LAUNCH(CLOT_PROBE_TR_ASM, k_tr_assemble<T>, dim3(gb.x, NTR), tb, 0, st, G, F, top, M);
        if (eta_side) {
            const clot_status r = eta_side_join();
            if (r < 0) return r;
        }
        {
            KVec<T, NTR> V = bicg_vecs<NTR>(0);
            for (int k = 0; k < NTR; ++k) {
                V.x[k] = F.dlt[k];  // delta form: each species' change, from zero
                V.b[k] = nullptr;   // TrOp forms the starting residual from its FP64 right-hand side
            }
            run_bicg<TrOp<T>, NTR>(top, V, prm.rtol_tr > 0.0 ? prm.rtol_tr : prm.rtol_s, allmask, 5,
                                   CLOT_PROBE_TR_B1);
            hipLaunchKernelGGL(k_add_change<T>, gb, tb, 0, st, G, F);
            record(ST_TR, ST_REST, NTR, false, nullptr, ST_SYSIT_TR);
        }
        if (eta_side) {   // the transport solve's polls have synchronised the main stream
            const clot_status r = eta_side_finish();
            if (r < 0) return r;
        }
        // Crank-Nicolson history of u and the transported species (before the reactions)
        if (M.psi > 0.0) hipLaunchKernelGGL(k_ddt_close<T>, gb, tb, 0, st, G, F);
        // O-6 reactions (wall first: it reads the transported S1)
        if (NINJ > 0)
            hipLaunchKernelGGL(k_wall_rxn<T>, dim3((NINJ + NT - 1) / NT), tb, 0, st, d_ch, d_f2c, NINJ, F, M);
#ifndef CLOT_INHIBITOR
        if (rxn_mode == CLOT_RXN_SURROGATE) {
            fill(fb_count, 0, 1);
            fill(fb_chan, 0, nch);
            MLPWeights w{mlp_wb + MLP_OFF_W1, mlp_wb + MLP_OFF_W2, mlp_wb + MLP_OFF_W3,
                         mlp_wf + MLP_OFF_B1, mlp_wf + MLP_OFF_B2, mlp_wf + MLP_OFF_B3};
            CLOT_LAUNCH(CLOT_PROBE_RXN, k_rxn_surr<T>, gb, dim3(256), 0, st, G, F, rxn_consts<T>(M), w, surr_tb, surr_tol, fb_list,
                        fb_count, fb_chan);
            CLOT_LAUNCH(CLOT_PROBE_RXN_FALLBACK, k_rxn_list<T>, dim3((unsigned)std::min<int64_t>((N + NT - 1) / NT, 1024)), tb, 0, st, d_ch, nch, F, (int)M.M_rxn, rxn_consts<T>(M),
                        fb_list, fb_count);
            hipLaunchKernelGGL(k_record_fallback, dim3(1), dim3(64), 0, st, fb_chan, d_ch, dstats, NSTAT, nch,
                               (int)ST_FALLBACK);
        } else
#endif
        {
            CLOT_LAUNCH(CLOT_PROBE_RXN, k_rxn<T>, gb, tb, 0, st, G, F, (int)M.M_rxn, rxn_consts<T>(M));
        }
        // the next step's ddt coefficients and variable step
        if (M.psi > 0.0 || M.max_co > 0.0)
            hipLaunchKernelGGL(k_time_end, dim3(nch), dim3(256), 0, st, d_ch, (const double*)F.co_part, M);
        // O-7 rotate theta_B and the flux
        rotate();
        HIPCHK(hipGetLastError());
        return CLOT_OK;
    }

    // Host side of the end of a step: buffer rotation and the channel clocks.
    void rotate() {
        std::swap(F.thB, F.thB_prev);
        for (int c = 0; c < 3; ++c) std::swap(F.phi[c], F.phin[c]);
        parity ^= 1;
        for (ChanHost& h : ch) {
            h.n += 1;
        }
    }

    static SigState fresh_sig() {
        SigState s{};
        s.t = 0.0;
        s.n = 0;
        s.next_push = 0;
        s.head = -1;
        s.npushed = 0;
        for (int q = 0; q < NHIST; ++q) s.hist_t[q] = -1e300;
        return s;
    }

    void drop_graphs() {
        for (auto& v : gseg) {
            for (hipGraphExec_t g : v) (void)hipGraphExecDestroy(g);
            v.clear();
        }
    }

    // Ends the recording in progress, keeps it as the next graph of the chain, and
    // starts recording again.
    clot_status seg_close(bool reopen) {
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (e != hipSuccess || !g) {
            err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
            return CLOT_EHIP;
        }
        size_t nn = 0;
        (void)hipGraphGetNodes(g, nullptr, &nn);
        g_nodes += (int64_t)nn;
        hipGraphExec_t x = nullptr;
        const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
            return CLOT_EHIP;
        }
        cap_out->push_back(x);
        g_segs += 1;
        if (reopen) HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        return CLOT_OK;
    }
    void seg_point() {
        if (!capturing || seg_err) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipGraph_t g = nullptr;
        if (hipStreamGetCaptureInfo_v2(st, &cs, nullptr, &g, nullptr, nullptr) != hipSuccess ||
            cs != hipStreamCaptureStatusActive || !g) {
            err = "graph recording: stream is not recording";
            seg_err = CLOT_EHIP;
            return;
        }
        size_t nn = 0;
        if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) {
            err = "graph recording: hipGraphGetNodes failed";
            seg_err = CLOT_EHIP;
            return;
        }
        if (nn >= SEG_NODES) seg_err = seg_close(true);
    }

    // Records one step of the current parity into a graph.  The host state that the
    // recording advances (buffer rotation, clocks) is restored afterwards: capture
    // enqueues work without running it.
    clot_status capture() {
        if (!cst) HIPCHK(hipStreamCreateWithFlags(&cst, hipStreamNonBlocking));
        auto bud = [&](int m) { return std::min(prm.max_iter, (int)std::ceil(g_scale * m) + g_pad); };
        for (int s = 0; s < 8; ++s) budget[s] = bud(it_max[s]);
        // refinement passes: the most seen (plus one per budget overflow so far); a
        // pass budget follows the count seen in that pass (an extra pass takes the
        // last one's)
        budget[6] = std::min(12, it_max[6] + (int)g_overflows);
        for (int q = 0; q < 3; ++q)
            for (int ps = 0; ps < 12; ++ps)
                pbudget[q][ps] = bud(ps < it_max[6] ? it_pmax[q][ps] : (it_max[6] > 0 ? it_pmax[q][it_max[6] - 1] : 0));
        const Fields<T> F0 = F;
        const int par0 = parity;
        std::vector<ChanHost> ch0 = ch;
        hipStream_t st0 = st;
        std::vector<hipGraphExec_t>& out = gseg[parity];
        for (hipGraphExec_t x : out) (void)hipGraphExecDestroy(x);
        out.clear();
        g_nodes = 0;
        g_segs = 0;
        HIPCHK(hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal));
        st = cst;
        capturing = true;
        cap_out = &out;
        seg_err = CLOT_OK;
        clot_status r = one_step();
        capturing = false;
        if (r >= 0 && seg_err >= 0) {
            r = seg_close(false);
        } else {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cst, &g);
            if (g) (void)hipGraphDestroy(g);
            if (r >= 0) r = seg_err;
        }
        st = st0;
        cap_out = nullptr;
        F = F0;
        parity = par0;
        ch = ch0;
        if (r < 0) {
            for (hipGraphExec_t x : out) (void)hipGraphExecDestroy(x);
            out.clear();
            return r;
        }
        g_captures += 1;
        return CLOT_OK;
    }

    // ---- rollback of a call window that meets a non-finite value ------------------
    // The persistent state (the workspace's first state_bytes) is copied aside on the
    // stream when a window opens: at a blocking clot_step, or at the first
    // clot_step_async after a synchronisation.  The synchronisation that closes it scans
    // the fields; if they or any reduction of the window met a NaN or infinity, the copy
    // is put back with the host side of the window's start (buffer parity, step counts).
    clot_status snapshot() {
        HIPCHK(hipMemcpyAsync(snap, ws_base, state_bytes, hipMemcpyDeviceToDevice, st));
        fill(nanflag, 0, 2);
        snap_parity = parity;
        snap_F = F;
        snap_n.resize(ch.size());
        for (size_t i = 0; i < ch.size(); ++i) snap_n[i] = ch[i].n;
        snap_valid = true;
        return CLOT_OK;
    }
    clot_status close_window() {
        snap_valid = false;
        hipLaunchKernelGGL(k_nonfinite_scan<T>, dim3(ntiles), dim3(NT), 0, st, grid(), F, NINJ, nanflag + 1);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h_nact + 8, nanflag, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!h_nact[8] && !h_nact[9]) return CLOT_OK;
        HIPCHK(hipMemcpyAsync(ws_base, snap, state_bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        F = snap_F;
        parity = snap_parity;
        for (size_t i = 0; i < ch.size(); ++i) ch[i].n = snap_n[i];
        err = std::string("a non-finite value appeared (") + (h_nact[8] ? "in a linear solve" : "in the fields") +
              "); the state is rolled back to the start of the call";
        return CLOT_ENAN;
    }

    clot_status step(int nsteps, bool wait) override {
        if (!snap_valid) {
            const clot_status r = snapshot();
            if (r < 0) return r;
        }
        for (int s = 0; s < nsteps; ++s) {
            if (graph_on && calib_left == 0) {
                if (gseg[parity].empty()) {
                    const clot_status r = capture();
                    if (r < 0) return r;
                }
                for (hipGraphExec_t x : gseg[parity]) HIPCHK(hipGraphLaunch(x, st));
                g_replays += 1;
                rotate();
                continue;
            }
            clot_status r = one_step();
            if (r < 0) return r;
            if (calib_left > 0) --calib_left;
        }
        if (wait) return sync();
        return CLOT_OK;
    }
    clot_status sync() override {
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (graph_on && g_replays > 0) {
            int32_t f = 0;
            HIPCHK(hipMemcpy(&f, gflag, 4, hipMemcpyDeviceToHost));
            if (f) {   // a budget was too small: count it, widen the budgets, re-record
                g_overflows += 1;
                const int32_t z = 0;
                HIPCHK(hipMemcpy(gflag, &z, 4, hipMemcpyHostToDevice));
                g_scale *= 2.0;
                g_pad += 2;
                drop_graphs();
            }
        }
        if (snap_valid) return close_window();
        return CLOT_OK;
    }

    clot_status set_brick(int kernel, int shape) override {
        static_assert(MGM_NSHAPE == 4 && MGB_NSHAPE == 4, "four shapes per bricked kernel");
        if (kernel < 0 || kernel >= CLOT_NBRICK_KERNELS || shape < 0 || shape >= MGM_NSHAPE) {
            err = "set_brick_shape: kernel in [0, 5), shape in [0, 4)";
            return CLOT_EINVAL;
        }
        HIPCHK(hipStreamSynchronize(st));
        drop_graphs();   // recorded steps hold the old launches
        brick_shape[kernel] = shape;
        return CLOT_OK;
    }
    clot_status set_graph(int on, double scale, int pad) override {
        HIPCHK(hipStreamSynchronize(st));
        drop_graphs();
        graph_on = on != 0;
        if (!graph_on) return CLOT_OK;
        if (!(scale >= 0.0) || pad < 1) {
            err = "set_graph_mode: budget scale must be >= 0 and pad >= 1";
            graph_on = false;
            return CLOT_EINVAL;
        }
        g_scale = scale;
        g_pad = pad;
        for (int& m : it_max) m = 0;
        for (auto& r : it_pmax)
            for (int& m : r) m = 0;
        calib_left = 2;   // one eager step of each parity sets the budgets
        return CLOT_OK;
    }
    clot_status graph_info(int64_t* info) override {
        info[0] = graph_on ? 1 : 0;
        info[1] = g_captures;
        info[2] = g_replays;
        info[3] = g_overflows;
        for (int s = 0; s < 7; ++s) info[4 + s] = budget[s];
        for (int s = 0; s < 7; ++s) info[11 + s] = it_max[s];
        info[18] = g_nodes;
        info[19] = g_segs;
        return CLOT_OK;
    }
    // ---- checkpoint and resume ----------------------------------------------------
    struct StateHead {
        uint64_t magic;
        int32_t version, prec, nch, parity;
        int64_t N, NFX, NFY, NFZ, NINJ, ntiles, ws;
        int32_t eta_budget, rxn_mode;
        float surr_tol, pad;
        int32_t last_it[8];
        SurrTables surr_tb;
    };
    struct StateChan {
        int64_t n;
        double t;          // the channel's simulated time (informative: the clock is in the workspace)
        clot_channel d;    // the descriptor: the workspace's channel tables derive from it
    };
    static constexpr uint64_t STATE_MAGIC = 0x54415453544f4c43ull;   // "CLOTSTAT"
    clot_status state_size(size_t* bytes) const override {
        *bytes = sizeof(StateHead) + ch.size() * sizeof(StateChan) + ws_bytes;
        return CLOT_OK;
    }
    clot_status save_state(void* host, size_t bytes) override {
        size_t need = 0;
        state_size(&need);
        if (!host || bytes < need) {
            err = "save_state: buffer of " + std::to_string(need) + " bytes needed";
            return CLOT_EINVAL;
        }
        HIPCHK(hipStreamSynchronize(st));
        if (st2) HIPCHK(hipStreamSynchronize(st2));
        StateHead h{};
        h.magic = STATE_MAGIC;
        h.version = 3;
        h.prec = (int32_t)prec;
        h.nch = (int32_t)ch.size();
        h.parity = parity;
        h.N = N;
        h.NFX = NFX;
        h.NFY = NFY;
        h.NFZ = NFZ;
        h.NINJ = NINJ;
        h.ntiles = ntiles;
        h.ws = (int64_t)ws_bytes;
        h.eta_budget = eta_budget;
        h.rxn_mode = (int32_t)rxn_mode;
        h.surr_tol = surr_tol;
        for (int i = 0; i < 8; ++i) h.last_it[i] = last_it[i];
        h.surr_tb = surr_tb;
        std::vector<SigState> clocks(ch.size());
        HIPCHK(hipMemcpy(clocks.data(), sig, ch.size() * sizeof(SigState), hipMemcpyDeviceToHost));
        char* p = static_cast<char*>(host);
        std::memcpy(p, &h, sizeof(h));
        p += sizeof(h);
        for (size_t i = 0; i < ch.size(); ++i) {
            const ChanHost& c = ch[i];
            StateChan sc{};
            sc.n = c.n;
            sc.t = clocks[i].t;
            sc.d = c.d;
            std::memcpy(p, &sc, sizeof(sc));
            p += sizeof(sc);
        }
        HIPCHK(hipMemcpy(p, ws_base, ws_bytes, hipMemcpyDeviceToHost));
        return CLOT_OK;
    }
    clot_status load_state(const void* host, size_t bytes) override {
        size_t need = 0;
        state_size(&need);
        if (!host || bytes < need) {
            err = "load_state: blob of " + std::to_string(need) + " bytes expected";
            return CLOT_EINVAL;
        }
        StateHead h;
        const char* p = static_cast<const char*>(host);
        std::memcpy(&h, p, sizeof(h));
        p += sizeof(h);
        if (h.magic != STATE_MAGIC || h.version != 3 || h.prec != (int32_t)prec || h.nch != (int32_t)ch.size() ||
            h.N != N || h.NFX != NFX || h.NFY != NFY || h.NFZ != NFZ || h.NINJ != NINJ || h.ntiles != ntiles ||
            h.ws != (int64_t)ws_bytes || (h.parity != 0 && h.parity != 1)) {
            err = "load_state: the blob was saved from a context of another layout";
            return CLOT_EINVAL;
        }
        std::vector<StateChan> sc(ch.size());
        for (size_t i = 0; i < ch.size(); ++i) {
            std::memcpy(&sc[i], p, sizeof(StateChan));
            p += sizeof(StateChan);
            // every field of the descriptor (extents, injury patch, shear, margination, step)
            // must match: the blob carries the channel tables and clocks built from it
            if (std::memcmp(&sc[i].d, &ch[i].d, sizeof(clot_channel)) != 0) {
                err = "load_state: channel " + std::to_string(i) + " differs from the saved one";
                return CLOT_EINVAL;
            }
        }
        HIPCHK(hipStreamSynchronize(st));
        if (st2) HIPCHK(hipStreamSynchronize(st2));
        drop_graphs();
        snap_valid = false;
        HIPCHK(hipMemcpy(ws_base, p, ws_bytes, hipMemcpyHostToDevice));
        {   // the inflow profiles follow this context's parameters
            const clot_status r = upload_inflow();
            if (r) return r;
        }
        for (size_t i = 0; i < ch.size(); ++i) {
            ch[i].n = sc[i].n;
        }
        if (parity != h.parity) {   // the buffer pair that holds the current flux and theta_B
            std::swap(F.thB, F.thB_prev);
            for (int c = 0; c < 3; ++c) std::swap(F.phi[c], F.phin[c]);
            parity = h.parity;
        }
        eta_budget = h.eta_budget;
        for (int i = 0; i < 8; ++i) last_it[i] = h.last_it[i];
        rxn_mode = (clot_rxn_mode)h.rxn_mode;
        surr_tol = h.surr_tol;
        surr_tb = h.surr_tb;
        if (graph_on) {             // budgets are measured again
            for (int& m : it_max) m = 0;
            for (auto& r : it_pmax)
                for (int& m : r) m = 0;
            calib_left = 2;
        }
        return CLOT_OK;
    }

    clot_status stats(int c, clot_stats* s) const override {
        // diagnostics of the current state, after whatever the context stream holds
        hipLaunchKernelGGL(k_diag_tiles<T>, dim3(ntiles), dim3(NT), 0, st, grid(), F, M, S.part);
        hipLaunchKernelGGL(k_diag_finish, dim3((int)ch.size()), dim3(256), 0, st, d_ch, (const double*)S.part, dstats,
                           NSTAT, (int)ST_DIAG);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return CLOT_EHIP;
        std::vector<double> v(NSTAT);
        if (hipMemcpy(v.data(), dstats + (size_t)c * NSTAT, NSTAT * 8, hipMemcpyDeviceToHost) != hipSuccess) return CLOT_EHIP;
        std::memset(s, 0, sizeof(*s));
        s->it_mom = (int)v[ST_MOM];
        s->it_eta = (int)v[ST_ETA];
        s->it_tr = (int)v[ST_TR];
        for (int k = 0; k < 8; ++k) {
            s->it_p[k] = (int)v[ST_P + k];
            s->refine_p[k] = (int)v[ST_REF + k];
        }
        s->res_mom = v[ST_RESM];
        s->res_p = v[ST_RESP];
        s->res_eta = v[ST_RESE];
        s->res_tr = v[ST_REST];
        s->fallback_frac = v[ST_FALLBACK];
        s->steps = ch[c].n;
        SigState sg;
        ChanDev cd;
        if (hipMemcpy(&sg, sig + c, sizeof(SigState), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&cd, d_ch + c, sizeof(ChanDev), hipMemcpyDeviceToHost) != hipSuccess)
            return CLOT_EHIP;
        s->t = sg.t;
        s->dt = cd.dt;
        s->div_rel = v[ST_DIAG + 1] > 0.0 ? v[ST_DIAG] / v[ST_DIAG + 1] : v[ST_DIAG];
        s->min_species = v[ST_DIAG + 2];
        s->sysit_tr = (int32_t)v[ST_SYSIT_TR];
        return v[ST_FAIL] >= 2 ? CLOT_W_NONFINITE : v[ST_FAIL] > 0 ? CLOT_W_NOTCONV : CLOT_OK;
    }
};

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
static clot_ctx* make_ctx(clot_precision prec) {
    if (prec == CLOT_FP64) return new Ctx<double>();
    return new Ctx<float>();
}

template <class T>
static size_t ws_size(Ctx<T>* c) {
    return c->layout(nullptr);
}

static ModelDev model_from_params(const clot_params& q) {
    ModelDev M{q.nu, q.C_CK, q.D_P, q.D_ADP, q.D_chem, q.P_diam, q.P_max, q.P_0, q.k_adh, q.kcoh_Pmax,
               q.eta_t, q.eta_star, 0.0, q.k_adp, q.adp_crit, q.k_e2, q.e2_crit,
               q.A_hat, q.tau_f, q.dtau, q.N_A, q.N1, q.N2,
               q.kC0p, q.kC0m, q.kC0cat, q.kC1p, q.kC1m, q.kC1cat, q.kC2p, q.kC2m, q.kC2cat,
               q.kS1p, q.kS1m, q.kE1p, q.kE1m, q.kS2p, q.kS2m, q.kE2p, q.kE2m,
               q.S1_0, q.S2_0, q.E0_0, q.p_out, 0.0, q.M_rxn};
    const double Le = q.L_eta_over_Pdiam * q.P_diam;
    M.kappa_eta = Le * Le / 4.0;
    M.g0 = (std::pow(q.eta_star, 3) + std::pow(1.0 - q.eta_t, 3)) / std::pow(1.0 - q.eta_t, 3);
    M.psi = q.ddt_psi;
    M.max_co = q.max_co;
    M.dt_growth = q.dt_growth;
    M.k_I = q.k_I;
    M.I_0 = q.I_0;
    return M;
}

template <class T>
static clot_status create_t(Ctx<T>* c, const clot_channel* chs, int n_ch, const clot_params* p, void* ws, size_t wsb,
                            void* stream) {
    clot_status s = c->setup(chs, n_ch, p);
    if (s) return s;
    s = c->lds_limits();
    if (s) return s;
    const size_t need = c->layout(nullptr);
    if (wsb < need) {
        c->err = "workspace too small: need " + std::to_string(need) + " bytes";
        return CLOT_ENOMEM;
    }
    if (((uintptr_t)ws & 255) != 0) {
        c->err = "workspace must be 256-byte aligned";
        return CLOT_EWORKSPACE;
    }
    c->layout((char*)ws);
    c->nchan = n_ch;
    c->ws_base = (char*)ws;
    c->ws_bytes = need;
    c->st = (hipStream_t)stream;
    hipError_t he = hipHostMalloc((void**)&c->h_nact, 64, hipHostMallocDefault);
    if (he != hipSuccess) {
        // an error left by an earlier call can surface here: clear it and try once more
        (void)hipGetLastError();
        he = hipHostMalloc((void**)&c->h_nact, 64, hipHostMallocDefault);
    }
    if (he != hipSuccess) {
        c->h_nact = nullptr;
        c->err = std::string("hipHostMalloc of the 64-byte poll buffer failed: ") + hipGetErrorName(he) + " (" +
                 hipGetErrorString(he) + ")";
        return CLOT_EHIP;
    }
    return c->upload_tables();
}

// Message of the last failed clot_create (its context no longer exists) or failed
// context-free call on this thread.
static thread_local std::string g_create_err;

// ---- the MLP backward without allocation --------------------------------------------
// Per-block gradient partials of clot_mlp_backward_noalloc: one MLP_NPARAM slice per
// block of 64 samples, for at most NOALLOC_MAX samples (7.5 MB).  Each device holds its
// own copy for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the name is a host-side stand-in).
constexpr int64_t NOALLOC_MAX = 16384;
constexpr int64_t NOALLOC_BLOCKS = NOALLOC_MAX / 64;
static __device__ __align__(256) float scratch[NOALLOC_BLOCKS * MLP_NPARAM];

static std::mutex g_scratch_mu;
static std::array<float*, 64> g_scratch_ptr{};   // per device id

// The current device's copy of `scratch`, looked up once per device.
static clot_status noalloc_scratch(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= (int)g_scratch_ptr.size()) {
        g_create_err = std::string("mlp_backward_noalloc: no usable current device: ") + hipGetErrorString(e);
        return CLOT_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_create_err = std::string("mlp_backward_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
            return CLOT_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return CLOT_OK;
}

extern "C" {

clot_status clot_params_default(clot_params* p) {
    if (!p) return CLOT_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->nu = 2.62507;
    p->C_CK = 1.0e6;
    p->D_P = 2.5e-5;
    p->D_ADP = 5.0e-4;
    p->D_chem = 5.0e-5;
    p->P_diam = 3.0e-3;
    p->P_max = 6.67e7;
    p->P_0 = 2.5e5;
    p->k_adh = 3.3212e-8;
    p->kcoh_Pmax = 1.0e4;
    p->eta_t = 0.1;
    p->eta_star = 0.4;
    p->L_eta_over_Pdiam = 2.0;
    p->k_adp = 0.34;
    p->adp_crit = 2.0e-3;
    p->k_e2 = 0.5;
    p->e2_crit = 1.0e-6;
    p->A_hat = 2.0e-8;
    p->tau_f = 6.0;
    p->dtau = 0.25;
    p->N_A = 6.02214076e14;
    p->N1 = 2700.0;
    p->N2 = 2000.0;
    p->kC0p = 8.95e3;
    p->kC0m = 1.0;
    p->kC0cat = 1.15;
    p->kC1p = 1.03e5;
    p->kC1m = 1.0;
    p->kC1cat = 30.0;
    p->kC2p = 1.73e4;
    p->kC2m = 1.0;
    p->kC2cat = 0.23;
    p->kS1p = 5.7e4;
    p->kS1m = 0.17;
    p->kE1p = 1.0e4;
    p->kE1m = 2.5e-2;
    p->kS2p = 1.0e4;
    p->kS2m = 5.9;
    p->kE2p = 1.0e4;
    p->kE2m = 5.9;
    p->S1_0 = 1.7e-4;
    p->S2_0 = 1.4e-3;
    p->E0_0 = 1.5e-7;
    p->p_out = 0.0;
    p->M_rxn = 2;
    p->n_corr = 0;
    p->max_iter = 5000;
    p->marg_m = 19;
    p->marg_n = 2;
    p->rtol_p = 1e-13;
    p->rtol_s = 1e-13;
    p->rtol_inner = 1e-4;
    p->mg_tail = 1024;
    p->mg_sweeps = 0;
    p->ddt_psi = 0.0;
    p->max_co = 0.0;
    p->dt_growth = 1.2;
    p->k_I = 7.1;
    p->I_0 = 3.4e-3;
    p->rtol_tr = 1e-13;
    p->mom_mg = 1;
    p->mg_brick = 1;
    return CLOT_OK;
}

clot_status clot_query_workspace(const clot_channel* chs, int32_t n_ch, clot_precision prec, size_t* bytes) {
    if (!chs || n_ch < 1 || !bytes || (prec != CLOT_FP64 && prec != CLOT_FP32_MIXED)) return CLOT_EINVAL;
    clot_params p;
    clot_params_default(&p);
    clot_ctx* c = make_ctx(prec);
    clot_status s;
    if (prec == CLOT_FP64) {
        auto* d = static_cast<Ctx<double>*>(c);
        s = d->setup(chs, n_ch, &p);
        if (s == CLOT_OK) *bytes = ws_size(d);
    } else {
        auto* d = static_cast<Ctx<float>*>(c);
        s = d->setup(chs, n_ch, &p);
        if (s == CLOT_OK) *bytes = ws_size(d);
    }
    delete c;
    return s;
}

clot_status clot_create(const clot_channel* chs, int32_t n_ch, const clot_params* p, clot_precision prec, void* ws,
                        size_t wsb, void* stream, clot_ctx** out) {
    if (!chs || n_ch < 1 || !p || !ws || !out || (prec != CLOT_FP64 && prec != CLOT_FP32_MIXED)) return CLOT_EINVAL;
    *out = nullptr;
    if (p->M_rxn < 1 || p->n_corr < 0 || p->n_corr > MAXCORR || p->max_iter < 1 || p->mg_tail < 0 ||
        p->mg_sweeps < 0 || p->mg_sweeps > 4 || !(p->ddt_psi >= 0.0 && p->ddt_psi <= 1.0) ||
        !(p->max_co >= 0.0) || !(p->dt_growth >= 1.0) || !(p->k_I >= 0.0) || !(p->I_0 >= 0.0) ||
        (p->mom_mg != 0 && p->mom_mg != 1) || (p->mg_brick != 0 && p->mg_brick != 1))
        return CLOT_EINVAL;
    clot_ctx* c = make_ctx(prec);
    c->prec = prec;
    clot_status s = prec == CLOT_FP64 ? create_t(static_cast<Ctx<double>*>(c), chs, n_ch, p, ws, wsb, stream)
                                      : create_t(static_cast<Ctx<float>*>(c), chs, n_ch, p, ws, wsb, stream);
    if (s < 0) {
        g_create_err = c->err;
        delete c;
        return s;
    }
    g_create_err.clear();
    *out = c;
    return CLOT_OK;
}

// A channel index outside [0, n_ch) is refused before anything is touched.
static bool bad_channel(const clot_ctx* c, int32_t chn) {
    if (chn >= 0 && chn < c->nchan) return false;
    const_cast<clot_ctx*>(c)->err =
        "channel index " + std::to_string(chn) + " outside [0, " + std::to_string(c->nchan) + ")";
    return true;
}

clot_status clot_init_state(clot_ctx* c, int32_t chn, const double* xc, size_t nc, const double* xf, size_t nf) {
    if (!c || bad_channel(c, chn)) return CLOT_EINVAL;
    return c->init_state(chn, xc, nc, xf, nf);
}
clot_status clot_field_count(const clot_ctx* c, int32_t chn, clot_field f, size_t* n) {
    if (!c || !n || bad_channel(c, chn)) return CLOT_EINVAL;
    return c->count(chn, f, n);
}
clot_status clot_set_field(clot_ctx* c, int32_t chn, clot_field f, const double* h, size_t n) {
    if (!c || bad_channel(c, chn)) return CLOT_EINVAL;
    return c->set(chn, f, h, n);
}
clot_status clot_get_field(clot_ctx* c, int32_t chn, clot_field f, double* h, size_t n) {
    if (!c || bad_channel(c, chn)) return CLOT_EINVAL;
    return c->get(chn, f, h, n);
}
clot_status clot_step(clot_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return CLOT_EINVAL;
    return c->step(nsteps, true);
}
clot_status clot_step_async(clot_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return CLOT_EINVAL;
    return c->step(nsteps, false);
}
clot_status clot_sync(clot_ctx* c) {
    if (!c) return CLOT_EINVAL;
    return c->sync();
}
clot_status clot_get_stats(const clot_ctx* c, int32_t chn, clot_stats* s) {
    if (!c || !s || bad_channel(c, chn)) return CLOT_EINVAL;
    return c->stats(chn, s);
}
clot_status clot_state_size(const clot_ctx* c, size_t* bytes) {
    if (!c || !bytes) return CLOT_EINVAL;
    return c->state_size(bytes);
}
clot_status clot_save_state(clot_ctx* c, void* host, size_t bytes) {
    if (!c) return CLOT_EINVAL;
    return c->save_state(host, bytes);
}
clot_status clot_load_state(clot_ctx* c, const void* host, size_t bytes) {
    if (!c) return CLOT_EINVAL;
    return c->load_state(host, bytes);
}
clot_status clot_set_reaction_mode(clot_ctx* c, clot_rxn_mode mode, const void* blob, size_t nb, double tol) {
    if (!c) return CLOT_EINVAL;
    return c->set_rxn(mode, blob, nb, tol);
}

// ---- surrogate training and data preparation (device pointers, caller's stream) ----
#define CHK_LAUNCH()                                              \
    do {                                                          \
        if (hipGetLastError() != hipSuccess) return CLOT_EHIP;    \
    } while (0)

static MLPWeights mlp_ptrs(const float* wf, const uint16_t* wb) {
    return MLPWeights{wb + MLP_OFF_W1, wb + MLP_OFF_W2, wb + MLP_OFF_W3, wf + MLP_OFF_B1, wf + MLP_OFF_B2, wf + MLP_OFF_B3};
}

int64_t clot_mlp_nparam(void) { return MLP_NPARAM; }

size_t clot_mlp_backward_workspace(int64_t n) {
    const int64_t nblk = (n + 63) / 64;
    return (size_t)nblk * MLP_NPARAM * sizeof(float);
}

clot_status clot_mlp_forward(const float* wf, const uint16_t* wb, const uint16_t* x, int64_t n, float* y, uint16_t* cache,
                             void* stream) {
    if (!wf || !wb || !x || !y || n < 0) return CLOT_EINVAL;
    if (n == 0) return CLOT_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, mlp_ptrs(wf, wb), x,
                       n, y, cache);
    CHK_LAUNCH();
    return CLOT_OK;
}

clot_status clot_mlp_backward(const float* wf, const uint16_t* wb, const uint16_t* x, const uint16_t* cache,
                              const float* dy, int64_t n, float* part, float* dw, void* stream) {
    if (!wf || !wb || !x || !cache || !dy || !part || !dw || n <= 0) return CLOT_EINVAL;
    const int nblk = (int)((n + 63) / 64);
    hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(256), 0, (hipStream_t)stream, mlp_ptrs(wf, wb), x, cache, dy, n,
                       part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, part, nblk, dw);
    CHK_LAUNCH();
    return CLOT_OK;
}

clot_status clot_mlp_backward_noalloc(const float* wf, const uint16_t* wb, const uint16_t* x, const uint16_t* cache,
                                      const float* dy, int64_t n, float* dw, void* stream) {
    if (!wf || !wb || !x || !cache || !dy || !dw || n <= 0) return CLOT_EINVAL;
    if (n > NOALLOC_MAX) {
        g_create_err = "mlp_backward_noalloc: n = " + std::to_string(n) + " exceeds the limit of " +
                       std::to_string(NOALLOC_MAX) + " samples";
        return CLOT_EINVAL;
    }
    float* part = nullptr;
    const clot_status r = noalloc_scratch(&part);
    if (r) return r;
    // the same kernels as clot_mlp_backward: every block writes its whole slice, the
    // reduction reads exactly nblk slices, so nothing needs clearing between calls
    const int nblk = (int)((n + 63) / 64);
    hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(256), 0, (hipStream_t)stream, mlp_ptrs(wf, wb), x, cache, dy, n,
                       part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, part, nblk, dw);
    CHK_LAUNCH();
    return CLOT_OK;
}

clot_status clot_mlp_adam(float* wf, uint16_t* wb, const float* g, float* m, float* v, int64_t t, double lr, double b1,
                          double b2, double eps, void* stream) {
    if (!wf || !wb || !g || !m || !v || t < 1) return CLOT_EINVAL;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)t)), bc2 = (float)(1.0 - std::pow(b2, (double)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, wf, wb, g, m, v,
                       (int64_t)MLP_NPARAM, (float)lr, (float)b1, (float)b2, (float)eps, bc1, bc2);
    CHK_LAUNCH();
    return CLOT_OK;
}

clot_status clot_mlp_mse(const float* y, const float* t, int64_t n, int32_t nuse, float* dy, double* lpart,
                         void* stream) {
    if (!y || !t || !dy || !lpart || n <= 0 || nuse < 1 || nuse > MLP_OUT) return CLOT_EINVAL;
    hipLaunchKernelGGL(k_mlp_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, t, n, nuse, dy,
                       lpart);
    CHK_LAUNCH();
    return CLOT_OK;
}

clot_status clot_rxn_rk4_batch(const clot_params* p, const double* rows, int64_t n, double* inc, void* stream) {
#ifdef CLOT_INHIBITOR
    (void)p, (void)rows, (void)n, (void)inc, (void)stream;
    return CLOT_EINVAL;   // rows hold the base model's 14 species
#else
    if (!p || !rows || !inc || n < 0 || p->M_rxn < 1) return CLOT_EINVAL;
    if (n == 0) return CLOT_OK;
    const ModelDev M = model_from_params(*p);
    hipLaunchKernelGGL(k_rxn_batch, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, (hipStream_t)stream, rows, n,
                       (int)M.M_rxn, rxn_consts<double>(M), inc);
    CHK_LAUNCH();
    return CLOT_OK;
#endif
}

clot_status clot_surr_dataset(const clot_params* p, const double* rows, const double* inc, int64_t n,
                              const float* scales, uint16_t* x, float* t, double* stats, void* stream) {
#ifdef CLOT_INHIBITOR
    (void)p, (void)rows, (void)inc, (void)n, (void)scales, (void)x, (void)t, (void)stats, (void)stream;
    return CLOT_EINVAL;   // the learned step covers the base model only
#else
    if (!p || !rows || !inc || n <= 0 || (!stats && (!scales || !x || !t))) return CLOT_EINVAL;
    const ModelDev M = model_from_params(*p);
    SurrTables tb{};
    for (int i = 0; i < MLP_NSP; ++i) {
        tb.sf[i] = scales ? scales[i] : 1.f;
        tb.sc[i] = scales ? scales[MLP_NSP + i] : 1.f;
    }
    surr_tables_finish(M, tb);
    hipLaunchKernelGGL(k_surr_dataset, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, (hipStream_t)stream, rows, inc, n,
                       rxn_consts<double>(M), tb, x, t, stats);
    CHK_LAUNCH();
    return CLOT_OK;
#endif
}

clot_status clot_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, void* stream) {
    if (!A || !B || !D) return CLOT_EINVAL;
    hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, D);
    CHK_LAUNCH();
    return CLOT_OK;
}
clot_status clot_probe(clot_ctx* c, int32_t kernel) {
    if (!c) return CLOT_EINVAL;
    return c->probe(kernel);
}
clot_status clot_probe_read(clot_ctx* c, double* ms, int64_t* n) {
    if (!c || !ms || !n) return CLOT_EINVAL;
    return c->probe_read(ms, n);
}
int32_t clot_tile_cells(void) { return TILE; }

int32_t clot_cell_species(void) { return NSPC; }
clot_status clot_set_graph_mode(clot_ctx* c, int32_t on, double budget_scale, int32_t budget_pad) {
    if (!c) return CLOT_EINVAL;
    return c->set_graph(on, budget_scale, budget_pad);
}
clot_status clot_graph_info(clot_ctx* c, int64_t* info) {
    if (!c || !info) return CLOT_EINVAL;
    return c->graph_info(info);
}
clot_status clot_set_brick_shape(clot_ctx* c, int32_t kernel, int32_t shape) {
    if (!c) return CLOT_EINVAL;
    return c->set_brick(kernel, shape);
}
clot_status clot_brick_kernel_dims(int32_t kernel, int32_t dim, int32_t shape, int32_t* dims) {
    if (!dims || (dim != 2 && dim != 3) || shape < 0 || shape >= MGM_NSHAPE || kernel < 0 ||
        kernel >= CLOT_NBRICK_KERNELS)
        return CLOT_EINVAL;
    int bx, by, bz;
    if (kernel == CLOT_BRICK_P_DOWN || kernel == CLOT_BRICK_P_UP)
        pbrick_dims(dim, shape, bx, by, bz);
    else
        brick_dims(dim, shape, bx, by, bz);
    dims[0] = bx;
    dims[1] = by;
    dims[2] = bz;
    return CLOT_OK;
}
clot_status clot_brick_dims(int32_t dim, int32_t shape, int32_t* dims) {
    return clot_brick_kernel_dims(CLOT_BRICK_RESTRICT, dim, shape, dims);
}
void clot_destroy(clot_ctx* c) { delete c; }
const char* clot_last_error(const clot_ctx* c) {
    if (c) return c->err.c_str();
    return g_create_err.empty() ? "null context" : g_create_err.c_str();
}

}  // extern "C"
