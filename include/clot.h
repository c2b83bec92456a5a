/*
 * clot.h — C ABI of the MI355X (gfx950) clotting-step library.
 *
 * The library advances the clotting model of clotFoam (arXiv 2304.09180) by whole
 * time steps on one GPU.  One step is, in order:
 *   1. theta_B, theta_T and the Carman-Kozeny permeability alpha (section 2, eq. NSB;
 *      Appendix A for theta_T);
 *   2. the PISO pressure-velocity update: one implicit momentum predictor with the
 *      Darcy term nu*alpha(theta_B) on the diagonal, then n_corr pressure
 *      corrections (section 3.2);
 *   3. the virtual substance eta - (L_eta^2/4) lap eta = theta_B (Appendix A, eq. eta);
 *   4. the ADP release source sigma by the coarse-tau trapezoid (section 3.2,
 *      eqs. ADP_source and sigma_disc);
 *   5. implicit transport of Pmu, Pma, S1, S2, E1, E2, ADP with van Leer TVD
 *      convection, hindered platelet fluxes (downwind / localMax theta_T, section
 *      3.2 and Appendix D) and the reactive injury-wall conditions (Appendix B,
 *      Appendix C table);
 *   6. the reactions, M_rxn classical RK4 sub-steps per cell and per injury face
 *      (section 3.2 fractional step; Appendix A and B right-hand sides).
 *
 * Conventions
 *   - Every call returns clot_status: 0 success, >0 warning (state valid),
 *     <0 error (state unchanged; clot_last_error() says why).  A channel index
 *     outside [0, n_ch) is an error (CLOT_EINVAL).
 *   - Units: mm, s, nmol, platelets/mm^3 (Appendix E tables).
 *   - Cell fields cross the ABI as float64 in x-fastest order, cell id
 *     i + nx*(j + ny*k).  Face fluxes (mm^3/s, positive along +axis) are x-faces
 *     i + (nx+1)*(j + ny*k), y-faces i + nx*(j + (ny+1)*k), z-faces
 *     i + nx*(j + ny*k) with k in [0, nz].  Injury-face fields follow the injury
 *     faces x-fastest, then z.
 *   - Ownership: host buffers are caller-owned and used only during the call.
 *     The device workspace and the HIP stream are caller-owned and must outlive
 *     the context; the library allocates no device memory of its own.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef CLOT_H
#define CLOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CLOT_OK = 0,
    CLOT_W_NOTCONV = 1,     /* a linear solve stopped at max_iter; the step completed        */
    CLOT_W_FALLBACK = 2,    /* surrogate step: some cells fell back to the plain integrator  */
    CLOT_W_NONFINITE = 3,   /* reported by clot_get_stats: a linear solve met a NaN or
                               infinity (in the fields or its system) and stopped; the call
                               that ran it returned CLOT_ENAN and rolled the state back      */
    CLOT_EINVAL = -1,       /* bad argument                                                  */
    CLOT_ENOMEM = -2,       /* workspace too small                                           */
    CLOT_EWORKSPACE = -3,   /* workspace pointer misaligned                                  */
    CLOT_EHIP = -4,         /* a HIP runtime call failed                                     */
    CLOT_ESTATE = -5,       /* call not valid in the current state                           */
    CLOT_ENAN = -6          /* a non-finite value appeared: clot_set_field refuses it; a
                               step call (or the clot_sync that closes asynchronous steps)
                               restores the state of the call's start                         */
} clot_status;

typedef enum { CLOT_FP64 = 0, CLOT_FP32_MIXED = 1 } clot_precision;
typedef enum { CLOT_RXN_PLAIN = 0, CLOT_RXN_SURROGATE = 1 } clot_rxn_mode;

typedef enum {
    CLOT_UX = 0, CLOT_UY, CLOT_UZ, CLOT_P, CLOT_PHIX, CLOT_PHIY, CLOT_PHIZ,
    CLOT_PMU, CLOT_PMA, CLOT_PBA, CLOT_PBSE, CLOT_ADP, CLOT_S1, CLOT_S2, CLOT_E1, CLOT_E2,
    CLOT_S1B, CLOT_S2B, CLOT_E1B, CLOT_E2B, CLOT_C1, CLOT_C2,   /* 15 cell species          */
    CLOT_E0, CLOT_C0,                                            /* injury-face species     */
    CLOT_ETA, CLOT_THETAB, CLOT_SIGMA,                           /* derived, read only      */
    CLOT_HADH,                                                   /* adhesion mask, read only */
    CLOT_I, CLOT_E2I,            /* inhibitor build only (section 3.4, I + E2 -> E2i): the
                                    inhibitor I and the inhibited thrombin E2i, both
                                    transported and reacting; other builds refuse them
                                    with CLOT_EINVAL                                      */
    CLOT_NFIELDS
} clot_field;

/* One straight channel [0,Lx]x[0,Ly](x[0,Lz]): inlet x=0, outlet x=Lx, walls elsewhere.
 * 2-D channels have nz = 1 and Lz the cell depth.  The injury patch is the set of
 * y=0 wall faces whose centre lies in [inj_x0,inj_x1] x [inj_z0,inj_z1]
 * (section 3.1, injuryWalls).  The inflow is the parabola of eq. parabolicVelocity
 * (2-D) or the rectangular-duct Poiseuille profile (3-D), scaled to the wall shear
 * rate `shear` on the bottom-wall centre line; platelets enter with the
 * margination profile of Appendix C.1 (amplitudes K_y, K_z). */
typedef struct {
    int32_t dim, nx, ny, nz;
    double Lx, Ly, Lz;
    double inj_x0, inj_x1, inj_z0, inj_z1;
    double shear;
    double K_y, K_z;
    double dt;
} clot_channel;

/* Model constants (Appendix E) and solver settings.  The release history (section
 * 3.2, eq. for sigma) keeps tau_f/dtau + 1 = 25 snapshots: tau_f/dtau must be 24,
 * else clot_create returns CLOT_EINVAL. */
typedef struct {
    double nu, C_CK, D_P, D_ADP, D_chem, P_diam, P_max, P_0, k_adh, kcoh_Pmax;
    double eta_t, eta_star, L_eta_over_Pdiam, k_adp, adp_crit, k_e2, e2_crit;
    double A_hat, tau_f, dtau, N_A, N1, N2;
    double kC0p, kC0m, kC0cat, kC1p, kC1m, kC1cat, kC2p, kC2m, kC2cat;
    double kS1p, kS1m, kE1p, kE1m, kS2p, kS2m, kE2p, kE2m;
    double S1_0, S2_0, E0_0, p_out;
    int32_t M_rxn;        /* reaction sub-steps per step (section 3.2; default 2)          */
    int32_t n_corr;       /* PISO pressure corrections per step; 0 = by the diffusion number
                             D = nu dt / h_min^2: 2 (D <= 10), 3 (30), 4 (50), 5 (80),
                             6 (120), else 8                                              */
    int32_t max_iter;     /* per linear solve                                              */
    int32_t marg_m, marg_n;
    double rtol_p;        /* pressure: ||b - A p|| <= rtol_p ||b|| (FP64 residual)           */
    double rtol_s;        /* momentum, eta (and transport when rtol_tr is 0)               */
    double rtol_inner;    /* FP32 inner pressure solve of each refinement pass             */
    int32_t mg_tail;      /* pressure multigrid: the levels whose channels all have at most
                             this many cells run as one launch (one block per channel);
                             0 = every level its own launches.  Default 1024.            */
    int32_t mg_sweeps;    /* pressure multigrid: weighted-Jacobi sweeps before and after each
                             restriction, 1 to 4, or 0 (default): 3 when every channel is
                             3-D, else 2.  Each sweep costs one stencil pass per level;
                             more sweeps need fewer CG iterations                       */
    double ddt_psi;       /* Crank-Nicolson off-centring of every ddt term (Appendix D
                             table), in [0,1]; 0 = implicit Euler (default).  The time
                             derivative over a step is k (f' - f)/dt - w D, D the stored
                             derivative of the previous step (updated by the same
                             expression), k = 1+psi, w = psi; the first step after
                             clot_init_state is implicit Euler.  A species' stored
                             derivative is that of its transport sub-step.               */
    double max_co;        /* > 0: variable step (Appendix D: maxCo) holding the largest cell
                             Courant number 0.5 dt sum_f |phi_f| / V of the current flux at
                             max_co; the channel's dt is the largest step, the first step
                             the largest the initial flux allows.  0 = the channel's fixed
                             dt (default).  The corrector count (n_corr = 0) follows the
                             channel's dt.                                               */
    double dt_growth;     /* variable step: largest growth factor per step, >= 1 (default 1.2) */
    double k_I;           /* inhibitor variant: rate of I + E2 -> E2i, (nmol/mm^3)^-1 s^-1,
                             >= 0 (default 7.1); other builds ignore it                   */
    double I_0;           /* inhibitor variant: inlet and initial I, nmol/mm^3, >= 0
                             (default 3.4e-3); other builds ignore it                     */
    double rtol_tr;       /* the 7 transport solves (each solves for the step's change,
                             from an FP64 residual); 0 = rtol_s                          */
    int32_t mom_mg;       /* momentum predictor (eq. NSB, section 3.2): 1 (default) =
                             BiCGStab with one multigrid V-cycle per direction (the
                             aggregation levels of the pressure solver carrying the mass
                             and viscous parts of the momentum matrix); 0 = BiCGStab with
                             the Jacobi preconditioner.  Both stop at rtol_s.             */
    int32_t mg_brick;     /* pressure multigrid, where every channel is coarsened along every
                             axis: 1 (default) = the mesh's restriction over 1024-cell
                             bricks and its prolongation by index halving, and (FP32, 2 or
                             3 sweeps) each leg of every coarse level above the fused tail
                             as one launch over LDS-staged 1024-cell bricks with a halo of
                             one cell per sweep; 0 = the general separate launches.  Bit
                             for bit the same.                                            */
} clot_params;

/* Per-channel statistics of the last step. */
typedef struct {
    int32_t it_mom, it_p[8], it_eta, it_tr;   /* Krylov iterations (it_p per corrector)   */
    int32_t refine_p[8];                        /* FP64 refinement passes per corrector      */
    double res_mom, res_p, res_eta, res_tr;     /* final relative residuals, max over the
                                                   solve's systems; an FP32 transport species
                                                   stopped by the absolute floor is measured
                                                   against the norm that floor stands for      */
    double fallback_frac;                       /* surrogate cells sent to the plain RK4     */
    int64_t steps;
    double t;                                   /* simulated time                            */
    double dt;                                  /* step the next clot_step takes             */
    double div_rel;                             /* largest |net outflow| of a cell over the
                                                   largest face flux (discrete continuity)   */
    double min_species;                         /* smallest species value over its scale
                                                   (P_max, ADP*, S1_0, S2_0): < 0 if negative */
    int32_t sysit_tr;                           /* transport: iterations summed over the
                                                   systems (a system leaves the batched solve
                                                   when it converges, so sysit_tr / it_tr
                                                   systems work per iteration on average)     */
} clot_stats;

typedef struct clot_ctx clot_ctx;

/* Fills the Appendix E constants; M_rxn = 2, n_corr = 0 (automatic), max_iter 5000,
 * rtol_p = rtol_s = rtol_tr = 1e-13, rtol_inner = 1e-4 (FP64 settings; the FP32 path
 * is run with rtol_s 1e-7, rtol_tr 1e-8, rtol_p 1e-8, rtol_inner 1e-4).  Never fails
 * for a non-NULL pointer. */
clot_status clot_params_default(clot_params* p);

/* Bytes of device workspace clot_create needs for these channels and precision. */
clot_status clot_query_workspace(const clot_channel* ch, int32_t n_ch, clot_precision prec, size_t* bytes);

/* Creates a context over n_ch independent channels.  dev_workspace: device memory of
 * at least the queried size, 256-byte aligned; hip_stream: a hipStream_t (NULL =
 * default stream).  Builds the mesh tables and the inflow profiles; all fields are
 * zero until clot_init_state or clot_set_field.  On its first step the context
 * creates one internal non-blocking stream of default priority, on which the eta
 * solve and the pressure preconditioner set-up run concurrently with the rest of the
 * step; it is joined into hip_stream by events within every step, so a step's
 * results are ordered on hip_stream.  It is destroyed with the context. */
clot_status clot_create(const clot_channel* ch, int32_t n_ch, const clot_params* p, clot_precision prec,
                        void* dev_workspace, size_t ws_bytes, void* hip_stream, clot_ctx** out);

/* Initial state of channel ch (fully developed inflow, its Poiseuille pressure,
 * margination platelets, S1_0, S2_0, E0_0, zero for the other species), every
 * species value multiplied by (1 + 0.01*xi).  xi_cell: 15*ncell float64 normal
 * draws (species in field order CLOT_PMU..CLOT_C2, cells x-fastest); xi_face:
 * 2*nface draws (E0 then C0). */
clot_status clot_init_state(clot_ctx* c, int32_t ch, const double* xi_cell, size_t n_cell,
                            const double* xi_face, size_t n_face);

clot_status clot_field_count(const clot_ctx* c, int32_t ch, clot_field f, size_t* n);
clot_status clot_set_field(clot_ctx* c, int32_t ch, clot_field f, const double* host, size_t n);
clot_status clot_get_field(clot_ctx* c, int32_t ch, clot_field f, double* host, size_t n);

/* Advances every channel by nsteps time steps; blocks until done.  Before the first
 * step the call copies the context's persistent state (fields, fluxes, clocks, release
 * and time-derivative histories) aside in its workspace, on the context stream; after
 * the last it scans the velocity, pressure and species for NaN or infinity.  If the scan
 * or any linear-solve reduction of the call met one, the state of the call's start is
 * restored (every channel) and CLOT_ENAN is returned; clot_get_stats then reports the
 * failed step's statistics and CLOT_W_NONFINITE. */
clot_status clot_step(clot_ctx* c, int32_t nsteps);

/* Enqueues nsteps steps on the context stream without waiting; returns a warning
 * only through clot_get_stats after a later synchronising call.  The first
 * asynchronous call after a synchronisation opens a window (the state is copied aside
 * as by clot_step); clot_sync closes it with the same scan and, on a non-finite value,
 * restores the window's start and returns CLOT_ENAN.  clot_set_field, clot_init_state
 * and clot_load_state end an open window without a check (the state they set is the
 * next window's start). */
clot_status clot_step_async(clot_ctx* c, int32_t nsteps);
clot_status clot_sync(clot_ctx* c);

/* Statistics of channel ch's last step.  Returns CLOT_OK, or the worst warning of any
 * step since the channel's last clot_init_state: CLOT_W_NOTCONV, CLOT_W_NONFINITE. */
clot_status clot_get_stats(const clot_ctx* c, int32_t ch, clot_stats* s);

/* Checkpoint and resume.  A context's state is its device workspace and its host side
 * (channel clocks and step counts, buffer parity, solver budgets, reaction mode); it
 * goes to and from a host blob of clot_state_size bytes, owned by the caller.
 * clot_load_state accepts a blob saved from a context created with the same channels
 * (every field of every clot_channel equal: the blob holds channel tables and clocks
 * built from them), precision and workspace size, else CLOT_EINVAL and the context is
 * unchanged; the model parameters remain the loading context's (its inflow profiles are
 * rebuilt from them after the load).  Both calls
 * wait for the context's streams; recorded graphs are dropped on load (graph mode
 * calibrates again).  Steps after a load continue bit for bit as from the saved one. */
clot_status clot_state_size(const clot_ctx* c, size_t* bytes);
clot_status clot_save_state(clot_ctx* c, void* host, size_t bytes);
clot_status clot_load_state(clot_ctx* c, const void* host, size_t bytes);

/* Selects the reaction integrator.  mode CLOT_RXN_SURROGATE takes a weight blob
 * (layout of clot_mlp_layout) and a residual threshold; a cell whose residual
 * exceeds it is recomputed by the plain RK4 integrator. */
clot_status clot_set_reaction_mode(clot_ctx* c, clot_rxn_mode mode, const void* mlp_blob, size_t blob_bytes,
                                   double resid_tol);

/* Cells per tile this library was built for (256, 512 or 1024): a tile is the
 * group of cells one 256-thread block owns, with its own partial sums.  The tile
 * size is a build option; the autotuner chooses among the built libraries. */
int32_t clot_tile_cells(void);

/* Cell species this library carries: 15 (the model of section 2 and Appendix B), or
 * 17 for the inhibitor build (section 3.4's extensibility example), which appends the
 * inhibitor I and the inhibited thrombin E2i (fields CLOT_I, CLOT_E2I).  That build
 * solves 9 transport equations and 16 reaction equations; I has the fixed inlet value
 * I_0 and starts there, E2i starts at zero, neither takes an initial-noise draw; its
 * learned reaction step, clot_rxn_rk4_batch and clot_surr_dataset return CLOT_EINVAL
 * (the network covers the base model's 14 reacting species). */
int32_t clot_cell_species(void);

/* Graph replay of whole steps (for ensembles stepped many times).
 * on != 0: the next two clot_step steps run as usual and record, per solve, the
 * largest Krylov iteration count (and the number of FP64 pressure refinement
 * passes).  Each later step replays a HIP graph recorded once per buffer parity
 * (the step rotates theta_B and the face fluxes between two buffers), in which
 * every solve runs a fixed budget of ceil(budget_scale * count) + budget_pad
 * iterations, and the pressure corrector the number of refinement passes seen (one
 * more per overflow noticed so far).  Channels that converge earlier skip the remaining iterations on the
 * device, so a replayed step gives bit-for-bit the result of the eager step.  A
 * channel still unconverged when its budget ends is counted as a failed solve in
 * the statistics (as max_iter is eagerly); the next synchronisation (clot_step with
 * wait, clot_sync) notices it, doubles the scale, adds 2 to the pad and re-records
 * the graphs.  Changing the reaction mode re-records them.  The probe does not time
 * replayed steps.  on == 0 returns to eager steps.  budget_scale >= 0, budget_pad
 * >= 1, else CLOT_EINVAL. */
clot_status clot_set_graph_mode(clot_ctx* c, int32_t on, double budget_scale, int32_t budget_pad);
/* info[0] graph mode on, [1] graphs recorded, [2] steps replayed, [3] budget
 * overflows noticed, [4..10] current budgets: momentum, pressure corrector 1, 2,
 * later correctors, eta, transport, pressure refinement passes; [11..17] the largest
 * counts seen by the calibrating eager steps, in the same order; [18] nodes of the
 * last recorded step, [19] the graphs it was recorded as (a step is cut into a chain
 * of graphs of about 1500 nodes each).  info: 20 entries. */
clot_status clot_graph_info(clot_ctx* c, int64_t* info);

/* Tile shapes of the LDS-staged kernels: the finest-level kernels of the momentum
 * preconditioner (a block owns a brick of 1024 cells and stages it with a one-cell halo
 * in LDS) and the legs of the pressure hierarchy's coarse levels (a brick of 1024 cells
 * with a halo of one cell per sweep; FP32 contexts, see mg_brick).  The tile autotuner
 * times each kernel in each shape and sets its choice; shape 0 is the default of every
 * kernel, and every shape gives the same step bit for bit.  Shapes (BX x BY x BZ cells),
 * one shape index naming a 3-D and a 2-D shape: momentum 3-D 32x8x4, 16x16x4, 32x4x8,
 * 16x8x8, 2-D 64x16, 128x8, 32x32, 256x4; pressure legs 3-D 16x8x8, 32x8x4, 8x8x16,
 * 16x16x4, 2-D 64x16, 128x8, 32x32, 256x4.  Contexts that do not run a bricked kernel
 * still record the choice. */
typedef enum {
    CLOT_BRICK_RESTRICT = 0,   /* momentum: residual restriction with the formed right-hand side */
    CLOT_BRICK_PROLONG = 1,    /* momentum: prolongation + smoothing sweep                        */
    CLOT_BRICK_SWEEP = 2,      /* momentum: the last smoothing sweep                              */
    CLOT_BRICK_P_DOWN = 3,     /* pressure: a coarse level's sweeps and restriction               */
    CLOT_BRICK_P_UP = 4,       /* pressure: a coarse level's prolongation and sweeps              */
    CLOT_NBRICK_KERNELS = 5
} clot_brick_kernel;
/* kernel in [0, CLOT_NBRICK_KERNELS), shape in [0, 4), else CLOT_EINVAL.  Recorded
 * graphs are dropped (re-recorded at the next step in graph mode). */
clot_status clot_set_brick_shape(clot_ctx* c, int32_t kernel, int32_t shape);
/* dims[0..2] = BX, BY, BZ of a momentum kernel's shape for channels of dimension dim
 * (2 or 3). */
clot_status clot_brick_dims(int32_t dim, int32_t shape, int32_t* dims);
/* dims[0..2] = BX, BY, BZ of the shape of the given bricked kernel (clot_brick_kernel)
 * for channels of dimension dim; CLOT_EINVAL for an invalid kernel, dim or shape. */
clot_status clot_brick_kernel_dims(int32_t kernel, int32_t dim, int32_t shape, int32_t* dims);

/* Kernel-phase timing probe.  While a phase is selected, every launch of it is
 * bracketed by HIP events on the context stream; clot_probe_read synchronises,
 * returns the summed event time (ms) and the launch count since the selection,
 * and keeps counting.  Selecting CLOT_PROBE_OFF stops it. */
typedef enum {
    CLOT_PROBE_OFF = 0,
    CLOT_PROBE_P_CG_A = 1,      /* pressure MG-PCG: direction update + stencil product   */
    CLOT_PROBE_P_CG_B = 2,      /* pressure MG-PCG: solution/residual update              */
    CLOT_PROBE_TR_B1 = 3,       /* transport BiCGStab phase 1 (p, v = A M^-1 p)           */
    CLOT_PROBE_TR_B2 = 4,       /* transport BiCGStab phase 2 (t = A M^-1 s)              */
    CLOT_PROBE_TR_B3 = 5,       /* transport BiCGStab phase 3 (x, r update)               */
    CLOT_PROBE_MOM_B1 = 6,
    CLOT_PROBE_MOM_B2 = 7,
    CLOT_PROBE_MOM_B3 = 8,
    CLOT_PROBE_RXN = 9,         /* cell reactions (RK4)                                   */
    CLOT_PROBE_TR_ASM = 10,     /* transport assembly                                     */
    CLOT_PROBE_ETA_CG_A = 11,
    CLOT_PROBE_ETA_CG_B = 12,
    CLOT_PROBE_P_RESID = 13,    /* FP64 pressure residual                                 */
    CLOT_PROBE_CORRECT = 14,    /* PISO flux and velocity correction                      */
    CLOT_PROBE_HBYA = 15,
    CLOT_PROBE_PRHS = 16,
    CLOT_PROBE_MOM_ASM = 17,
    CLOT_PROBE_P_MG_POST = 18,  /* pressure multigrid: finest-level smoothing sweep + r.z  */
    CLOT_PROBE_RXN_FALLBACK = 19, /* plain RK4 on the cells the surrogate rejected          */
    CLOT_PROBE_MOM_MG_R = 20,   /* momentum V-cycle: finest-level sweep + restriction      */
    CLOT_PROBE_MOM_MG_P1 = 21,  /* momentum V-cycle: prolongation + finest-level sweep     */
    CLOT_PROBE_MOM_MG_P2 = 22,  /* momentum V-cycle: last finest-level sweep               */
    CLOT_PROBE_P_MG_DOWN = 23,  /* pressure multigrid, bricked: a coarse level's down leg   */
    CLOT_PROBE_P_MG_UP = 24,    /* pressure multigrid, bricked: a coarse level's up leg     */
    CLOT_PROBE_P_MG_MESH_DOWN = 25, /* pressure multigrid: the mesh's down leg in one launch */
    CLOT_PROBE_P_MG_MESH_UP = 26,   /* pressure multigrid: the mesh's prolongation and next sweep */
    CLOT_PROBE_NKERNELS
} clot_probe_kernel;
clot_status clot_probe(clot_ctx* c, int32_t kernel);
clot_status clot_probe_read(clot_ctx* c, double* total_ms, int64_t* launches);

/* ---- learned reaction step: training and data (device pointers, caller's stream) ----
 * The surrogate (clot_set_reaction_mode) predicts the reaction increment of one
 * step as f (1 + clamp(sc_i c_i, -1/2, 1/2)) with f = Dt R(y + Dt R(y)/2) the
 * explicit-midpoint increment and c = MLP(features): 32 inputs -> 64 tanh -> 64 tanh -> 16 outputs (14 used),
 * BF16 weights/activations, FP32 accumulate.  The parameter vector (float32,
 * clot_mlp_nparam() entries) is W1[64][32] b1[64] W2[64][64] b2[64] W3[16][64]
 * b3[16]; the mode blob appends sf[14] and sc[14], the RMS over the training set of
 * the scaled explicit increments f/s and of the relative corrections (RK4 - f)/|f|.  The plain RK4 step (section 3.2) is the arbiter: a cell whose
 * midpoint defect relative to the increment, max over species of
 * |Delta_i - Dt R_i(y + Delta/2)| / (|Delta_i| + 1e-5 |y_i| + 1e-6 s_i) with s_i the
 * species scale (P_max for the platelets, S1_0 or S2_0 for the chemicals), exceeds
 * resid_tol is recomputed by it.
 * State rows for the batch calls: 18 float64 each = 14 species (Pmu Pma Pba Pbse S1
 * S2 E1 E2 S1b S2b E1b E2b C1 C2), ADP, eta, H_adh, Dt. */
int64_t clot_mlp_nparam(void);
size_t clot_mlp_backward_workspace(int64_t n);
/* y = MLP(x); x bf16 [n][32], y f32 [n][16]; cache (optional) bf16 [n][128] activations */
clot_status clot_mlp_forward(const float* w_f32, const uint16_t* w_bf16, const uint16_t* x_bf16, int64_t n,
                             float* y_f32, uint16_t* cache_bf16, void* hip_stream);
/* dw = d loss / d params given dy = d loss / d y; part: clot_mlp_backward_workspace(n) bytes */
clot_status clot_mlp_backward(const float* w_f32, const uint16_t* w_bf16, const uint16_t* x_bf16,
                              const uint16_t* cache_bf16, const float* dy_f32, int64_t n, float* part, float* dw_f32,
                              void* hip_stream);
/* The same gradient as clot_mlp_backward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops, harnesses
 * that forbid hipMalloc): the per-block partials live in a static device array inside
 * the library (7.5 MB, one copy per GPU, held until the process ends), so the call
 * allocates nothing and needs no workspace.  n <= 16384 samples, else CLOT_EINVAL
 * (message through clot_last_error(NULL)).  All
 * calls on one GPU share that array: calls that overlap on one GPU (concurrent
 * streams or threads) race and must be serialised by the caller; the first call on
 * each device looks the array up (hipGetSymbolAddress) with that device current. */
clot_status clot_mlp_backward_noalloc(const float* w_f32, const uint16_t* w_bf16, const uint16_t* x_bf16,
                                      const uint16_t* cache_bf16, const float* dy_f32, int64_t n, float* dw_f32,
                                      void* hip_stream);
/* Adam step t (>= 1) on the float32 master parameters; refreshes the bf16 copy */
clot_status clot_mlp_adam(float* w_f32, uint16_t* w_bf16, const float* grad, float* m, float* v, int64_t t,
                          double lr, double beta1, double beta2, double eps, void* hip_stream);
/* mean squared error over the first nuse outputs: dy, and per-256-sample loss partials */
clot_status clot_mlp_mse(const float* y, const float* target, int64_t n, int32_t nuse, float* dy, double* loss_part,
                         void* hip_stream);
/* plain RK4 reaction increments (M_rxn sub-steps, FP64) of n state rows: inc [n][14] */
clot_status clot_rxn_rk4_batch(const clot_params* p, const double* rows, int64_t n, double* inc, void* hip_stream);
/* training set from rows and their RK4 increments: bf16 features [n][32] and f32 targets
 * [n][16] with scales = sf[14], sc[14]; or, with stats != NULL, per-256-row block sums
 * (42 per block): squares of f/s, squares of the relative corrections, count of f != 0 */
clot_status clot_surr_dataset(const clot_params* p, const double* rows, const double* inc, int64_t n,
                              const float* scales, uint16_t* x_bf16, float* target, double* stats, void* hip_stream);
/* checks the MFMA operand layout: D = A B for 16x16 bf16 A, B (row major), f32 D */
clot_status clot_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, void* hip_stream);

void clot_destroy(clot_ctx* c);
/* the context's last error message; with c == NULL, that of the last failed clot_create
 * or context-free call that sets one (clot_mlp_backward_noalloc) on the calling thread */
const char* clot_last_error(const clot_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
