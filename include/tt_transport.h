/*
 * tt_transport.h -- C ABI of the MI355X (gfx950) tensor-train multigroup
 * radiation transport library.
 *
 * What the library computes (arXiv 2602.00290):
 *
 *   * The intensity is a tensor train over (space x group, polar angle,
 *     azimuthal angle):  I[k, l, p] = sum_{a,b} Z[k,a] Theta[a,l,b] Phi[b,p]
 *     with the merged spatio-spectral row index k = cell * N_nu + g
 *     (Section 3.1, the merged decomposition; cell = ix + Nx*(iy + Ny*iz)).
 *   * One time step applies the discretised multigroup discrete-ordinates
 *     operator: forward-Euler streaming with the upwind flux, then the
 *     backward-Euler operator-split absorption/emission update at fixed
 *     medium temperature with zero scattering and density 1 (Section 2.1,
 *     the discrete source equation), i.e.
 *        I* = I - sum_d lambda_d [n_d^+ (I_c - I_{c-e_d}) + n_d^- (I_{c+e_d} - I_c)]
 *        I' = (I* + c dt kappa eps) / (1 + c dt kappa),   lambda_d = c dt / dx_d,
 *     as a sum of n = 2 d_X rank-1 TT operators plus rank-1 boundary and
 *     emission terms (Appendix A), so the ranks grow to (n+1) r + n_bc + 1.
 *     Options: the Rusanov flux instead of upwind (tt_problem.flux), still
 *     two rank-1 operators per axis (Appendix A, "Value of n"); isotropic
 *     scattering (tt_problem.kappa_s_full), which enters the same rank-1
 *     isotropic source column; and the coupled medium temperature
 *     (tt_problem.heat_capacity).
 *   * Rank is restored by TT-SVD rounding (Oseledets 2011, the SVD rounding
 *     the paper uses, Section 3.1 footnote): right-to-left QR
 *     orthogonalisation, then left-to-right delta-truncated SVDs with
 *     delta = tol * ||I||_F / sqrt(2); each rank is also capped.  The first
 *     core's factorisation is Householder QR or an FP64 Gram matrix (the
 *     footnote's SVD and Gram methods); the footnote's randomized method
 *     compresses the sum to sketch ranks first (tt_problem.round_method).
 *   * Group emission eps_g(T) = 2 T^4 int x^3/(e^x - 1) dx over the group
 *     in units h = k = c_light = 1 (Section 2, group emission; the solver's
 *     own c is a separate input).
 *
 * Conventions for every entry point:
 *   * Host arrays passed in are read during the call and copied; the caller
 *     keeps ownership.  Device memory is never allocated by the library: the
 *     caller passes one device workspace (e.g. a torch uint8 tensor) of at
 *     least tt_transport_workspace_bytes() bytes, owns it, and must keep it
 *     alive until tt_transport_destroy().
 *   * `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on that stream and return without waiting, except
 *     those documented as synchronising.
 *   * Every call returns a tt_status; nothing aborts or throws across the
 *     ABI.  tt_transport_last_error() gives a thread-local message for the
 *     last failing call.  A NaN/Inf produced on the device is reported as
 *     TT_ERR_NUMERIC by the next synchronising call.
 *   * One handle must not be used from two host threads at once.  Handles
 *     are independent of each other.
 */
#ifndef TT_TRANSPORT_H
#define TT_TRANSPORT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TT_OK = 0,
    TT_ERR_INVALID_ARG = -1,   /* bad sizes, pointers, or option values          */
    TT_ERR_OOM = -2,           /* workspace smaller than required               */
    TT_ERR_NUMERIC = -3,       /* NaN / Inf detected in the state               */
    TT_ERR_HIP = -4,           /* a HIP runtime call failed                     */
    TT_ERR_STATE = -5          /* call not valid in the handle's current state  */
} tt_status;

/* Precision of the large core contractions (Z and the first-core projection).
 * The R factors, the SVDs and the truncation thresholds are always FP64. */
typedef enum {
    TT_PREC_FP64 = 0,   /* Z stored and contracted in FP64                       */
    TT_PREC_FP32 = 1,   /* Z stored in FP32, contractions on FP32 MFMA            */
    TT_PREC_BF16X = 2   /* Z stored in FP32, contractions as split BF16 (hi+lo)
                           products on BF16 MFMA with FP32 accumulation          */
} tt_precision;

/* How the first (M-row) core is factorised inside the rounding. */
typedef enum {
    TT_ROUND_QR = 0,    /* Householder TSQR in FP64, then an FP64 SVD of R
                           (TT-SVD rounding)                                      */
    TT_ROUND_GRAM = 1,  /* FP64 Gram matrix of the projected core, then an FP64
                           symmetric eigensolver (Gram rounding, Section 3.1
                           footnote); accurate when tol >> 1e-8                  */
    TT_ROUND_AUTO = 2,  /* QR for TT_PREC_FP64; Gram for FP32 / split-BF16 data,
                           whose own rounding (>= 6e-8) is above the Gram's
                           FP64 accuracy floor (~1.5e-8 relative)                */
    TT_ROUND_RAND = 3   /* randomized rounding (Section 3.1 footnote): each pass
                           first compresses the TT sum to sketch ranks
                           (incoming ranks + rand_oversample, at most the
                           sum's orthogonalised ranks) by randomize-then-
                           orthogonalize with a random TT drawn from
                           Philox-4x32-10 (key rand_seed; counter = entry,
                           core, number of rounding passes since create,
                           set_cores or reset), then truncates
                           like TT_ROUND_GRAM.  The sketch acts on the Gram of
                           the projected core, so it adds one single-workgroup
                           kernel and no pass over Z; same accuracy floor as
                           TT_ROUND_GRAM.                                        */
} tt_round_method;

typedef enum {
    TT_BC_VACUUM = 0,          /* ghost intensity 0                              */
    TT_BC_INFLOW_PLANCK = 1,   /* isotropic ghost intensity eps_g(bc_T[face])    */
    TT_BC_PERIODIC = 2,        /* wrap-around; both faces of the axis            */
    TT_BC_INFLOW_VALUES = 3    /* isotropic ghost intensity bc_values[face*N+g]  */
} tt_bc;

/* Problem statement (Section 2 and 2.1; quadrature and group conventions of
 * Section 4).  Faces are ordered x-, x+, y-, y+, z-, z+. */
/* Streaming flux (Section 2.1 names upwind, Rusanov and HLL).
 * Rusanov: F_{i+1/2} = (c n_d / 2)(I_i + I_{i+1}) - (S+ / 2)(I_{i+1} - I_i)
 * with S+ = rusanov_s * c; a ghost value enters both neighbours of every
 * direction on an inflow face.
 * HLL (the asymptotic-preserving flux; its only multigroup change is a
 * per-group optical depth): F_{i+1/2} = (c n_d / 2)(I_i + I_{i+1})
 * - (c |n_d| eps / 2)(I_{i+1} - I_i) with eps = (1 - exp(-tau)) / tau and
 * tau = hll_beta dx_d (kappa_i + kappa_{i+1}) / 2 in the group (the inside
 * cell's on a boundary face): upwind in thin cells, central differences in
 * thick ones.  Still two rank-1 operators per axis, whose spatial parts vary
 * per (cell, group) row (Appendix A).  Provided for FP64 data without
 * scattering or a coupled temperature. */
typedef enum { TT_FLUX_UPWIND = 0, TT_FLUX_RUSANOV = 1, TT_FLUX_HLL = 2 } tt_flux;

typedef struct tt_problem {
    int dim;                        /* 1, 2 or 3                                    */
    int n_cells[3];                 /* cells per axis (unused axes: 1)              */
    double extent[3];               /* domain [0, extent_d] per axis                */
    int n_groups;                   /* N_nu >= 1                                    */
    const double* group_edges;      /* N_nu + 1 edges, [0] = 0, [N_nu] = +inf       */
    const double* kappa0;           /* N_X spatial opacity factor (>= 0); may be
                                       NULL when kappa_full is given              */
    const double* kappa_group_scale;/* N_nu: kappa[cell,g] = kappa0[cell]*scale[g]
                                       (NULL allowed with kappa_full)             */
    const double* T_cell;           /* N_X fixed medium temperature (>= 0)          */
    int n_theta;                    /* polar nodes                                  */
    int n_phi;                      /* azimuthal nodes (must be 1 when dim == 1)    */
    const double* mu;               /* n_theta cos(theta) nodes in (-1, 1)          */
    const double* w_theta;          /* n_theta polar weights                        */
    const double* phi;              /* n_phi azimuth nodes (ignored when dim == 1)  */
    const double* w_phi;            /* n_phi azimuthal weights                      */
    int bc[6];                      /* tt_bc per face                               */
    double bc_T[6];                 /* temperatures for TT_BC_INFLOW_PLANCK          */
    const double* bc_values;        /* 6*N_nu values for TT_BC_INFLOW_VALUES or NULL */
    double c;                       /* propagation speed                            */
    double cfl;                     /* dt = cfl / (c * sum_d 1/dx_d)                */
    double tol;                     /* relative rounding tolerance                  */
    int rank_cap;                   /* cap on both TT ranks (>= 1)                  */
    int precision;                  /* tt_precision                                 */
    int round_method;               /* tt_round_method                              */
    int paper_step_order;           /* 0: one rounding per step after transport and
                                       source; 1: round after transport and again
                                       after the source (Section 3.1)              */
    double heat_capacity;           /* rho c_v per unit volume (the density and
                                       specific heat of Section 2).  0: the medium
                                       temperature stays T_cell.  > 0: it is coupled
                                       (Section 2.1, the coupled source stage): each
                                       step takes the stage temperature T+ of every
                                       cell as the root of the paper's scalar
                                       equation, updates the intensity with
                                       eps_g(T+), and advances T by total-energy
                                       conservation with the angle means of the
                                       rounded new state.  With paper_step_order 1
                                       the stage acts on the rounded state after
                                       transport (its angle means are J*) and is
                                       rounded again.  Such a problem advances only
                                       through tt_transport_solve / step_batch /
                                       solve_batch.                                 */
    const double* T_rad0;           /* N_X initial radiation temperature (isotropic
                                       Planck initial state), or NULL for T_cell  */
    const double* kappa_full;       /* N_X * N_nu opacities kappa_{a,g}(x) (>= 0),
                                       row cell * N_nu + g, for fields that do not
                                       factor (several materials: the opacity
                                       matrix then has rank N_materials, Section 4
                                       and the internal-structure discussion), or
                                       NULL for kappa0 x kappa_group_scale.  Copied
                                       to the workspace (N_X N_nu doubles more).  */
    int flux;                       /* tt_flux (0: upwind)                          */
    double rusanov_s;               /* S+ / c of the Rusanov flux, in [0, 1] (1: S+ = c;
                                       0: central differences, the Gaussian
                                       diffusion setting of Section 4)              */
    const double* kappa_s_full;     /* N_X * N_nu isotropic scattering opacities
                                       kappa_{s,g}(x) >= 0, row cell * N_nu + g, or
                                       NULL for none.  The source update becomes
                                       I' = (I* + a eps + b J') / (1 + a + b) with
                                       a = c dt kappa, b = c dt kappa_s and
                                       J' = (J* + a eps) / (1 + a) the angle mean
                                       of the update (J* that of I*): a per-step
                                       pre-pass computes J* from the cores (from
                                       the rounded state after transport with
                                       paper_step_order 1).  Such a problem advances
                                       only through solve / step_batch / solve_batch
                                       (apply_op returns TT_ERR_STATE).  Adds 2 N_X
                                       N_nu doubles of workspace (3 without a
                                       coupled temperature).                        */
    int rand_oversample;            /* TT_ROUND_RAND: sketch ranks = solution ranks
                                       + this, in [1, 128] (the paper's comparison
                                       uses 4); ignored by the other methods        */
    unsigned long long rand_seed;   /* TT_ROUND_RAND: generator key; the same key
                                       reproduces a solve bit for bit              */
    double hll_beta;                /* TT_FLUX_HLL: optical-depth factor beta of the
                                       interface wave-speed reduction (> 0; the
                                       paper's HLL runs use 20)                      */
} tt_problem;

/* Statistics of the last solve / round (Section 3.2 metrics). */
typedef struct tt_stats {
    int steps;            /* steps taken by the last solve                           */
    int r1, r2;           /* current ranks                                            */
    int max_R1, max_R2;   /* largest pre-rounding ranks seen                          */
    int nan_flag;         /* 1 if a NaN/Inf was seen                                  */
    double norm;          /* ||I||_F before the last truncation                       */
    double discarded_rel; /* sqrt(sum of discarded sigma^2) / norm, last rounding     */
    double energy;        /* dV * sum_k sum_lp w_l w_p I[k,l,p] of the current state */
    double k_s;           /* storage factor of the last rounding pass (Section 3.2
                             k_s): entries of the TT sum before rounding (ranks
                             R1, R2, as SVD rounding forms it) over the entries
                             of the rounded TT; 1 before the first pass          */
    double compression;   /* N_X N_nu N_theta N_phi / TT entries (Section 3.2 eq.)    */
    double seconds;       /* wall time of the last solve (host clock, synchronised)  */
    double kernel_ms[10]; /* summed HIP-event durations per kernel class when timing
                             is on: [0] prep, [1] project (the gathered first-core
                             contraction; a few microseconds when the pass runs
                             in direction space), [2] factor (TSQR or Gram),
                             [3] factor tree / reduce, [4] small-core SVD chain,
                             [5] output contraction, [6] diagnostics, [7] source
                             pre-pass (coupled medium temperature and / or
                             scattering), [8] angle (Y = Z W of the direction-space
                             projection), [9] stencil (its per-direction stencil;
                             both launched on every eligible pass, a few
                             microseconds when the pass is not in direction space) */
    long long kernel_launches[10]; /* launches counted per class                     */
    double flops[10];     /* executed flops per class, summed over the solve          */
    double medium_energy; /* dV * heat_capacity * sum_x T[x] (0 when T is fixed); the
                             radiation energy is energy / c                          */
    int sketch_r1, sketch_r2; /* TT_ROUND_RAND: ranks of the last randomized
                             compression after null sketch directions were
                             dropped (0 for the other methods)                       */
    double k_s_impl;      /* this library's peak storage in the last pass (input Z,
                             stored projected core M x k1 unless the pass is
                             fused, and Y = Z W beside it when the pass projected
                             in direction space, output Z, the R1 x N_theta x R2
                             core) over the
                             entries of the rounded TT; the TT sum itself is
                             never formed                                             */
    int direction_space_rounds; /* rounding passes since create / reset whose
                             projection ran in direction space (FP64 data,
                             128-column cores, both small-core factors square):
                             Y = Z W, then the operator's stencil on Y          */
} tt_stats;

/* Internal delta-ranks of the combined core Z (section "Internal structure of
 * the combined core" and its relative compression equations). */
typedef struct tt_internal_ranks {
    int r_nux;        /* delta-rank of the N_nu x (N_X r1) unfolding of Z'        */
    int r_xnu;        /* delta-rank of the N_X x (N_nu r1) unfolding of Z'        */
    double C_rel_nu;  /* TT entries / entries with Z split as (frequency, space)  */
    double C_rel_x;   /* TT entries / entries with Z split as (space, frequency)  */
    int n_sv_nu;      /* number of singular values of the first unfolding        */
    int n_sv_x;       /* number of singular values of the second unfolding       */
} tt_internal_ranks;

typedef struct tt_handle tt_handle;

/* Bytes of device workspace needed for `p` at its rank cap.  FP64 and FP32
 * problems whose projected first core can exceed 64 columns also hold
 * Y = Z W (M rows of up to 128 elements of the data type, 32 elements of
 * padding each; FP32 also an FP32 copy of W) for the direction-space
 * projection.  Returns 0 for an
 * invalid problem (see tt_transport_last_error). */
size_t tt_transport_workspace_bytes(const tt_problem* p);

/* Create a solver.  Validates `p`, computes host-side setup in FP64 (dt,
 * group emission, angular factors), carves `dev_workspace` and uploads the
 * inputs and the rank-1 initial state I0 = eps_g(T_cell) (x) 1 (x) 1
 * (isotropic Planck state at the medium temperature).  Synchronises.
 * Errors: TT_ERR_INVALID_ARG, TT_ERR_OOM (bytes too small), TT_ERR_HIP. */
tt_status tt_transport_create(const tt_problem* p, void* dev_workspace, size_t bytes,
                              void* stream, tt_handle** out);

/* The same as tt_transport_create, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the workspace is a static array of 64 MiB that the
 * library holds on each device from module load until the process ends, so
 * this call allocates nothing.  It serves problems whose
 * tt_transport_workspace_bytes() is at most 64 MiB (small requests such as
 * the 1D slab, ~1 MiB); larger ones fail with TT_ERR_INVALID_ARG.  One
 * handle at a time may hold a device's array: a second call on the same
 * device fails with TT_ERR_STATE until the first handle is destroyed.
 * Work of a destroyed handle still in flight on a stream races with the
 * next handle's: synchronise the stream before tt_transport_destroy.  The
 * array keeps the last handle's contents; creation initialises everything a
 * solve reads.  Synchronises like tt_transport_create.
 * Errors: TT_ERR_INVALID_ARG, TT_ERR_STATE, TT_ERR_HIP. */
tt_status tt_transport_create_noalloc(const tt_problem* p, void* stream, tt_handle** out);

/* Apply the transport + source operator once without rounding (Appendix A):
 * afterwards the handle holds the unrounded TT sum with ranks
 * (n+1) r + n_bc + 1; tt_transport_get_cores materialises it.  With
 * paper_step_order = 1 this applies the transport half only. */
tt_status tt_transport_apply_op(tt_handle* h, void* stream);

/* Round the handle's TT (a pending unrounded sum or a plain state) with the
 * given tolerance and rank cap (rank_cap <= the problem's cap). */
tt_status tt_transport_round(tt_handle* h, double tol, int rank_cap, void* stream);

/* n_steps full steps (apply + round, or the paper's two-round order).  No host
 * synchronisation inside; `out` (may be NULL) is filled after a final
 * synchronisation. */
tt_status tt_transport_solve(tt_handle* h, int n_steps, tt_stats* out, void* stream);

/* Reset the state to the rank-1 initial condition. */
tt_status tt_transport_reset(tt_handle* h, void* stream);

/* Current ranks (synchronises). */
tt_status tt_transport_get_ranks(tt_handle* h, int* r1, int* r2);

/* Copy the current cores to host FP64 arrays: Z (M x r1, row-major),
 * Theta (r1 x n_theta x r2), Phi (r2 x n_phi).  Any pointer may be NULL.
 * Synchronises.  A pending unrounded sum is returned as its explicit cores. */
tt_status tt_transport_get_cores(tt_handle* h, double* Z, double* Theta, double* Phi,
                                 void* stream);

/* Replace the state by host FP64 cores of ranks (r1, r2) <= the caps
 * (checkpoint restore, tests).  Synchronises. */
tt_status tt_transport_set_cores(tt_handle* h, int r1, int r2, const double* Z,
                                 const double* Theta, const double* Phi, void* stream);

/* Copy the medium temperature per cell (N_X doubles, cell = ix + Nx*(iy + Ny*iz))
 * to host memory owned by the caller: the current values of a coupled problem
 * (heat_capacity > 0), else T_cell as given.  Synchronises `stream` for a
 * coupled problem.  Errors: TT_ERR_INVALID_ARG (NULL handle or T), TT_ERR_HIP. */
tt_status tt_transport_get_temperature(tt_handle* h, double* T, void* stream);

/* Internal delta-ranks of the current combined core (section "Internal
 * structure of the combined core").  Z' = Z L_Theta is Z in the gauge where
 * Theta and Phi are right-orthonormal, so that a truncation of Z' carries the
 * same Frobenius error as of the whole tensor.  r_nux is the smallest k whose
 * singular-value tail of reshape(Z', [N_nu, N_X r1]) is <= delta times the
 * norm of all of them, r_xnu the same for reshape(Z', [N_X, N_nu r1]); C_rel_nu
 * and C_rel_x are the paper's relative compression ratios for the two split
 * topologies.  The singular values (descending; out->n_sv_nu = N_nu and
 * out->n_sv_x = min(N_X, N_nu r1) of them) are copied to sv_nu / sv_x, at most
 * n_sv_nu / n_sv_x each; either pointer may be NULL.  The Gram of the
 * N_X x (N_nu ld) unfolding is formed in FP64 on the device in the handle's
 * round scratch, then reduced on the host, so singular values below about
 * 1e-8 of the largest are not resolved.  Synchronises `stream`.
 * Errors: TT_ERR_INVALID_ARG (NULL handle/out, delta < 0, N_nu * ld > 2048),
 * TT_ERR_STATE (an unrounded sum is pending, or the scratch is too small),
 * TT_ERR_HIP. */
tt_status tt_transport_internal_ranks(tt_handle* h, double delta, tt_internal_ranks* out, double* sv_nu,
                                      int n_sv_nu, double* sv_x, int n_sv_x, void* stream);

/* Replay the step sequence as a HIP graph (on = 1) or launch every kernel
 * (on = 0, the default).  With graphs on, tt_transport_solve captures two
 * steps (the kernels of every rounding pass of both, and nothing else) into a
 * graph on first use, then launches that graph once per two steps; an odd
 * last step is launched kernel by kernel.  The result is bitwise the same as
 * without graphs.  Needs a non-null stream; graphs are not used while kernel
 * timing is on or an unrounded operator is pending.  on = 0 frees the graphs. */
tt_status tt_transport_set_graph(tt_handle* h, int on);

/* Launch shapes (grid sizes) of the persistent contraction kernels, for
 * tt_transport_tune, tt_transport_set_launch and tt_transport_get_launch.  A
 * block count of 0 means the plan launches no such kernel (on input: keep).
 * The kernels are the projection B = Z_new L_Theta (FP64 MFMA contractions;
 * with FP32 data the fused projection + FP64 Gram), the output
 * Z_out = B V_r (or its fused FP32 form from Z), and the FP64 Gram of a
 * stored first core (one row range and one partial per block; its grid is
 * rounded to whole row ranges of a multiple of 16 rows, at least 64).  These
 * are the contractions of the rounding pass (Sec. 3.1, the first-core steps
 * of the TT rounding); their grids change only the order of the Gram's
 * partial sums, never what is computed. */
typedef struct tt_tuning {
    int project_blocks;            /* blocks of the projection kernel */
    int output_blocks;             /* blocks of the output kernel */
    int gram_blocks;               /* blocks of the Gram kernel */
    int from_cache;                /* out (tune): 1 if the shapes came from the cache file, untimed */
    double project_ms, output_ms, gram_ms;                 /* out (tune): ms per launch at the chosen shapes */
    double project_ms_default, output_ms_default, gram_ms_default;   /* out (tune): ms per launch at the plan's defaults */
} tt_tuning;

/* Launch-shape autotuning (batching extension: launch shapes per workload).
 * Times candidate grids of each tunable kernel of the handle's rounding pass
 * (64 to 1024 blocks, up to the plan's maximum) on the handle's current state
 * and keeps the fastest for this handle, unless it is within 2 % of the
 * plan's default.  The state is not changed: the kernels write only the
 * handle's round scratch (B, Gram partials, the next Z buffer), and the gather
 * operand the tuner prepares is the one the next rounding pass prepares
 * again.  Tune once the ranks are representative (after the first steps of a
 * solve), since the best grid depends on them.  cache_path (may be NULL) names
 * a text file, one line per tuned problem: "key project output gram", the key
 * naming the device (architecture, compute units) and the problem's shape
 * (precision, rounding route, rows, groups, dimension, angles, rank caps,
 * flux), not the current ranks; a matching line is applied without timing or
 * touching the device (out->from_cache = 1), so a new handle of a tuned
 * problem can take its grids before its first step; otherwise the result is
 * appended.
 * One writer per file.  Drops captured graphs.  Synchronises `stream`.
 * Errors: TT_ERR_INVALID_ARG (NULL handle/out, cache file not writable),
 * TT_ERR_STATE (an unrounded operator is pending), TT_ERR_HIP. */
tt_status tt_transport_tune(tt_handle* h, const char* cache_path, tt_tuning* out, void* stream);

/* Set launch shapes explicitly (the *_ms fields and from_cache are ignored;
 * a block count of 0 keeps the current one).  Errors: TT_ERR_INVALID_ARG
 * (NULL arguments, a count outside [1, maximum], or a count for a kernel the
 * plan does not launch).  Drops captured graphs. */
tt_status tt_transport_set_launch(tt_handle* h, const tt_tuning* shapes);

/* The current launch shapes and the largest allowed (either may be NULL). */
tt_status tt_transport_get_launch(tt_handle* h, tt_tuning* current, tt_tuning* maximum);

/* Fill `out` with the statistics of the current state (synchronises). */
tt_status tt_transport_get_stats(tt_handle* h, tt_stats* out);

/* Record HIP events around every kernel launch and accumulate their
 * durations into tt_stats.kernel_ms (on = 1) or stop (on = 0). */
tt_status tt_transport_set_timing(tt_handle* h, int on);

/* One full step for each of n independent handles (batched solves).  Handle i
 * runs on streams[i % n_streams] (hipStream_t values), and the host enqueues
 * the handles' steps interleaved, so requests on different streams overlap on
 * the device (the single-workgroup SVD kernels of different handles run on
 * different compute units).  Handles must be distinct.  Asynchronous. */
tt_status tt_transport_step_batch(tt_handle** hs, int n, void** streams, int n_streams);

/* n_steps steps of every handle as in tt_transport_step_batch, then a
 * synchronisation of all streams; out (may be NULL) receives n stats. */
tt_status tt_transport_solve_batch(tt_handle** hs, int n, int n_steps, void** streams, int n_streams,
                                   tt_stats* out);

/* Advance many small independent requests with one persistent ragged kernel
 * (the batching of many solves with different grids, group counts, ranks and
 * step counts): handle i takes n_steps[i] full steps, each request in one
 * 1024-thread workgroup that runs the whole apply + round path of every step
 * (small-core QR, gather projection, Householder QR of the first core, SVD
 * chain, output contraction) without a launch per kernel, up to 256 requests
 * per launch side by side.  Eligible handles: FP64 data, Householder QR
 * rounding (TT_ROUND_QR, or AUTO with FP64), a projected first core of at most
 * 16 columns (N_theta N_phi <= 16, e.g. 1D slabs with up to 16 directions),
 * one rounding per step, no coupled temperature or scattering, timing off;
 * others fail with TT_ERR_INVALID_ARG naming the reason.  A request's result
 * does not depend on the other requests of the batch.  Runs on `stream`,
 * then synchronises it; out (may be NULL) receives n stats. */
tt_status tt_transport_solve_small_batch(tt_handle** hs, int n, const int* n_steps, void* stream, tt_stats* out);

/* Release the handle's host resources.  Never frees the caller's workspace. */
tt_status tt_transport_destroy(tt_handle* h);

/* Message of the last failing call on this thread ("" if none). */
const char* tt_transport_last_error(void);

/* Group emission coefficients eps_g(T), N_nu values, computed by the
 * library's host routine (series evaluation, see the source). */
tt_status tt_transport_group_emission(const double* edges, int n_groups, double T, double* out);

#ifdef __cplusplus
}
#endif

#endif /* TT_TRANSPORT_H */
