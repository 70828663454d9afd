/*
 * cuth.h - C ABI of the MI355X (gfx950) layered-stencil thermal solver.
 *
 * The library solves the symmetric positive definite 7-point finite-volume
 * system of a layered 3D-IC grid (paper Section 3.2):
 *
 *   steady:     sum_i g_{0,i}(T_0 - T_i) + h S_0 T_0 = p_0 V_0 + h S_0 T_amb
 *               (eq. "steady-state"), i.e. G T = P;
 *   transient:  C_0 V_0 (T_{0,n+1} - T_{0,n}) / dt + sum_i g_{0,i}(T_{0,n+1} - T_{i,n+1})
 *               + h S_0 T_{0,n+1} = p_{0,n+1} V_0 + h S_0 T_amb
 *               (eq. "transient", backward Euler), i.e. (C/dt + G) T_{n+1} = P + (C/dt) T_n;
 *
 * with preconditioned conjugate gradient (Algorithm 1), the Chebyshev polynomial
 * preconditioner (Section 4.3, "Chebyshev Polynomial Preconditioning") and
 * spectral bounds from an FP32 Lanczos process with an FP64 eigensolve of the
 * tridiagonal on the host (Section 4.3 last paragraph, Section 4.4
 * "component-wise precision in Lanczos").  In mixed precision the inner PCG runs
 * in FP32 and the residual r = P - G T and the update of T run in FP64
 * (iterative refinement; the FP64 "true residual" and "hot restart" of
 * Section 4.4).
 *
 * Grid: cell (i, j, l), i along x, j along y, l the layer counted from the
 * bottom; every vector is contiguous in the flat order  i + nx*(j + ny*l).
 * Units: lengths m, conductivity W/(m K), heat capacity J/(m^3 K), h W/(m^2 K),
 * power W per cell (the p_0 V_0 product), temperature K.
 *
 * Conventions for every call:
 *  - Vectors named "device" are caller-owned device memory on the handle's
 *    device (e.g. torch tensor data pointers), contiguous, of the stated type.
 *    The library never frees them.  Host arrays are copied before returning.
 *  - All device work is ordered on the HIP stream given at create time.  Calls
 *    that return results or statistics synchronise that stream before return.
 *  - Errors are reported by return code only; cuth_last_error() gives a
 *    thread-local message for the last non-OK status of the calling thread.
 *    CUTH_E_INVALID is returned before any device work when host-side
 *    arguments are bad.
 *  - A handle may be used by one thread at a time.
 *
 * Environment (tuning and diagnostics; none is needed for correct results):
 *  - CUTH_FUSE=0/1: never / always fuse the general FP32 Chebyshev sweeps in
 *    pairs (unset: chosen per grid or batch by timing); CUTH_FUSE_SHAPE="R,zc"
 *    with CUTH_FUSE=1: rows per workgroup and layers per chunk (default 2,8).
 *  - CUTH_FUSE3=0/1: never / always fuse them in triples, with pairs for the
 *    sweeps left over (unset: chosen by timing against the single sweeps or
 *    pairs that won; with CUTH_FUSE unset, =1 takes the first triple shape
 *    that fits);
 *    CUTH_FUSE3_SHAPE="R,zc" with CUTH_FUSE=1 and CUTH_FUSE3=1 (default 4,8).
 *  - CUTH_AUTOTUNE_CACHE=<file>: keep the tuned tile shapes of batches there.
 *  - CUTH_GRAPH=0/1: replay CG chunks from captured HIP graphs, kept by the
 *    handle between solves (default: batches, and single solves of grids of
 *    at most 2^21 unknowns, whose kernels are shorter than a host launch).
 *  - CUTH_REDUCE_ABOVE=<n>: workgroups per problem above which the CG sums go
 *    through a separate reduce launch (default 4096).
 *  - CUTH_LOG=1: tuning results and one line per refinement cycle on stderr.
 * Fused and single sweeps compute the same polynomial in the same order of
 * operations; the choice changes speed, not results beyond FP32 rounding.
 */
#ifndef CUTH_H
#define CUTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cuth_grid_s *cuth_grid;

typedef enum {
    CUTH_OK = 0,
    CUTH_E_INVALID = 1,        /* bad argument (checked before device work)          */
    CUTH_E_NOMEM = 2,          /* device allocation failed                            */
    CUTH_E_DEVICE = 3,         /* a HIP call failed                                   */
    CUTH_E_NOT_CONVERGED = 4,  /* iteration limit hit; best iterate returned          */
    CUTH_E_BREAKDOWN = 5       /* p^T A p <= 0 or a non-finite value in the iteration */
} cuth_status;

typedef enum {
    CUTH_FP64 = 0,    /* every step in FP64                                         */
    CUTH_MIXED = 1,   /* FP32 inner PCG + FP64 residual and refinement update        */
    CUTH_MIXED16 = 2, /* as CUTH_MIXED, and the Chebyshev sweeps read the lateral
                         conductances from FP16 copies (Section 4.2, the
                         half-precision copy of the in-plane diagonals; Section
                         4.4, component-wise precision in preconditioning).  Each
                         layer's values are stored as fp16(fp32(g * 2^e_l)),
                         e_l = 14 - ceil(log2(max g of the layer)), and promoted
                         to FP32 and scaled by 2^-e_l before use.  CG products,
                         checks and Lanczos use the FP32 conductances.  Same as
                         CUTH_MIXED for grids without k_lat_mult.             */
    CUTH_ADAPTIVE = 3, /* the paper's stage-switched scheme (Section 4.4): CG
                         vectors, scalars and inner products in FP64; the
                         Chebyshev preconditioner in FP32 with the FP16-stored
                         lateral conductances (as CUTH_MIXED16); the CG product
                         with FP32-stored conductances promoted to FP64 in the
                         early stage, FP64 ones in the late stage.  The early
                         stage ends when ||r_low|| <= sqrt(tol) ||b|| (eq.
                         switching a, relative), or when the FP64 true residual,
                         checked every check_period iterations, stagnates (b)
                         or drifts from r_low (c); the switch recomputes
                         r = b - A T in FP64 and restarts p (hot restart).
                         Stops at ||b - A T|| <= tol ||b|| (tol as CUTH_FP64). */
    CUTH_FP32 = 4     /* ablation baseline (Section 5, Ablation II, fixed FP32): one
                         PCG entirely in FP32 (vectors, scalars, operator,
                         preconditioner) that stops when its own recursive FP32
                         residual meets ||r|| <= tol ||b|| (tol as CUTH_FP64), with
                         no FP64 refinement and no drift or stagnation test.  The
                         result is the FP32 iterate; stats.rel_residual is its
                         FP64 true residual, which may be far above tol (the
                         drift this baseline exists to show).  CUTH_OK unless a
                         breakdown or max_inner ends the iteration.           */
} cuth_precision;

/* cuth_options.cheb_degree: pick the degree from the spectral interval. */
#define CUTH_DEGREE_AUTO (-1)

/* Preconditioner of the inner PCG.  The Chebyshev polynomial is the paper's
 * (Section 4.3); Jacobi and none are the baselines of its Ablation III
 * (Section 5), here as single element-wise passes. */
typedef enum {
    CUTH_PC_CHEBYSHEV = 0,  /* z = q(A) r, degree cheb_degree, Lanczos bounds     */
    CUTH_PC_JACOBI = 1,     /* z = r / diag(A), diag = sink + face conductances   */
    CUTH_PC_NONE = 2,       /* z = r (plain CG); no Lanczos setup either         */
    CUTH_PC_CHEBYSHEV_JACOBI = 3 /* beyond the paper: z = q(D^{-1} A) D^{-1} r, the
                               Chebyshev polynomial of the Jacobi-scaled operator
                               (D = diag(A) = sink + face conductances), degree
                               cheb_degree, on the interval of D^{-1} A from
                               Lanczos on D^{-1/2} A D^{-1/2} (upper end capped
                               by 2, a bound of that spectrum).  Narrows the
                               interval of layered stacks (config 0: condition
                               number 7.2e4 -> 1.25e4).  Not with CSR storage. */
} cuth_preconditioner;

/* Storage of the operator in the CG and Chebyshev products.  The matrix-free
 * layered stencil is the paper's (Section 4.2: direct addressing, coalesced
 * loads); CSR with one thread per row is the baseline of its Ablation I (and of
 * the optimisation-off columns of Ablation III), Section 5.  CSR runs the same
 * PCG kernels with only the product changed; it needs precision CUTH_FP64 and
 * fewer than 2^31 nonzeros (7 per cell at most), builds the CSR copy of each
 * operator (steady, and per dt) on first use and keeps it with the grid; the
 * Lanczos bounds and the once-per-restart FP64 residual still use the stencil,
 * and stats.alg_bytes still counts the stencil's bytes.  Single solves and
 * transient steps only (cuth_solve_batch returns CUTH_E_INVALID). */
typedef enum {
    CUTH_STORAGE_STENCIL = 0,  /* matrix-free stencil (default)                   */
    CUTH_STORAGE_CSR = 1       /* CSR copy of the FP64 operator, row-wise products */
} cuth_storage;

/* Grid descriptor.  Conductances follow the series (harmonic) half-cell rule:
 * a lateral face between cells a and b of layer l has
 *   g = (face area) / (d/(2 k_a) + d/(2 k_b)),  k = k_lat[l] * k_lat_mult[cell];
 * a vertical face between layers l and l+1 has
 *   g = dx dy / (dz[l]/(2 k_vert[l]) + dz[l+1]/(2 k_vert[l+1])).
 * The top layer has a convective conductance h_top*dx*dy to ambient, the bottom
 * layer h_bottom*dx*dy; the four sides are adiabatic. */
typedef struct {
    int32_t nx, ny, nz;          /* cells per axis, each >= 1, nz <= 64               */
    double dx, dy;               /* lateral cell pitch (m), > 0                       */
    const double *dz;            /* host [nz] layer thickness (m), > 0                */
    const double *k_lat;         /* host [nz] lateral conductivity, > 0               */
    const double *k_vert;        /* host [nz] vertical conductivity, > 0              */
    const double *k_lat_mult;    /* device [nx*ny*nz] lateral multiplier (> 0, finite)
                                    or NULL for per-layer-uniform conductivity        */
    const double *heat_cap;      /* host [nz] volumetric heat capacity (> 0), or NULL
                                    (then transient calls are invalid)                */
    double h_top, h_bottom;      /* >= 0; steady solves need h_top + h_bottom > 0     */
    double t_amb;                /* ambient temperature (K), finite                    */
} cuth_grid_desc;

typedef struct {
    int32_t precision;           /* cuth_precision                                     */
    double tol;                  /* 0 selects the default.  CUTH_MIXED(16): target
                                    relative error of the rise T - T_amb (inf-norm),
                                    default 1e-8.  CUTH_FP64, CUTH_ADAPTIVE: relative
                                    residual ||b - A T|| / ||b||, default 1e-10 for
                                    steady and 1e-12 for transient solves; a
                                    transient solve at the default whose residual
                                    stops falling between the two ends without
                                    error (a stiff step, large dt, can have an
                                    FP64 floor above 1e-12).                          */
    int32_t cheb_degree;         /* Chebyshev degree k, 1..256 (default 30), or
                                    CUTH_DEGREE_AUTO: the smallest k >= 2 with
                                    2 s^k <= 0.3, s = (sqrt(c) - 1)/(sqrt(c) + 1),
                                    c = lambda_max/lambda_min of the preconditioner's
                                    interval, at most 64 (the damping the Chebyshev
                                    polynomial gives on that interval; not from the
                                    paper); a batch takes the largest over its
                                    systems.  stats.cheb_degree reports the choice. */
    int32_t lanczos_steps;       /* Lanczos steps m, 2..256 (default 30)               */
    int32_t max_inner;           /* CG iterations per inner solve (default 2000)       */
    int32_t max_outer;           /* refinement cycles, CUTH_MIXED (default 12)         */
    int32_t use_initial_guess;   /* 1: T holds the initial guess on entry (cuth_solve) */
    int32_t check_period;        /* iterations between true-residual checks, 0 = the
                                    default (20 steady, 5 transient)                   */
    int32_t preconditioner;      /* cuth_preconditioner (default CUTH_PC_CHEBYSHEV)    */
    int32_t storage;             /* cuth_storage (default CUTH_STORAGE_STENCIL)        */
} cuth_options;

typedef struct {
    int32_t outer_cycles;        /* FP64 residual evaluations that fed an inner solve  */
    int32_t cg_iters;            /* total CG iterations                                */
    int64_t stencil_applies;     /* operator applications incl. Chebyshev and checks   */
    int32_t stop_reason;         /* last inner solve: 1 tol, 2 drift, 3 stagnation,
                                    4 breakdown, 5 iteration limit                      */
    int32_t cheb_degree;         /* Chebyshev degree used (1 without Chebyshev)        */
    int32_t drift_stops;         /* inner solves stopped by the drift test (Section 4.4,
                                    eq. switching c: ||r_true - r_low|| >= 0.5 ||r_true||) */
    int32_t stagnation_stops;    /* inner solves stopped by the stagnation test (eq.
                                    switching b: ||r_true|| > 0.9 ||r_true|| of the
                                    previous check while ||r_low|| fell since it)     */
    double rel_residual;         /* final ||b - A theta||_2 / ||b||_2 (FP64)           */
    double err_est;              /* mixed: last correction ||delta||_inf/||theta||_inf */
    double setup_ms;             /* coefficient/Lanczos setup inside this call         */
    double solve_ms;             /* solve phase                                        */
    double alg_bytes;            /* algorithmic HBM bytes of the solve phase           */
    double lambda_min, lambda_max; /* spectral bounds used by the preconditioner       */
} cuth_stats;

/* Fill *o with the defaults listed above. */
void cuth_default_options(cuth_options *o);

/* Create a handle for one grid on the current HIP device.  hip_stream is a
 * hipStream_t (NULL = the default stream).  Builds the face conductances on the
 * device (FP64 and FP32 copies when k_lat_mult is given).  Validates the
 * descriptor on the host; the multiplier field is checked on the device
 * (CUTH_E_INVALID if any entry is <= 0 or not finite). */
cuth_status cuth_grid_create(const cuth_grid_desc *desc, void *hip_stream, cuth_grid *out);

/* Release every allocation of the handle (NULL is a no-op). */
void cuth_grid_destroy(cuth_grid g);

/* New layer conductivities for an existing grid, e.g. the steps of a design
 * loop driven by the per-layer gradient of cuth_adjoint (the paper's use of
 * the solver under automatic differentiation, Section 4.2).  The face
 * conductances are rebuilt in place by the same kernels as cuth_grid_create,
 * so every later call returns what a grid created with these values would
 * return.  The handle keeps its buffers, captured graphs and launch shapes;
 * the layer coefficients of every time step size used so far are recomputed,
 * and the cached spectral intervals are dropped (the next solve reruns the
 * Lanczos setup).  k_lat, k_vert: host double [nz], finite and > 0.
 * k_lat_mult: device double [nx*ny*nz] lateral multiplier, required for a grid
 * created with one (it need not be the same field) and NULL for a grid created
 * without.  Waits for the handle's stream before it starts.  Errors:
 * CUTH_E_INVALID for bad host values or a multiplier given or missing against
 * the grid (the grid is unchanged); CUTH_E_INVALID also when the device check
 * finds a multiplier entry <= 0 or not finite, after which the handle refuses
 * every call except this one and cuth_grid_destroy until a call here
 * succeeds. */
cuth_status cuth_grid_set_conductivity(cuth_grid g, const double *k_lat, const double *k_vert,
                                       const double *k_lat_mult);

/* Steady solve G T = P (paper Section 3.2 eq. "steady-state"; PCG of
 * Algorithm 1 with the Chebyshev preconditioner).  P: device double [N] W per
 * cell; T: device double [N] K, output (input too if use_initial_guess).
 * opt/stats may be NULL (defaults / not reported).  CUTH_E_NOT_CONVERGED and
 * CUTH_E_BREAKDOWN leave the best iterate in T. */
cuth_status cuth_solve(cuth_grid g, const double *P, double *T,
                       const cuth_options *opt, cuth_stats *stats);

/* One backward-Euler step (eq. "transient"): solves
 * (C/dt + G) T_next = P_next + (C/dt) T_n, warm-started from T_n.  Spectral
 * bounds are computed once per distinct dt and cached in the handle.  T_next
 * may alias T_n.  dt > 0; the handle needs heat_cap. */
cuth_status cuth_transient_step(cuth_grid g, double dt, const double *P_next,
                                const double *T_n, double *T_next,
                                const cuth_options *opt, cuth_stats *stats);

/* Solve nsys independent steady systems, each with nrhs right-hand sides.
 * Every (system, right-hand side) pair is one problem; all problems advance
 * together: each kernel launch covers every active problem (per-problem
 * scalars, spectral bounds and convergence flags), a chunk of CG iterations is
 * captured once into a HIP graph and replayed, and the tile shape is picked by
 * timing candidate shapes on the batch (cached per batch signature, and in the
 * file named by the CUTH_AUTOTUNE_CACHE environment variable if set).
 * P[s] / T[s]: device double [nrhs * N_s] (right-hand side q at offset q*N_s).
 * stats: NULL or [nsys*nrhs] (setup_ms/solve_ms are 0 per problem).  All grids
 * must live on the same device; work is ordered after the first grid's stream.
 * The work vectors (about 56 B per unknown and right-hand side in mixed
 * precision) and launch descriptors are allocated on the first call and kept
 * by the batch's first grid for later calls with the same sizes, precision and
 * number of right-hand sides; destroying that grid releases them. */
cuth_status cuth_solve_batch(int32_t nsys, const cuth_grid *grids, int32_t nrhs,
                             const double *const *P, double *const *T,
                             const cuth_options *opt, cuth_stats *stats);

/* Adjoint of the steady solve (a gradient of a loss through the solve of
 * Section 3.2's steady system; the method of Sections 4.3-4.4 applied to
 * G^T lambda = dL/dT).  Given the forward solution T (device double [N]) and
 * dL/dT (device double [N]), solves G lambda = dL/dT (G = G^T) and returns
 * dL/dP = lambda (device double [N], W^-1 per cell) and the gradient with
 * respect to each layer's conductivity (device double [nz]):
 *   dL_dk[l] = dL/dk_lat[l] + dL/dk_vert[l]
 *            = -(1/k_lat[l]) sum over lateral faces f of layer l of
 *                  g_f (lambda_a - lambda_b)(theta_a - theta_b)
 *              - sum over vertical faces touching layer l of
 *                  (dg_f/dk_vert[l]) (lambda_a - lambda_b)(theta_a - theta_b),
 *   dg/dk_vert[l] = g^2 dz[l] / (2 k_vert[l]^2 dx dy),  theta = T - T_amb,
 * with the lateral multiplier field held fixed.  For a layer whose lateral and
 * vertical conductivities are one value k_l (every layer of an isotropic
 * stack), dL_dk[l] is dL/dk_l; otherwise it is the derivative along an equal
 * increment of both.  dL_dk is written on the device in a fixed summation
 * order (run-to-run identical). */
cuth_status cuth_adjoint(cuth_grid g, const double *T, const double *dL_dT,
                         double *dL_dP, double *dL_dk,
                         const cuth_options *opt, cuth_stats *stats);

/* Thread-local message of the last non-OK status ("" if none). */
const char *cuth_last_error(void);

/* ---- step-level entry points (each runs one step of the solve path) ---- */

/* y = A x for the steady (dt == 0) or transient (dt > 0) operator.
 * precision CUTH_FP64: x, y device double [N]; CUTH_MIXED: the FP32 operator,
 * x, y device float [N]; CUTH_MIXED16: the FP32 operator with the FP16-stored
 * lateral conductances (the one the CUTH_MIXED16 Chebyshev sweeps apply), x, y
 * device float [N].  Paper Algorithm 2 computes the same product. */
cuth_status cuth_apply(cuth_grid g, double dt, int32_t precision, const void *x, void *y);

/* y = A x with the operator stored as a CSR matrix (FP64 values, 32-bit column
 * indices, rows in cell order, columns ascending, the diagonal formed from the
 * face conductances as in the stencil) and one thread per row: the storage
 * baseline of the paper's Ablation I (Section 5, Quad-Diag against CSR),
 * compared with the matrix-free stencil of cuth_apply.  The matrix of (grid,
 * dt) is built on first use (host row pointers, device fill) and kept by the
 * handle.  x, y: device double [N].  CUTH_E_INVALID if the grid has 2^31 or
 * more nonzeros. */
cuth_status cuth_apply_csr(cuth_grid g, double dt, const double *x, double *y);

/* r = b - A (T - t_amb) in FP64 (the true residual of Section 4.4).
 * b, T, r: device double [N]. */
cuth_status cuth_residual(cuth_grid g, double dt, const double *b, const double *T, double *r);

/* z = M^{-1} r: one application of a preconditioner as the solver applies it.
 * preconditioner (cuth_preconditioner): CUTH_PC_CHEBYSHEV, z = q(A) r, the
 * Chebyshev polynomial of degree `degree` on [lmin, lmax] (Section 4.3);
 * CUTH_PC_CHEBYSHEV_JACOBI, z = q(D^{-1} A) D^{-1} r with [lmin, lmax] an
 * interval of D^{-1} A (beyond the paper); CUTH_PC_JACOBI, z = r / diag(A);
 * CUTH_PC_NONE, z = r (lmin, lmax and degree still validated, then unused).
 * precision selects FP64 (double vectors), FP32 (CUTH_MIXED: float vectors,
 * FP32 operator) or FP32 with the FP16-stored lateral conductances in the
 * Chebyshev sweeps (CUTH_MIXED16, float vectors). */
cuth_status cuth_precond_apply(cuth_grid g, double dt, int32_t precision, int32_t preconditioner,
                               double lmin, double lmax, int32_t degree, const void *r, void *z);

/* ---- allocation-free entry point ---- */

/* Bytes of device memory the library holds on every GPU it runs on, until the
 * process ends, for cuth_precond_apply_noalloc. */
#define CUTH_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same z = M^{-1} r
 * as cuth_precond_apply, with the same arguments, validation and result, but
 * the call allocates nothing.  Every device buffer it needs besides r, z and
 * the operator the handle built at creation (the problem descriptor and its
 * state, the polynomial's constants, the layer coefficients of dt, the
 * reduction partials and the one iterate that is not z) lives in a per-device
 * scratch array of CUTH_NOALLOC_SCRATCH_BYTES; the small parts are written into
 * it by kernel arguments, and the state is cleared on every call.  The sweeps
 * run one per launch (never fused).  Scratch needed: about N * 4 bytes (FP32,
 * CUTH_MIXED and CUTH_MIXED16) or N * 8 bytes (CUTH_FP64), plus a few KiB and
 * 384 bytes per stencil workgroup; a grid that needs more returns
 * CUTH_E_INVALID before any device work, with the sizes in cuth_last_error().
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (other host threads, other streams) race and give undefined results.  Returns
 * after the handle's stream has completed the work, like cuth_precond_apply. */
cuth_status cuth_precond_apply_noalloc(cuth_grid g, double dt, int32_t precision,
                                       int32_t preconditioner, double lmin, double lmax,
                                       int32_t degree, const void *r, void *z);

/* FP32 Lanczos with `steps` steps on the FP32 operator (preconditioner
 * CUTH_PC_CHEBYSHEV: A; CUTH_PC_CHEBYSHEV_JACOBI: D^{-1/2} A D^{-1/2}, whose
 * spectrum is that of D^{-1} A; other values CUTH_E_INVALID), start vector v0
 * (device float [N], or NULL for the library's own counter-based start vector),
 * followed by the FP64 host eigensolve of the tridiagonal.  alpha (host
 * [steps]) and beta (host [steps-1]) receive the tridiagonal (either may be
 * NULL); ritz_min/ritz_max its extreme eigenvalues; lmin/lmax the bounds the
 * solver uses: lmin = ritz_min, lmax = min(Gershgorin bound, 1.05 ritz_max),
 * the Gershgorin bound of D^{-1} A being 2. */
cuth_status cuth_spectral_bounds(cuth_grid g, double dt, int32_t preconditioner, int32_t steps,
                                 const float *v0, double *alpha, double *beta, double *ritz_min,
                                 double *ritz_max, double *lmin, double *lmax);

/* ---- setup control and measurement ---- */

/* Drop the cached spectral bounds of every operator of the handle, so the next
 * solve reruns the Lanczos setup (Section 4.3 last paragraph).  No device work. */
cuth_status cuth_grid_reset_bounds(cuth_grid g);

/* Kernel timing for measurement.  When on, each preconditioner application
 * brackets its run of back-to-back general Chebyshev launches from the third
 * sweep on (the fused triples of sweeps, else the fused pairs, else the single
 * sweeps before the last) with two HIP events on the handle's stream;
 * cuth_profile_read returns the summed duration of those runs (ms), the number
 * of launches they hold, the algorithmic bytes of one such launch (N times the
 * bytes per unknown) and the sweeps per timed launch minus one (*fused 2:
 * fused triples, 1: fused pairs, 0: single sweeps).
 * Any output pointer may be NULL.  Enabling resets the counters and
 * synchronises the stream. */
cuth_status cuth_profile_enable(cuth_grid g, int32_t on);
cuth_status cuth_profile_read(cuth_grid g, double *total_ms, int64_t *launches,
                              double *bytes_per_launch, int32_t *fused);

#ifdef __cplusplus
}
#endif

#endif /* CUTH_H */
