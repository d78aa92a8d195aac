/*
 * nrd.h -- C ABI of the MI355X library for the implicit AMR two-temperature
 * non-equilibrium radiation diffusion hot path (Philip et al., "Dynamic
 * Implicit 3D Adaptive Mesh Refinement for Non-Equilibrium Radiation
 * Diffusion", arXiv:1302.6303).
 *
 * The library evaluates, on one GPU, the pieces of a Jacobian-free
 * Newton-Krylov time step on a structured AMR hierarchy:
 *   - the flux-limited residual F(u) = c0 u - b - dt f(u)  (Sec. 3.1-3.3),
 *   - its Jacobian action and transpose                      (Sec. 4.1),
 *   - the physics-based preconditioner P^-1 = P2^-1 P1^-1 with FAC V(1,0)
 *     diffusion solves (Sec. 4.2-4.3, Alg. 1),
 *   - the whole BDF1/BDF2 implicit step with inexact Newton + FGMRES.
 *
 * Conventions (every call):
 *   - Return value: NRD_OK (0) or a negative nrd_status.  The message of the
 *     last failure on the calling thread is nrd_last_error().  No C++
 *     exception crosses the ABI.
 *   - Pointers named `dev_*` or documented as device pointers refer to GPU
 *     memory; all others are host memory.  Ownership never transfers: the
 *     caller keeps every buffer it passes.
 *   - The library allocates no device memory.  After nrd_hierarchy_create
 *     the caller queries nrd_workspace_size and binds ONE device buffer of
 *     at least that size with nrd_bind_workspace; it must stay alive until
 *     nrd_hierarchy_destroy.
 *   - All device work is queued on the HIP stream given at create.  Calls
 *     that return data to the host (norm values, statistics) synchronise
 *     that stream; the others are asynchronous.
 *   - A hierarchy is not thread safe; use one per host thread.
 *
 * Layouts:
 *   - compact: for every box in creation order, its cells with x fastest;
 *     all E values first, then all T values (length 2 * ncells).  z is one
 *     field (length ncells).
 *   - native: every box stored as a block of (nx+2)(ny+2)(nz+2) values with
 *     one ghost layer, x fastest; all E blocks, then all T blocks (length
 *     2 * native_len).  Ghost entries and covered-cell entries of native
 *     inputs are scratch that the library overwrites (restriction and ghost
 *     fill); outputs are written on interior cells only, covered cells = 0.
 */
#ifndef NRD_H
#define NRD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nrd_status;
enum {
    NRD_OK = 0,
    NRD_EINVAL = -1,     /* bad argument, size or option                  */
    NRD_ENESTING = -2,   /* boxes overlap, are misaligned or not nested   */
    NRD_ESTATE = -3,     /* call out of order (e.g. no workspace bound)   */
    NRD_ENONPOS = -4,    /* E, T or z not positive and finite             */
    NRD_ENOTCONV = -5,   /* Newton or Krylov failed; state rolled back     */
    NRD_EDEVICE = -6,    /* HIP runtime error                              */
    NRD_EUNSUPPORTED = -7
};

/* One refinement patch: half-open [lo, hi) in the index space of its level
 * (level l refines level 0 by 2^l per axis).  Level-0 boxes tile the base
 * grid (the coarsest level is a union of patches, Sec. 3.2): no overlap,
 * together exactly the base grid (NRD_ENESTING otherwise).  A base grid cut
 * into several boxes must coarsen at least once (even extents above 5) and
 * be cut at even planes, since the base multigrid coarsens across the cuts
 * (NRD_EUNSUPPORTED otherwise).  Finer boxes: even lo/hi, inside the
 * coarser level shrunk by one coarse cell away from the physical boundary
 * (proper nesting).  Boxes must be ordered by (problem, level). */
typedef struct {
    int32_t problem;
    int32_t level;
    int32_t lo[3];
    int32_t hi[3];
} nrd_box;

/* One independent problem on [lo, hi] with base_n cells per axis.
 * Faces are numbered 2*d + s (d = axis, s = 0 low / 1 high).
 * bc_E[f] = 0: zero flux; 1: Marshak/Robin face  1/2 n.D grad E + E/4 = R
 * with R = robin_R[f] (eqs. robinbc, bcs).  T has zero flux on every face. */
typedef struct {
    int32_t base_n[3];
    double lo[3];
    double hi[3];
    int32_t bc_E[6];
    double robin_R[6];
    double kappa;          /* D_T = kappa T^(5/2), kappa = 0.01 in Sec. 3.1  */
} nrd_problem;

enum { NRD_FP64 = 0, NRD_MIXED = 1 };            /* preconditioner precision */
enum { NRD_BATCHED = 0, NRD_PER_PATCH = 1 };     /* kernel launch grouping   */
enum { NRD_JVP_ANALYTIC = 0, NRD_JVP_FD = 1 };
enum { NRD_P2_PAPER = 0, NRD_P2_FROZEN4 = 1 };
enum { NRD_SMOOTH_RBGS = 0, NRD_SMOOTH_JACOBI = 1,   /* FAC level smoother */
       NRD_SMOOTH_LINE = 2 };
enum { NRD_BASE_MG = 0, NRD_BASE_SMOOTH = 1 };       /* FAC base level     */
enum { NRD_FAC_MULT = 0, NRD_FAC_AFACX = 1 };        /* P1 cycle           */
enum { NRD_EW_KELLEY = 0, NRD_EW_PETSC = 1 };         /* Newton forcing     */

typedef struct {
    int32_t precision;      /* NRD_FP64 or NRD_MIXED (V-cycles in float)     */
    int32_t launch;         /* NRD_BATCHED: one launch per operator over the
                               whole patch table; NRD_PER_PATCH: one launch
                               per patch (same kernels, same results)       */
    int32_t use_graph;      /* 1: capture each FGMRES iteration (precond,
                               Jacobian action, CGS2, Givens) as a HIP graph
                               on first use and replay it on the library
                               stream (results bitwise those of direct
                               launches; pays off when launches dominate,
                               e.g. a single problem of 32^3)                */
    int32_t jvp_mode;       /* analytic Jacobian action or finite difference  */
    double limiter;         /* lambda in D_h / (1 + lambda D_h |dE|/(h E_f));
                               0.5 = the printed pair (default), 1 = Wilson  */
    int32_t p2_mode;        /* coupling block entries                        */
    double newton_rtol;     /* ||F_k|| <= max(rtol ||F_0||, atol)            */
    double newton_atol;
    int32_t newton_maxit;
    int32_t gmres_restart;  /* Krylov dimension m <= 64                      */
    int32_t gmres_maxrestarts;
    int32_t mg_nu_pre;      /* base multigrid V(nu_pre, nu_post)             */
    int32_t mg_nu_post;
    int32_t adjoint_slots;  /* device state slots reserved for nrd_adjoint_run:
                               ceil(nsteps / ckpt_every) + ckpt_every + 3    */
    int32_t stencil;        /* residual / Jacobian kernel: 0 one thread per
                               cell in runs of 256 cells (six faces each),
                               1 plane-marching tiles (each face once, LDS),
                               2 wave runs (x faces shared across lanes),
                               3 staged planes (each plane slice read once
                               into LDS, 256-cell runs; a hierarchy with a
                               patch wider than about 250 cells in x runs
                               variant 1 instead)                            */
    int32_t zchunk;         /* planes per tile of variants 1, 2 (0: default)  */
    int32_t bdf_max_order;  /* 2 (default): BDF2 after the first step; 1: BDF1
                               throughout (the adjoint assumes BDF1)         */
    int32_t error_estimate; /* 1: every BDF2 step keeps its leapfrog predictor
                               and reports the scaled max norm of its local
                               error estimate (eq. bdf2le) in
                               nrd_step_stats.err_norm; needed by
                               nrd_adaptive_steps (0 default)                */
    int32_t fac_nu_pre;     /* FAC V(m, n) of Alg. 1 on hierarchies with more
                               than one level: m in [1, 8] smoothing sweeps
                               per level on the down-sweep (default 1)       */
    int32_t fac_nu_post;    /* n in [0, 8] sweeps per level on the up-sweep,
                               each level's right-hand side the composite
                               residual refreshed with every correction so
                               far (default 0: the paper's V(1,0))           */
    int32_t fac_smoother;   /* FAC level smoother (Sec. 4.3): NRD_SMOOTH_RBGS
                               (default), NRD_SMOOTH_JACOBI, damped point
                               Jacobi with weight 6/7, or NRD_SMOOTH_LINE,
                               block Gauss-Seidel whose blocks are the
                               x-lines of each patch (red-black by j + k,
                               each line solved exactly with the rest held) */
    double err_eta_E;       /* eta_E, eta_T of that norm,                    */
    double err_eta_T;       /* max |e / (u + eta)| over composite cells      */
    int32_t fac_base;       /* base level of FAC: NRD_BASE_MG (default), one
                               multigrid V-cycle, or NRD_BASE_SMOOTH, only
                               fac_nu_pre level sweeps there (the paper's
                               runs smooth on the coarsest level, Sec. 4.3)  */
    int32_t fac_cycle;      /* P1's cycle on refined hierarchies: NRD_FAC_MULT
                               (default), the multiplicative FAC of Alg. 1,
                               or NRD_FAC_AFACX, the asynchronous variant
                               named in Sec. 7 (after Lee, McCormick, Philip
                               and Quinlan): the base correction and, for
                               every refined level l at once, fac_nu_pre
                               red-black sweeps of the level-(l-1) operator
                               from zero on the cells level l covers (the
                               rest held at 0), their interpolation s onto
                               level l and fac_nu_pre sweeps of the level-l
                               operator from s, minus s; the corrections are
                               summed.  Needs the red-black smoother and
                               fac_nu_post = 0                              */
    int32_t newton_forcing; /* Eisenstat-Walker forcing term of the inexact
                               Newton solve (Sec. 4.1 points to Kelley's
                               algorithm and Sec. 6 to PETSc's
                               implementation): NRD_EW_PETSC (default):
                               eta_0 = 0.3, eta_k = (|F_k| / |F_k-1|)^a,
                               a = (1 + 5^1/2) / 2, at least eta_k-1^a when
                               that exceeds 0.1; or NRD_EW_KELLEY: eta_0 =
                               0.9, eta_k = 0.9 (|F_k| / |F_k-1|)^2, at least
                               0.9 eta_k-1^2 when that exceeds 0.1.  Both
                               capped at 0.9 and floored at 0.5 tau / |F_k|,
                               tau the Newton stopping tolerance          */
    int32_t pad_;
} nrd_options;

/* Fills *opt with the defaults: FP64, batched, no graph, analytic JVP,
 * limiter 1/2 (the printed pair), paper P2, rtol 1e-8, atol 1e-14, 20 Newton iterations,
 * PETSc's Eisenstat-Walker forcing terms, GMRES(30) with 10 restarts,
 * multiplicative FAC V(1,0), base multigrid V(1,1),
 * staged-plane stencil, BDF2, no error
 * estimate, eta_E = 1e-5 (the initial energy density of Sec. 6), eta_T =
 * 1e-5^(1/4). */
void nrd_default_options(nrd_options* opt);

typedef struct {
    int32_t newton_iters;        /* accepted Newton updates                  */
    int32_t krylov_iters;        /* total over the Newton iterations         */
    int32_t positivity_cuts;     /* rejected trial steps (a trial u - l s with
                                    a nonpositive E or T on a composite cell
                                    halves l; 31 rejections end the solve)  */
    int32_t converged;
    double fnorm0;
    double fnorm;
    int32_t krylov_per_newton[24];
    double dt;                   /* the step size of this step               */
    double err_norm;             /* scaled max norm of the local error
                                    estimate (error_estimate set, BDF2 step);
                                    -1 otherwise                             */
} nrd_step_stats;

/* Time-step control (Sec. 3.4-3.5, eqs. odets, pc47, bdf2le). */
enum { NRD_CTL_PC47 = 0, NRD_CTL_EPS = 1 };
typedef struct {
    double eps;                  /* target local error eps_t                 */
    double ratio_min;            /* bounds of dt_{n+1} / dt_n (variable-step */
    double ratio_max;            /* BDF2 is zero-stable below 1 + sqrt 2)    */
    int32_t controller;          /* NRD_CTL_PC47 (k_I = 0.4/3, k_P = 0.7/3;
                                    EPS for a problem's first estimate) or
                                    NRD_CTL_EPS (dt (eps / err)^(1/3))       */
    int32_t max_halvings;        /* retries of a step whose solve fails      */
} nrd_timectl;

typedef struct nrd_hierarchy nrd_hierarchy;

const char* nrd_last_error(void);

/* Builds the patch, ghost, restriction and flux-matching tables on the host
 * (Sec. 3.2.1: coarse-fine boundary fragments become a flat ghost table).
 * hip_stream: a hipStream_t (NULL = default stream).  Errors: NRD_EINVAL,
 * NRD_ENESTING.  *out is set only on success. */
nrd_status nrd_hierarchy_create(const nrd_problem* probs, int32_t nprob,
                                const nrd_box* boxes, int32_t nbox,
                                const nrd_options* opt, void* hip_stream,
                                nrd_hierarchy** out);
/* Releases host tables and graphs; never frees the bound workspace. */
nrd_status nrd_hierarchy_destroy(nrd_hierarchy* h);

/* Bytes of device workspace this hierarchy needs (Krylov basis included). */
nrd_status nrd_workspace_size(const nrd_hierarchy* h, size_t* bytes);
/* Binds dev_ptr (>= nrd_workspace_size bytes, 256-byte aligned) and uploads
 * the tables into it.  Synchronises the stream. */
nrd_status nrd_bind_workspace(nrd_hierarchy* h, void* dev_ptr, size_t bytes);

/* ncells: composite + covered cells of all boxes; native_len: ghosted cells
 * per field. */
nrd_status nrd_layout(const nrd_hierarchy* h, int64_t* ncells,
                      int64_t* native_len);
/* Device pointers; 2-field vectors in the layouts described above. */
nrd_status nrd_pack(nrd_hierarchy* h, const double* dev_native,
                    double* dev_compact);
nrd_status nrd_unpack(nrd_hierarchy* h, const double* dev_compact,
                      double* dev_native);

/* Copies the state E, T and the material z (device, compact) into the
 * library, restricts covered cells, fills ghosts and resets the time
 * history (the next implicit step is BDF1).  z must be given on every
 * level, covered cells included.  NRD_ENONPOS if any value <= 0 or not
 * finite (checked on the device; synchronises). */
nrd_status nrd_set_fields(nrd_hierarchy* h, const double* dev_E,
                          const double* dev_T, const double* dev_z);
/* Copies the current state out (compact; covered cells hold restricted
 * values).  Synchronises. */
nrd_status nrd_get_fields(nrd_hierarchy* h, double* dev_E, double* dev_T);

/* Fixes BDF order, alpha, c0, b = history combination and beta for the
 * following residual / jvp / precond calls, per problem (dt: host array of
 * nprob step sizes; eqs. be, bdf2). */
nrd_status nrd_begin_step(nrd_hierarchy* h, const double* dt);

/* F = c0 u - b - dt f(u) on composite cells (covered cells = 0) for a native
 * state u; u's ghost and covered entries are overwritten (restriction and
 * ghost fill).  Sec. 3.1-3.3, eq. nonlinearsystem. */
nrd_status nrd_residual(nrd_hierarchy* h, double* dev_u, double* dev_F);

/* Jv = F'(u) v (analytic derivative of the residual, or the finite
 * difference of eq. Jac-free with the step of Sec. 4.1 when jvp_mode is FD).
 * u and v native; their ghost/covered entries are overwritten. */
nrd_status nrd_jvp(nrd_hierarchy* h, double* dev_u, double* dev_v,
                   double* dev_Jv);

/* Freezes D_E, D_T, sigma at u (Sec. 4.2 L^k) and factors the coarsest
 * multigrid grid.  Then y = P2^-1 P1^-1 w, P1^-1 by one FAC V(1,0) cycle
 * (Alg. 1) in the configured precision.  w and y native double; covered
 * entries of y are unspecified. */
nrd_status nrd_precond_setup(nrd_hierarchy* h, double* dev_u);
nrd_status nrd_precond_apply(nrd_hierarchy* h, const double* dev_w,
                             double* dev_y);

/* Transposed action (Sec. 3.2.1's synchronisation run backwards on refined
 * hierarchies): JTlam = F'(u)^T lam in the composite unknowns (native,
 * interior written; covered entries 0: the covered cells' restricted values
 * pass their sensitivities to their children) and gz = (dF/dz)^T lam per
 * cell (compact, ncells, every level: covered cells' z reaches the fine
 * level through coarse-fine ghosts).  Covered entries of lam are ignored.
 * u's ghost/covered entries and lam's ghosts are overwritten; the ghost
 * slots of JTlam are used as scratch. */
nrd_status nrd_vjp(nrd_hierarchy* h, double* dev_u, double* dev_lam,
                   double* dev_JTlam, double* dev_gz);

/* One BDF step of the library-owned state for every problem: BDF1 after
 * set_fields, BDF2 with alpha = dt_n / dt_{n-1} afterwards, leapfrog
 * predictor as initial guess (eqs. be, bdf2, leapfrog), inexact Newton with
 * Eisenstat-Walker forcing and positivity-preserving step halving, FGMRES
 * right-preconditioned by P (eq. inexactNewtoneqns).  dt: host [nprob];
 * stats: host [nprob] or NULL.  On failure the state is rolled back and
 * NRD_ENOTCONV is returned.  Synchronises. */
nrd_status nrd_implicit_step(nrd_hierarchy* h, const double* dt,
                             nrd_step_stats* stats);

/* nsteps accepted steps of every problem with step sizes chosen by the
 * controller from each problem's own local error estimates (the hierarchy
 * must be created with error_estimate = 1).  dt: host [nprob], in: the next
 * step size of every problem, out: the size chosen for the step after the
 * last.  t: host [nprob] or NULL, advanced by the accepted steps.  A batch
 * whose solve fails for some problems is rolled back and retried with those
 * problems' steps halved (the others repeat the same step); more than
 * max_halvings retries of one problem's step give NRD_ENOTCONV with the state
 * of the last accepted step.  The first step after nrd_set_fields is BDF1 and
 * keeps its size.  stats: host [nsteps * nprob] (step-major) or NULL.
 * Synchronises. */
nrd_status nrd_adaptive_steps(nrd_hierarchy* h, const nrd_timectl* ctl, int32_t nsteps,
                              double* dt, double* t, nrd_step_stats* stats);

/* Discrete adjoint of nsteps BDF1 steps of size dt from the current state
 * for J = sum over cells of dJdE_final[c] * E_N(c) (device, compact E part;
 * a covered cell's E is the mean of its children's, so its weight reaches
 * them; NULL = 1 on every composite cell and 0 on covered cells).  Forward
 * states are checkpointed every ckpt_every steps and recomputed segment by
 * segment.  gz (device, ncells) receives dJ/dz for the z of every cell of
 * every level.  The state afterwards is u_N. */
nrd_status nrd_adjoint_run(nrd_hierarchy* h, const double* dt, int32_t nsteps,
                           int32_t ckpt_every, const double* dev_dJdE_final,
                           double* dev_gz);

/* ---- dynamic regridding (Sec. 5) ------------------------------------- */

/* Refinement criteria; a threshold <= 0 (or z_interface = 0) switches one
 * off, a cell is tagged when any enabled criterion holds.  With E_d the
 * centred difference of E along axis d (a neighbour beyond a physical face
 * is the cell itself):
 *   grad_E:  |grad E| / E > grad_E, grad E in physical units;
 *   tau_g:   sum_d |E_{+d} - E_{-d}| / 2 / (0.1 max|E|) > tau_g   (tau^g),
 *   tau_c:   sum_d |E_{+d} - 2 E + E_{-d}| / (0.1 max|E|) > tau_c  (tau^c),
 *            the paper's indicators, max|E| over the problem's composite
 *            cells;
 *   z_interface: a face neighbour lies in another material (a coarse-fine
 *            neighbour's material is its coarse parent's z). */
typedef struct {
    double grad_E;
    double tau_g;
    double tau_c;
    int32_t z_interface;
    int32_t pad_;
} nrd_tagging;

/* Tags of the current state (after nrd_set_fields or a step): dev_tags
 * (device, ncells bytes, compact layout) receives 1 for a tagged cell and 0
 * otherwise, for every cell of every box, covered cells included.  NRD_ESTATE
 * before nrd_set_fields.  Asynchronous. */
nrd_status nrd_tag(nrd_hierarchy* h, const nrd_tagging* crit, uint8_t* dev_tags);

/* Clustering options (cell counts on the level whose tags are clustered). */
typedef struct {
    int32_t max_levels;   /* levels of the new hierarchy, base included      */
    int32_t buffer;       /* tags grown by this many cells per axis          */
    double efficiency;    /* a box is kept when tagged / cells >= efficiency  */
    int32_t min_side;     /* cuts made for efficiency leave sides >= this    */
    int32_t max_side;     /* longer boxes are halved                         */
} nrd_cluster_opt;

/* Host only (no device, no hierarchy object): the boxes of a new hierarchy
 * for the problems probs from the boxes of the current one and their tags
 * (host_tags: ncells bytes in the compact layout of `boxes`, nonzero =
 * tagged).  Level 0 is kept.  Level l + 1 is built from tags on the new
 * level l, each cell taking the tag of the finest old level at or below l
 * that holds it; tags are grown by `buffer`, restricted to cells whose 26
 * neighbours lie on level l (proper nesting), and grouped into boxes by the
 * Berger-Rigoutsos algorithm (Sec. 5): bounding boxes accepted at the
 * efficiency target, else cut at a plane without tags, at the strongest
 * inflection of the tag signature, or in the middle.  Boxes longer than
 * max_side are halved.  The result (ordered by problem and level, level-l
 * boxes refined by 2) is written to out[0 .. *nout); NRD_EINVAL if it holds
 * more than cap boxes (*nout is then the count needed) or for bad options.
 * Deterministic. */
nrd_status nrd_cluster(const nrd_problem* probs, int32_t nprob, const nrd_box* boxes,
                       int32_t nbox, const uint8_t* host_tags,
                       const nrd_cluster_opt* opt, nrd_box* out, int32_t cap,
                       int32_t* nout);

/* Moves the time history of src to dst (both bound, created for the same
 * problems, possibly with other boxes; same device): the state u_n, the
 * previous state u_{n-1} and the last step's history vector b, by
 * conservative minmod-limited linear refinement (Sec. 5): dst level 0 copies
 * src level 0; every finer dst level is refined from the dst level below
 * (each child u_P +- s_d / 4 per axis, s_d the minmod of the two one-sided
 * differences of its parent, zero across a physical face) and then takes
 * src's values wherever src has that level (src covered cells hold the mean
 * of their children); the result is synced.  dev_z (device, compact layout
 * of dst) is dst's material field, sampled by the caller on every level.
 * The step-size history moves too; the next nrd_implicit_step continues
 * with BDF2 on the interpolated history (warm restart), its local error
 * estimate is not computed (err_norm = -1: it would rest on interpolated
 * data) and nrd_adaptive_steps keeps that step's size.  Call nrd_resolve
 * first to solve the last step again on the new grid.  src is unchanged.
 * Errors: NRD_EINVAL (other problems), NRD_ESTATE (unbound, no fields),
 * NRD_ENONPOS (z).  Synchronises both streams. */
nrd_status nrd_transfer(nrd_hierarchy* src, nrd_hierarchy* dst, const double* dev_z);

/* Solves the last step's system F(u) = c0 u - b - dt f(u) = 0 again on the
 * hierarchy a transfer moved it to (Sec. 5: a re-solve at the current time
 * with the interpolated history, starting from the interpolated state);
 * the solution replaces u_n and the time derivative for the next predictor
 * is recomputed from it.  stats: host [nprob] or NULL.  NRD_OK with no work
 * when no step had been taken before the transfer.  On failure the
 * transferred state is kept and NRD_ENOTCONV returned.  Synchronises. */
nrd_status nrd_resolve(nrd_hierarchy* h, nrd_step_stats* stats);

/* Inner product and norm of native 2-field vectors, per problem, volume
 * weighted over composite cells (host outputs of length nprob). */
nrd_status nrd_dot(nrd_hierarchy* h, const double* dev_x, const double* dev_y,
                   double* out);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): nrd_dot's inner products <x, y>
 * per problem written to dev_out (device, nprob doubles) on the library
 * stream, without synchronising.  Its per-tile partial sums live in a fixed
 * device array of 32768 doubles (256 KiB) that the library holds on every
 * GPU it runs on until the process ends, not in the workspace; the
 * hierarchy still needs its bound workspace (tables).  Same kernels and
 * summation order as nrd_dot, so the results are equal bit for bit.
 * NRD_EINVAL if the hierarchy has more reduction tiles (runs of at most
 * 2048 cells of one patch) than the array holds, or for a NULL argument.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or host threads) race and must be serialised by the
 * caller. */
nrd_status nrd_dot_noalloc(nrd_hierarchy* h, const double* dev_x,
                           const double* dev_y, double* dev_out);

/* Tile-shape tuner of the batching machinery (patch table + tile lists).
 * For every patch-size class (interior extents nx x ny x nz) the residual
 * kernel is timed on that class's patches with each candidate plane-tile
 * shape of the configured stencil variant (planes per tile, cells per plane
 * run) and the fastest shape is used for that class from then on; results
 * do not change (every shape evaluates the same face and cell formulas on
 * the same operands).  cache_path (may be NULL) is a text file of earlier
 * choices, one line "arch v<variant> <fmt> <nx>x<ny>x<nz> <planes> <run> <us>"
 * per class (<fmt> names the tile constants of the build that wrote it);
 * classes found for this device architecture, variant and format whose shape
 * is one this build would try are not timed again (other lines are ignored),
 * newly timed ones are appended.  *timed_classes (may be NULL)
 * returns how many classes were timed.  Needs a bound workspace and
 * nrd_set_fields (NRD_ESTATE otherwise); synchronises the stream; drops
 * captured graphs.  Variant 0 has nothing to tune (returns NRD_OK). */
nrd_status nrd_autotune(nrd_hierarchy* h, const char* cache_path,
                        int32_t* timed_classes);

/* Time of the kernels of one operator, for measurement: while timing is
 * enabled every call of the operator records HIP events on the library
 * stream around its launches; *ms_total is their summed elapsed time and
 * *count the number of calls since nrd_timer_enable.  RESIDUAL: the residual
 * launch(es) of a residual evaluation; JVP: one Jacobian action; PRECOND:
 * one preconditioner application; SMOOTH: one red-black sweep (both colour
 * launches) on the base level's multigrid grid starting from a nonzero
 * iterate; SMOOTH_ZERO: the first such sweep of a V-cycle, from a zero
 * iterate.  NRD_EINVAL for an unknown timer.  Synchronises. */
nrd_status nrd_timer_read(nrd_hierarchy* h, int32_t which, double* ms_total,
                          int32_t* count);
enum { NRD_TIMER_RESIDUAL = 0, NRD_TIMER_JVP = 1, NRD_TIMER_PRECOND = 2,
       NRD_TIMER_SMOOTH = 3, NRD_TIMER_SMOOTH_ZERO = 4, NRD_TIMER_COUNT = 5 };
nrd_status nrd_timer_enable(nrd_hierarchy* h, int32_t on);

/* Composite cells covered by the timed calls of a RESIDUAL or JVP timer
 * since nrd_timer_enable (a call over the problems still iterating in a
 * lock-step Newton solve covers only theirs); 0 for the other timers.  With
 * nrd_timer_read this gives the operator's cells per second.  NRD_EINVAL for
 * an unknown timer. */
nrd_status nrd_timer_cells(nrd_hierarchy* h, int32_t which, int64_t* cells);

#ifdef __cplusplus
}
#endif
#endif /* NRD_H */
