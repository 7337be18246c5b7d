/*
 * jfmg: Jacobian-free Newton-GMRES with an FV-subgrid multigrid preconditioner
 * for the well-balanced DG discretization of 2D compressible Euler / viscous
 * flow with gravity on Cartesian quadrilaterals, on AMD MI355X (gfx950).
 *
 * Method: P. Birken, A. Dedner, R. Kloefkorn, "A Jacobian-free Multigrid
 * Preconditioner for Discontinuous Galerkin Methods applied to Numerical
 * Weather Prediction", arXiv 2505.24504.
 *
 * Conventions for every entry point
 *  - Vectors are DEVICE pointers owned by the caller.  The library never
 *    allocates device memory after jfmg_create_problem: everything lives in
 *    the caller's workspace (size from jfmg_workspace_bytes).
 *  - DG vector layout: the perturbation U' of the well-balanced form (Sec.
 *    "euler-model", eq. perturbed-euler) as FP64 SoA [4][nz][nx][(k+1)^2],
 *    components (rho, rho u, rho w, rho theta); element e = ez*nx + ex; node
 *    b*(k+1) + a with a along x and nodes at the Gauss-Legendre points in
 *    ascending order.  N = 4 nx nz (k+1)^2 entries (jfmg_num_dofs).
 *  - FV vector layout (finest level = (k+1)nx x (k+1)nz subcells, each coarser
 *    level halves both counts): SoA [4][nzl][nxl], cell (I,J) at J*nxl + I, in
 *    the problem's multigrid precision (double for mg_precision 64, float for 32).
 *  - All work is stream ordered on the stream given at creation.  Entry points
 *    that return scalars or make convergence decisions synchronize that stream.
 *  - Every call returns a jfmg_status; jfmg_last_error gives a message.  No
 *    exception crosses the ABI.  A problem is used by one host thread at a time.
 */
#ifndef JFMG_H
#define JFMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    JFMG_OK = 0,
    JFMG_EINVAL = 1,      /* bad configuration or argument                     */
    JFMG_ENOMEM = 2,      /* workspace too small                               */
    JFMG_ENOCONV = 3,     /* Newton or GMRES hit its iteration cap             */
    JFMG_ENONFINITE = 4,  /* NaN/Inf in a norm                                 */
    JFMG_ESTATE = 5,      /* call needs a prior jfmg_linearize                 */
    JFMG_EDEVICE = 6      /* HIP runtime error                                 */
} jfmg_status;

typedef struct {
    int nx, nz, k;            /* quads in x and z; DG degree k in {1,2,3}                 */
    int physics;              /* 0 Euler, 1 viscous flux F_v (eq. compressible-euler)    */
    int background;           /* 0 neutral (theta = theta0), 1 constant N                */
    int bc;                   /* 0 slip walls, 1 periodic in x + slip walls in z        */
    int scheme;               /* 0 implicit Euler, 1 SDIRK2 of Ellsiepen (eq. ellsiep)   */
    int newton_maxit;         /* Newton cap (ENOCONV beyond)                            */
    int gmres_m;              /* FGMRES restart length, <= 64                           */
    int gmres_max_restarts;   /* restarts before ENOCONV                                */
    int fd_eps_mode;          /* DG FD step: 0 sqrt(eps)/||y||, 1 sqrt(eps)||U+Ubar||/||y|| */
    int mg_levels;            /* FV levels including the finest, 1..8                   */
    int rk_stages;            /* stages of the RK pseudo-time smoother, 1..4            */
    int mass_fix;             /* 1: mass-fixed transfers (eq. transfer-mass-fix)        */
    int mg_precision;         /* 64 or 32: precision of the whole multigrid             */
    int precond;              /* 1 multigrid Q^-1 = T^-1 q^-1 T, 0 identity             */
    char mg_key[16];          /* "mg a b c d e f G", e.g. "mg002222V" (one digit each)  */
    double x0, x1, z0, z1;    /* domain                                                 */
    double g, gamma, R, p0;   /* gravity, adiabatic index, gas constant, reference p    */
    double theta0, N, u_mean; /* background theta (surface), Brunt-Vaisala N, mean wind */
    double mu, c_ip;          /* kinematic viscosity [m^2/s]; interior-penalty constant */
    double dt, newton_rtol;   /* time step; Newton stops at ||G|| < rtol ||G^0||        */
    double ew_gamma, ew_alpha, ew_eta0, ew_eta_max; /* Eisenstat-Walker choice 2        */
    double rk_alpha[4];       /* smoother coefficients; 0 entries: 1/(s-j+1)            */
    double pseudo_cfl;        /* c* in the pseudo time step                             */
    double newton_stall;      /* > 0: a stage also ends, successfully, once ||G|| <=
                                 newton_stall ||G^0|| and a Newton step no longer halves
                                 ||G|| (the rounding floor of G lies above rtol); 0: off */
    int batch;                /* members of a lock-step batch (0 or 1: a single problem);
                                 see "lock-step batches" below                          */
    int transfer;             /* DG <-> FV transfer (Sec. "Transfer functions"): 0 the
                                 interpolation at the subcell centres (with mass_fix),
                                 1 the L2 projection onto the subcells (subcell averages;
                                 conserves mass, mass_fix does not apply)              */
    double pseudo_cfl_dg;     /* c* of the DG-level smoother's pseudo time step (key a, b):
                                 dtau_dg = c* / (1 + alpha dt (lam_0 (1/hx + 1/hz)
                                 + 2 mu (1/hx^2 + 1/hz^2))), hx, hz = element widths over
                                 2k+1, lam_0 = max |v| + c of the finest FV level      */
} jfmg_config;

typedef struct {
    int shape;                /* 0 cosine bubble (density current), 1 inertia-gravity  */
    int pad;
    double amp, xc, zc, xr, zr, a, Z;
} jfmg_perturbation;

typedef struct {
    int newton_its, gmres_its, lh_evals, jvps;
    int fv_matvecs[8];        /* FV operator evaluations per level (finest first)      */
    int host_syncs, status;
    int stall_stops;          /* stages ended at the rounding floor (newton_stall)     */
    int reorth_its;           /* FGMRES iterations (per member) whose second
                                 Gram-Schmidt pass ran                                 */
    double g0_norm, g_norm;   /* ||G(U^0)||, ||G|| at exit of the last stage          */
    double seconds;           /* host wall time of the call                           */
    double reached_rtol;      /* largest final ||G|| / ||G^0|| over the call's stages
                                 (and members): the Newton tolerance actually met      */
} jfmg_stats;

typedef struct jfmg_problem jfmg_problem;

/* Fill a configuration with the defaults (16x16, k=1, Euler, neutral 300 K,
   slip walls, SDIRK2, dt 1 s, rtol 1e-8, FGMRES(30), 3 levels, mg002222V,
   3 RK stages, mass fix, FP64 multigrid). */
jfmg_status jfmg_config_default(jfmg_config* cfg);

/* Device workspace bytes a problem with this configuration needs.
   EINVAL for an invalid configuration (k outside 1..3, an FV dimension that
   becomes odd before the last level, a or b of the key nonzero, m > 64, ...). */
jfmg_status jfmg_workspace_bytes(const jfmg_config* cfg, size_t* bytes);

/* Create a problem in the caller's device workspace (>= jfmg_workspace_bytes,
   256-byte aligned) on the HIP stream `hip_stream` (NULL = default stream).
   Builds the reference-element, background and index tables on the host and
   uploads them.  The workspace stays owned by the caller and must outlive the
   problem. */
jfmg_status jfmg_create_problem(const jfmg_config* cfg, void* workspace, size_t ws_bytes,
                                void* hip_stream, jfmg_problem** out);

/* Release the host-side handle; frees nothing the caller gave. */
jfmg_status jfmg_destroy_problem(jfmg_problem* p);

/* N = 4 nx nz (k+1)^2, and 4 nxl nzl of FV level `level` (0 = finest). */
size_t jfmg_num_dofs(const jfmg_problem* p);
size_t jfmg_fv_size(const jfmg_problem* p, int level);

/* Initial perturbation U' at the GL nodes: theta' inserted at constant
   pressure (eq. add-perturbation), rho theta' = 0, v = background wind. */
jfmg_status jfmg_initial_state(jfmg_problem* p, const jfmg_perturbation* pert, double* U);

/* out = <psi, L_h(U')> (eqs. convDiscr, elementint, surfaceint on the
   perturbation system), or f = M^-1 L_h (Sec. "Temporal discretization") when
   apply_minv = 1.  U and out are DG vectors; no host synchronization. */
jfmg_status jfmg_residual(jfmg_problem* p, const double* U, double* out, int apply_minv);

/* G = U - alpha_dt f(U) - Ubar (eq. newton) and, if norm != NULL, ||G||_2
   (host pointer; synchronizes). */
jfmg_status jfmg_stage_residual(jfmg_problem* p, const double* U, const double* Ubar,
                                double alpha_dt, double* G, double* norm);

/* Set the Newton iterate U (copied) and alpha*dt for jfmg_jvp / jfmg_mg_apply:
   ||U + Ubar||, the FV linearization states u_L = T^mf U, u_{l-1} = R u_l,
   f_low(u_l) and the pseudo time steps of every level. */
jfmg_status jfmg_linearize(jfmg_problem* p, const double* U, double alpha_dt);

/* out = G'(U) y by finite differences (Sec. "Solver"):
   y - (alpha dt/eps) M^-1 (L_h(U + eps y) - L_h(U)), eps per fd_eps_mode.
   ESTATE without jfmg_linearize.  y = 0 gives 0. */
jfmg_status jfmg_jvp(jfmg_problem* p, const double* y, double* out);

/* z = Q^-1 r = T^-1 MG(0, T r; u_L) (eq. preconditioner); identity when
   precond = 0.  With the DG smoothing counts a, b of mg_key nonzero the DG data
   are the finest level of the cycle (Sec. "Smoother / Pseudo time iteration":
   pseudo-time smoothing on the DG data before the transfer and after the
   reconstruction): a sweeps of the s-stage smoother
   z_j = z_0 + alpha_j dtau_dg (r - G' z_{j-1}) from z = 0, the coarse
   correction z += T^-1 MG(0, T(r - G' z)), then b sweeps.  Workspace vectors of
   the problem hold the intermediate vectors.  ESTATE without jfmg_linearize. */
jfmg_status jfmg_mg_apply(jfmg_problem* p, const double* r, double* z);

/* ---- lock-step batches (config.batch = B > 1) ----
   B members of one configuration (an ensemble: same grid, physics and solver,
   different states) share one problem: jfmg_workspace_bytes returns B times
   the bytes of one member, every kernel covers all members in one launch
   (launch grid z = member), and the Newton and FGMRES iterations run in lock
   step with per-member norms, forcing terms, Hessenberg matrices and stopping
   tests; a member that has converged takes no further part (its updates are
   zero).  Each member's result is bitwise the one it gives as a single problem.
   State vectors passed in are B * N doubles, members back to back.  Only
   jfmg_implicit_step, jfmg_initial_state (the same state for every member),
   jfmg_linearize (every member at its own state), the tile-shape calls and
   jfmg_autotune accept batched problems; the other calls return EINVAL.  Stats
   count the lock-step iterations. */

/* ---- ragged batches: ensemble members of different grid sizes ----
   n configurations that differ only in nx, nz and the domain (x0, x1, z0, z1)
   form one lock-step batch: every member has a workspace region laid out for the
   envelope grid (the largest nx and nz), a device table carries each member's
   sizes, geometry and background tables, and every kernel still covers all
   members in one launch (grid z = member): its work-groups beyond a smaller
   member's elements or tiles stay idle and store zero partial sums, so each
   member's result is bitwise the one it gives as a single problem with the same
   FV tile shapes (the tile shapes apply to all members).  State vectors are the
   members' DG vectors back to back, member m with jfmg_member_dofs(p, m)
   entries; initial states come from single problems.  The calls accepted are
   those of lock-step batches except jfmg_initial_state; the multigrid key must
   not use DG-level smoothing (a, b = 0).  EINVAL for members that differ in
   anything else, ENOMEM for a short workspace. */
jfmg_status jfmg_ensemble_workspace_bytes(const jfmg_config* cfgs, int n, size_t* bytes);
jfmg_status jfmg_create_ensemble(const jfmg_config* cfgs, int n, void* workspace, size_t ws_bytes,
                                 void* hip_stream, jfmg_problem** out);
/* DG entries of member `member` (N of a single problem or a lock-step batch's
   member; 0 for a member index out of range). */
size_t jfmg_member_dofs(const jfmg_problem* p, int member);

/* One implicit step U^n -> U^{n+1} in place (implicit Euler or SDIRK2), each
   stage by inexact Newton with Eisenstat-Walker forcing and right-preconditioned
   FGMRES (Sec. "Solver").  On any error U is left unchanged.  stats may be NULL.
   FGMRES iterations are launched kernel by kernel; with the environment variable
   JFMG_GRAPH=1 when the problem is created, each iteration index is captured
   once as a HIP graph and replayed instead (bitwise the same results). */
jfmg_status jfmg_implicit_step(jfmg_problem* p, double* U, jfmg_stats* stats);

/* One stage equation G(U) = U - alpha_dt f(U) - Ubar = 0 (eq. newton) solved
   as inside jfmg_implicit_step: inexact Newton from U^0 = Ubar with
   Eisenstat-Walker forcing and preconditioned FGMRES (Sec. "Solver").  Ubar
   (read) and U (written with the solution) are device DG vectors; U is left
   unchanged on any error.  Host-synchronous.  SDIRK2 is the stage with
   alpha_dt = (1 - sqrt(2)/2) dt and Ubar = U^n, then the stage with the same
   alpha_dt and Ubar = U^n + (sqrt(2)/2) dt f(U_1) (eq. ellsiep).  EINVAL for a
   batched problem or alpha_dt not positive and finite. */
jfmg_status jfmg_newton_stage(jfmg_problem* p, const double* Ubar, double alpha_dt, double* U, jfmg_stats* stats);

/* nsteps explicit steps U^n -> U^{n+1} in place with the four-stage,
   third-order strong-stability-preserving Runge-Kutta method (Ketcheson 2008)
   that the paper's reference runs use (Sec. "Numerical Experiments", set-up):
   U1 = U + dt/2 f(U), U2 = U1 + dt/2 f(U1), U3 = 2/3 U + 1/3 U2 + dt/6 f(U2),
   U^{n+1} = U3 + dt/2 f(U3), with f = M^-1 L_h.  U is a device DG vector; the
   call is queued on the problem's stream without host synchronization and uses
   the problem's workspace (do not overlap it with other calls on the problem).
   dt is not limited here: a step beyond the CFL limit diverges.  EINVAL for a
   batched problem, a non-finite dt or nsteps < 0. */
jfmg_status jfmg_explicit_steps(jfmg_problem* p, double* U, double dt, int nsteps);

/* ---- finer-grained calls on the preconditioner's pieces (FV vectors in the
        problem's multigrid precision) ---- */

/* u = T^mf U (DG -> finest FV level) or U = T^-1,mf u (FV -> DG), dir 0 / 1
   (Sec. "Transfer functions", eq. transfer-mass-fix, appendix weights). */
jfmg_status jfmg_transfer(jfmg_problem* p, int dir, const void* in, void* out);
/* coarse = R fine (agglomeration average, fine_level -> fine_level+1) */
jfmg_status jfmg_restrict(jfmg_problem* p, int fine_level, const void* fine, void* coarse);
/* fine = P coarse (injection, coarse_level -> coarse_level-1) */
jfmg_status jfmg_prolong(jfmg_problem* p, int coarse_level, const void* coarse, void* fine);
/* Copy of the linearization state u_l of `level`; ESTATE without linearize. */
jfmg_status jfmg_fv_level_state(jfmg_problem* p, int level, void* u);
/* Pseudo time step of `level` (host double; synchronizes). */
jfmg_status jfmg_fv_dtau(jfmg_problem* p, int level, double* dtau);
/* Pseudo time step of the DG-level smoother (Sec. "Smoother / Pseudo time
   iteration"; formula at pseudo_cfl_dg; host double; synchronizes).  ESTATE
   without jfmg_linearize; EINVAL when a = b = 0. */
jfmg_status jfmg_dg_dtau(jfmg_problem* p, double* dtau);
/* out = g'_l(u_l) x = x - (alpha dt/eps)(f_low(u_l + eps x) - f_low(u_l)),
   eps = sqrt(eps_p) ||u_l + Ubar|| / ||x||. */
jfmg_status jfmg_fv_matvec(jfmg_problem* p, int level, const void* x, void* out);
/* x = MG_L(0, b; u_L): one multigrid cycle on the FV levels from x = 0. */
jfmg_status jfmg_mg_fv(jfmg_problem* p, const void* b, void* x);
/* fv_to_dg[J*nxf + I] = e*(k+1)^2 + node of the DG node whose subcell is (I,J). */
jfmg_status jfmg_subgrid_map(jfmg_problem* p, int* fv_to_dg);

/* ---- tile shapes of the FV operator kernels, per multigrid level ----
   The smoother stage, matvec, defect and linearization kernels of a level (the
   FV operator of Sec. "Multigrid preconditioner for finite volume
   approximations") run with one of these work-group tiles of cells:
     JFMG_TILE_64x4  256 threads, one wave per 64-cell row
     JFMG_TILE_64x8  512 threads, one wave per 64-cell row
     JFMG_TILE_16x4  256 threads, every face of the tile on its own thread
     JFMG_TILE_8x4   128 threads, every face of the tile on its own thread
     JFMG_TILE_32x4  256 threads, two per cell
     JFMG_TILE_64x4_512  512 threads, two per cell
   A new problem uses, by level width in cells, 64x8 from 1024, 64x4_512 from
   512, 16x4 from 256 and 8x4 below.
   Shapes change the order of the partial sums of the FD step norms only, so
   results agree to rounding; the same shapes give bitwise the same results. */
typedef enum {
    JFMG_TILE_64x4 = 0,
    JFMG_TILE_64x8 = 1,
    JFMG_TILE_16x4 = 2,
    JFMG_TILE_8x4 = 3,
    JFMG_TILE_32x4 = 4,
    JFMG_TILE_64x4_512 = 5,
    JFMG_TILE_NSHAPE = 6
} jfmg_tile;
/* shapes: host array of mg_levels entries (finest level first). */
jfmg_status jfmg_get_tiles(const jfmg_problem* p, int* shapes);
/* EINVAL for an unknown shape (nothing changed).  Drops captured HIP graphs. */
jfmg_status jfmg_set_tiles(jfmg_problem* p, const int* shapes);
/* Autotuner: on every level, time every shape with `reps` back-to-back launches
   (after one warm-up launch) of the smoother stage kernel at the current
   linearization state, with a fixed nonzero test vector, and keep the fastest.
   A lock-step batch times all its members in each launch.  shapes (mg_levels
   entries) receives the choice and times_us (mg_levels * JFMG_TILE_NSHAPE
   entries, level-major) the mean launch time in microseconds; either may be
   NULL.  ESTATE without jfmg_linearize; EINVAL for reps outside 1..1000.
   Synchronizes the stream and overwrites the multigrid work vectors. */
jfmg_status jfmg_autotune(jfmg_problem* p, int reps, int* shapes, double* times_us);

/* ---- kernel-class timing (benchmark instrumentation) ----
   When a class's bit is set in class_mask, every launch of that class records
   the start and stop events of its own dispatch (hipExtLaunchKernel) on the
   stream it runs on; jfmg_profile_read returns per class the summed event time
   [ms], the launch count and the summed algorithmic HBM bytes (what the launch
   must read and write at minimum, e.g. 6 FV vectors for a smoother stage with a
   matvec).  While a mask is set, implicit steps launch kernel by kernel even
   with JFMG_GRAPH=1 (event timing inside graphs is not available).  Enabling
   resets the counters and synchronizes the stream. */
typedef enum {
    JFMG_K_DG_RESIDUAL = 0,   /* stage residual G and ||G||                         */
    JFMG_K_DG_JVP = 1,        /* fused FD Jacobian-vector product                   */
    JFMG_K_FV_STAGE = 2,      /* RK smoother stage with an FV matvec, levels >= 512
                                 cells wide (wide-tile kernel)                      */
    JFMG_K_FV_STAGE_ZERO = 3, /* first stage from x = 0 (no matvec)                 */
    JFMG_K_FV_DEFECT = 4,     /* defect + agglomeration restriction                 */
    JFMG_K_FV_PROLONG = 5,    /* injection prolongation + correction               */
    JFMG_K_FV_LINEARIZE = 6,  /* f_low(u_l), ||u_l + Ubar||, pseudo time step       */
    JFMG_K_TRANSFER_T = 7,    /* DG -> FV                                           */
    JFMG_K_TRANSFER_TINV = 8, /* FV -> DG                                           */
    JFMG_K_MULTIDOT = 9,      /* Arnoldi <w, v_i>                                   */
    JFMG_K_UPDATE = 10,       /* Arnoldi w -= V h                                   */
    JFMG_K_FV_STAGE_SMALL = 11, /* the same on narrower levels (small-tile kernel)    */
    JFMG_K_DG_SMOOTH = 12,    /* DG-level smoother stage combination (key a, b)     */
    JFMG_K_DG_LINEARIZE = 13, /* fluxes of the linearization state for the JVPs     */
    JFMG_K_NCLASS = 14
} jfmg_kernel_class;
jfmg_status jfmg_profile_enable(jfmg_problem* p, unsigned class_mask);
/* ms, launches and bytes are host arrays of JFMG_K_NCLASS entries. */
jfmg_status jfmg_profile_read(jfmg_problem* p, double* ms, long long* launches, double* bytes);

/* ---- ensembles and served requests: many independent problems, one arena ----
   A batch advances independent members (an ensemble of perturbed forecasts, or
   requests of a solver service) concurrently.  Each member is an ordinary
   problem whose workspace is a first-fit, 256-byte aligned range of the
   caller's device arena, taken at admission and returned at retirement
   (admission fails with ENOMEM when no range is large enough: the arena is the
   HBM budget).  A pool of host worker threads advances the members one
   implicit step at a time, each step on the member's private stream, so the
   small kernels of different members overlap on the GPU.  A member's state U
   is a caller-owned device vector updated in place after every step.  Members
   share no device memory and every kernel reduces in a fixed order, so a
   member's result is bitwise the same alone and in any mix.  The batch
   functions are called from one host thread. */
typedef struct jfmg_batch jfmg_batch;
/* arena: device memory of arena_bytes (256-byte aligned), owned by the caller
   and unused by it while the batch exists; max_members slots; workers host
   threads (0: min(max_members, 8)); hip_stream: the stream member creation and
   jfmg_initial_state on members use, and that run/start order after. */
jfmg_status jfmg_batch_create(size_t arena_bytes, void* arena, int max_members, int workers, void* hip_stream,
                              jfmg_batch** out);
/* Stops the workers after their current steps and destroys every member. */
jfmg_status jfmg_batch_destroy(jfmg_batch* b);
/* Admit a member that will take n_steps implicit steps of U (device, caller
   owned, N = 4 nx nz (k+1)^2 doubles).  With pert non-NULL, U is first set to
   that initial state (as jfmg_initial_state, on the batch stream); else U must
   hold the state.  ENOMEM: no free slot or arena range; EINVAL: invalid
   configuration.  In background mode the member starts at once. */
jfmg_status jfmg_batch_admit(jfmg_batch* b, const jfmg_config* cfg, const jfmg_perturbation* pert, double* U,
                             int n_steps, int* slot);
/* The member's problem, e.g. for jfmg_initial_state on U; only while the
   member is not being advanced (before run/start, or once finished). */
jfmg_problem* jfmg_batch_member(jfmg_batch* b, int slot);
/* Advance every unfinished member by up to max_steps steps (all remaining if
   max_steps <= 0) and return when they are done.  ESTATE in background mode. */
jfmg_status jfmg_batch_run(jfmg_batch* b, int max_steps);
/* Background mode: the workers keep advancing every member, including members
   admitted later, until it has taken all its steps; jfmg_batch_stop ends it
   (after the steps in flight). */
jfmg_status jfmg_batch_start(jfmg_batch* b);
jfmg_status jfmg_batch_stop(jfmg_batch* b);
/* Wait up to timeout_s seconds (forever if < 0) for a member to finish; *slot
   is the finished member, each reported once, or -1 on timeout or when no
   member is active. */
jfmg_status jfmg_batch_wait_any(jfmg_batch* b, double timeout_s, int* slot);
/* finished = 1 once every step is done or a step failed; steps_done; stats
   summed over the member's steps (status: the first failure).  Returns the
   member's status. */
jfmg_status jfmg_batch_poll(jfmg_batch* b, int slot, int* finished, int* steps_done, jfmg_stats* stats);
/* Destroy a member that is not being advanced and return its arena range. */
jfmg_status jfmg_batch_retire(jfmg_batch* b, int slot);
/* Largest free arena range in bytes. */
size_t jfmg_batch_arena_free(jfmg_batch* b);
const char* jfmg_batch_last_error(const jfmg_batch* b);

/* ---- allocation-free stage residual ----
   For callers that cannot allocate device memory: code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc.  The same
   G = U - alpha_dt f(U) - Ubar as jfmg_stage_residual, for the single problem
   described by cfg, without a problem handle or a workspace: the background
   tables of the DG kernel and the block partials of the norm live in a
   file-scope device array of JFMG_NOALLOC_SCRATCH_BYTES (1 MiB) per GPU, held
   until the process ends.  U, Ubar, G: caller-owned device DG vectors of
   N = 4 nx nz (k+1)^2 doubles (layout as everywhere above); norm2: NULL or a
   caller-owned device double that receives ||G||_2^2.  Stream ordered on
   hip_stream (NULL = default stream); no host synchronization, no device
   memory allocation (the first call on a device resolves the array's address
   once).  Errors: EINVAL for a null vector, an invalid configuration, batch > 1
   or a non-finite alpha_dt; ENOMEM when the tables and partials of the problem
   exceed the array (tables of 88 bytes per node row, nz (k+1) rows, and 80 per
   element face row, nz + 1 rows, plus 8 bytes per DG work-group of 8 to 16
   elements, each region 256-byte aligned: every configuration with
   nz (k+1) <= 2048 and nx nz <= 65536 fits);
   EDEVICE for a HIP error.  Messages through jfmg_last_error(NULL).  Every call
   on one GPU uses that GPU's array: calls that overlap on one GPU (different
   streams or threads) race on it and must be serialized by the caller.  The
   background tables are evaluated on the device, so G agrees with
   jfmg_stage_residual to rounding, not bitwise. */
#define JFMG_NOALLOC_SCRATCH_BYTES ((size_t)1 << 20)
jfmg_status jfmg_stage_residual_noalloc(const jfmg_config* cfg, const double* U, const double* Ubar,
                                        double alpha_dt, double* G, double* norm2, void* hip_stream);

/* Message of the last failed call on p (or of the last failed creation if p is NULL). */
const char* jfmg_last_error(const jfmg_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* JFMG_H */
