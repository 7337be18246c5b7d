/*
 * Oracle for the Jacobian-free Newton-GMRES / FV-subgrid multigrid method of
 * Birken, Dedner & Kloefkorn, "A Jacobian-free Multigrid Preconditioner for
 * Discontinuous Galerkin Methods applied to Numerical Weather Prediction".
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 reference written
 * from the paper (OpenMP over the element and cell loops, results independent
 * of the thread count).  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the GPU library and the GPU library never calls it.
 *
 * Vector layouts (chosen for the whole project; the paper fixes none):
 *   DG vector   [4][nz][nx][(k+1)^2]  components (rho, rho u, rho w, rho theta)
 *               of the perturbation U' (well-balanced form, Sec. "euler-model"),
 *               element e = ez*nx+ex, node b*(k+1)+a, a along x, GL order.
 *   FV vector   [4][nzl][nxl]         cell (I,J) at index J*nxl+I.
 */
#ifndef ORC_H
#define ORC_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, nz, k;
    int physics;        /* 0 Euler, 1 viscous (F_v of eq. compressible-euler) */
    int background;     /* 0 neutral (theta const), 1 constant Brunt-Vaisala N */
    int bc;             /* 0 slip walls everywhere, 1 periodic x + slip z      */
    int mass_fix;       /* 1: transfer with the mass fix (eq. transfer-mass-fix) */
    int transfer;       /* 0 interpolation at the subcell centres, 1 L2 projection
                           onto the subcells (subcell averages; no mass fix)       */
    int mg_levels;      /* number of FV levels, finest included               */
    int nu_pre_fine, nu_post_fine, nu_pre, nu_post; /* key mg a b c d e f G: c d e f */
    int cycle;          /* 1 V-cycle, 2 W-cycle                               */
    int rk_stages;      /* explicit RK pseudo-time smoother stages            */
    int fd_eps_mode;    /* DG FD step: 0 paper literal, 1 state scaled         */
    int gmres_m, gmres_max_restarts, newton_maxit;
    int scheme;         /* 0 implicit Euler, 1 SDIRK2 (Ellsiepen)             */
    int precond;        /* 1 multigrid preconditioner, 0 identity             */
    double x0, x1, z0, z1;
    double g, gamma, R, p0, theta0, N, u_mean, mu, c_ip;
    double rk_alpha[4];
    double pseudo_cfl;
    double newton_rtol, ew_gamma, ew_alpha, ew_eta0, ew_eta_max;
    double dt;
    double newton_stall; /* > 0: also stop at the rounding floor of G (see orc_newton_stage) */
    int nu_pre_dg, nu_post_dg; /* key mg a b c d e f G: a b, pseudo-time sweeps on the DG data */
    double pseudo_cfl_dg;      /* c* of the DG-level pseudo time step                      */
} orc_cfg;

typedef struct {
    int shape;          /* 0 cosine bubble, 1 inertia-gravity profile */
    int pad;
    double amp, xc, zc, xr, zr, a, Z;
} orc_pert;

typedef struct {
    int newton_its, gmres_its, lh_evals, jvps;
    int fv_matvecs[8];
    int status;
    int stalls;         /* stages stopped at the rounding floor of G */
    double g0_norm, g_norm;
} orc_stats;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOCONV = 3, ORC_ENONFINITE = 4 };

typedef struct orc_ctx orc_ctx;

int  orc_ref_tables(int k, double* xi, double* w, double* D, double* em, double* ep,
                    double* dm, double* dp, double* V, double* Vinv, double* wnc);
/* L2 projection onto the k+1 equal subintervals of [-1, 1]: P[i][a] = mean of the
   Lagrange basis function l_a over subinterval i, and its inverse. */
int  orc_proj_tables(int k, double* P, double* Pinv);
orc_ctx* orc_create(const orc_cfg* cfg);
void orc_destroy(orc_ctx* X);
long orc_num_dofs(const orc_ctx* X);
int  orc_fv_dims(const orc_ctx* X, int level, int* nxl, int* nzl);

void orc_background(const orc_ctx* X, double z, double* Ub, double* dUb);
void orc_flux(const orc_ctx* X, const double* U, double nx, double nz, double* F);
void orc_hllc(const orc_ctx* X, const double* UL, const double* UR, double nx, double nz, double* F);
void orc_initial_state(const orc_ctx* X, const orc_pert* P, double* U);

/* mode 0: <psi, L_h(U)>; 1: f = M^-1 L_h(U); 2: non-well-balanced <psi, L(U'+Ubar)>;
   3: rounding scale (sums of absolute values of the unsubtracted terms) */
void orc_residual(orc_ctx* X, const double* U, double* out, int mode);
void orc_stage_residual(orc_ctx* X, const double* U, const double* Ubar, double alpha_dt, double* G);

void orc_transfer_T(const orc_ctx* X, const double* U, double* u);
void orc_transfer_Tinv(const orc_ctx* X, const double* u, double* U);
void orc_restrict(const orc_ctx* X, int fine_level, const double* uf, double* uc);
void orc_prolong(const orc_ctx* X, int coarse_level, const double* uc, double* uf);
void orc_fv_residual(const orc_ctx* X, int level, const double* u, double* f);
void orc_subgrid_map(const orc_ctx* X, int* fv_to_dg);

int  orc_linearize(orc_ctx* X, const double* U, double alpha_dt);
void orc_fv_level_state(const orc_ctx* X, int level, double* u);
double orc_fv_dtau(const orc_ctx* X, int level);
double orc_dg_dtau(const orc_ctx* X);
/* operation counts (FV matvecs per level, JVPs, L_h calls) since creation or the
   last call with reset = 1; test instrumentation */
void orc_counters(orc_ctx* X, int* fv_matvecs, int* jvps, int* lh_evals, int reset);
void orc_fv_matvec(orc_ctx* X, int level, const double* x, double* out);
void orc_jvp(orc_ctx* X, const double* y, double* out);
void orc_mg_fv(orc_ctx* X, const double* b, double* x);
void orc_mg_apply(orc_ctx* X, const double* r, double* z);

typedef void (*orc_op)(void* ctx, const double* in, double* out);
int  orc_fgmres(long n, orc_op A, void* actx, orc_op P, void* pctx, const double* rhs,
                double tol_abs, int m, int max_restarts, double* x, int* its);

int  orc_newton_stage(orc_ctx* X, const double* Ubar, double alpha_dt, double* U, orc_stats* st);
int  orc_implicit_step(orc_ctx* X, double* U, orc_stats* st);
/* nsteps explicit SSP RK(4,3) steps of size dt (the paper's reference method) */
void orc_explicit_steps(orc_ctx* X, double* U, double dt, int nsteps);

#ifdef __cplusplus
}
#endif
#endif
