/*
 * Oracle for the Jacobian-free Newton-GMRES solver with the FV-subgrid
 * multigrid preconditioner of Birken, Dedner & Kloefkorn (arXiv 2505.24504).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow FP64 C written from the paper, used by
 * the tests, the smoke check and the CPU-baseline leg of the benchmark.  It
 * shares no code with the GPU library.  The element loop of L_h and the cell
 * loop of f_low run on all host cores (OpenMP; every element's and cell's
 * arithmetic is the serial one, so results do not depend on the thread count);
 * everything else is serial.
 *
 * Where the paper leaves a choice open the oracle takes the readings listed in
 * the project's design notes; each function below names the passage it
 * follows and the reading it takes.  Parity-pinned by tests/test_oracle_*.py;
 * no function here is "parity unpinned".
 */
#include "orc.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXK 3
#define MAXN (MAXK + 1)
#define MAXLEV 8

struct orc_ctx {
    orc_cfg c;
    int n1, np;                 /* k+1, (k+1)^2 */
    long ne, ndof;              /* elements, 4*ne*np */
    double dx, dz, J;           /* element sizes, |J| = dx dz / 4 */
    double xi[MAXN], w[MAXN], D[MAXN][MAXN], em[MAXN], ep[MAXN], dm[MAXN], dp[MAXN];
    double V[MAXN][MAXN], Vinv[MAXN][MAXN], wnc[MAXN];
    double P[MAXN][MAXN], Pinv[MAXN][MAXN];   /* L2 projection onto subcells (transfer = 1) */
    int nlev, nxl[MAXLEV], nzl[MAXLEV];
    double hx[MAXLEV], hz[MAXLEV];
    /* linearization (Newton iterate) */
    int have_lin;
    double adt;                 /* alpha * dt */
    double* Ulin;               /* DG perturbation state */
    double* Llin;               /* <psi, L_h(Ulin)> */
    double utot_dg;             /* || Ulin + Ubar ||_2 over all DG nodes */
    double* ulev[MAXLEV];       /* FV linearization states u_l (perturbation) */
    double* flev[MAXLEV];       /* f_low(u_l) */
    double utot[MAXLEV], lam[MAXLEV], dtau[MAXLEV];
    double dtau_dg;             /* pseudo time step of the DG-level smoother */
    int* mv_count;              /* counts FV matvecs per level (stats) */
    int mv_local[MAXLEV];
    int lh_count, jvp_count;
};

/* ------------------------------------------------------------------------ */
/* Reference element (Sec. "Discontinuous Galerkin Discretization"): Lagrange */
/* basis on tensor-product Gauss-Legendre nodes, FV subcell centres (figure  */
/* lgl_fv_points) and the modified Newton-Cotes weights of the appendix.     */
/* ------------------------------------------------------------------------ */

static void legendre(int n, double x, double* P, double* dP)
{
    /* P_n(x) and P_n'(x) by the three-term recurrence */
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    *dP = n * (x * p1 - p0) / (x * x - 1.0);
}

static void gauss_legendre(int n, double* x, double* w)
{
    /* roots of P_n by Newton's method, ascending; w_i = 2/((1-x^2) P_n'^2) */
    for (int i = 0; i < n; ++i) {
        double r = -cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, r, &P, &dP);
            double dr = P / dP;
            r -= dr;
            if (fabs(dr) < 1e-16) break;
        }
        double P, dP;
        legendre(n, r, &P, &dP);
        x[i] = r;
        w[i] = 2.0 / ((1.0 - r * r) * dP * dP);
    }
}

static double lagrange(int n, const double* xs, int j, double x)
{
    double v = 1.0;
    for (int m = 0; m < n; ++m)
        if (m != j) v *= (x - xs[m]) / (xs[j] - xs[m]);
    return v;
}

static double lagrange_deriv(int n, const double* xs, int j, double x)
{
    double s = 0.0;
    for (int l = 0; l < n; ++l) {
        if (l == j) continue;
        double t = 1.0 / (xs[j] - xs[l]);
        for (int m = 0; m < n; ++m)
            if (m != j && m != l) t *= (x - xs[m]) / (xs[j] - xs[m]);
        s += t;
    }
    return s;
}

/* Solve A X = B (n x n, nr right-hand sides) by Gauss-Jordan with partial pivoting. */
static int solve_dense(int n, double* A, double* B, int nr)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) return -1;
        if (piv != col) {
            for (int j = 0; j < n; ++j) { double t = A[col * n + j]; A[col * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            for (int j = 0; j < nr; ++j) { double t = B[col * nr + j]; B[col * nr + j] = B[piv * nr + j]; B[piv * nr + j] = t; }
        }
        double d = A[col * n + col];
        for (int j = 0; j < n; ++j) A[col * n + j] /= d;
        for (int j = 0; j < nr; ++j) B[col * nr + j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = A[r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) A[r * n + j] -= f * A[col * n + j];
            for (int j = 0; j < nr; ++j) B[r * nr + j] -= f * B[col * nr + j];
        }
    }
    return 0;
}

int orc_ref_tables(int k, double* xi, double* w, double* D, double* em, double* ep,
                   double* dm, double* dp, double* V, double* Vinv, double* wnc)
{
    if (k < 1 || k > MAXK) return ORC_EINVAL;
    int n = k + 1;
    gauss_legendre(n, xi, w);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) D[i * n + j] = lagrange_deriv(n, xi, j, xi[i]);
    for (int j = 0; j < n; ++j) {
        em[j] = lagrange(n, xi, j, -1.0);
        ep[j] = lagrange(n, xi, j, 1.0);
        dm[j] = lagrange_deriv(n, xi, j, -1.0);
        dp[j] = lagrange_deriv(n, xi, j, 1.0);
    }
    /* subcell centres c_i = -1 + (2i+1)/(k+1) (equidistant subdivision) */
    double A[MAXN * MAXN];
    for (int i = 0; i < n; ++i) {
        double ci = -1.0 + (2.0 * i + 1.0) / n;
        for (int j = 0; j < n; ++j) V[i * n + j] = lagrange(n, xi, j, ci);
    }
    memcpy(A, V, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) Vinv[i] = 0.0;
    for (int i = 0; i < n; ++i) Vinv[i * n + i] = 1.0;
    if (solve_dense(n, A, Vinv, n)) return ORC_EINVAL;
    /* modified Newton-Cotes weights on [0,1] at G_i = (2i+1)/(2(k+1)): the
       interpolatory rule w_i = int_0^1 l_i(s) ds with l_i the Lagrange basis on
       the points G_i, so that it is exact for degree <= k.  The integral of the
       degree-k polynomial l_i is taken with the (k+1)-point GL rule, which is
       exact for it. */
    double G[MAXN];
    for (int i = 0; i < n; ++i) G[i] = (2.0 * i + 1.0) / (2.0 * n);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += 0.5 * w[q] * lagrange(n, G, i, 0.5 * (1.0 + xi[q]));
        wnc[i] = s;
    }
    return ORC_OK;
}

/* L2 projection of the element polynomial onto the piecewise constants of the
   (k+1)^2 subcells (the alternative to interpolation that Sec. "Transfer
   functions" names; it conserves mass by construction): in 1D the average of l_a
   over subinterval i = [-1 + 2i/(k+1), -1 + 2(i+1)/(k+1)],
       P[i][a] = (1/2) sum_q w_q l_a(s_i + (1 + xi_q)/(k+1)),
   the (k+1)-point GL rule on the subinterval (exact: l_a has degree k), and the
   element map is the tensor product P (x) P.  Its inverse gives T^-1. */
int orc_proj_tables(int k, double* P, double* Pinv)
{
    if (k < 1 || k > MAXK) return ORC_EINVAL;
    int n = k + 1;
    double xi[MAXN], w[MAXN], A[MAXN * MAXN];
    gauss_legendre(n, xi, w);
    for (int i = 0; i < n; ++i) {
        double si = -1.0 + 2.0 * i / n;
        for (int a = 0; a < n; ++a) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += w[q] * lagrange(n, xi, a, si + (1.0 + xi[q]) / n);
            P[i * n + a] = 0.5 * s;
        }
    }
    memcpy(A, P, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) Pinv[i] = 0.0;
    for (int i = 0; i < n; ++i) Pinv[i * n + i] = 1.0;
    if (solve_dense(n, A, Pinv, n)) return ORC_EINVAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Physics (eq. compressible-euler) and background atmospheres              */
/* ------------------------------------------------------------------------ */

static double cp_of(const orc_cfg* c) { return c->gamma * c->R / (c->gamma - 1.0); }

/* Equation of state p = p0 (R rho theta / p0)^gamma, the inverse of the
   pressure-preserving insertion formula eq:add-perturbation. */
static double pressure(const orc_cfg* c, double rt) { return c->p0 * pow(c->R * rt / c->p0, c->gamma); }

/* background potential temperature: theta0, or theta0 e^{z/H} with H = g/N^2 */
static double bg_theta(const orc_cfg* c, double z)
{
    if (c->background == 0) return c->theta0;
    return c->theta0 * exp(z / (c->g / (c->N * c->N)));
}

/* Background atmosphere Ubar(z) and d/dz Ubar(z).
   Neutral (rising bubble / density current): theta = theta0,
     T = theta0 - g z / cp, p = p0 (T/theta0)^(cp/R).
   Constant N (inertia-gravity): theta = T0 e^{z/H}, T = T0 (a - (a-1) e^{z/H}),
     p = p0 exp(cp/R (ln(T/T0) - z/H)), H = g/N^2, a = g H/(cp T0), T0 = theta0.
   rho theta = p0^{R/cp} p^{1/gamma} / R, rho = (rho theta)/theta, momentum rho*u_mean. */
void orc_background(const orc_ctx* X, double z, double* Ub, double* dUb)
{
    const orc_cfg* c = &X->c;
    double cp = cp_of(c);
    double th, dth, p, dp;
    if (c->background == 0) {
        double T = c->theta0 - c->g * z / cp;
        th = bg_theta(c, z);
        dth = 0.0;
        p = c->p0 * pow(T / c->theta0, cp / c->R);
        dp = -(c->g * c->p0 / (c->R * c->theta0)) * pow(T / c->theta0, cp / c->R - 1.0);
    } else {
        double H = c->g / (c->N * c->N);
        double a = c->g * H / (cp * c->theta0);
        double ez = exp(z / H);
        double T = c->theta0 * (a - (a - 1.0) * ez);
        double dT = -c->theta0 * (a - 1.0) * ez / H;
        th = bg_theta(c, z);
        dth = th / H;
        p = c->p0 * exp((cp / c->R) * (log(T / c->theta0) - z / H));
        dp = p * (cp / c->R) * (dT / T - 1.0 / H);
    }
    double C = pow(c->p0, c->R / cp) / c->R;
    double rt = C * pow(p, 1.0 / c->gamma);
    double drt = C * (1.0 / c->gamma) * pow(p, 1.0 / c->gamma - 1.0) * dp;
    double rho = rt / th;
    double drho = (drt - rho * dth) / th;
    Ub[0] = rho;
    Ub[1] = rho * c->u_mean;
    Ub[2] = 0.0;
    Ub[3] = rt;
    if (dUb) {
        dUb[0] = drho;
        dUb[1] = drho * c->u_mean;
        dUb[2] = 0.0;
        dUb[3] = drt;
    }
}

/* Convective flux F_c(U) . n (eq. compressible-euler), n axis aligned. */
void orc_flux(const orc_ctx* X, const double* U, double nx, double nz, double* F)
{
    double rho = U[0], u = U[1] / rho, w = U[2] / rho;
    double p = pressure(&X->c, U[3]);
    double q = u * nx + w * nz;
    F[0] = U[1] * nx + U[2] * nz;
    F[1] = U[1] * q + p * nx;
    F[2] = U[2] * q + p * nz;
    F[3] = U[3] * q;
}

/* HLLC flux (Toro) with Davis wave-speed estimates; the star flux is written
   in the S*-factored form, algebraically identical to F_K + S_K (U*_K - U_K). */
void orc_hllc(const orc_ctx* X, const double* UL, const double* UR, double nx, double nz, double* F)
{
    const orc_cfg* c = &X->c;
    double rL = UL[0], uL = UL[1] / rL, wL = UL[2] / rL, pL = pressure(c, UL[3]);
    double rR = UR[0], uR = UR[1] / rR, wR = UR[2] / rR, pR = pressure(c, UR[3]);
    double qL = uL * nx + wL * nz, qR = uR * nx + wR * nz;
    double cL = sqrt(c->gamma * pL / rL), cR = sqrt(c->gamma * pR / rR);
    double SL = fmin(qL - cL, qR - cR);
    double SR = fmax(qL + cL, qR + cR);
    if (SL >= 0.0) { orc_flux(X, UL, nx, nz, F); return; }
    double Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) / (rL * (SL - qL) - rR * (SR - qR));
    const double* UK;
    double SK, rK, qK, pK;
    if (Ss >= 0.0) { UK = UL; SK = SL; rK = rL; qK = qL; pK = pL; }
    else if (SR > 0.0) { UK = UR; SK = SR; rK = rR; qK = qR; pK = pR; }
    else { orc_flux(X, UR, nx, nz, F); return; }
    double FK[4];
    orc_flux(X, UK, nx, nz, FK);
    double pstar = pK + rK * (SK - qK) * (Ss - qK);
    double den = SK - Ss;
    F[0] = (Ss * (SK * UK[0] - FK[0])) / den;
    F[1] = (Ss * (SK * UK[1] - FK[1]) + SK * pstar * nx) / den;
    F[2] = (Ss * (SK * UK[2] - FK[2]) + SK * pstar * nz) / den;
    F[3] = (Ss * (SK * UK[3] - FK[3])) / den;
}

/* Viscous flux F_v(U, G) . n = mu rho grad(U_c/rho) . n written with the
   gradient G of the conserved variables: mu (G_c - (U_c/rho) G_rho). */
static void visc_flux(const orc_cfg* c, const double* U, const double* Gx, const double* Gz,
                      double nx, double nz, double* F)
{
    F[0] = 0.0;
    for (int m = 1; m < 4; ++m) {
        double r = U[m] / U[0];
        F[m] = c->mu * ((Gx[m] - r * Gx[0]) * nx + (Gz[m] - r * Gz[0]) * nz);
    }
}

static void mirror(const double* U, int xface, double* M)
{
    M[0] = U[0]; M[1] = U[1]; M[2] = U[2]; M[3] = U[3];
    if (xface) M[1] = -U[1]; else M[2] = -U[2];
}

/* ------------------------------------------------------------------------ */
/* Context                                                                  */
/* ------------------------------------------------------------------------ */

orc_ctx* orc_create(const orc_cfg* cfg)
{
    if (cfg->k < 1 || cfg->k > MAXK || cfg->nx < 1 || cfg->nz < 1) return NULL;
    if (cfg->mg_levels < 1 || cfg->mg_levels > MAXLEV) return NULL;
    if (cfg->rk_stages < 1 || cfg->rk_stages > 4) return NULL;
    orc_ctx* X = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    X->c = *cfg;
    X->n1 = cfg->k + 1;
    X->np = X->n1 * X->n1;
    X->ne = (long)cfg->nx * cfg->nz;
    X->ndof = 4 * X->ne * X->np;
    X->dx = (cfg->x1 - cfg->x0) / cfg->nx;
    X->dz = (cfg->z1 - cfg->z0) / cfg->nz;
    X->J = X->dx * X->dz / 4.0;
    double D[MAXN * MAXN], V[MAXN * MAXN], Vi[MAXN * MAXN];
    orc_ref_tables(cfg->k, X->xi, X->w, D, X->em, X->ep, X->dm, X->dp, V, Vi, X->wnc);
    double Pp[MAXN * MAXN], Pi[MAXN * MAXN];
    orc_proj_tables(cfg->k, Pp, Pi);
    for (int i = 0; i < X->n1; ++i)
        for (int j = 0; j < X->n1; ++j) {
            X->D[i][j] = D[i * X->n1 + j];
            X->V[i][j] = V[i * X->n1 + j];
            X->Vinv[i][j] = Vi[i * X->n1 + j];
            X->P[i][j] = Pp[i * X->n1 + j];
            X->Pinv[i][j] = Pi[i * X->n1 + j];
        }
    /* FV levels: finest = (k+1)nx x (k+1)nz subcells, each coarser level
       agglomerates 2x2 cells (Sec. "Multigrid preconditioner for finite volume") */
    X->nlev = cfg->mg_levels;
    int nxf = X->n1 * cfg->nx, nzf = X->n1 * cfg->nz;
    for (int l = 0; l < X->nlev; ++l) {
        if (l > 0 && ((X->nxl[l - 1] & 1) || (X->nzl[l - 1] & 1))) { free(X); return NULL; }
        X->nxl[l] = l ? X->nxl[l - 1] / 2 : nxf;
        X->nzl[l] = l ? X->nzl[l - 1] / 2 : nzf;
        X->hx[l] = (cfg->x1 - cfg->x0) / X->nxl[l];
        X->hz[l] = (cfg->z1 - cfg->z0) / X->nzl[l];
    }
    X->Ulin = (double*)calloc(X->ndof, sizeof(double));
    X->Llin = (double*)calloc(X->ndof, sizeof(double));
    for (int l = 0; l < X->nlev; ++l) {
        long n = 4L * X->nxl[l] * X->nzl[l];
        X->ulev[l] = (double*)calloc(n, sizeof(double));
        X->flev[l] = (double*)calloc(n, sizeof(double));
    }
    X->mv_count = X->mv_local;
    return X;
}

void orc_destroy(orc_ctx* X)
{
    if (!X) return;
    free(X->Ulin);
    free(X->Llin);
    for (int l = 0; l < X->nlev; ++l) { free(X->ulev[l]); free(X->flev[l]); }
    free(X);
}

long orc_num_dofs(const orc_ctx* X) { return X->ndof; }

int orc_fv_dims(const orc_ctx* X, int level, int* nxl, int* nzl)
{
    if (level < 0 || level >= X->nlev) return ORC_EINVAL;
    *nxl = X->nxl[level];
    *nzl = X->nzl[level];
    return ORC_OK;
}

#define UIDX(X, c, e, node) ((long)(c) * (X)->ne * (X)->np + (long)(e) * (X)->np + (node))

static double node_x(const orc_ctx* X, int ex, int a) { return X->c.x0 + (ex + 0.5 * (1.0 + X->xi[a])) * X->dx; }
static double node_z(const orc_ctx* X, int ez, int b) { return X->c.z0 + (ez + 0.5 * (1.0 + X->xi[b])) * X->dz; }

/* ------------------------------------------------------------------------ */
/* Initial data: potential temperature perturbation inserted at constant     */
/* pressure (eq:add-perturbation), taken at the GL nodes (collocated L2      */
/* projection, Sec. "Temporal discretization").                             */
/* ------------------------------------------------------------------------ */

void orc_initial_state(const orc_ctx* X, const orc_pert* P, double* U)
{
    const orc_cfg* c = &X->c;
    for (int ez = 0; ez < c->nz; ++ez)
        for (int ex = 0; ex < c->nx; ++ex)
            for (int b = 0; b < X->n1; ++b)
                for (int a = 0; a < X->n1; ++a) {
                    double x = node_x(X, ex, a), z = node_z(X, ez, b);
                    double th1 = 0.0;
                    if (P->shape == 0) {
                        double rx = (x - P->xc) / P->xr, rz = (z - P->zc) / P->zr;
                        double r = sqrt(rx * rx + rz * rz);
                        if (r < 1.0) th1 = 0.5 * P->amp * (1.0 + cos(M_PI * r));
                    } else {
                        double s = (x - P->xc) / P->a;
                        th1 = P->amp / (1.0 + s * s) * sin(M_PI * z / P->Z);
                    }
                    double Ub[4];
                    orc_background(X, z, Ub, NULL);
                    double rho = Ub[3] / (bg_theta(c, z) + th1);
                    long e = (long)ez * c->nx + ex;
                    int node = b * X->n1 + a;
                    U[UIDX(X, 0, e, node)] = rho - Ub[0];
                    U[UIDX(X, 1, e, node)] = rho * c->u_mean - Ub[1];
                    U[UIDX(X, 2, e, node)] = 0.0;
                    U[UIDX(X, 3, e, node)] = 0.0;
                }
}

/* ------------------------------------------------------------------------ */
/* DG operator <psi, L_h(U')> (eqs. convDiscr, elementint, surfaceint) in the */
/* well-balanced perturbation form (eq. perturbed-euler).  Collocated GL     */
/* quadrature; HLLC convective flux; symmetric interior penalty diffusion   */
/* flux with eta = c_ip (k+1)^2 / h; slip walls carry no viscous flux.       */
/* ------------------------------------------------------------------------ */

static void dg_residual_mode(orc_ctx* X, const double* U, double* L, int wb, int mag);

static void dg_residual(orc_ctx* X, const double* U, double* L, int wb) { dg_residual_mode(X, U, L, wb, 0); }

/* wb = 1: well-balanced perturbation form; wb = 0: plain form on U' + Ubar.
   mag = 1: rounding scale, i.e. the same sums taken over absolute values of the
   unsubtracted terms (used only to scale parity tolerances). */
static void dg_residual_mode(orc_ctx* X, const double* U, double* L, int wb, int mag)
{
    const orc_cfg* c = &X->c;
    const int n1 = X->n1, np = X->np;
    const int ns = (c->physics == 1);
    const double dx = X->dx, dz = X->dz, J = X->J;
    X->lh_count++;
    /* elements are independent (each writes only its own nodes): spread over the host
       cores, the arithmetic of every element unchanged */
#pragma omp parallel for collapse(2) schedule(static)
    for (int ez = 0; ez < c->nz; ++ez)
        for (int ex = 0; ex < c->nx; ++ex) {
            double Fx[4][MAXN * MAXN], Fz[4][MAXN * MAXN], Ue[4][MAXN * MAXN], Un[4][MAXN * MAXN];
            long e = (long)ez * c->nx + ex;
            for (int cc = 0; cc < 4; ++cc)
                for (int i = 0; i < np; ++i) Ue[cc][i] = U[UIDX(X, cc, e, i)];
            double Le[4][MAXN * MAXN];
            memset(Le, 0, sizeof(Le));
            /* element integral: (F_c - F_v) : grad psi + S . psi */
            for (int b = 0; b < n1; ++b) {
                double z = node_z(X, ez, b), Ub[4], dUb[4];
                orc_background(X, z, Ub, dUb);
                for (int a = 0; a < n1; ++a) {
                    int i = b * n1 + a;
                    double Ut[4], fx[4], fz[4];
                    for (int cc = 0; cc < 4; ++cc) Ut[cc] = Ue[cc][i] + Ub[cc];
                    orc_flux(X, Ut, 1.0, 0.0, fx);
                    orc_flux(X, Ut, 0.0, 1.0, fz);
                    if (mag) for (int cc = 0; cc < 4; ++cc) { fx[cc] = fabs(fx[cc]); fz[cc] = fabs(fz[cc]); }
                    if (wb && !mag) {
                        double bx[4], bz[4];
                        orc_flux(X, Ub, 1.0, 0.0, bx);
                        orc_flux(X, Ub, 0.0, 1.0, bz);
                        for (int cc = 0; cc < 4; ++cc) { fx[cc] -= bx[cc]; fz[cc] -= bz[cc]; }
                    }
                    if (ns) {
                        double Gx[4], Gz[4], vx[4], vz[4];
                        for (int cc = 0; cc < 4; ++cc) {
                            double sx = 0.0, sz = 0.0;
                            for (int j = 0; j < n1; ++j) {
                                sx += X->D[a][j] * Ue[cc][b * n1 + j];
                                sz += X->D[b][j] * Ue[cc][j * n1 + a];
                            }
                            Gx[cc] = (2.0 / dx) * sx;
                            Gz[cc] = (2.0 / dz) * sz + dUb[cc];
                        }
                        visc_flux(c, Ut, Gx, Gz, 1.0, 0.0, vx);
                        visc_flux(c, Ut, Gx, Gz, 0.0, 1.0, vz);
                        if (mag) for (int cc = 0; cc < 4; ++cc) { fx[cc] += fabs(vx[cc]); fz[cc] += fabs(vz[cc]); }
                        else for (int cc = 0; cc < 4; ++cc) { fx[cc] -= vx[cc]; fz[cc] -= vz[cc]; }
                    }
                    for (int cc = 0; cc < 4; ++cc) { Fx[cc][i] = fx[cc]; Fz[cc][i] = fz[cc]; }
                }
            }
            for (int b = 0; b < n1; ++b) {
                double Ub[4];
                orc_background(X, node_z(X, ez, b), Ub, NULL);
                for (int a = 0; a < n1; ++a) {
                    int i = b * n1 + a;
                    for (int cc = 0; cc < 4; ++cc) {
                        double sx = 0.0, sz = 0.0;
                        for (int q = 0; q < n1; ++q) sx += X->w[q] * (mag ? fabs(X->D[q][a]) : X->D[q][a]) * Fx[cc][b * n1 + q];
                        for (int r = 0; r < n1; ++r) sz += X->w[r] * (mag ? fabs(X->D[r][b]) : X->D[r][b]) * Fz[cc][r * n1 + a];
                        Le[cc][i] += J * ((2.0 / dx) * X->w[b] * sx + (2.0 / dz) * X->w[a] * sz);
                    }
                    /* gravity source S = (0, 0, -rho g, 0); perturbation form: -g rho' */
                    double rho_src = (wb && !mag) ? Ue[0][i] : Ue[0][i] + Ub[0];
                    Le[2][i] += X->w[a] * X->w[b] * J * (mag ? fabs(c->g * rho_src) : -c->g * rho_src);
                }
            }
            /* surface integrals over the four faces, own-side test functions */
            for (int f = 0; f < 4; ++f) {
                int xface = (f < 2);
                int side = (f == 0 || f == 2) ? -1 : 1;
                double nx = xface ? side : 0.0, nz = xface ? 0.0 : side;
                const double* es = side > 0 ? X->ep : X->em;    /* own trace row   */
                const double* eo = side > 0 ? X->em : X->ep;    /* neighbour row   */
                const double* ds = side > 0 ? X->dp : X->dm;
                const double* dso = side > 0 ? X->dm : X->dp;
                double hperp = xface ? dx : dz, flen = xface ? dz : dx;
                int wall = 0;
                long en = -1;
                if (xface) {
                    int exn = ex + side;
                    if (exn < 0 || exn >= c->nx) {
                        if (c->bc == 1) exn = (exn + c->nx) % c->nx;
                        else wall = 1;
                    }
                    if (!wall) en = (long)ez * c->nx + exn;
                } else {
                    int ezn = ez + side;
                    if (ezn < 0 || ezn >= c->nz) wall = 1;
                    else en = (long)ezn * c->nx + ex;
                }
                if (!wall)
                    for (int cc = 0; cc < 4; ++cc)
                        for (int i = 0; i < np; ++i) Un[cc][i] = U[UIDX(X, cc, en, i)];
                /* traces at the k+1 face GL points */
                double tro[4][MAXN], trx[4][MAXN];
                for (int cc = 0; cc < 4; ++cc)
                    for (int r = 0; r < n1; ++r) {
                        double so = 0.0, sx = 0.0;
                        for (int j = 0; j < n1; ++j) {
                            int io = xface ? r * n1 + j : j * n1 + r;
                            so += es[j] * Ue[cc][io];
                            if (!wall) sx += eo[j] * Un[cc][io];
                        }
                        tro[cc][r] = so;
                        trx[cc][r] = sx;
                    }
                for (int r = 0; r < n1; ++r) {
                    double zp = xface ? node_z(X, ez, r) : c->z0 + (ez + (side > 0 ? 1 : 0)) * dz;
                    double Ub[4], dUb[4];
                    orc_background(X, zp, Ub, dUb);
                    double Uo[4], Ux[4], H[4], flux[4], sym[4] = {0, 0, 0, 0};
                    for (int cc = 0; cc < 4; ++cc) Uo[cc] = tro[cc][r] + Ub[cc];
                    if (wall) mirror(Uo, xface, Ux);
                    else for (int cc = 0; cc < 4; ++cc) Ux[cc] = trx[cc][r] + Ub[cc];
                    orc_hllc(X, Uo, Ux, nx, nz, H);
                    if (mag) for (int cc = 0; cc < 4; ++cc) H[cc] = -fabs(H[cc]);
                    if (wb && !mag) {
                        double Hb[4], Um[4];
                        if (wall) mirror(Ub, xface, Um);
                        else memcpy(Um, Ub, sizeof(Um));
                        orc_hllc(X, Ub, Um, nx, nz, Hb);
                        for (int cc = 0; cc < 4; ++cc) H[cc] -= Hb[cc];
                    }
                    for (int cc = 0; cc < 4; ++cc) flux[cc] = -H[cc];
                    if (ns && !wall) {
                        double Gxo[4], Gzo[4], Gxx[4], Gzx[4], Fo[4], Fxx[4];
                        for (int cc = 0; cc < 4; ++cc) {
                            double sn_o = 0.0, sn_x = 0.0, st_o = 0.0, st_x = 0.0;
                            for (int j = 0; j < n1; ++j) {
                                int io = xface ? r * n1 + j : j * n1 + r;
                                sn_o += ds[j] * Ue[cc][io];
                                sn_x += dso[j] * Un[cc][io];
                                st_o += X->D[r][j] * tro[cc][j];
                                st_x += X->D[r][j] * trx[cc][j];
                            }
                            if (xface) {
                                Gxo[cc] = (2.0 / dx) * sn_o;
                                Gxx[cc] = (2.0 / dx) * sn_x;
                                Gzo[cc] = (2.0 / dz) * st_o + dUb[cc];
                                Gzx[cc] = (2.0 / dz) * st_x + dUb[cc];
                            } else {
                                Gzo[cc] = (2.0 / dz) * sn_o + dUb[cc];
                                Gzx[cc] = (2.0 / dz) * sn_x + dUb[cc];
                                Gxo[cc] = (2.0 / dx) * st_o;
                                Gxx[cc] = (2.0 / dx) * st_x;
                            }
                        }
                        visc_flux(c, Uo, Gxo, Gzo, nx, nz, Fo);
                        visc_flux(c, Ux, Gxx, Gzx, nx, nz, Fxx);
                        double eta = c->c_ip * n1 * n1 / hperp;
                        double Dl[4], Um[4];
                        for (int cc = 0; cc < 4; ++cc) {
                            Dl[cc] = tro[cc][r] - trx[cc][r];
                            Um[cc] = 0.5 * (Uo[cc] + Ux[cc]);
                        }
                        for (int cc = 1; cc < 4; ++cc) {
                            double pen = eta * c->mu * (Dl[cc] - (Um[cc] / Um[0]) * Dl[0]);
                            if (mag) {
                                flux[cc] += 0.5 * (fabs(Fo[cc]) + fabs(Fxx[cc])) + fabs(pen);
                                sym[cc] = fabs(0.5 * c->mu * (Dl[cc] - (Uo[cc] / Uo[0]) * Dl[0]));
                            } else {
                                flux[cc] += 0.5 * (Fo[cc] + Fxx[cc]) - pen;
                                sym[cc] = 0.5 * c->mu * (Dl[cc] - (Uo[cc] / Uo[0]) * Dl[0]);
                            }
                        }
                    }
                    double W = X->w[r] * flen / 2.0;
                    for (int j = 0; j < n1; ++j) {
                        int io = xface ? r * n1 + j : j * n1 + r;
                        double dn = side * (2.0 / hperp) * ds[j];
                        if (mag)
                            for (int cc = 0; cc < 4; ++cc) Le[cc][io] += W * (flux[cc] * fabs(es[j]) + sym[cc] * fabs(dn));
                        else
                            for (int cc = 0; cc < 4; ++cc) Le[cc][io] += W * (flux[cc] * es[j] + sym[cc] * dn);
                    }
                }
            }
            for (int cc = 0; cc < 4; ++cc)
                for (int i = 0; i < np; ++i) L[UIDX(X, cc, e, i)] = Le[cc][i];
        }
}

/* M^-1 with the diagonal GL mass m_ab = w_a w_b |J| (Sec. "Temporal discretization") */
static void apply_minv(const orc_ctx* X, double* v)
{
    for (int cc = 0; cc < 4; ++cc)
        for (long e = 0; e < X->ne; ++e)
            for (int b = 0; b < X->n1; ++b)
                for (int a = 0; a < X->n1; ++a)
                    v[UIDX(X, cc, e, b * X->n1 + a)] /= X->w[a] * X->w[b] * X->J;
}

void orc_residual(orc_ctx* X, const double* U, double* out, int mode)
{
    if (mode == 3) dg_residual_mode(X, U, out, 0, 1);
    else dg_residual(X, U, out, mode == 2 ? 0 : 1);
    if (mode == 1) apply_minv(X, out);
}

/* G(U) = U - alpha dt f(U) - Ubar (eq. newton) */
void orc_stage_residual(orc_ctx* X, const double* U, const double* Ubar, double alpha_dt, double* G)
{
    orc_residual(X, U, G, 1);
    for (long i = 0; i < X->ndof; ++i) G[i] = U[i] - alpha_dt * G[i] - Ubar[i];
}

static double norm2(long n, const double* v)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

static double dot(long n, const double* a, const double* b)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Transfers between V_h^k and the FV subgrid V_h^0 (Sec. "Transfer          */
/* functions", eq. transfer-mass-fix, appendix quadrature).                   */
/*   T:       t_ij = sum_ab V_ia V_jb u_ab (interpolation at subcell centres)   */
/*   mass fix: t -= (mean(t) - sum_ij w_i w_j t_ij)                             */
/*   T^-1:    u = (V^-1 x V^-1) t  - (sum w_i w_j t_ij - mean(t))  (inverse)    */
/* ------------------------------------------------------------------------ */

void orc_subgrid_map(const orc_ctx* X, int* fv_to_dg)
{
    int n1 = X->n1, nxf = X->nxl[0];
    for (int ez = 0; ez < X->c.nz; ++ez)
        for (int ex = 0; ex < X->c.nx; ++ex)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int I = ex * n1 + i, Jc = ez * n1 + j;
                    fv_to_dg[(long)Jc * nxf + I] = (int)(((long)ez * X->c.nx + ex) * X->np + j * n1 + i);
                }
}

void orc_transfer_T(const orc_ctx* X, const double* U, double* u)
{
    int n1 = X->n1, np = X->np, nxf = X->nxl[0], nzf = X->nzl[0];
    long nc = (long)nxf * nzf;
    for (int ez = 0; ez < X->c.nz; ++ez)
        for (int ex = 0; ex < X->c.nx; ++ex) {
            long e = (long)ez * X->c.nx + ex;
            for (int cc = 0; cc < 4; ++cc) {
                double t[MAXN][MAXN];
                double mean = 0.0, quad = 0.0;
                const int proj = X->c.transfer == 1;   /* subcell averages instead of centre values */
                for (int j = 0; j < n1; ++j)
                    for (int i = 0; i < n1; ++i) {
                        double s = 0.0;
                        for (int b = 0; b < n1; ++b)
                            for (int a = 0; a < n1; ++a)
                                s += (proj ? X->P[i][a] * X->P[j][b] : X->V[i][a] * X->V[j][b]) *
                                     U[UIDX(X, cc, e, b * n1 + a)];
                        t[j][i] = s;
                        mean += s;
                        quad += X->wnc[i] * X->wnc[j] * s;
                    }
                mean /= np;
                double shift = (X->c.mass_fix && !proj) ? (mean - quad) : 0.0;
                for (int j = 0; j < n1; ++j)
                    for (int i = 0; i < n1; ++i)
                        u[cc * nc + (long)(ez * n1 + j) * nxf + ex * n1 + i] = t[j][i] - shift;
            }
        }
}

void orc_transfer_Tinv(const orc_ctx* X, const double* u, double* U)
{
    int n1 = X->n1, np = X->np, nxf = X->nxl[0], nzf = X->nzl[0];
    long nc = (long)nxf * nzf;
    for (int ez = 0; ez < X->c.nz; ++ez)
        for (int ex = 0; ex < X->c.nx; ++ex) {
            long e = (long)ez * X->c.nx + ex;
            for (int cc = 0; cc < 4; ++cc) {
                double t[MAXN][MAXN];
                double mean = 0.0, quad = 0.0;
                for (int j = 0; j < n1; ++j)
                    for (int i = 0; i < n1; ++i) {
                        t[j][i] = u[cc * nc + (long)(ez * n1 + j) * nxf + ex * n1 + i];
                        mean += t[j][i];
                        quad += X->wnc[i] * X->wnc[j] * t[j][i];
                    }
                mean /= np;
                const int proj = X->c.transfer == 1;
                double shift = (X->c.mass_fix && !proj) ? (quad - mean) : 0.0;
                for (int b = 0; b < n1; ++b)
                    for (int a = 0; a < n1; ++a) {
                        double s = 0.0;
                        for (int j = 0; j < n1; ++j)
                            for (int i = 0; i < n1; ++i)
                                s += (proj ? X->Pinv[a][i] * X->Pinv[b][j] : X->Vinv[a][i] * X->Vinv[b][j]) * t[j][i];
                        U[UIDX(X, cc, e, b * n1 + a)] = s - shift;
                    }
            }
        }
}

/* Agglomeration restriction (average of the 4 children, summed pairwise
   ((c00 + c10) + (c01 + c11)) / 4) and injection prolongation. */
void orc_restrict(const orc_ctx* X, int fl, const double* uf, double* uc)
{
    int nxf = X->nxl[fl], nzf = X->nzl[fl], nxc = X->nxl[fl + 1], nzc = X->nzl[fl + 1];
    for (int cc = 0; cc < 4; ++cc)
        for (int J = 0; J < nzc; ++J)
            for (int I = 0; I < nxc; ++I) {
                const double* f = uf + (long)cc * nxf * nzf;
                double c00 = f[(long)(2 * J) * nxf + 2 * I], c10 = f[(long)(2 * J) * nxf + 2 * I + 1];
                double c01 = f[(long)(2 * J + 1) * nxf + 2 * I], c11 = f[(long)(2 * J + 1) * nxf + 2 * I + 1];
                uc[(long)cc * nxc * nzc + (long)J * nxc + I] = ((c00 + c10) + (c01 + c11)) * 0.25;
            }
}

void orc_prolong(const orc_ctx* X, int cl, const double* uc, double* uf)
{
    int nxc = X->nxl[cl], nzc = X->nzl[cl], nxf = X->nxl[cl - 1], nzf = X->nzl[cl - 1];
    for (int cc = 0; cc < 4; ++cc)
        for (int J = 0; J < nzf; ++J)
            for (int I = 0; I < nxf; ++I)
                uf[(long)cc * nxf * nzf + (long)J * nxf + I] = uc[(long)cc * nxc * nzc + (long)(J / 2) * nxc + I / 2];
}

/* ------------------------------------------------------------------------ */
/* FV operator f_low on level l: the DG method with k = 0 on the subgrid     */
/* (Sec. "Low order approximation preconditioner").  With piecewise         */
/* constants the element integral has no flux part; the face total states  */
/* are cell value + Ubar(face point); the diffusion flux is the k = 0 form  */
/* of the interior-penalty flux with penalty 1/h (two-point flux).           */
/* ------------------------------------------------------------------------ */

void orc_fv_residual(const orc_ctx* X, int l, const double* u, double* f)
{
    const orc_cfg* c = &X->c;
    int nxl = X->nxl[l], nzl = X->nzl[l];
    long nc = (long)nxl * nzl;
    double hx = X->hx[l], hz = X->hz[l], area = hx * hz;
    /* cells are independent (each writes only its own values) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int J = 0; J < nzl; ++J)
        for (int I = 0; I < nxl; ++I) {
            long q = (long)J * nxl + I;
            double L[4] = {0, 0, 0, 0};
            for (int f4 = 0; f4 < 4; ++f4) {
                int xface = (f4 < 2);
                int side = (f4 == 0 || f4 == 2) ? -1 : 1;
                double nx = xface ? side : 0.0, nz = xface ? 0.0 : side;
                double elen = xface ? hz : hx, hn = xface ? hx : hz;
                double zf = xface ? c->z0 + (J + 0.5) * hz : c->z0 + (J + (side > 0 ? 1 : 0)) * hz;
                int wall = 0;
                long qn = -1;
                if (xface) {
                    int In = I + side;
                    if (In < 0 || In >= nxl) {
                        if (c->bc == 1) In = (In + nxl) % nxl;
                        else wall = 1;
                    }
                    if (!wall) qn = (long)J * nxl + In;
                } else {
                    int Jn = J + side;
                    if (Jn < 0 || Jn >= nzl) wall = 1;
                    else qn = (long)Jn * nxl + I;
                }
                double Ub[4], dUb[4], Uq[4], Un[4], H[4], Hb[4], Um[4];
                orc_background(X, zf, Ub, dUb);
                for (int cc = 0; cc < 4; ++cc) Uq[cc] = u[cc * nc + q] + Ub[cc];
                if (wall) { mirror(Uq, xface, Un); mirror(Ub, xface, Um); }
                else {
                    for (int cc = 0; cc < 4; ++cc) Un[cc] = u[cc * nc + qn] + Ub[cc];
                    memcpy(Um, Ub, sizeof(Um));
                }
                orc_hllc(X, Uq, Un, nx, nz, H);
                orc_hllc(X, Ub, Um, nx, nz, Hb);
                for (int cc = 0; cc < 4; ++cc) L[cc] -= elen * (H[cc] - Hb[cc]);
                if (c->physics == 1 && !wall) {
                    double G0[4] = {0, 0, 0, 0}, Fq[4], Fn[4], Av[4];
                    visc_flux(c, Uq, G0, dUb, nx, nz, Fq);
                    visc_flux(c, Un, G0, dUb, nx, nz, Fn);
                    double Dl[4];
                    for (int cc = 0; cc < 4; ++cc) {
                        Dl[cc] = u[cc * nc + q] - u[cc * nc + qn];
                        Av[cc] = 0.5 * (Uq[cc] + Un[cc]);
                    }
                    for (int cc = 1; cc < 4; ++cc) {
                        double pen = (1.0 / hn) * c->mu * (Dl[cc] - (Av[cc] / Av[0]) * Dl[0]);
                        L[cc] += elen * (0.5 * (Fq[cc] + Fn[cc]) - pen);
                    }
                }
            }
            L[2] += area * (-c->g * u[0 * nc + q]);
            for (int cc = 0; cc < 4; ++cc) f[cc * nc + q] = L[cc] / area;
        }
}

/* ------------------------------------------------------------------------ */
/* Linearization at a Newton iterate: u_L = T^mf U, u_{l-1} = R u_l, and per  */
/* level the pseudo time step Delta tau_l from a pseudo CFL condition        */
/* (Sec. "Smoother / Pseudo time iteration").                               */
/* ------------------------------------------------------------------------ */

static void fv_level_stats(orc_ctx* X, int l)
{
    const orc_cfg* c = &X->c;
    int nxl = X->nxl[l], nzl = X->nzl[l];
    long nc = (long)nxl * nzl;
    double s = 0.0, lam = 0.0;
    for (int J = 0; J < nzl; ++J) {
        double Ub[4];
        orc_background(X, c->z0 + (J + 0.5) * X->hz[l], Ub, NULL);
        for (int I = 0; I < nxl; ++I) {
            long q = (long)J * nxl + I;
            double Ut[4];
            for (int cc = 0; cc < 4; ++cc) {
                Ut[cc] = X->ulev[l][cc * nc + q] + Ub[cc];
                s += Ut[cc] * Ut[cc];
            }
            double u = Ut[1] / Ut[0], w = Ut[2] / Ut[0];
            double p = pressure(c, Ut[3]);
            double a = sqrt(u * u + w * w) + sqrt(c->gamma * p / Ut[0]);
            if (a > lam) lam = a;
        }
    }
    X->utot[l] = sqrt(s);
    X->lam[l] = lam;
    double hx = X->hx[l], hz = X->hz[l];
    X->dtau[l] = c->pseudo_cfl /
                 (1.0 + X->adt * (lam * (1.0 / hx + 1.0 / hz) + 2.0 * c->mu * (1.0 / (hx * hx) + 1.0 / (hz * hz))));
}

int orc_linearize(orc_ctx* X, const double* U, double alpha_dt)
{
    X->adt = alpha_dt;
    memcpy(X->Ulin, U, sizeof(double) * X->ndof);
    dg_residual(X, U, X->Llin, 1);
    double s = 0.0;
    for (int ez = 0; ez < X->c.nz; ++ez)
        for (int b = 0; b < X->n1; ++b) {
            double Ub[4];
            orc_background(X, node_z(X, ez, b), Ub, NULL);
            for (int ex = 0; ex < X->c.nx; ++ex)
                for (int a = 0; a < X->n1; ++a) {
                    long e = (long)ez * X->c.nx + ex;
                    for (int cc = 0; cc < 4; ++cc) {
                        double v = U[UIDX(X, cc, e, b * X->n1 + a)] + Ub[cc];
                        s += v * v;
                    }
                }
        }
    X->utot_dg = sqrt(s);
    orc_transfer_T(X, U, X->ulev[0]);
    for (int l = 1; l < X->nlev; ++l) orc_restrict(X, l - 1, X->ulev[l - 1], X->ulev[l]);
    for (int l = 0; l < X->nlev; ++l) {
        orc_fv_residual(X, l, X->ulev[l], X->flev[l]);
        fv_level_stats(X, l);
    }
    /* DG-level pseudo time step: the level formula with the element widths divided
       by 2k+1 (the explicit DG step scale) and the wave speed of the finest FV level */
    {
        const orc_cfg* c = &X->c;
        double hx = (c->x1 - c->x0) / c->nx / (2.0 * c->k + 1.0);
        double hz = (c->z1 - c->z0) / c->nz / (2.0 * c->k + 1.0);
        X->dtau_dg = c->pseudo_cfl_dg /
                     (1.0 + X->adt * (X->lam[0] * (1.0 / hx + 1.0 / hz) +
                                      2.0 * c->mu * (1.0 / (hx * hx) + 1.0 / (hz * hz))));
    }
    X->have_lin = 1;
    if (!isfinite(X->utot_dg)) return ORC_ENONFINITE;
    return ORC_OK;
}

void orc_fv_level_state(const orc_ctx* X, int l, double* u)
{
    memcpy(u, X->ulev[l], sizeof(double) * 4 * X->nxl[l] * X->nzl[l]);
}

double orc_fv_dtau(const orc_ctx* X, int l) { return X->dtau[l]; }

double orc_dg_dtau(const orc_ctx* X) { return X->dtau_dg; }

/* Operation counts since the context was created or last reset (instrumentation
   for the tests, no arithmetic): FV matvecs per level, DG JVPs, L_h calls. */
void orc_counters(orc_ctx* X, int* fv_matvecs, int* jvps, int* lh_evals, int reset)
{
    for (int l = 0; l < MAXLEV; ++l) {
        if (fv_matvecs) fv_matvecs[l] = X->mv_local[l];
        if (reset) X->mv_local[l] = 0;
    }
    if (jvps) *jvps = X->jvp_count;
    if (lh_evals) *lh_evals = X->lh_count;
    if (reset) { X->jvp_count = 0; X->lh_count = 0; }
}

/* FV Jacobian-free matvec g'_l(u) x = x - (alpha dt / eps)(f_low(u + eps x) - f_low(u)),
   eps = sqrt(eps_mach) ||u + Ubar||_2 / ||x||_2; x = 0 gives 0. */
void orc_fv_matvec(orc_ctx* X, int l, const double* x, double* out)
{
    long n = 4L * X->nxl[l] * X->nzl[l];
    double xn = norm2(n, x);
    X->mv_count[l]++;
    if (xn == 0.0) { memset(out, 0, sizeof(double) * n); return; }
    double eps = sqrt(DBL_EPSILON) * X->utot[l] / xn;
    double* up = (double*)malloc(sizeof(double) * n);
    double* fp = (double*)malloc(sizeof(double) * n);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) up[i] = X->ulev[l][i] + eps * x[i];
    orc_fv_residual(X, l, up, fp);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = x[i] - (X->adt / eps) * (fp[i] - X->flev[l][i]);
    free(up);
    free(fp);
}

/* DG Jacobian-free product G'(U) y = y - (alpha dt / eps) M^-1 (L_h(U + eps y) - L_h(U))
   (Sec. "Solver"); the identity part of G is differenced exactly.
   eps = sqrt(eps_mach)/||y|| (paper) or sqrt(eps_mach) ||U + Ubar|| / ||y||. */
void orc_jvp(orc_ctx* X, const double* y, double* out)
{
    long n = X->ndof;
    double yn = norm2(n, y);
    X->jvp_count++;
    if (yn == 0.0) { memset(out, 0, sizeof(double) * n); return; }
    double eps = X->c.fd_eps_mode == 0 ? sqrt(DBL_EPSILON) / yn : sqrt(DBL_EPSILON) * X->utot_dg / yn;
    double* Up = (double*)malloc(sizeof(double) * n);
    double* Lp = (double*)malloc(sizeof(double) * n);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) Up[i] = X->Ulin[i] + eps * y[i];
    dg_residual(X, Up, Lp, 1);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) Lp[i] -= X->Llin[i];
    apply_minv(X, Lp);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = y[i] - (X->adt / eps) * Lp[i];
    free(Up);
    free(Lp);
}

/* ------------------------------------------------------------------------ */
/* Multigrid MG_l(x, b; u) (Sec. "Multigrid preconditioner for finite volume */
/* approximations"): pre-smooth, defect, restrict, coarse call(s) with the   */
/* restricted linearization, x := x - P v, post-smooth.  The smoother is the */
/* explicit RK pseudo-time iteration x_j = x_0 + alpha_j dtau (b - g' x_{j-1}) */
/* (low-storage form); a flag skips the matvec with the zero vector.         */
/* Levels here run 0 (finest) .. nlev-1 (coarsest).                          */
/* ------------------------------------------------------------------------ */

static void smooth(orc_ctx* X, int l, double* x, const double* b, int nu, int* xzero)
{
    long n = 4L * X->nxl[l] * X->nzl[l];
    double* x0 = (double*)malloc(sizeof(double) * n);
    double* xp = (double*)malloc(sizeof(double) * n);
    double* Ax = (double*)malloc(sizeof(double) * n);
    for (int sweep = 0; sweep < nu; ++sweep) {
        memcpy(x0, x, sizeof(double) * n);
        memcpy(xp, x, sizeof(double) * n);
        for (int j = 0; j < X->c.rk_stages; ++j) {
            if (j == 0 && *xzero) memset(Ax, 0, sizeof(double) * n);
            else orc_fv_matvec(X, l, xp, Ax);
            double s = X->c.rk_alpha[j] * X->dtau[l];
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) xp[i] = x0[i] + s * (b[i] - Ax[i]);
        }
        memcpy(x, xp, sizeof(double) * n);
        *xzero = 0;
    }
    free(x0);
    free(xp);
    free(Ax);
}

static void mg_cycle(orc_ctx* X, int l, double* x, const double* b, int* xzero)
{
    const orc_cfg* c = &X->c;
    int fine = (l == 0);
    int nu_pre = fine ? c->nu_pre_fine : c->nu_pre;
    int nu_post = fine ? c->nu_post_fine : c->nu_post;
    smooth(X, l, x, b, nu_pre, xzero);
    if (l < X->nlev - 1) {
        long n = 4L * X->nxl[l] * X->nzl[l];
        long nc = 4L * X->nxl[l + 1] * X->nzl[l + 1];
        double* d = (double*)malloc(sizeof(double) * n);
        double* r = (double*)malloc(sizeof(double) * nc);
        double* v = (double*)calloc(nc, sizeof(double));
        double* pv = (double*)malloc(sizeof(double) * n);
        if (*xzero) memset(d, 0, sizeof(double) * n);
        else orc_fv_matvec(X, l, x, d);
        for (long i = 0; i < n; ++i) d[i] -= b[i];
        orc_restrict(X, l, d, r);
        int vzero = 1;
        for (int cyc = 0; cyc < c->cycle; ++cyc) mg_cycle(X, l + 1, v, r, &vzero);
        orc_prolong(X, l + 1, v, pv);
        for (long i = 0; i < n; ++i) x[i] -= pv[i];
        *xzero = 0;
        free(d);
        free(r);
        free(v);
        free(pv);
    }
    smooth(X, l, x, b, nu_post, xzero);
}

void orc_mg_fv(orc_ctx* X, const double* b, double* x)
{
    long n = 4L * X->nxl[0] * X->nzl[0];
    memset(x, 0, sizeof(double) * n);
    int xzero = 1;
    mg_cycle(X, 0, x, b, &xzero);
}

/* T^-1 q^-1 T r (eq. preconditioner), q^-1 = one MG cycle from x = 0 */
static void coarse_correction(orc_ctx* X, const double* r, double* z)
{
    long n = 4L * X->nxl[0] * X->nzl[0];
    double* b = (double*)malloc(sizeof(double) * n);
    double* x = (double*)malloc(sizeof(double) * n);
    orc_transfer_T(X, r, b);
    orc_mg_fv(X, b, x);
    orc_transfer_Tinv(X, x, z);
    free(b);
    free(x);
}

/* Pseudo-time smoothing on the DG data (Sec. "Smoother / Pseudo time iteration":
   the FV smoother's iteration applied to G'(U) z = r before the transfer to the
   FV grid or after the reconstruction): nu sweeps of
   z_j = z_0 + alpha_j dtau_dg (r - G' z_{j-1}), the zero flag skipping G' 0. */
static void smooth_dg(orc_ctx* X, double* z, const double* r, int nu, int* zzero)
{
    long n = X->ndof;
    double* z0 = (double*)malloc(sizeof(double) * n);
    double* zp = (double*)malloc(sizeof(double) * n);
    double* Az = (double*)malloc(sizeof(double) * n);
    for (int sweep = 0; sweep < nu; ++sweep) {
        memcpy(z0, z, sizeof(double) * n);
        memcpy(zp, z, sizeof(double) * n);
        for (int j = 0; j < X->c.rk_stages; ++j) {
            if (j == 0 && *zzero) memset(Az, 0, sizeof(double) * n);
            else orc_jvp(X, zp, Az);
            double s = X->c.rk_alpha[j] * X->dtau_dg;
            for (long i = 0; i < n; ++i) zp[i] = z0[i] + s * (r[i] - Az[i]);
        }
        memcpy(z, zp, sizeof(double) * n);
        *zzero = 0;
    }
    free(z0);
    free(zp);
    free(Az);
}

/* Q^-1 r: with the DG smoothing counts a = b = 0 of the key, T^-1 q^-1 T r
   (eq. preconditioner); otherwise the DG data are the finest level of the cycle:
   a DG sweeps from z = 0, the coarse correction z += T^-1 q^-1 T (r - G' z),
   b DG sweeps. */
void orc_mg_apply(orc_ctx* X, const double* r, double* z)
{
    if (!X->c.precond) { memcpy(z, r, sizeof(double) * X->ndof); return; }
    int a = X->c.nu_pre_dg, b = X->c.nu_post_dg;
    if (a == 0 && b == 0) { coarse_correction(X, r, z); return; }
    long n = X->ndof;
    double* d = (double*)malloc(sizeof(double) * n);
    double* cc = (double*)malloc(sizeof(double) * n);
    memset(z, 0, sizeof(double) * n);
    int zzero = 1;
    smooth_dg(X, z, r, a, &zzero);
    if (zzero) {
        coarse_correction(X, r, z);
    } else {
        orc_jvp(X, z, d);
        for (long i = 0; i < n; ++i) d[i] = r[i] - d[i];
        coarse_correction(X, d, cc);
        for (long i = 0; i < n; ++i) z[i] += cc[i];
    }
    zzero = 0;
    smooth_dg(X, z, r, b, &zzero);
    free(d);
    free(cc);
}

/* ------------------------------------------------------------------------ */
/* Right-preconditioned flexible GMRES(m) with modified Gram-Schmidt and     */
/* Givens rotations; x0 = 0; stops when the residual estimate |g_{j+1}| is   */
/* at most tol_abs; restarts from the true residual rhs - A x.               */
/* ------------------------------------------------------------------------ */

int orc_fgmres(long n, orc_op A, void* actx, orc_op P, void* pctx, const double* rhs,
               double tol_abs, int m, int max_restarts, double* x, int* its)
{
    double* V = (double*)malloc(sizeof(double) * n * (m + 1));
    double* Z = (double*)malloc(sizeof(double) * n * m);
    double* w = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* g = (double*)malloc(sizeof(double) * (m + 1));
    double* y = (double*)malloc(sizeof(double) * m);
    int status = ORC_ENOCONV;
    *its = 0;
    memset(x, 0, sizeof(double) * n);
    memcpy(r, rhs, sizeof(double) * n);
    double beta = norm2(n, r);
    if (!isfinite(beta)) { status = ORC_ENONFINITE; goto done; }
    if (beta <= tol_abs) { status = ORC_OK; goto done; }
    for (int cycle = 0; cycle <= max_restarts; ++cycle) {
        for (long i = 0; i < n; ++i) V[i] = r[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int jend = 0, conv = 0;
        for (int j = 0; j < m; ++j) {
            P(pctx, V + (long)j * n, Z + (long)j * n);
            A(actx, Z + (long)j * n, w);
            for (int i = 0; i <= j; ++i) {
                double h = dot(n, w, V + (long)i * n);
                H[i * m + j] = h;
                #pragma omp parallel for schedule(static)
                for (long t = 0; t < n; ++t) w[t] -= h * V[(long)i * n + t];
            }
            double hn = norm2(n, w);
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0)
                #pragma omp parallel for schedule(static)
                for (long t = 0; t < n; ++t) V[(long)(j + 1) * n + t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double rr = sqrt(a * a + b * b);
            cs[j] = a / rr;
            sn[j] = b / rr;
            H[j * m + j] = rr;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            (*its)++;
            jend = j + 1;
            if (!isfinite(g[j + 1])) { status = ORC_ENONFINITE; goto done; }
            if (fabs(g[j + 1]) <= tol_abs || hn == 0.0) { conv = 1; break; }
        }
        for (int i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < jend; ++t) s -= H[i * m + t] * y[t];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < jend; ++i)
            #pragma omp parallel for schedule(static)
            for (long t = 0; t < n; ++t) x[t] += y[i] * Z[(long)i * n + t];
        if (conv) { status = ORC_OK; break; }
        A(actx, x, w);
        for (long t = 0; t < n; ++t) r[t] = rhs[t] - w[t];
        beta = norm2(n, r);
        if (!isfinite(beta)) { status = ORC_ENONFINITE; break; }
        if (beta <= tol_abs) { status = ORC_OK; break; }
    }
done:
    free(V); free(Z); free(w); free(r); free(H); free(cs); free(sn); free(g); free(y);
    return status;
}

static void op_jvp(void* ctx, const double* in, double* out) { orc_jvp((orc_ctx*)ctx, in, out); }
static void op_prec(void* ctx, const double* in, double* out) { orc_mg_apply((orc_ctx*)ctx, in, out); }

/* ------------------------------------------------------------------------ */
/* Inexact Newton for one stage G(U_s) = 0 (eqs. newton, krylov) from        */
/* U^0 = Ubar_s, stopping when ||G(U^k)|| < TOL ||G(U^0)||; linear tolerance */
/* by Eisenstat-Walker choice 2 (gamma = 0.1, alpha = 1), eta_0 = 0.1,        */
/* eta_max = 0.9; ||G(U^0)|| = 0 is converged with no iteration.             */
/* ------------------------------------------------------------------------ */

int orc_newton_stage(orc_ctx* X, const double* Ubar, double alpha_dt, double* U, orc_stats* st)
{
    long n = X->ndof;
    const orc_cfg* c = &X->c;
    double* G = (double*)malloc(sizeof(double) * n);
    double* rhs = (double*)malloc(sizeof(double) * n);
    double* d = (double*)malloc(sizeof(double) * n);
    int status = ORC_ENOCONV;
    memcpy(U, Ubar, sizeof(double) * n);
    orc_stage_residual(X, U, Ubar, alpha_dt, G);
    double g0 = norm2(n, G), gk = g0, gprev = g0, eta = c->ew_eta0;
    if (st) st->g0_norm = g0;
    if (!isfinite(g0)) { status = ORC_ENONFINITE; goto done; }
    if (g0 == 0.0) { status = ORC_OK; goto done; }
    for (int it = 0; it < c->newton_maxit; ++it) {
        if (it > 0) {
            double eta_new = c->ew_gamma * pow(gk / gprev, c->ew_alpha);
            double safe = c->ew_gamma * pow(eta, c->ew_alpha);
            if (safe > 0.1 && safe > eta_new) eta_new = safe;
            eta = fmin(eta_new, c->ew_eta_max);
        }
        int rc = orc_linearize(X, U, alpha_dt);
        if (rc) { status = rc; goto done; }
        for (long i = 0; i < n; ++i) rhs[i] = -G[i];
        int its = 0;
        rc = orc_fgmres(n, op_jvp, X, op_prec, X, rhs, eta * gk, c->gmres_m, c->gmres_max_restarts, d, &its);
        if (st) { st->gmres_its += its; st->newton_its++; }
        if (rc) { status = rc; goto done; }
        for (long i = 0; i < n; ++i) U[i] += d[i];
        orc_stage_residual(X, U, Ubar, alpha_dt, G);
        gprev = gk;
        gk = norm2(n, G);
        if (st) st->g_norm = gk;
        if (!isfinite(gk)) { status = ORC_ENONFINITE; goto done; }
        if (gk < c->newton_rtol * g0) { status = ORC_OK; goto done; }
        /* rounding floor: the step no longer halves ||G|| although ||G|| is
           already below newton_stall ||G^0|| (G = U - adt f(U) - Ubar cannot be
           evaluated more accurately than its rounding; the relative tolerance
           may lie below that floor for weak perturbations on fine grids) */
        if (c->newton_stall > 0.0 && gk <= c->newton_stall * g0 && gk > 0.5 * gprev) {
            if (st) st->stalls++;
            status = ORC_OK;
            goto done;
        }
    }
done:
    free(G);
    free(rhs);
    free(d);
    return status;
}

/* Explicit reference time stepping (the paper's reference runs use a 4-stage,
   third-order SSP Runge-Kutta method, cited to Ketcheson 2008): for
   dU/dt = f(U) = M^-1 L_h(U), with SSP coefficient 2,
       U1 = U + dt/2 f(U)
       U2 = U1 + dt/2 f(U1)
       U3 = 2/3 U + 1/3 U2 + dt/6 f(U2)
       U_new = U3 + dt/2 f(U3).
   nsteps steps of size dt, U updated in place. */
void orc_explicit_steps(orc_ctx* X, double* U, double dt, int nsteps)
{
    long n = X->ndof;
    double* U1 = (double*)malloc(sizeof(double) * n);
    double* f = (double*)malloc(sizeof(double) * n);
    for (int it = 0; it < nsteps; ++it) {
        orc_residual(X, U, f, 1);
        for (long i = 0; i < n; ++i) U1[i] = U[i] + 0.5 * dt * f[i];
        orc_residual(X, U1, f, 1);
        for (long i = 0; i < n; ++i) U1[i] = U1[i] + 0.5 * dt * f[i];
        orc_residual(X, U1, f, 1);
        for (long i = 0; i < n; ++i) U1[i] = (2.0 / 3.0) * U[i] + (1.0 / 3.0) * U1[i] + (dt / 6.0) * f[i];
        orc_residual(X, U1, f, 1);
        for (long i = 0; i < n; ++i) U[i] = U1[i] + 0.5 * dt * f[i];
    }
    free(U1);
    free(f);
}

/* One implicit step (Sec. "Temporal discretization"): implicit Euler, or
   SDIRK2 of Ellsiepen, alpha = 1 - sqrt(2)/2, tableau [[a,0],[1-a,a]]:
   U_1 solves G with Ubar_1 = U^n; Ubar_2 = U^n + (1-a) dt f(U_1); U^{n+1} = U_2.
   On failure U is left unchanged. */
int orc_implicit_step(orc_ctx* X, double* U, orc_stats* st)
{
    long n = X->ndof;
    const orc_cfg* c = &X->c;
    orc_stats local;
    memset(&local, 0, sizeof(local));
    memset(X->mv_local, 0, sizeof(X->mv_local));
    X->lh_count = 0;
    X->jvp_count = 0;
    double* U1 = (double*)malloc(sizeof(double) * n);
    double* Ub = (double*)malloc(sizeof(double) * n);
    int rc;
    if (c->scheme == 0) {
        rc = orc_newton_stage(X, U, c->dt, U1, &local);
    } else {
        double a = 1.0 - sqrt(2.0) / 2.0;
        rc = orc_newton_stage(X, U, a * c->dt, U1, &local);
        if (rc == ORC_OK) {
            orc_residual(X, U1, Ub, 1);
            for (long i = 0; i < n; ++i) Ub[i] = U[i] + (1.0 - a) * c->dt * Ub[i];
            rc = orc_newton_stage(X, Ub, a * c->dt, U1, &local);
        }
    }
    if (rc == ORC_OK) memcpy(U, U1, sizeof(double) * n);
    local.status = rc;
    local.lh_evals = X->lh_count;
    local.jvps = X->jvp_count;
    for (int l = 0; l < MAXLEV; ++l) local.fv_matvecs[l] = X->mv_local[l];
    if (st) *st = local;
    free(U1);
    free(Ub);
    return rc;
}
