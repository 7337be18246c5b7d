// DG space operator of the well-balanced perturbation system (paper eqs.
// convDiscr, elementint, surfaceint and perturbed-euler) on gfx950.
//
// One work-group holds EPB whole elements, one thread per GL node (k = 3: 8
// elements x 16 nodes = 128 threads).  Element values are staged in LDS; each
// thread then
//   B  evaluates the volume flux at its node (total state U' + Ubar minus the
//      background flux, minus the viscous flux) into LDS,
//   C  loads the neighbour element's trace and normal derivative at one face
//      point from global memory into registers (faces are recomputed from both
//      sides; this costs flops, not HBM bytes) and evaluates HLLC minus the
//      background HLLC, the interior-penalty terms and the symmetric term there,
//   D  contracts the volume fluxes with the GL derivative matrix, lifts the
//      face terms to its node and writes the requested output.
// The same kernel in JVP mode carries two states, U' and U' + eps y, and
// differences the fluxes point by point before contracting.
#include "jfmg_internal.h"

namespace jfmg {

template <int N1> struct DgShape {
    static constexpr int NP = N1 * N1;
    static constexpr int NTH = (N1 == 2) ? 64 : 128;
    static constexpr int EPB = NTH / NP;
};

__device__ __forceinline__ int face_nb(int f, int ex, int ez, int nx, int nz, int bc)
{
    // returns neighbour element index, or -1 for a slip wall
    if (f == 0) { if (ex > 0) return ez * nx + ex - 1; return bc == 1 ? ez * nx + nx - 1 : -1; }
    if (f == 1) { if (ex < nx - 1) return ez * nx + ex + 1; return bc == 1 ? ez * nx : -1; }
    if (f == 2) return ez > 0 ? (ez - 1) * nx + ex : -1;
    return ez < nz - 1 ? (ez + 1) * nx + ex : -1;
}

// At most 168 VGPRs so that three waves fit per SIMD (with 24 KB of LDS per
// 128-thread work-group, LDS allows six work-groups per CU).
template <int N1, bool NS, int MODE>
__global__ void __launch_bounds__(DgShape<N1>::NTH, 3)
dg_kernel(DgArgs A, const double* __restrict__ U, const double* __restrict__ Y, const double* __restrict__ Ubar,
          double* __restrict__ out, const double* __restrict__ yn2p, const double* __restrict__ ut2p, int eps_mode,
          double adt, Red red, long ms, ExStage rk)
{
    if (gridDim.z > 1) {   // member of a lock-step batch
        U = mbr(U, ms);
        Y = mbr(Y, ms);
        Ubar = mbr(Ubar, ms);
        out = mbr(out, ms);
        yn2p = mbr(yn2p, ms);
        ut2p = mbr(ut2p, ms);
        red = mbr(red, ms);
    }
    constexpr int NP = DgShape<N1>::NP, NTH = DgShape<N1>::NTH, EPB = DgShape<N1>::EPB;
    constexpr int NSt = (MODE == 3) ? 2 : 1;
    __shared__ double sS[NSt][EPB][4][NP];
    __shared__ double sFx[EPB][4][NP], sFz[EPB][4][NP];
    __shared__ double sFc[EPB][4][N1][4];
    __shared__ double sSy[NS ? EPB : 1][4][N1][4];

    const int t = threadIdx.x;
    const int le = t / NP, nd = t - le * NP;
    const bool act = le < EPB;
    const long e = (long)xcd_tile(blockIdx.x, gridDim.x) * EPB + le;   // XCD-contiguous element ranges
    const bool valid = act && e < A.ne;
    const int ez = valid ? (int)(e / A.nx) : 0;
    const int ex = valid ? (int)(e - (long)ez * A.nx) : 0;
    const long N = A.ne * NP;
    const RefTab& R = A.R;

    double eps = 0.0;
    if constexpr (MODE == 3) {
        const double yn2 = yn2p[0];
        if (!(yn2 > 0.0)) {   // y = 0: the product is 0 (uniform over the grid)
            if (valid)
                for (int c = 0; c < 4; ++c) out[c * N + e * NP + nd] = 0.0;
            return;
        }
        eps = eps_mode == 0 ? FdEps<double>::sqrt_eps / sqrt(yn2)
                            : FdEps<double>::sqrt_eps * sqrt(ut2p[0]) / sqrt(yn2);
    }

    // ---- A: stage element values ----
    double yv[4] = {0, 0, 0, 0};
    if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double u = valid ? U[c * N + e * NP + nd] : 0.0;
            sS[0][le][c][nd] = u;
            if constexpr (MODE == 3) {
                yv[c] = valid ? Y[c * N + e * NP + nd] : 0.0;
                sS[1][le][c][nd] = u + eps * yv[c];
            }
        }
    }
    __syncthreads();

    const int a = nd % N1, b = nd / N1;
    // ---- B: volume fluxes ----
    if (act) {
        double Ub[4], dUb[4];
        const int zi = ez * N1 + b;
#pragma unroll
        for (int c = 0; c < 4; ++c) { Ub[c] = A.bg_node[zi * 4 + c]; dUb[c] = A.dbg_node[zi * 4 + c]; }
        const double pbz = A.pb_node[zi], irz = A.irt_node[zi];
        double fx[4], fz[4];
#pragma unroll
        for (int s = 0; s < NSt; ++s) {
            double Ut[4], Fx[4], Fz[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) Ut[c] = sS[s][le][c][nd] + Ub[c];
            const double pt = pert_pressure(A.gas, sS[s][le][3][nd], irz, pbz);
            conv_flux_xz(Ut, pt, Fx, Fz);
            if constexpr (MODE != 3) {
                double Bx[4], Bz[4];
                conv_flux_xz(Ub, pbz, Bx, Bz);
#pragma unroll
                for (int c = 0; c < 4; ++c) { Fx[c] -= Bx[c]; Fz[c] -= Bz[c]; }
            }
            if constexpr (NS) {
                // F_v^x and F_v^z: mu (G_c - (U_c/rho) G_rho) with the x- and z-derivatives
                double Gx[4], Gz[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double sx = 0.0, sz = 0.0;
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        sx += R.D[a][j] * sS[s][le][c][b * N1 + j];
                        sz += R.D[b][j] * sS[s][le][c][j * N1 + a];
                    }
                    Gx[c] = (2.0 / A.dx) * sx;
                    Gz[c] = (2.0 / A.dz) * sz + dUb[c];
                }
                const double ir = frcp(Ut[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c) {
                    const double rc = Ut[c] * ir;
                    Fx[c] -= A.mu * (Gx[c] - rc * Gx[0]);
                    Fz[c] -= A.mu * (Gz[c] - rc * Gz[0]);
                }
            }
            if (s == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) { fx[c] = Fx[c]; fz[c] = Fz[c]; }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) { fx[c] = Fx[c] - fx[c]; fz[c] = Fz[c] - fz[c]; }
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) { sFx[le][c][nd] = fx[c]; sFz[le][c][nd] = fz[c]; }
    }

    // ---- C: face fluxes; the neighbour element's trace and normal derivative at
    // the face point come straight from global memory into registers ----
    if (act) {
        for (int fp = nd; fp < 4 * N1; fp += NP) {
            const int f = fp / N1, r = fp - f * N1;
            const bool xf = f < 2;
            const int side = (f == 0 || f == 2) ? -1 : 1;
            const double nxn = xf ? (double)side : 0.0, nzn = xf ? 0.0 : (double)side;
            const double* es = side > 0 ? R.ep : R.em;
            const double* ds = side > 0 ? R.dp : R.dm;
            const double hperp = xf ? A.dx : A.dz;
            const double flen = xf ? A.dz : A.dx;
            const int nb = valid ? face_nb(f, ex, ez, A.nx, A.nz, A.bc) : -1;
            const bool wall = nb < 0;
            double trx[NSt][4], dnx[NSt][4];   // other side: trace and normal derivative (d/d xi of the neighbour)
            {
                const double* eo = side > 0 ? R.em : R.ep;
                const double* dso = side > 0 ? R.dm : R.dp;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int st = 0; st < NSt; ++st) { trx[st][c] = 0.0; dnx[st][c] = 0.0; }
                    if (!wall) {
#pragma unroll
                        for (int j = 0; j < N1; ++j) {
                            const int idx = xf ? r * N1 + j : j * N1 + r;
                            const double v = U[c * N + (long)nb * NP + idx];
                            trx[0][c] += eo[j] * v;
                            if constexpr (NS) dnx[0][c] += dso[j] * v;
                            if constexpr (MODE == 3) {
                                const double v1 = v + eps * Y[c * N + (long)nb * NP + idx];
                                trx[1][c] += eo[j] * v1;
                                if constexpr (NS) dnx[1][c] += dso[j] * v1;
                            }
                        }
                    }
                }
            }
            double Ub[4], dUb[4];
            const int zrow = xf ? (ez * N1 + r) : (ez + (side > 0 ? 1 : 0));
            const double* bgp = xf ? A.bg_node : A.bg_face;
            const double* dbgp = xf ? A.dbg_node : A.dbg_face;
#pragma unroll
            for (int c = 0; c < 4; ++c) { Ub[c] = bgp[zrow * 4 + c]; dUb[c] = dbgp[zrow * 4 + c]; }
            const double pbz = xf ? A.pb_node[zrow] : A.pb_face[zrow];
            const double irz = xf ? A.irt_node[zrow] : A.irt_face[zrow];
            double flux[4] = {0, 0, 0, 0}, sym[4] = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < NSt; ++s) {
                double tro[4], Uo[4], Ux[4], H[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double v = 0.0;
#pragma unroll
                    for (int j = 0; j < N1; ++j) v += es[j] * sS[s][le][c][xf ? r * N1 + j : j * N1 + r];
                    tro[c] = v;
                    Uo[c] = v + Ub[c];
                }
                const double po = pert_pressure(A.gas, tro[3], irz, pbz);
                double px = po;
                if (wall) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) Ux[c] = Uo[c];
                    if (xf) Ux[1] = -Uo[1]; else Ux[2] = -Uo[2];
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) Ux[c] = trx[s][c] + Ub[c];
                    px = pert_pressure(A.gas, trx[s][3], irz, pbz);
                }
                hllc(A.gas, Uo, Ux, po, px, nxn, nzn, H);
                double fl[4], sy[4] = {0, 0, 0, 0};
                if constexpr (MODE != 3) {
                    double Um[4], Hb[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) Um[c] = Ub[c];
                    if (wall) { if (xf) Um[1] = -Ub[1]; else Um[2] = -Ub[2]; }
                    hllc(A.gas, Ub, Um, pbz, pbz, nxn, nzn, Hb);
#pragma unroll
                    for (int c = 0; c < 4; ++c) H[c] -= Hb[c];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) fl[c] = -H[c];
                if constexpr (NS) {
                    if (!wall) {
                        // F_v(U, G) . n of a Cartesian face involves only the normal derivative
                        // G_n (the tangential part enters multiplied by 0): own side from the
                        // element's values, other side from the neighbour's trace derivative,
                        // plus the background's z-derivative on z-faces
                        const double gs = 2.0 / hperp, sg = (double)side;
                        const double iro = frcp(Uo[0]), irx = frcp(Ux[0]);
                        double Gno[4], Gnx[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            double sn = 0.0;
#pragma unroll
                            for (int j = 0; j < N1; ++j) sn += ds[j] * sS[s][le][c][xf ? r * N1 + j : j * N1 + r];
                            const double db = xf ? 0.0 : dUb[c];
                            Gno[c] = gs * sn + db;
                            Gnx[c] = gs * dnx[s][c] + db;
                        }
                        const double eta = A.c_ip * (double)(N1 * N1) / hperp;
                        const double Dl0 = tro[0] - trx[s][0];
                        const double irm = frcp(0.5 * (Uo[0] + Ux[0]));
#pragma unroll
                        for (int c = 1; c < 4; ++c) {
                            const double ro = Uo[c] * iro;
                            const double Fo = sg * A.mu * (Gno[c] - ro * Gno[0]);
                            const double Fxx = sg * A.mu * (Gnx[c] - Ux[c] * irx * Gnx[0]);
                            const double Dlc = tro[c] - trx[s][c];
                            const double pen = eta * A.mu * (Dlc - (0.5 * (Uo[c] + Ux[c]) * irm) * Dl0);
                            fl[c] += 0.5 * (Fo + Fxx) - pen;
                            sy[c] = 0.5 * A.mu * (Dlc - ro * Dl0);
                        }
                    }
                }
                if (s == 0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) { flux[c] = fl[c]; sym[c] = sy[c]; }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) { flux[c] = fl[c] - flux[c]; sym[c] = sy[c] - sym[c]; }
                }
            }
            const double W = R.w[r] * flen * 0.5;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sFc[le][f][r][c] = W * flux[c];
                if constexpr (NS) sSy[le][f][r][c] = W * sym[c];
            }
        }
    }
    __syncthreads();

    // ---- D: contraction, lifting and output ----
    double nrm = 0.0;
    if (valid) {
        const double m = R.w[a] * R.w[b] * A.J, im = frcp(m);
        const double sc = MODE == 3 ? adt / eps : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double sx = 0.0, sz = 0.0;
#pragma unroll
            for (int q = 0; q < N1; ++q) sx += R.w[q] * R.D[q][a] * sFx[le][c][b * N1 + q];
#pragma unroll
            for (int q = 0; q < N1; ++q) sz += R.w[q] * R.D[q][b] * sFz[le][c][q * N1 + a];
            double L = A.J * ((2.0 / A.dx) * R.w[b] * sx + (2.0 / A.dz) * R.w[a] * sz);
            L += sFc[le][0][b][c] * R.em[a] + sFc[le][1][b][c] * R.ep[a];
            L += sFc[le][2][a][c] * R.em[b] + sFc[le][3][a][c] * R.ep[b];
            if constexpr (NS) {
                L += sSy[le][0][b][c] * (-(2.0 / A.dx) * R.dm[a]) + sSy[le][1][b][c] * ((2.0 / A.dx) * R.dp[a]);
                L += sSy[le][2][a][c] * (-(2.0 / A.dz) * R.dm[b]) + sSy[le][3][a][c] * ((2.0 / A.dz) * R.dp[b]);
            }
            if (c == 2) {
                if constexpr (MODE == 3) L += m * (-A.g * (sS[1][le][0][nd] - sS[0][le][0][nd]));
                else L += m * (-A.g * sS[0][le][0][nd]);
            }
            const long o = c * N + e * NP + nd;
            if constexpr (MODE == 0) out[o] = L;
            else if constexpr (MODE == 1) out[o] = L * im;
            else if constexpr (MODE == 2) {
                const double G = sS[0][le][c][nd] - adt * (L * im) - Ubar[o];
                out[o] = G;
                nrm += G * G;
            } else if constexpr (MODE == 3) {
                out[o] = yv[c] - sc * (L * im);
            } else {   // explicit Runge-Kutta stage
                const double base = rk.a0 != 0.0 ? rk.a0 * Ubar[o] : 0.0;
                out[o] = base + rk.a1 * sS[0][le][c][nd] + rk.c * (L * im);
            }
        }
    }
    if constexpr (MODE == 2) put_partial<NTH>(red, nrm);
}

int dg_grid(int k, long ne)
{
    const int epb = k == 1 ? DgShape<2>::EPB : k == 2 ? DgShape<3>::EPB : DgShape<4>::EPB;
    return (int)((ne + epb - 1) / epb);
}

template <int N1, bool NS>
static void launch_dg_n(int mode, const DgArgs& A, const double* U, const double* Y, const double* Ubar,
                        double* out, const double* yn2, const double* ut2, int eps_mode, double adt, Red red,
                        hipStream_t st, const Mb& mb, const ExStage& ex)
{
    const dim3 grid(dg_grid(N1 - 1, A.ne), 1, mb.n), block(DgShape<N1>::NTH);
    if (mode == 2 && red.out) {
        timed_launch(dg_kernel<N1, NS, 2>, grid, block, st, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, mb.ms,
                     ex);
        launch_finalize(red.partials, (int)grid.x, 1, red.out, st, Gate{}, mb);
        return;
    }
#define JFMG_DG_CASE(M)                                                                                             \
    case M:                                                                                                         \
        timed_launch(dg_kernel<N1, NS, M>, grid, block, st, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, mb.ms, \
                     ex);                                                                                           \
        break;
    switch (mode) {
        JFMG_DG_CASE(0)
        JFMG_DG_CASE(1)
        JFMG_DG_CASE(2)
        JFMG_DG_CASE(4)
    default:
        timed_launch(dg_kernel<N1, NS, 3>, grid, block, st, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, mb.ms,
                     ex);
        break;
    }
#undef JFMG_DG_CASE
}

void launch_dg(int k, bool ns, int mode, const DgArgs& A, const double* U, const double* Y, const double* Ubar,
               double* out, const double* yn2, const double* ut2, int eps_mode, double adt, Red red, hipStream_t st,
               const Mb& mb, const ExStage& ex)
{
    if (k == 1) { if (ns) launch_dg_n<2, true>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex);
                  else launch_dg_n<2, false>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex); }
    else if (k == 2) { if (ns) launch_dg_n<3, true>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex);
                       else launch_dg_n<3, false>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex); }
    else { if (ns) launch_dg_n<4, true>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex);
           else launch_dg_n<4, false>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex); }
}

// ---------------------------------------------------------------------------
// Initial data (eq. add-perturbation): theta' inserted at constant pressure.
// ---------------------------------------------------------------------------
template <int N1>
__global__ void __launch_bounds__(256)
init_kernel(DgArgs A, int shape, double amp, double xc, double zc, double xr, double zr, double aa, double Z,
            double x0, double z0, double u_mean, double* __restrict__ U, long ms)
{
    U = mbr(U, ms);
    constexpr int NP = N1 * N1;
    const long n = A.ne * NP;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const long e = i / NP;
    const int nd = (int)(i - e * NP);
    const int a = nd % N1, b = nd / N1;
    const int ez = (int)(e / A.nx), ex = (int)(e - (long)ez * A.nx);
    const double x = x0 + (ex + 0.5 * (1.0 + A.R.xi[a])) * A.dx;
    const double z = z0 + (ez + 0.5 * (1.0 + A.R.xi[b])) * A.dz;
    double th1 = 0.0;
    if (shape == 0) {
        const double rx = (x - xc) / xr, rz = (z - zc) / zr;
        const double r = sqrt(rx * rx + rz * rz);
        if (r < 1.0) th1 = 0.5 * amp * (1.0 + cos(M_PI * r));
    } else {
        const double s = (x - xc) / aa;
        th1 = amp / (1.0 + s * s) * sin(M_PI * z / Z);
    }
    const int zi = ez * N1 + b;
    const double rt = A.bg_node[zi * 4 + 3], rhob = A.bg_node[zi * 4 + 0], mb = A.bg_node[zi * 4 + 1];
    const double rho = rt / (A.th_node[zi] + th1);
    U[i] = rho - rhob;
    U[n + i] = rho * u_mean - mb;
    U[2 * n + i] = 0.0;
    U[3 * n + i] = 0.0;
}

void launch_initial_state(int k, const DgArgs& A, int shape, double amp, double xc, double zc, double xr, double zr,
                          double a, double Z, double x0, double z0, double u_mean, double* U, hipStream_t st,
                          const Mb& mb)
{
    const long n = A.ne * (k + 1) * (k + 1);
    const dim3 grid((unsigned)((n + 255) / 256), 1, mb.n), block(256);
    if (k == 1) init_kernel<2><<<grid, block, 0, st>>>(A, shape, amp, xc, zc, xr, zr, a, Z, x0, z0, u_mean, U, mb.ms);
    else if (k == 2) init_kernel<3><<<grid, block, 0, st>>>(A, shape, amp, xc, zc, xr, zr, a, Z, x0, z0, u_mean, U, mb.ms);
    else init_kernel<4><<<grid, block, 0, st>>>(A, shape, amp, xc, zc, xr, zr, a, Z, x0, z0, u_mean, U, mb.ms);
}

// sum over all nodes and components of (U' + Ubar)^2
template <int N1>
__global__ void __launch_bounds__(256) norm_total_kernel(DgArgs A, const double* __restrict__ U, Red red, long ms)
{
    U = mbr(U, ms);
    red = mbr(red, ms);
    constexpr int NP = N1 * N1;
    const long n = A.ne * NP;
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const long e = i / NP;
        const int b = (int)(i - e * NP) / N1;
        const int zi = (int)(e / A.nx) * N1 + b;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = U[c * n + i] + A.bg_node[zi * 4 + c];
            s += v * v;
        }
    }
    put_partial<256>(red, s);
}

int norm_total_grid(long n)
{
    long b = (n + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

void launch_norm2_total(int k, const DgArgs& A, const double* U, Red red, hipStream_t st, const Mb& mb)
{
    const long n = A.ne * (k + 1) * (k + 1);
    const dim3 grid(norm_total_grid(n), 1, mb.n), block(256);
    if (k == 1) norm_total_kernel<2><<<grid, block, 0, st>>>(A, U, red, mb.ms);
    else if (k == 2) norm_total_kernel<3><<<grid, block, 0, st>>>(A, U, red, mb.ms);
    else norm_total_kernel<4><<<grid, block, 0, st>>>(A, U, red, mb.ms);
    launch_finalize(red.partials, (int)grid.x, 1, red.out, st, Gate{}, mb);
}

}  // namespace jfmg
