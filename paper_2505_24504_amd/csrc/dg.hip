// DG space operator of the well-balanced perturbation system (paper eqs.
// convDiscr, elementint, surfaceint and perturbed-euler) on gfx950.
//
// One work-group holds EPB whole elements, one thread per GL node (k = 3: 8
// elements x 16 nodes = 128 threads).  Element values are staged in LDS; each
// thread then
//   B  evaluates the volume flux at its node (total state U' + Ubar minus the
//      background flux, minus the viscous flux) into LDS,
//   C  loads the neighbour element's trace and normal derivative at one face
//      point from global memory into registers (faces are evaluated from both
//      sides; this costs flops, not HBM bytes) and evaluates HLLC minus the
//      background HLLC, the interior-penalty terms and the symmetric term there,
//   D  contracts the volume fluxes with the GL derivative matrix, lifts the
//      face terms to its node and writes the requested output.
// In JVP mode the kernel evaluates the fluxes of U' + eps y and differences them
// point by point with those of U' before contracting.  The fluxes of U' are the
// same for every product with one linearization state: mode 5 writes them (volume
// fluxes per node, face terms per face point) once per linearization, and each
// product reads them back instead of evaluating a second state.
#include "jfmg_internal.h"

namespace jfmg {

template <int N1> struct DgShape {
    static constexpr int NP = N1 * N1;
    static constexpr int NTH = (N1 == 2) ? 64 : 128;
    static constexpr int EPB = NTH / NP;
    static constexpr int FPE = 4 * N1;   // face points per element
};

__device__ __forceinline__ int face_nb(int f, int ex, int ez, int nx, int nz, int bc)
{
    // returns neighbour element index, or -1 for a slip wall
    if (f == 0) { if (ex > 0) return ez * nx + ex - 1; return bc == 1 ? ez * nx + nx - 1 : -1; }
    if (f == 1) { if (ex < nx - 1) return ez * nx + ex + 1; return bc == 1 ? ez * nx : -1; }
    if (f == 2) return ez > 0 ? (ez - 1) * nx + ex : -1;
    return ez < nz - 1 ? (ez + 1) * nx + ex : -1;
}

// Face terms of one state at face point r of an x-face (xf) or z-face of element
// row ez with outward normal +e_D (pos) or -e_D, before the quadrature weight:
//   fl = -H(U_in, U_out; n) (minus the background's H when BGSUB) plus, for
//        viscous flow, the average of both sides' F_v . n minus the interior
//        penalty on the jump of the velocity-like variables,
//   sy = the symmetric term's jump mu (U_c,in - U_c,out - (U_c/rho)_in (rho_in - rho_out)).
// The element's own values come from its LDS block sv; the neighbour nb (-1: a
// slip wall, mirrored state) is read from U, plus eps Y when PLUSY.  When pos is
// uniform over the wave the trace weights are scalar loads.
template <int N1, bool NS, bool BGSUB, bool PLUSY>
__device__ __forceinline__ void dg_face(const DgArgs& A, const double (&sv)[4][N1 * N1], const double* __restrict__ U,
                                        const double* __restrict__ Y, double eps, long N, int nb, bool xf, bool pos,
                                        int r, int ez, double (&fl)[4], double (&sy)[4])
{
    constexpr int NP = N1 * N1;
    const RefTab& R = A.R;
    const double sg = pos ? 1.0 : -1.0;
    const bool wall = nb < 0;
    // trace and normal-derivative weights of the own and the other side
    const double* es = pos ? R.ep : R.em;
    const double* ds = pos ? R.dp : R.dm;
    const double* eo = pos ? R.em : R.ep;
    const double* dso = pos ? R.dm : R.dp;
    double Ub[4], dUb[4];
    const int zrow = xf ? (ez * N1 + r) : (ez + (pos ? 1 : 0));
    const double* bgp = xf ? A.bg_node : A.bg_face;
    const double* dbgp = xf ? A.dbg_node : A.dbg_face;
#pragma unroll
    for (int c = 0; c < 4; ++c) { Ub[c] = bgp[zrow * 4 + c]; dUb[c] = dbgp[zrow * 4 + c]; }
    const double pbz = xf ? A.pb_node[zrow] : A.pb_face[zrow];
    const double irz = xf ? A.irt_node[zrow] : A.irt_face[zrow];
    double trx[4], dnx[4];   // the neighbour's trace and normal derivative (d/d xi)
#pragma unroll
    for (int c = 0; c < 4; ++c) trx[c] = dnx[c] = 0.0;
    if (!wall) {
        // every load of the neighbour's nodes first (one block: one memory round trip
        // instead of one per component), then the sums in the same order
        double vu[4][N1], vy[PLUSY ? 4 : 1][PLUSY ? N1 : 1];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < N1; ++j) {
                const unsigned o = (unsigned)nb * NP + (xf ? r * N1 + j : j * N1 + r);
                vu[c][j] = ld(U + c * N, o);
                if constexpr (PLUSY) vy[c][j] = ld(Y + c * N, o);
            }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < N1; ++j) {
                double v = vu[c][j];
                if constexpr (PLUSY) v = v + eps * vy[c][j];
                trx[c] += eo[j] * v;
                if constexpr (NS) dnx[c] += dso[j] * v;
            }
    }
    double tro[4], Uo[4], Ux[4], H[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) v += es[j] * sv[c][xf ? r * N1 + j : j * N1 + r];
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
        for (int c = 0; c < 4; ++c) Ux[c] = trx[c] + Ub[c];
        px = pert_pressure(A.gas, trx[3], irz, pbz);
    }
    const double iro = frcp(Uo[0]), irx = frcp(Ux[0]);
    hllc_face(A.gas, Uo, Ux, po, px, iro, irx, xf, sg, H);
    if constexpr (BGSUB) {
        double Um[4], Hb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) Um[c] = Ub[c];
        if (wall) { if (xf) Um[1] = -Ub[1]; else Um[2] = -Ub[2]; }
        const double irb = frcp(Ub[0]);
        hllc_face(A.gas, Ub, Um, pbz, pbz, irb, irb, xf, sg, Hb);
#pragma unroll
        for (int c = 0; c < 4; ++c) H[c] -= Hb[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) { fl[c] = -H[c]; sy[c] = 0.0; }
    if constexpr (NS) {
        if (!wall) {
            // F_v(U, G) . n of a Cartesian face involves only the normal derivative
            // G_n (the tangential part enters multiplied by 0): own side from the
            // element's values, other side from the neighbour's trace derivative,
            // plus the background's z-derivative on z-faces
            const double gs = xf ? A.rdx2 : A.rdz2;
            double Gno[4], Gnx[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double sn = 0.0;
#pragma unroll
                for (int j = 0; j < N1; ++j) sn += ds[j] * sv[c][xf ? r * N1 + j : j * N1 + r];
                const double db = xf ? 0.0 : dUb[c];
                Gno[c] = gs * sn + db;
                Gnx[c] = gs * dnx[c] + db;
            }
            const double eta = xf ? A.eta_x : A.eta_z;
            const double Dl0 = tro[0] - trx[0];
            const double irm = frcp(0.5 * (Uo[0] + Ux[0]));
#pragma unroll
            for (int c = 1; c < 4; ++c) {
                const double ro = Uo[c] * iro;
                const double Fo = sg * A.mu * (Gno[c] - ro * Gno[0]);
                const double Fxx = sg * A.mu * (Gnx[c] - Ux[c] * irx * Gnx[0]);
                const double Dlc = tro[c] - trx[c];
                const double pen = eta * A.mu * (Dlc - (0.5 * (Uo[c] + Ux[c]) * irm) * Dl0);
                fl[c] += 0.5 * (Fo + Fxx) - pen;
                sy[c] = 0.5 * A.mu * (Dlc - ro * Dl0);
            }
        }
    }
}

// k = 3: at most 128 VGPRs (four waves per SIMD) and 20 KB of LDS per 128-thread
// work-group, so that eight work-groups fit per CU; lower degrees at most 168.
template <int N1, bool NS, int MODE, bool RG>
__global__ void __launch_bounds__(DgShape<N1>::NTH, N1 == 4 ? 4 : 3)
dg_kernel(DgArgs Aa, const MemberArgs* __restrict__ mt, const double* __restrict__ U, const double* __restrict__ Y,
          const double* __restrict__ Ubar, double* __restrict__ out, const double* __restrict__ yn2p,
          const double* __restrict__ ut2p, int eps_mode, double adt, Red red, long ms, ExStage rk, int ycount)
{
    const DgArgs& A = dg_of<RG>(Aa, mt);
    double* lin0 = A.lin0;
    if (gridDim.z > 1) {   // member of a lock-step batch
        U = mbr(U, ms);
        Y = mbr(Y, ms);
        Ubar = mbr(Ubar, ms);
        out = mbr(out, ms);
        yn2p = mbr(yn2p, ms);
        ut2p = mbr(ut2p, ms);
        red = mbr(red, ms);
        if (!RG) lin0 = mbr(lin0, ms);   // a ragged member's pointer is its own
    }
    constexpr int NP = DgShape<N1>::NP, NTH = DgShape<N1>::NTH, EPB = DgShape<N1>::EPB, FPE = DgShape<N1>::FPE;
    const int nbm = (int)((A.ne + EPB - 1) / EPB);   // this member's work-groups
    if ((int)blockIdx.x >= nbm || (RG && sits_out(mt))) {   // beyond a smaller member, or one that sits out
        if (MODE == 2 && threadIdx.x == 0) red.partials[block_linear()] = 0.0;
        return;
    }
    constexpr bool OUTL = MODE != 5;   // the fluxes stay in LDS for the contraction
    __shared__ double sS[EPB][4][NP];
    __shared__ double sFx[OUTL ? EPB : 1][4][NP], sFz[OUTL ? EPB : 1][4][NP];
    __shared__ double sFc[OUTL ? EPB : 1][4][N1][4];
    __shared__ double sSy[OUTL && NS ? EPB : 1][4][N1][4];

    const int t = threadIdx.x;
    const int le = t / NP, nd = t - le * NP;
    const bool act = le < EPB;
    const long eb = (long)xcd_tile(blockIdx.x, nbm) * EPB;   // XCD-contiguous element ranges
    const long e = eb + le;
    const bool valid = act && e < A.ne;
    const int ez = valid ? (int)(e / A.nx) : 0;
    const long N = A.ne * NP, NF = A.ne * FPE;
    const RefTab& R = A.R;
    double* vol0 = lin0;              // [8][N]
    double* face0 = lin0 + 8 * N;     // [8][NF]

    const unsigned no = (unsigned)(e * NP + nd);   // the thread's node in component arrays
    // ---- A: stage the element values (JVP: of U' + eps y).  The loads are issued
    // before the step size is known (it depends on a device scalar). ----
    double u0[4], y0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        u0[c] = valid ? ld(U + c * N, no) : 0.0;
        y0[c] = (MODE == 3 && valid) ? ld(Y + c * N, no) : 0.0;
    }
    // the node row's background and (JVP) the stored volume fluxes of U', with the loads above
    const int a = nd % N1, b = nd / N1;
    double Ub[4], dUb[4], v0x[4], v0z[4];
    double pbz = 0.0, irz = 0.0;
    {
        const int zi = ez * N1 + b;
#pragma unroll
        for (int c = 0; c < 4; ++c) { Ub[c] = act ? A.bg_node[zi * 4 + c] : 0.0; dUb[c] = act ? A.dbg_node[zi * 4 + c] : 0.0; }
        pbz = act ? A.pb_node[zi] : 0.0;
        irz = act ? A.irt_node[zi] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v0x[c] = (MODE == 3 && valid) ? ld(vol0 + c * N, no) : 0.0;
            v0z[c] = (MODE == 3 && valid) ? ld(vol0 + (4 + c) * N, no) : 0.0;
        }
    }
    double eps = 0.0;
    if constexpr (MODE == 3) {
        const double ut2 = eps_mode == 0 ? 0.0 : ut2p[0];
        // ||y||^2: yn2p[0], or with ycount > 0 the sum of the ycount block partials at yn2p
        // (fixed order; sFx serves as scratch until phase B writes it)
        double yn2;
        if (ycount > 0) {
            double a = 0.0;
            for (int i = t; i < ycount; i += NTH) a += yn2p[i];
            a = wave_sum(a);
            double* scr = &sFx[0][0][0];
            if ((t & 63) == 0) scr[t >> 6] = a;
            __syncthreads();
            yn2 = scr[0];
#pragma unroll
            for (int w = 1; w < NTH / 64; ++w) yn2 += scr[w];
        } else {
            yn2 = yn2p[0];
        }
        if (!(yn2 > 0.0)) {   // y = 0: the product is 0 (uniform over the grid)
            if (valid)
                for (int c = 0; c < 4; ++c) st(out + c * N, no, 0.0);
            return;
        }
        eps = uniform(eps_mode == 0 ? FdEps<double>::sqrt_eps / sqrt(yn2)
                                    : FdEps<double>::sqrt_eps * sqrt(ut2) / sqrt(yn2));
    }
    if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sS[le][c][nd] = MODE == 3 ? u0[c] + eps * y0[c] : u0[c];
    }
    __syncthreads();

    // ---- B: volume fluxes (JVP: minus those of U') ----
    if (act) {
        double Ut[4], Fx[4], Fz[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) Ut[c] = sS[le][c][nd] + Ub[c];
        const double pt = pert_pressure(A.gas, sS[le][3][nd], irz, pbz);
        conv_flux_xz(Ut, pt, Fx, Fz);
        if constexpr (MODE != 3 && MODE != 5) {
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
                    sx += R.D[a][j] * sS[le][c][b * N1 + j];
                    sz += R.D[b][j] * sS[le][c][j * N1 + a];
                }
                Gx[c] = A.rdx2 * sx;
                Gz[c] = A.rdz2 * sz + dUb[c];
            }
            const double ir = frcp(Ut[0]);
#pragma unroll
            for (int c = 1; c < 4; ++c) {
                const double rc = Ut[c] * ir;
                Fx[c] -= A.mu * (Gx[c] - rc * Gx[0]);
                Fz[c] -= A.mu * (Gz[c] - rc * Gz[0]);
            }
        }
        if constexpr (MODE == 5) {
            if (valid) {
#pragma unroll
                for (int c = 0; c < 4; ++c) { st(vol0 + c * N, no, Fx[c]); st(vol0 + (4 + c) * N, no, Fz[c]); }
            }
        } else {
            if constexpr (MODE == 3) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    Fx[c] = Fx[c] - v0x[c];
                    Fz[c] = Fz[c] - v0z[c];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) { sFx[le][c][nd] = Fx[c]; sFz[le][c][nd] = Fz[c]; }
        }
    }

    // ---- C: face terms (JVP: minus those of U'); the neighbour element's trace
    // and normal derivative at the face point come straight from global memory
    // into registers.  With k = 3 (16 face points and 16 threads per element)
    // wave 0 takes the faces with outward normal -e_x / -e_z of all eight
    // elements and wave 1 those with +e_x / +e_z, so that the side, and with it
    // every trace weight, is uniform per wave. ----
    auto face_point = [&](int fle, int f, int r, bool pos) {
        const int fe = (int)eb + fle;
        const bool fvalid = fe < A.ne;
        const int fez = fvalid ? fe / A.nx : 0;
        const int fex = fvalid ? fe - fez * A.nx : 0;
        const int nb = fvalid ? face_nb(f, fex, fez, A.nx, A.nz, A.bc) : -1;
        const bool xf = f < 2;
        const unsigned q = (unsigned)fe * FPE + f * N1 + r;
        double fl[4], sy[4];
        dg_face<N1, NS, MODE != 3 && MODE != 5, MODE == 3>(A, sS[fle], U, Y, eps, N, nb, xf, pos, r, fez, fl, sy);
        if constexpr (MODE == 5) {
            if (fvalid) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    st(face0 + c * NF, q, fl[c]);
                    if constexpr (NS) st(face0 + (4 + c) * NF, q, sy[c]);
                }
            }
            return;
        }
        if constexpr (MODE == 3) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                fl[c] = fl[c] - (fvalid ? ld(face0 + c * NF, q) : 0.0);
                if constexpr (NS) sy[c] = sy[c] - (fvalid ? ld(face0 + (4 + c) * NF, q) : 0.0);
            }
        }
        const double W = R.w[r] * (xf ? A.dz : A.dx) * 0.5;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            sFc[fle][f][r][c] = W * fl[c];
            if constexpr (NS) sSy[fle][f][r][c] = W * sy[c];
        }
    };
    if constexpr (N1 == 4 && NTH == 128) {
        const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // wave index, uniform
        const int l = t & 63, qf = l & 7;
        face_point(l >> 3, ((qf >> 2) << 1) | w, qf & 3, w != 0);
    } else if (act) {
        for (int fp = nd; fp < FPE; fp += NP) {
            const int f = fp / N1;
            face_point(le, f, fp - f * N1, (f & 1) != 0);
        }
    }
    if constexpr (MODE == 5) return;
    // U'_rho and y are read again for the output (not held through the face phase);
    // the loads are issued before the barrier so that their latency overlaps it
    double y_d[4] = {0.0, 0.0, 0.0, 0.0}, urho_d = 0.0;
    if constexpr (MODE == 3) {
        if (valid) {
            const double* Ud = opaque(U);
            const double* Yd = opaque(Y);
            urho_d = ld(Ud, no);
#pragma unroll
            for (int c = 0; c < 4; ++c) y_d[c] = ld(Yd + c * N, no);
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
            double L = A.J * (A.rdx2 * R.w[b] * sx + A.rdz2 * R.w[a] * sz);
            L += sFc[le][0][b][c] * R.em[a] + sFc[le][1][b][c] * R.ep[a];
            L += sFc[le][2][a][c] * R.em[b] + sFc[le][3][a][c] * R.ep[b];
            if constexpr (NS) {
                L += sSy[le][0][b][c] * (-A.rdx2 * R.dm[a]) + sSy[le][1][b][c] * (A.rdx2 * R.dp[a]);
                L += sSy[le][2][a][c] * (-A.rdz2 * R.dm[b]) + sSy[le][3][a][c] * (A.rdz2 * R.dp[b]);
            }
            if (c == 2) {
                // gravity; JVP: of (U' + eps y)_rho - U'_rho
                if constexpr (MODE == 3) L += m * (-A.g * (sS[le][0][nd] - urho_d));
                else L += m * (-A.g * sS[le][0][nd]);
            }
            if constexpr (MODE == 0) st(out + c * N, no, L);
            else if constexpr (MODE == 1) st(out + c * N, no, L * im);
            else if constexpr (MODE == 2) {
                const double G = sS[le][c][nd] - adt * (L * im) - ld(Ubar + c * N, no);
                st(out + c * N, no, G);
                nrm += G * G;
            } else if constexpr (MODE == 3) {
                st(out + c * N, no, y_d[c] - sc * (L * im));
            } else {   // explicit Runge-Kutta stage
                const double base = rk.a0 != 0.0 ? rk.a0 * ld(Ubar + c * N, no) : 0.0;
                st(out + c * N, no, base + rk.a1 * sS[le][c][nd] + rk.c * (L * im));
            }
            // one component at a time: keeps the LDS reads of the next component
            // from being hoisted into this one (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if constexpr (MODE == 2) put_partial<NTH>(red, nrm);
}

int dg_grid(int k, long ne)
{
    const int epb = k == 1 ? DgShape<2>::EPB : k == 2 ? DgShape<3>::EPB : DgShape<4>::EPB;
    return (int)((ne + epb - 1) / epb);
}

template <int N1, bool NS, bool RG>
static void launch_dg_n(int mode, const DgArgs& A0, const double* U, const double* Y, const double* Ubar,
                        double* out, const double* yn2, const double* ut2, int eps_mode, double adt, Red red,
                        hipStream_t st, const Mb& mb, const ExStage& ex, int ycount)
{
    DgArgs A = A0;
    A.rdx2 = 2.0 / A.dx;
    A.rdz2 = 2.0 / A.dz;
    A.eta_x = A.c_ip * (double)(N1 * N1) / A.dx;
    A.eta_z = A.c_ip * (double)(N1 * N1) / A.dz;
    const dim3 grid(dg_grid(N1 - 1, A.ne), 1, mb.n), block(DgShape<N1>::NTH);
    if (mode == 2 && red.out) {
        timed_launch(dg_kernel<N1, NS, 2, RG>, grid, block, st, A, mb.tab, U, Y, Ubar, out, yn2, ut2, eps_mode, adt,
                     red, mb.ms, ex, 0);
        launch_finalize(red.partials, (int)grid.x, 1, red.out, st, Gate{}, mb);
        return;
    }
#define JFMG_DG_CASE(M)                                                                                            \
    case M:                                                                                                        \
        timed_launch(dg_kernel<N1, NS, M, RG>, grid, block, st, A, mb.tab, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, \
                     red, mb.ms, ex, 0);                                                                           \
        break;
    switch (mode) {
        JFMG_DG_CASE(0)
        JFMG_DG_CASE(1)
        JFMG_DG_CASE(2)
        JFMG_DG_CASE(4)
        JFMG_DG_CASE(5)
    default:
        timed_launch(dg_kernel<N1, NS, 3, RG>, grid, block, st, A, mb.tab, U, Y, Ubar, out, yn2, ut2, eps_mode, adt,
                     red, mb.ms, ex, ycount);
        break;
    }
#undef JFMG_DG_CASE
}

template <int N1>
static void launch_dg_k(bool ns, int mode, const DgArgs& A, const double* U, const double* Y, const double* Ubar,
                        double* out, const double* yn2, const double* ut2, int eps_mode, double adt, Red red,
                        hipStream_t st, const Mb& mb, const ExStage& ex, int yc)
{
    if (mb.tab) {
        if (ns) launch_dg_n<N1, true, true>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, yc);
        else launch_dg_n<N1, false, true>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, yc);
    } else {
        if (ns) launch_dg_n<N1, true, false>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, yc);
        else launch_dg_n<N1, false, false>(mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, yc);
    }
}

void launch_dg(int k, bool ns, int mode, const DgArgs& A, const double* U, const double* Y, const double* Ubar,
               double* out, const double* yn2, const double* ut2, int eps_mode, double adt, Red red, hipStream_t st,
               const Mb& mb, const ExStage& ex, int ycount)
{
    if (k == 1) launch_dg_k<2>(ns, mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, ycount);
    else if (k == 2) launch_dg_k<3>(ns, mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, ycount);
    else launch_dg_k<4>(ns, mode, A, U, Y, Ubar, out, yn2, ut2, eps_mode, adt, red, st, mb, ex, ycount);
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
template <int N1, bool RG>
__global__ void __launch_bounds__(256)
norm_total_kernel(DgArgs Aa, const MemberArgs* __restrict__ mt, const double* __restrict__ U, Red red, long ms)
{
    const DgArgs& A = dg_of<RG>(Aa, mt);
    U = mbr(U, ms);
    red = mbr(red, ms);
    constexpr int NP = N1 * N1;
    const long n = sits_out(mt) ? 0 : A.ne * NP;
    const long nb = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;   // this member's work-groups
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) {
        const long e = i / NP;
        const int b = (int)(i - e * NP) / N1;
        const int zi = (int)(e / A.nx) * N1 + b;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = U[c * n + i] + A.bg_node[zi * 4 + c];
            s += v * v;
        }
    }
    put_partial<256>(red, s);   // 0 from the work-groups beyond a smaller member
}

int norm_total_grid(long n)
{
    long b = (n + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

template <int N1>
static void launch_norm_total_k(const DgArgs& A, const double* U, Red red, hipStream_t st, const Mb& mb, dim3 grid)
{
    if (mb.tab) norm_total_kernel<N1, true><<<grid, dim3(256), 0, st>>>(A, mb.tab, U, red, mb.ms);
    else norm_total_kernel<N1, false><<<grid, dim3(256), 0, st>>>(A, nullptr, U, red, mb.ms);
}

void launch_norm2_total(int k, const DgArgs& A, const double* U, Red red, hipStream_t st, const Mb& mb)
{
    const long n = A.ne * (k + 1) * (k + 1);
    const dim3 grid(norm_total_grid(n), 1, mb.n);
    if (k == 1) launch_norm_total_k<2>(A, U, red, st, mb, grid);
    else if (k == 2) launch_norm_total_k<3>(A, U, red, st, mb, grid);
    else launch_norm_total_k<4>(A, U, red, st, mb, grid);
    launch_finalize(red.partials, (int)grid.x, 1, red.out, st, Gate{}, mb);
}

}  // namespace jfmg
