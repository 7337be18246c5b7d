// FV-subgrid multigrid kernels (paper Sec. "Multigrid preconditioner for
// finite volume approximations" and "Smoother / Pseudo time iteration").
//
// f_low on level l is the DG scheme with k = 0 on the subgrid: HLLC on the face
// total states (cell value + Ubar at the face), the k = 0 interior-penalty
// diffusion flux with penalty 1/h, and the gravity source.  The kernels carry
// the flux sum without the constant background-flux term, and each face's
// normal-momentum flux without the face's background pressure pb (the HLLC flux
// is affine in the pressure: F = F' + pb e_D, F' computed from p - pb); every
// use is a difference f(u + eps x) - f(u), in which those state-independent
// terms cancel, and the difference then loses digits only at the scale of
// p - pb and of the other fluxes, not at that of pb (about 10^5 Pa).
//
// Layout: SoA [4][nzl][nxl].  A work-group is a 64 x 4 tile of cells (one
// wave per row of 64 cells along x, so loads of a component are 256-byte
// coalesced); neighbours come through the caches.  Every kernel that produces
// a vector the next FD product needs also produces its squared norm through a
// deterministic two-level reduction.
#include "jfmg_internal.h"

namespace jfmg {

constexpr int FV_TX = 64, FV_TZ = 4, FV_NTH = FV_TX * FV_TZ;

enum { FVM_LIN = 0, FVM_STAGE = 1, FVM_MATVEC = 2, FVM_DEFECT = 3, FVM_STAGE_PC = 4, FVM_STAGE_TINV = 5 };

// Tile shapes of the FV operator kernels (jfmg_tile; chosen per level, by
// jfmg_autotune or by default):
//   64x4 / 256 threads: one wave per row of 64 cells (loads of a component are
//         512-byte rows); own-cell operands loaded after the face loop and at most
//         128 VGPRs, so four waves fit per SIMD
//   64x8 / 512 threads: the same with fewer halo faces per cell (2.14 vs 2.27)
//   16x4 / 256 threads: more threads than cells, so every face of the tile gets
//         its own thread (latency-bound narrow levels)
//   8x4 / 128 threads: the same with a quarter of the work per work-group
//   32x4 / 256 threads: two threads per cell (x-faces on the first threads,
//         z-faces from the last down), two waves per SIMD
//   64x4 / 512 threads: the 64x4 tile with two threads per cell (twice the waves
//         of the 256-thread form on a level too small to fill the chip)
// z-faces are handed out from the last thread down, so that the threads with a
// second x-face are not those with a second z-face.  Default by level width: 64x8
// from 1024 cells, 64x4 with 512 threads from 512, 16x4 from 256, 8x4 below (the
// autotuner's choice on the density-current levels 1024x256 ... 128x32; earlier
// measurements also ruled out 32x8, 16x4 with 128/192 threads, 64x4 with 2/3 waves
// per SIMD and early own-cell loads).

// Net flux through one face of a tile (HLLC minus the k = 0 interior-penalty diffusion
// flux, along +x or +z, times the face length) from the tile's staged states; face
// idx of the x-faces (XF) or z-faces in row-major order of the tile.
template <typename T, int TX, int TZ, int HZ, int HX, bool XF>
__device__ __forceinline__ void fv_face(const FvArgs<T>& A, const T (&sw)[4][HZ][HX], const T (&sBc)[TZ][6],
                                        const T (&sBf)[TZ + 1][10], T (&sFx)[TZ][TX + 1][4], T (&sFz)[TZ + 1][TX][4],
                                        int I0, int J0, int nxl, int nzl, int idx)
{
    constexpr int D = XF ? 1 : 2;   // normal momentum component
    int rl, cl, rr, cr, brow;       // LDS row/col of the low (L) and high (R) cell; background row of the tile
    bool skip, wallL, wallR;
    if constexpr (XF) {
        const int jj = idx / (TX + 1), fi = idx - jj * (TX + 1);
        const int Jf = J0 + jj, Ir = I0 + fi, Il = Ir - 1;
        skip = (Jf >= nzl) || (Il >= nxl);
        wallL = (Ir == 0) && A.bc != 1;
        wallR = (Il == nxl - 1) && A.bc != 1;
        rl = jj + 1; rr = jj + 1; cl = fi; cr = fi + 1;
        brow = jj;
    } else {
        const int fj = idx / TX, ii = idx - fj * TX;
        const int If = I0 + ii, Ja = J0 + fj, Jb = Ja - 1;
        skip = (If >= nxl) || (Jb >= nzl);
        wallL = (Jb < 0);
        wallR = (Ja == nzl);
        rl = fj; rr = fj + 1; cl = ii + 1; cr = ii + 1;
        brow = fj;
    }
    T Phi[4] = {T(0), T(0), T(0), T(0)};
    if (!skip) {
        const T* bg = XF ? &sBc[brow][0] : &sBf[brow][0];   // Ubar, then p, 1/(rho theta)
        const T* pr = bg + 4;
        const bool wall = wallL || wallR;
        // a slip wall: the missing side is the inside cell mirrored (normal momentum negated)
        const int rlx = wallL ? rr : rl, clx = wallL ? cr : cl;
        const int rrx = wallR ? rl : rr, crx = wallR ? cl : cr;
        T wL[4], wR[4], UL[4], UR[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            wL[c] = sw[c][rlx][clx];
            wR[c] = sw[c][rrx][crx];
            UL[c] = wL[c] + bg[c];
            UR[c] = wR[c] + bg[c];
        }
        if (wallL) UL[D] = -UL[D];
        if (wallR) UR[D] = -UR[D];
        const T pb = pr[0], irb = pr[1];
        // the face's background pressure is left out of the flux (see the file comment)
        const T dpL = pert_dpress(A.gas, wL[3], irb, pb), dpR = pert_dpress(A.gas, wR[3], irb, pb);
        const T pL = pb + dpL, pR = pb + dpR;
        const T irL = frcp<T>(UL[0]), irR = frcp<T>(UR[0]);
        hllc_ax_dp<T, D>(A.gas, UL, UR, pL, pR, dpL, dpR, irL, irR, Phi);
        if (A.physics == 1 && !wall) {
            // k = 0 diffusion: mean of mu (G_c - (U_c/rho) G_rho) over both sides, where the
            // only gradient is the background's (z-faces), minus the interior penalty
            // (mu/h) (dw_c - (U_c/rho)_avg dw_rho), dw = w_L - w_R, on the averaged state
            const T irs = frcp<T>(UL[0] + UR[0]);
            const T muh = A.mu / (XF ? A.hx : A.hz);
            const T* dbg = &sBf[brow][6];
            const T dw0 = wL[0] - wR[0];
#pragma unroll
            for (int c = 1; c < 4; ++c) {
                if constexpr (!XF) {
                    const T fl = A.mu * (dbg[c] - UL[c] * irL * dbg[0]);
                    const T fr = A.mu * (dbg[c] - UR[c] * irR * dbg[0]);
                    Phi[c] -= T(0.5) * (fl + fr);
                }
                const T rr = (UL[c] + UR[c]) * irs;
                Phi[c] += muh * ((wL[c] - wR[c]) - rr * dw0);
            }
        }
        const T elen = XF ? A.hz : A.hx;
#pragma unroll
        for (int c = 0; c < 4; ++c) Phi[c] *= elen;
    }
    if constexpr (XF) {
        const int jj = idx / (TX + 1), fi = idx - jj * (TX + 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) sFx[jj][fi][c] = Phi[c];
    } else {
        const int fj = idx / TX, ii = idx - fj * TX;
#pragma unroll
        for (int c = 0; c < 4; ++c) sFz[fj][ii][c] = Phi[c];
    }
}

// FV operator on one tile of TX x TZ cells, face-centric: the perturbed states
// w = u + eps x of the tile and a one-cell halo are staged in LDS, every face
// of the tile gets its net flux Phi (HLLC minus the interior-penalty diffusion
// flux, along +x or +z) exactly once, and each cell then sums its four faces:
//   |q| f~ = -hz (Phi_{I+1/2} - Phi_{I-1/2}) - hx (Phi_{J+1/2} - Phi_{J-1/2}) - |q| g w_rho.
// The flux through a face seen from the other cell is the same number with
// the opposite sign (HLLC(L,R;n) = -HLLC(R,L;-n)).  Modes:
//   LIN     out = F0 = f~(u); ||u + Ubar||^2 and max(|v| + c) block partials (the level
//           slots and dtau from them: fv_lin_finalize_kernel); with out2 also the next coarser
//           level's state R u
//   STAGE   out = x0 + alpha_j dtau (b - g'x), g'x = x - adt/eps (f~(u + eps x) - F0)
//   MATVEC  out = g'x
//   DEFECT  out(coarse) = R(g'x - b), 2x2 agglomeration inside the tile; with out2 also
//           the coarse level's first RK stage from zero, out2 = alpha_j dtau_c out (dtau_c in
//           slots2), and its ||.||^2 block partials into red
//   STAGE_PC the STAGE result v is not stored: it corrects the next finer level's x in
//           out2 by injection, x_f -= P v (x_f = -P v when fzero is set, x_f being zero), with the
//           ||x_f||^2 block partials into red (the last smoother stage of a coarse level)
//   STAGE_TINV (finest level, tiles of whole DG elements) the STAGE result v is not stored:
//           the tile's elements are transferred back to the DG space, tv.z = T^-1 v with the
//           mass fix when tv.mass_fix is set (the arithmetic of transfer_Tinv_kernel), with the
//           ||z||^2 block partials into red (the last smoother stage of the cycle)
template <typename T, int TX, int TZ, int NTH, int WPE, bool LATE, bool ZREV, bool MB, int MODE, bool RG>
__global__ void __launch_bounds__(NTH, WPE)
fv_tile_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, const T* __restrict__ u, const T* __restrict__ F0,
               const T* __restrict__ xp,
               const T* __restrict__ x0, const T* __restrict__ b, T* __restrict__ out, T* __restrict__ out2,
               const double* __restrict__ xpart, int xcount, double* __restrict__ slots,
               const double* __restrict__ slots2, double alpha_j, double adt, int fzero, Red red, long ms,
               TinvOut tv)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    if constexpr (MB) {   // member blockIdx.z of a lock-step batch
        u = mbr(u, ms);
        F0 = mbr(F0, ms);
        xp = mbr(xp, ms);
        x0 = mbr(x0, ms);
        b = mbr(b, ms);
        out = mbr(out, ms);
        out2 = mbr(out2, ms);
        slots2 = mbr(slots2, ms);
        xpart = mbr(xpart, ms);
        slots = mbr(slots, ms);
        red = mbr(red, ms);
    }
    double* const zout = MB ? mbr(tv.z, ms) : tv.z;   // STAGE_TINV output (tv stays in the arguments)
    constexpr int NCELL = TX * TZ, HX = TX + 2, HZ = TZ + 2;
    constexpr int NH = HX * HZ, HITEMS = (NH + NTH - 1) / NTH;
    constexpr int NFX = TZ * (TX + 1), NFZ = (TZ + 1) * TX;
    constexpr bool PERT = (MODE != FVM_LIN);
    constexpr bool STG = (MODE == FVM_STAGE || MODE == FVM_STAGE_PC || MODE == FVM_STAGE_TINV);
    constexpr bool TI = (MODE == FVM_STAGE_TINV);
    static_assert(NTH >= NCELL && NTH % 64 == 0, "tile shape");
    __shared__ T sw[4][HZ][HX];
    __shared__ T sFx[TZ][TX + 1][4];
    __shared__ T sFz[TZ + 1][TX][4];
    // background of the tile's rows: cell centres [Ubar(4), p, 1/(rho theta)], z-faces
    // [Ubar(4), p, 1/(rho theta), dUbar/dz(4)]
    __shared__ T sBc[TZ][6];
    __shared__ T sBf[TZ + 1][10];
    // STAGE_TINV: V^-1, the Newton-Cotes weights and the first contraction of T^-1
    __shared__ double sVi[TI ? MAXN1 : 1][MAXN1], sWn[TI ? MAXN1 : 1];
    __shared__ double sHt[TI ? 4 : 1][TI ? TZ : 1][TI ? TX : 1];
    const int tid = threadIdx.x;
    const long nc = A.nc;
    const int nxl = A.nxl, nzl = A.nzl;
    // tiles of this member (a one-dimensional grid; in a ragged batch the work-groups
    // beyond a smaller member's tiles only store zero partial sums)
    const unsigned ntx = (unsigned)((nxl + TX - 1) / TX), ntiles = ntx * (unsigned)((nzl + TZ - 1) / TZ);
    if (blockIdx.x >= ntiles || (RG && sits_out(mt))) {
        if (tid == 0) {
            if constexpr (MODE == FVM_LIN) {
                red.partials[blockIdx.x] = 0.0;
                red.partials[gridDim.x + blockIdx.x] = 0.0;
            } else if constexpr (STG) {
                red.partials[blockIdx.x] = 0.0;
            } else if constexpr (MODE == FVM_DEFECT) {
                if (out2) red.partials[blockIdx.x] = 0.0;
            }
        }
        return;
    }
    const unsigned tile = xcd_tile(blockIdx.x, ntiles);
    const int I0 = (int)(tile % ntx) * TX, J0 = (int)(tile / ntx) * TZ;
    // own cell (threads tid < NCELL)
    const int ti = tid % TX, tj = tid / TX;
    const int I = I0 + ti, J = J0 + tj;
    const bool valid = tid < NCELL && I < nxl && J < nzl;
    const long q = (long)J * nxl + I;

    // ---- every global load first (the level's scalars and background rows, the
    // own-cell operands, then the halo states), or the own-cell operands only after
    // the face loop (LATE: fewer live registers).  Nothing below waits on memory
    // before the partial sums of ||x||^2 have arrived. ----
    double s_utot = 0.0, s_iutot = 0.0, s_dtau = 0.0;
    if constexpr (PERT) {
        s_utot = slots[LV_UTOT];
        s_iutot = slots[LV_IUTOT];
    }
    if constexpr (STG) s_dtau = slots[LV_DTAU];
    if constexpr (TI) {
        if (tid < MAXN1 * MAXN1) sVi[tid / MAXN1][tid % MAXN1] = tv.Vinv[tid / MAXN1][tid % MAXN1];
        else if (tid < MAXN1 * MAXN1 + MAXN1) sWn[tid - MAXN1 * MAXN1] = tv.wnc[tid - MAXN1 * MAXN1];
    }
    if constexpr (MODE == FVM_DEFECT) s_dtau = out2 ? slots2[LV_DTAU] : 0.0;
    static_assert(NTH >= 6 * TZ + 10 * (TZ + 1), "background staging");
    T bg_v = T(0);   // this thread's entry of sBc / sBf
    if (tid < 6 * TZ) {
        const int r = tid / 6, k = tid - 6 * r, Jr = J0 + r;
        if (Jr < nzl) bg_v = k < 4 ? A.bgc[4 * Jr + k] : A.pc[2 * Jr + k - 4];
    } else if (tid < 6 * TZ + 10 * (TZ + 1)) {
        const int t2 = tid - 6 * TZ, r = t2 / 10, k = t2 - 10 * r, Jr = J0 + r;
        if (Jr <= nzl) bg_v = k < 4 ? A.bgf[4 * Jr + k] : k < 6 ? A.pf[2 * Jr + k - 4] : A.dbgf[4 * Jr + k - 6];
    }
    T own_x[4] = {T(0), T(0), T(0), T(0)}, own_f0[4] = {T(0), T(0), T(0), T(0)};
    T own_b[4] = {T(0), T(0), T(0), T(0)}, own_x0[4] = {T(0), T(0), T(0), T(0)};
    // STAGE_PC: the finer level's four children of the cell, read with the own-cell
    // operands (before any of them is written)
    T own_xf[4][4] = {};
    auto load_own = [&]() {
        if (valid) {
            if constexpr (MODE == FVM_STAGE_PC)
                if (!fzero) {
                    const long nxf = 2L * nxl, ncf = 4 * nc;
                    const long q00 = (long)(2 * J) * nxf + 2 * I, q10 = q00 + nxf;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const T* xf = out2 + c * ncf;
                        own_xf[c][0] = xf[q00]; own_xf[c][1] = xf[q00 + 1];
                        own_xf[c][2] = xf[q10]; own_xf[c][3] = xf[q10 + 1];
                    }
                }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (PERT) { own_x[c] = xp[c * nc + q]; own_f0[c] = F0[c * nc + q]; }
                if constexpr (STG || MODE == FVM_DEFECT)
                    own_b[c] = b[c * nc + q];
                // the first stage of a sweep has x^(0) = x^(j-1): no second load (the copy
                // is taken where x^(0) is used, so that no load waits for another)
                if constexpr (STG)
                    if (x0 && x0 != xp) own_x0[c] = x0[c * nc + q];
            }
        }
    };
    if constexpr (!LATE) load_own();
    T hu[HITEMS][4], hx[HITEMS][4];
#pragma unroll
    for (int it = 0; it < HITEMS; ++it) {
        const int h = tid + it * NTH;
        int Ih = I0 - 1 + h % HX;
        const int Jh = J0 - 1 + h / HX;
        bool ok = h < NH && Jh >= 0 && Jh < nzl;
        if (Ih < 0 || Ih >= nxl) {
            if (A.bc == 1) Ih = (Ih + nxl) % nxl;
            else ok = false;
        }
        const long qh = (long)Jh * nxl + Ih;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            hu[it][c] = ok ? u[c * nc + qh] : T(0);
            if constexpr (PERT) hx[it][c] = ok ? xp[c * nc + qh] : T(0);
        }
    }
    // eps = sqrt(eps_p) ||u + Ubar|| / ||x|| and adt / eps, from ||x|| and the stored 1/||u + Ubar||
    T eps = T(0), sc = T(0);
    bool xzero = false;   // uniform: g'x = 0 for x = 0
    if constexpr (PERT) {
        const double xn2 = sum_partials<NTH>(xpart, xcount);   // ||x||^2, same order in every block
        if (!(xn2 > 0.0)) {
            xzero = true;
        } else {
            const double xn = psqrt(xn2);
            eps = (T)(FdEps<T>::sqrt_eps * s_utot * frcp(xn));
            sc = (T)(adt * xn * (FdEps<T>::inv_sqrt_eps * s_iutot));
        }
    }

    if (!xzero) {
#pragma unroll
        for (int it = 0; it < HITEMS; ++it) {
            const int h = tid + it * NTH;
            if (h < NH)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    T v = hu[it][c];
                    if constexpr (PERT) v = v + eps * hx[it][c];
                    sw[c][h / HX][h % HX] = v;
                }
        }
        if (tid < 6 * TZ) {
            const int r = tid / 6, k = tid - 6 * r;
            if (J0 + r < nzl) sBc[r][k] = bg_v;
        } else if (tid < 6 * TZ + 10 * (TZ + 1)) {
            const int t2 = tid - 6 * TZ, r = t2 / 10, k = t2 - 10 * r;
            if (J0 + r <= nzl) sBf[r][k] = bg_v;
        }
        __syncthreads();
        // ---- one net flux per face: x-faces in thread order, z-faces in reverse
        // thread order (the threads with a second x-face are not those with a
        // second z-face) ----
        auto face = [&](auto xf_tag, int idx) {
            fv_face<T, TX, TZ, HZ, HX, decltype(xf_tag)::value>(A, sw, sBc, sBf, sFx, sFz, I0, J0, nxl, nzl, idx);
        };
        for (int fx = tid; fx < NFX; fx += NTH) face(std::true_type{}, fx);
        if constexpr (ZREV)   // z-faces from the last thread down
            for (int fz = NTH - 1 - tid; fz < NFZ; fz += NTH) face(std::false_type{}, fz);
        else                  // z-faces continue the numbering after the x-faces
            for (int fz = (tid + NTH - NFX % NTH) % NTH; fz < NFZ; fz += NTH) face(std::false_type{}, fz);
        if constexpr (LATE) load_own();
        __syncthreads();
    } else if constexpr (LATE) {
        load_own();
    }

    // ---- per cell ----
    T f[4] = {T(0), T(0), T(0), T(0)};
    if (valid && !xzero) {
        const T iarea = A.iarea;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            T L = -(sFx[tj][ti + 1][c] - sFx[tj][ti][c]) - (sFz[tj + 1][ti][c] - sFz[tj][ti][c]);
            if (c == 2) L += A.area * (-A.g * sw[0][tj + 1][ti + 1]);
            f[c] = L * iarea;
        }
    }
    if constexpr (MODE == FVM_LIN) {
        // with out2: the next coarser level's state R u from the staged tile (the 2 x 2
        // means of fv_restrict_kernel, in its order)
        if (out2 && valid && !(ti & 1) && !(tj & 1)) {
            const int nxc = nxl / 2;
            const long ncc = (long)nxc * (nzl / 2), qc = (long)(J / 2) * nxc + I / 2;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                out2[c * ncc + qc] =
                    ((sw[c][tj + 1][ti + 1] + sw[c][tj + 1][ti + 2]) + (sw[c][tj + 2][ti + 1] + sw[c][tj + 2][ti + 2])) * T(0.25);
        }
        double ss = 0.0, lam = 0.0;
        if (valid) {
            T Ut[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                out[c * nc + q] = f[c];   // F0
                Ut[c] = u[c * nc + q] + A.bgc[4 * J + c];
                ss += (double)Ut[c] * (double)Ut[c];
            }
            const double rho = Ut[0], uu = Ut[1] / rho, ww = Ut[2] / rho;
            const double p = (double)A.gas.p0 * pow((double)A.gas.R * (double)Ut[3] / (double)A.gas.p0,
                                                    (double)A.gas.gamma);
            lam = sqrt(uu * uu + ww * ww) + sqrt((double)A.gas.gamma * p / rho);
        }
        __shared__ double sh[NTH / 64];
        const double bs = block_sum<NTH>(ss, sh);
        const double bm = block_max<NTH>(lam, sh);
        if (tid == 0) {
            red.partials[blockIdx.x] = bs;
            red.partials[gridDim.x + blockIdx.x] = bm;
        }
        return;
    } else {
        T Ax[4] = {T(0), T(0), T(0), T(0)};
        if (valid && !xzero) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Ax[c] = own_x[c] - sc * (f[c] - own_f0[c]);
        }
        if constexpr (MODE == FVM_MATVEC) {
            if (valid)
#pragma unroll
                for (int c = 0; c < 4; ++c) out[c * nc + q] = Ax[c];
        } else if constexpr (MODE == FVM_STAGE) {
            double nrm = 0.0;
            if (valid) {
                const T s = (T)(alpha_j * s_dtau);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const T v = (x0 == xp ? own_x[c] : own_x0[c]) + s * (own_b[c] - Ax[c]);
                    out[c * nc + q] = v;
                    nrm += (double)v * (double)v;
                }
            }
            put_partial<NTH>(red, nrm);
        } else if constexpr (MODE == FVM_STAGE_PC) {
            double nrm = 0.0;
            if (valid) {
                const T s = (T)(alpha_j * s_dtau);
                const long nxf = 2L * nxl, ncf = 4 * nc;
                const long q00 = (long)(2 * J) * nxf + 2 * I, q10 = q00 + nxf;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const T v = (x0 == xp ? own_x[c] : own_x0[c]) + s * (own_b[c] - Ax[c]);
                    T* xf = out2 + c * ncf;
                    T f00 = -v, f01 = -v, f10 = -v, f11 = -v;
                    if (!fzero) {
                        f00 = own_xf[c][0] - v; f01 = own_xf[c][1] - v;
                        f10 = own_xf[c][2] - v; f11 = own_xf[c][3] - v;
                    }
                    xf[q00] = f00; xf[q00 + 1] = f01;
                    xf[q10] = f10; xf[q10 + 1] = f11;
                    nrm += ((double)f00 * (double)f00 + (double)f01 * (double)f01) +
                           ((double)f10 * (double)f10 + (double)f11 * (double)f11);
                }
            }
            put_partial<NTH>(red, nrm);
        } else if constexpr (MODE == FVM_STAGE_TINV) {
            T v[4] = {T(0), T(0), T(0), T(0)};
            if (valid) {
                const T s = (T)(alpha_j * s_dtau);
#pragma unroll
                for (int c = 0; c < 4; ++c) v[c] = (x0 == xp ? own_x[c] : own_x0[c]) + s * (own_b[c] - Ax[c]);
            }
            __syncthreads();   // the staged states are read no more: the tile of v replaces them
            if (valid)
#pragma unroll
                for (int c = 0; c < 4; ++c) sw[c][tj][ti] = v[c];
            __syncthreads();
            // T^-1 with k + 1 = N1 known at compile time (tiles of whole elements: N1 = 2 or 4)
            double nrm = 0.0;
            auto tinv = [&](auto n1c) {
                constexpr int N1 = decltype(n1c)::value, NP = N1 * N1;
                // first contraction, one thread per subcell (a, bb) of its element:
                // h_{bb,a} = sum_i Vinv_ai t_{i,bb}
                // the element sums of the mass fix (mean and Newton-Cotes quadrature of each
                // component, each in the order of transfer_Tinv_kernel) in the flux rows, which
                // the cell sums have finished reading: one (sum, component) pair per thread
                constexpr int NEX = TX / N1, NEL = NEX * (TZ / N1);
                static_assert(8 * NEL * sizeof(double) <= sizeof(sFz), "element sums");
                double* const sSum = reinterpret_cast<double*>(&sFz[0][0][0]);   // [8][NEL]
                if (valid) {
                    const int a = ti % N1, ea = ti - a, b1 = tj % N1, eb = tj - b1;
                    double va[N1];
#pragma unroll
                    for (int ii = 0; ii < N1; ++ii) va[ii] = sVi[a][ii];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        double s = 0.0;
#pragma unroll
                        for (int ii = 0; ii < N1; ++ii) s += va[ii] * (double)sw[c][tj][ea + ii];
                        sHt[c][tj][ti] = s;
                    }
                    if (tv.mass_fix) {
                        const int el = (eb / N1) * NEX + ea / N1;
                        for (int qs = b1 * N1 + a; qs < 8; qs += NP) {
                            const int c = qs & 3;
                            double acc = 0.0;
                            if (qs < 4) {
#pragma unroll
                                for (int jj = 0; jj < N1; ++jj)
#pragma unroll
                                    for (int ii = 0; ii < N1; ++ii) acc += (double)sw[c][eb + jj][ea + ii];
                            } else {
#pragma unroll
                                for (int jj = 0; jj < N1; ++jj)
#pragma unroll
                                    for (int ii = 0; ii < N1; ++ii) {
                                        const double w = sw[c][eb + jj][ea + ii];
                                        acc += sWn[ii] * sWn[jj] * w;
                                    }
                            }
                            sSum[qs * NEL + el] = acc;
                        }
                    }
                }
                __syncthreads();
                // second contraction and mass fix, one thread per DG node in the order of the
                // DG vector (the tile's elements of one element row are consecutive there)
                constexpr int ROW = TX * N1;   // nodes of one element row of the tile
                if (tid < NCELL) {
                    const int er = tid / ROW, rem = tid - er * ROW, el = rem / NP, nd = rem - el * NP;
                    const int a = nd % N1, bb = nd / N1, ea = el * N1, eb = er * N1;
                    if (I0 + ea < nxl && J0 + eb < nzl) {
                        const long e = (long)((J0 + eb) / N1) * (nxl / N1) + (I0 + ea) / N1;
                        double vb[N1];
#pragma unroll
                        for (int jj = 0; jj < N1; ++jj) vb[jj] = sVi[bb][jj];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            double s = 0.0;
#pragma unroll
                            for (int jj = 0; jj < N1; ++jj) s += vb[jj] * sHt[c][eb + jj][ea + a];
                            double shift = 0.0;
                            if (tv.mass_fix) {
                                const int el2 = er * NEX + el;
                                shift = sSum[(4 + c) * NEL + el2] - sSum[c * NEL + el2] / NP;
                            }
                            const double z = s - shift;
                            zout[c * nc + e * NP + nd] = z;   // the DG vector has nc nodes per component
                            nrm += z * z;
                        }
                    }
                }
            };
            if (tv.n1 == 4) tinv(std::integral_constant<int, 4>{});
            else tinv(std::integral_constant<int, 2>{});
            put_partial<NTH>(red, nrm);
        } else {   // DEFECT: reuse the state tile for d = g'x - b, then agglomerate 2x2
            __syncthreads();
            if (valid)
#pragma unroll
                for (int c = 0; c < 4; ++c) sw[c][tj][ti] = Ax[c] - own_b[c];
            __syncthreads();
            double nrm = 0.0;
            if (valid && !(ti & 1) && !(tj & 1)) {
                const int nxc = nxl / 2;
                const long ncc = (long)nxc * (nzl / 2), qc = (long)(J / 2) * nxc + I / 2;
                const T s1 = out2 ? (T)(alpha_j * s_dtau) : T(0);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const T r = ((sw[c][tj][ti] + sw[c][tj][ti + 1]) + (sw[c][tj + 1][ti] + sw[c][tj + 1][ti + 1])) * T(0.25);
                    out[c * ncc + qc] = r;
                    if (out2) {
                        const T v = s1 * r;
                        out2[c * ncc + qc] = v;
                        nrm += (double)v * (double)v;
                    }
                }
            }
            if (out2) put_partial<NTH>(red, nrm);
        }
    }
}

// first stage of a sweep from x = 0: out = alpha_1 dtau b, with ||out||^2
template <typename T, bool RG>
__global__ void __launch_bounds__(256)
fv_stage_zero_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, const T* __restrict__ b, T* __restrict__ out,
                     const double* __restrict__ slots, double alpha_j, Red red, long ms)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    b = mbr(b, ms);
    out = mbr(out, ms);
    slots = mbr(slots, ms);
    red = mbr(red, ms);
    const long n = sits_out(mt) ? 0 : 4 * A.nc;
    const long nb = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;   // this member's work-groups
    const T s = (T)(alpha_j * slots[LV_DTAU]);
    double nrm = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) {
        const T v = s * b[i];
        out[i] = v;
        nrm += (double)v * (double)v;
    }
    put_partial<256>(red, nrm);
}

// coarse = R(-b): the defect of x = 0
template <typename T, bool RG>
__global__ void __launch_bounds__(256)
fv_restrict_neg_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, const T* __restrict__ f, T* __restrict__ c,
                       long ms)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    if (RG && sits_out(mt)) return;
    f = mbr(f, ms);
    c = mbr(c, ms);
    const int nxc = A.nxl / 2, nzc = A.nzl / 2;
    const int Ic = blockIdx.x * 64 + (threadIdx.x & 63);
    const int Jc = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (Ic >= nxc || Jc >= nzc) return;
    const long ncc = (long)nxc * nzc, qc = (long)Jc * nxc + Ic;
    const long q00 = (long)(2 * Jc) * A.nxl + 2 * Ic, q01 = q00 + A.nxl;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        const T* g = f + cc * A.nc;
        c[cc * ncc + qc] = ((-g[q00] + -g[q00 + 1]) + (-g[q01] + -g[q01 + 1])) * T(0.25);
    }
}

// x -= P v (injection) on the fine level, with ||x||^2
template <typename T, bool RG>
__global__ void __launch_bounds__(FV_NTH)
fv_prolong_correct_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, T* __restrict__ x, const T* __restrict__ v,
                          Red red, long ms)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    x = mbr(x, ms);
    v = mbr(v, ms);
    red = mbr(red, ms);
    // a one-dimensional grid over this member's 64 x 4 tiles (row-major)
    const unsigned gx = (unsigned)((A.nxl + FV_TX - 1) / FV_TX), nt = gx * (unsigned)((A.nzl + FV_TZ - 1) / FV_TZ);
    if (blockIdx.x >= nt || sits_out(mt)) {   // beyond a smaller member, or one that sits out
        if (threadIdx.x == 0) red.partials[blockIdx.x] = 0.0;
        return;
    }
    const int I = (blockIdx.x % gx) * FV_TX + (threadIdx.x & (FV_TX - 1));
    const int J = (blockIdx.x / gx) * FV_TZ + (threadIdx.x / FV_TX);
    double nrm = 0.0;
    if (I < A.nxl && J < A.nzl) {
        const long q = (long)J * A.nxl + I;
        const long ncc = (long)(A.nxl / 2) * (A.nzl / 2), qc = (long)(J / 2) * (A.nxl / 2) + I / 2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T val = x[c * A.nc + q] - v[c * ncc + qc];
            x[c * A.nc + q] = val;
            nrm += (double)val * (double)val;
        }
    }
    put_partial<FV_NTH>(red, nrm);
}

template <typename T, bool RG>
__global__ void __launch_bounds__(FV_NTH)
fv_restrict_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, const T* __restrict__ f, T* __restrict__ c, long ms)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    if (RG && sits_out(mt)) return;
    f = mbr(f, ms);
    c = mbr(c, ms);
    const int nxc = A.nxl / 2, nzc = A.nzl / 2;
    const int Ic = blockIdx.x * FV_TX + (threadIdx.x & (FV_TX - 1));
    const int Jc = blockIdx.y * FV_TZ + (threadIdx.x / FV_TX);
    if (Ic >= nxc || Jc >= nzc) return;
    const long ncc = (long)nxc * nzc, qc = (long)Jc * nxc + Ic;
    const long q00 = (long)(2 * Jc) * A.nxl + 2 * Ic, q01 = q00 + A.nxl;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        const T* g = f + cc * A.nc;
        c[cc * ncc + qc] = ((g[q00] + g[q00 + 1]) + (g[q01] + g[q01 + 1])) * T(0.25);
    }
}

template <typename T, bool RG>
__global__ void __launch_bounds__(FV_NTH)
fv_prolong_kernel(FvArgs<T> Aa, const MemberArgs* __restrict__ mt, const T* __restrict__ c, T* __restrict__ f, long ms)
{
    const FvArgs<T>& A = fv_of<T, RG>(Aa, mt);
    if (RG && sits_out(mt)) return;
    c = mbr(c, ms);
    f = mbr(f, ms);
    const int I = blockIdx.x * FV_TX + (threadIdx.x & (FV_TX - 1));
    const int J = blockIdx.y * FV_TZ + (threadIdx.x / FV_TX);
    if (I >= A.nxl || J >= A.nzl) return;
    const long q = (long)J * A.nxl + I;
    const long ncc = (long)(A.nxl / 2) * (A.nzl / 2), qc = (long)(J / 2) * (A.nxl / 2) + I / 2;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) f[cc * A.nc + q] = c[cc * ncc + qc];
}

template <typename T>
__global__ void __launch_bounds__(256) fv_norm2_kernel(const T* __restrict__ x, long n, Red red, long ms)
{
    x = mbr(x, ms);
    red = mbr(red, ms);
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double v = x[i];
        s += v * v;
    }
    put_partial<256>(red, s);
}

// level slots from the LIN partials: ||u + Ubar||, max(|v| + c), pseudo time step
// The slots of every level from the LIN partials (one work-group per level, level l's
// 2 x nb[l] partials at p + l * pstride): ||u + Ubar||, its inverse, max(|v| + c), dtau
template <typename T>
__global__ void __launch_bounds__(256)
fv_lin_finalize_kernel(const double* __restrict__ p, long pstride, LinLevels lv, double* __restrict__ slots,
                       double mu, double adt, double cfl, long ms, const MemberArgs* __restrict__ mt)
{
    const int lev = blockIdx.x;
    p = mbr(p, ms) + lev * pstride;
    slots = mbr(slots, ms) + 4 * lev;
    const int nb = lv.nb[lev];
    double hx = lv.hx[lev], hz = lv.hz[lev];
    if (mt) {   // a ragged member's own cell widths
        const FvArgs<T>& A = fv_entry<T>(mt, lev);
        hx = (double)A.hx;
        hz = (double)A.hz;
    }
    __shared__ double sh[4];
    double a = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) { a += p[i]; m = fmax(m, p[nb + i]); }
    a = block_sum<256>(a, sh);
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) {
        slots[LV_UTOT] = sqrt(a);
        slots[LV_IUTOT] = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
        slots[LV_LAM] = m;
        slots[LV_DTAU] = cfl / (1.0 + adt * (m * (1.0 / hx + 1.0 / hz) + 2.0 * mu * (1.0 / (hx * hx) + 1.0 / (hz * hz))));
    }
}

static inline dim3 tile_grid(int nx, int nz, int members = 1)
{
    return dim3((unsigned)((nx + FV_TX - 1) / FV_TX), (unsigned)((nz + FV_TZ - 1) / FV_TZ), (unsigned)members);
}
// the same 64 x 4 tiles as a one-dimensional grid
static inline dim3 tile_grid_1d(int nx, int nz, int members = 1)
{
    const dim3 g = tile_grid(nx, nz);
    return dim3(g.x * g.y, 1, (unsigned)members);
}

template <typename T, int TX, int TZ, int NTH, int WPE, bool LATE, bool ZREV, int MODE>
static int tile_launch_shape(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b,
                             T* out, T* out2, const double* xpart, int xcount, double* slots, const double* slots2,
                             double alpha_j, double adt, int fzero, Red red, hipStream_t st, const Mb& mb,
                             const TinvOut& tv)
{
    const unsigned nt = (unsigned)((A.nxl + TX - 1) / TX) * (unsigned)((A.nzl + TZ - 1) / TZ);
    const dim3 g(nt, 1, (unsigned)mb.n);
    if (mb.tab)
        timed_launch(fv_tile_kernel<T, TX, TZ, NTH, WPE, LATE, ZREV, true, MODE, true>, g, dim3(NTH), st, A, mb.tab, u,
                     F0, xp, x0, b, out, out2, xpart, xcount, slots, slots2, alpha_j, adt, fzero, red, mb.ms, tv);
    else if (mb.n > 1)
        timed_launch(fv_tile_kernel<T, TX, TZ, NTH, WPE, LATE, ZREV, true, MODE, false>, g, dim3(NTH), st, A, mb.tab,
                     u, F0, xp, x0, b, out, out2, xpart, xcount, slots, slots2, alpha_j, adt, fzero, red, mb.ms, tv);
    else
        timed_launch(fv_tile_kernel<T, TX, TZ, NTH, WPE, LATE, ZREV, false, MODE, false>, g, dim3(NTH), st, A, mb.tab,
                     u, F0, xp, x0, b, out, out2, xpart, xcount, slots, slots2, alpha_j, adt, fzero, red, 0L, tv);
    return (int)nt;
}

template <typename T, int MODE>
static int tile_launch(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b, T* out,
                       const double* xpart, int xcount, double* slots, double alpha_j, double adt, int fzero,
                       Red red, hipStream_t st, const Mb& mb, T* out2 = nullptr, const double* slots2 = nullptr,
                       const TinvOut& tv = TinvOut{})
{
    switch (A.tile) {
    case JFMG_TILE_64x8:
        return tile_launch_shape<T, 64, 8, 512, 4, true, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                       slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    case JFMG_TILE_16x4:
        return tile_launch_shape<T, 16, 4, 256, 1, false, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                        slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    case JFMG_TILE_8x4:
        return tile_launch_shape<T, 8, 4, 128, 1, false, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                       slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    case JFMG_TILE_32x4:
        return tile_launch_shape<T, 32, 4, 256, 2, false, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                        slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    case JFMG_TILE_64x4_512:
        return tile_launch_shape<T, 64, 4, 512, 4, true, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                       slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    default:
        return tile_launch_shape<T, 64, 4, 256, 4, true, true, MODE>(A, u, F0, xp, x0, b, out, out2, xpart, xcount,
                                                                       slots, slots2, alpha_j, adt, fzero, red, st, mb, tv);
    }
}

template <typename T>
int FvLaunch<T>::lin_level(const FvArgs<T>& A, const T* u, T* F0, T* uc, Red red, double adt, hipStream_t st,
                           const Mb& mb)
{
    return tile_launch<T, FVM_LIN>(A, u, nullptr, nullptr, nullptr, nullptr, F0, nullptr, 0, nullptr, 0.0, adt, 0, red,
                                   st, mb, uc);
}
template <typename T>
void FvLaunch<T>::lin_finalize(const double* partials, long pstride, const LinLevels& lv, int nlev, double* slots,
                               double mu, double adt, double cfl, hipStream_t st, const Mb& mb)
{
    fv_lin_finalize_kernel<T><<<dim3(nlev, 1, mb.n), dim3(256), 0, st>>>(partials, pstride, lv, slots, mu, adt, cfl,
                                                                         mb.ms, mb.tab);
}
template <typename T>
int FvLaunch<T>::stage(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b, T* xo,
                       const double* xpart, int xcount, const double* slots, double alpha_j, double adt, int zero,
                       Red red, hipStream_t st, const Mb& mb)
{
    if (zero) {
        const long n = 4 * A.nc;
        const int nb = norm_blocks(n);
        if (mb.tab)
            timed_launch(fv_stage_zero_kernel<T, true>, dim3(nb, 1, mb.n), dim3(256), st, A, mb.tab, b, xo, slots,
                         alpha_j, red, mb.ms);
        else
            timed_launch(fv_stage_zero_kernel<T, false>, dim3(nb, 1, mb.n), dim3(256), st, A, mb.tab, b, xo, slots,
                         alpha_j, red, mb.ms);
        return nb;
    }
    return tile_launch<T, FVM_STAGE>(A, u, F0, xp, x0, b, xo, xpart, xcount, const_cast<double*>(slots), alpha_j,
                                     adt, 0, red, st, mb);
}
template <typename T>
int FvLaunch<T>::stage_prolong(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b,
                               T* xf, bool fine_zero, const double* xpart, int xcount, const double* slots,
                               double alpha_j, double adt, Red red, hipStream_t st, const Mb& mb)
{
    return tile_launch<T, FVM_STAGE_PC>(A, u, F0, xp, x0, b, nullptr, xpart, xcount, const_cast<double*>(slots),
                                        alpha_j, adt, fine_zero ? 1 : 0, red, st, mb, xf);
}
template <typename T>
int FvLaunch<T>::stage_tinv(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b,
                            const TinvOut& tv, const double* xpart, int xcount, const double* slots, double alpha_j,
                            double adt, Red red, hipStream_t st, const Mb& mb)
{
    return tile_launch<T, FVM_STAGE_TINV>(A, u, F0, xp, x0, b, nullptr, xpart, xcount, const_cast<double*>(slots),
                                          alpha_j, adt, 0, red, st, mb, nullptr, nullptr, tv);
}
template <typename T>
void FvLaunch<T>::matvec(const FvArgs<T>& A, const T* u, const T* F0, const T* x, T* out, const double* xpart,
                         int xcount, const double* slots, double adt, hipStream_t st, const Mb& mb)
{
    tile_launch<T, FVM_MATVEC>(A, u, F0, x, nullptr, nullptr, out, xpart, xcount, const_cast<double*>(slots), 0.0,
                               adt, 0, Red{nullptr, nullptr}, st, mb);
}
template <typename T>
int FvLaunch<T>::defect_restrict(const FvArgs<T>& A, const T* u, const T* F0, const T* x, const T* b, T* rc,
                                 const double* xpart, int xcount, const double* slots, double adt, int zero,
                                 hipStream_t st, const Mb& mb, const ZeroStage<T>& z0)
{
    if (zero) {
        const dim3 g((unsigned)((A.nxl / 2 + 63) / 64), (unsigned)((A.nzl / 2 + 3) / 4), (unsigned)mb.n);
        if (mb.tab) timed_launch(fv_restrict_neg_kernel<T, true>, g, dim3(256), st, A, mb.tab, b, rc, mb.ms);
        else timed_launch(fv_restrict_neg_kernel<T, false>, g, dim3(256), st, A, mb.tab, b, rc, mb.ms);
        return 0;
    }
    const int nb = tile_launch<T, FVM_DEFECT>(A, u, F0, x, nullptr, b, rc, xpart, xcount, const_cast<double*>(slots),
                                              z0.alpha, adt, 0, z0.red, st, mb, z0.x1, z0.slots);
    return z0.x1 ? nb : 0;
}
template <typename T>
int FvLaunch<T>::prolong_correct(const FvArgs<T>& Af, T* x, const T* v, Red red, hipStream_t st, const Mb& mb)
{
    const dim3 g = tile_grid_1d(Af.nxl, Af.nzl, mb.n);
    if (mb.tab) timed_launch(fv_prolong_correct_kernel<T, true>, g, dim3(FV_NTH), st, Af, mb.tab, x, v, red, mb.ms);
    else timed_launch(fv_prolong_correct_kernel<T, false>, g, dim3(FV_NTH), st, Af, mb.tab, x, v, red, mb.ms);
    return (int)g.x;
}
template <typename T>
void FvLaunch<T>::restrict_(const FvArgs<T>& Af, const T* f, T* c, hipStream_t st, const Mb& mb)
{
    const dim3 g = tile_grid(Af.nxl / 2, Af.nzl / 2, mb.n);
    if (mb.tab) fv_restrict_kernel<T, true><<<g, dim3(FV_NTH), 0, st>>>(Af, mb.tab, f, c, mb.ms);
    else fv_restrict_kernel<T, false><<<g, dim3(FV_NTH), 0, st>>>(Af, mb.tab, f, c, mb.ms);
}
template <typename T>
void FvLaunch<T>::prolong(const FvArgs<T>& Af, const T* c, T* f, hipStream_t st, const Mb& mb)
{
    const dim3 g = tile_grid(Af.nxl, Af.nzl, mb.n);
    if (mb.tab) fv_prolong_kernel<T, true><<<g, dim3(FV_NTH), 0, st>>>(Af, mb.tab, c, f, mb.ms);
    else fv_prolong_kernel<T, false><<<g, dim3(FV_NTH), 0, st>>>(Af, mb.tab, c, f, mb.ms);
}
template <typename T>
void FvLaunch<T>::norm2(const T* x, long n, Red red, hipStream_t st, const Mb& mb)
{
    fv_norm2_kernel<T><<<dim3(norm_blocks(n), 1, mb.n), dim3(256), 0, st>>>(x, n, red, mb.ms);
    if (red.out) launch_finalize(red.partials, norm_blocks(n), 1, red.out, st, Gate{}, mb);
}
int fv_default_tile(long nxl)
{
    return nxl >= 1024 ? JFMG_TILE_64x8
           : nxl >= 512 ? JFMG_TILE_64x4_512
           : nxl >= 256 ? JFMG_TILE_16x4 : JFMG_TILE_8x4;
}
bool fv_wide_tile(int tile) { return tile == JFMG_TILE_64x4 || tile == JFMG_TILE_64x8 || tile == JFMG_TILE_64x4_512; }
bool fv_tile_fits_elements(int tile, int n1)
{
    const int tx = tile == JFMG_TILE_16x4 ? 16 : tile == JFMG_TILE_8x4 ? 8 : tile == JFMG_TILE_32x4 ? 32 : 64;
    const int tz = tile == JFMG_TILE_64x8 ? 8 : 4;
    return (n1 == 2 || n1 == 4) && tx % n1 == 0 && tz % n1 == 0;   // the stage kernel's two N1
}

long fv_partial_blocks(long nxl, long nzl)
{
    // the most work-groups of any tile shape (8x4) or of the 64x4 streaming kernels, at least 1024
    const long smallest = ((nxl + 7) / 8) * ((nzl + 3) / 4);
    const long pro = ((nxl + FV_TX - 1) / FV_TX) * ((nzl + FV_TZ - 1) / FV_TZ);
    return std::max(std::max(smallest, pro), 1024L);
}
template <typename T> int FvLaunch<T>::norm_blocks(long n)
{
    long b = (n + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

template struct FvLaunch<double>;
template struct FvLaunch<float>;

}  // namespace jfmg
