// Transfers between the DG space and its FV subgrid (paper Sec. "Transfer
// functions", eq. transfer-mass-fix and the appendix quadrature).
//
//   T^mf:  t_ij = sum_ab V_ia V_jb u_ab  (DG polynomial at the subcell centres),
//          t -= mean(t) - sum_ij w_i w_j t_ij  (mass of the DG function from the
//          centre values with the modified Newton-Cotes weights w)
//   T^-1,mf: u_ab = sum_ij Vinv_ai Vinv_bj t_ij - (sum_ij w_i w_j t_ij - mean(t))
//
// One thread per node/subcell, EPB elements per work-group; the (k+1)^2 x
// (k+1)^2 operator is applied as two 1D contractions through LDS.  The kernels
// are bound by HBM (<= 2 x 16 FMAs per output value), so no matrix cores.
// Subcell (i, j) of element (ex, ez) is FV cell (ex (k+1) + i, ez (k+1) + j).
#include "jfmg_internal.h"

namespace jfmg {

template <int N1> struct TrShape {
    static constexpr int NP = N1 * N1;
    static constexpr int NTH = (N1 == 2) ? 64 : 128;
    static constexpr int EPB = NTH / NP;
};

__device__ __forceinline__ long subcell_index(int ex, int ez, int i, int j, int n1, int nxf)
{
    return (long)(ez * n1 + j) * nxf + (long)ex * n1 + i;
}

// snrm2 != nullptr: the input is sgn U / ||U|| (||U||^2 = snrm2[0]); the scaled DG
// vector is also written to Us (may alias U: every value is read and written by
// the same thread).
// With x1 != nullptr the kernel also takes the first RK stage of the finest FV
// level from x = 0: x1 = (alpha dtau) u and the block partials of ||x1||^2.
template <int N1, typename T, bool RG>
__global__ void __launch_bounds__(TrShape<N1>::NTH)
transfer_T_kernel(DgArgs Aa, const MemberArgs* __restrict__ mt, int mass_fix, const double* U, T* __restrict__ u,
                  int nxf, const double* snrm2, double* Us, T* __restrict__ x1, const double* __restrict__ slots,
                  double alpha, Red red, long ms, double sgn)
{
    const DgArgs& A = dg_of<RG>(Aa, mt);
    if (RG) nxf = N1 * A.nx;
    U = mbr(U, ms);
    u = mbr(u, ms);
    snrm2 = mbr(snrm2, ms);
    Us = mbr(Us, ms);
    x1 = mbr(x1, ms);
    slots = mbr(slots, ms);
    red = mbr(red, ms);
    constexpr int NP = TrShape<N1>::NP, EPB = TrShape<N1>::EPB;
    if ((long)blockIdx.x * EPB >= A.ne || sits_out(mt)) {   // beyond a smaller member, or one that sits out
        if (x1 && threadIdx.x == 0) red.partials[block_linear()] = 0.0;
        return;
    }
    __shared__ double sU[EPB][4][NP];
    __shared__ double sH[EPB][4][NP];
    const int t = threadIdx.x, le = t / NP, nd = t - le * NP;
    const bool act = le < EPB;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = act && e < A.ne;
    const long N = A.ne * NP;
    const long nc = N;   // number of finest FV cells
    const int i = nd % N1, j = nd / N1;   // this thread: x-index i, z-index j
    // every global load first (the node's four components, ||U||^2, the pseudo time
    // step and this thread's rows of V), so that their latencies overlap
    double uv[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid)
#pragma unroll
        for (int c = 0; c < 4; ++c) uv[c] = U[c * N + e * NP + nd];
    const double sn2 = snrm2 ? snrm2[0] : 1.0;
    const double dtau = x1 ? slots[LV_DTAU] : 0.0;
    double Vi[N1], Vj[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) {
        Vi[a] = A.R.V[i][a];
        Vj[a] = A.R.V[j][a];
    }
    const double s = snrm2 ? sgn / sqrt(sn2) : 1.0;
    if (act)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double v = uv[c];
            if (valid && snrm2) {
                v = v * s;
                Us[c * N + e * NP + nd] = v;
            }
            sU[le][c][nd] = v;
        }
    __syncthreads();
    // first contraction along x: h_{b,i} = sum_a V_ia u_ab (stored at node slot b*N1+i)
    if (act)
        for (int c = 0; c < 4; ++c) {
            double s2 = 0.0;
#pragma unroll
            for (int a = 0; a < N1; ++a) s2 += Vi[a] * sU[le][c][j * N1 + a];
            sH[le][c][j * N1 + i] = s2;
        }
    __syncthreads();
    double tv[4];
    if (act)
        for (int c = 0; c < 4; ++c) {
            double s2 = 0.0;
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) s2 += Vj[bb] * sH[le][c][bb * N1 + i];
            tv[c] = s2;
        }
    __syncthreads();
    if (act)
        for (int c = 0; c < 4; ++c) sU[le][c][nd] = tv[c];
    __syncthreads();
    // the element's mass-fix sums (mean and Newton-Cotes quadrature of each component, each
    // summed in the order below by one of the element's threads) into sH, which the
    // contractions are done with: [le] as 8 consecutive doubles
    double* const ssum = &sH[act ? le : 0][0][0];
    if (mass_fix) {
        if (act)
            for (int q = nd; q < 8; q += NP) {
                const int c = q & 3;
                double acc = 0.0;
                if (q < 4) {
#pragma unroll
                    for (int jj = 0; jj < N1; ++jj)
#pragma unroll
                        for (int ii = 0; ii < N1; ++ii) acc += sU[le][c][jj * N1 + ii];
                } else {
#pragma unroll
                    for (int jj = 0; jj < N1; ++jj)
#pragma unroll
                        for (int ii = 0; ii < N1; ++ii) {
                            const double v = sU[le][c][jj * N1 + ii];
                            acc += A.R.wnc[ii] * A.R.wnc[jj] * v;
                        }
                }
                ssum[q] = acc;
            }
        __syncthreads();
    }
    double nrm = 0.0;
    if (valid) {
        const int ez = (int)(e / A.nx), ex = (int)(e - (long)ez * A.nx);
        const long o = subcell_index(ex, ez, i, j, N1, nxf);
        const T s1 = x1 ? (T)(alpha * dtau) : T(0);
        for (int c = 0; c < 4; ++c) {
            double shift = 0.0;
            if (mass_fix) shift = ssum[c] / NP - ssum[4 + c];   // mean / NP - quad
            const T b = (T)(tv[c] - shift);
            u[c * nc + o] = b;
            if (x1) {
                const T v = s1 * b;
                x1[c * nc + o] = v;
                nrm += (double)v * (double)v;
            }
        }
    }
    if (x1) put_partial<TrShape<N1>::NTH>(red, nrm);
}

template <int N1, typename T, bool RG>
__global__ void __launch_bounds__(TrShape<N1>::NTH)
transfer_Tinv_kernel(DgArgs Aa, const MemberArgs* __restrict__ mt, int mass_fix, const T* __restrict__ u,
                     double* __restrict__ U, int nxf, Red red, long ms)
{
    const DgArgs& A = dg_of<RG>(Aa, mt);
    if (RG) nxf = N1 * A.nx;
    u = mbr(u, ms);
    U = mbr(U, ms);
    red = mbr(red, ms);
    constexpr int NP = TrShape<N1>::NP, NTH = TrShape<N1>::NTH, EPB = TrShape<N1>::EPB;
    if ((long)blockIdx.x * EPB >= A.ne || sits_out(mt)) {   // beyond a smaller member, or one that sits out
        if (red.partials && threadIdx.x == 0) red.partials[block_linear()] = 0.0;
        return;
    }
    __shared__ double sT[EPB][4][NP];
    __shared__ double sH[EPB][4][NP];
    const int t = threadIdx.x, le = t / NP, nd = t - le * NP;
    const bool act = le < EPB;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = act && e < A.ne;
    const long N = A.ne * NP;
    const int ez = valid ? (int)(e / A.nx) : 0, ex = valid ? (int)(e - (long)ez * A.nx) : 0;
    const int i = nd % N1, j = nd / N1;
    // every global load first: the subcell's four components and this thread's rows
    // of V^-1
    T tv[4] = {T(0), T(0), T(0), T(0)};
    if (valid)
#pragma unroll
        for (int c = 0; c < 4; ++c) tv[c] = u[c * N + subcell_index(ex, ez, i, j, N1, nxf)];
    // thread slot nd = b*N1 + a computes DG node (a, b)
    const int a = i, b = j;
    double Va[N1], Vb[N1];
#pragma unroll
    for (int q = 0; q < N1; ++q) {
        Va[q] = A.R.Vinv[a][q];
        Vb[q] = A.R.Vinv[b][q];
    }
    if (act)
#pragma unroll
        for (int c = 0; c < 4; ++c) sT[le][c][nd] = (double)tv[c];
    __syncthreads();
    if (act)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;   // h_{jj,a} = sum_i Vinv_ai t_{i,jj}, stored at slot jj*N1+a
#pragma unroll
            for (int ii = 0; ii < N1; ++ii) s += Va[ii] * sT[le][c][b * N1 + ii];
            sH[le][c][b * N1 + a] = s;
        }
    __syncthreads();
    double nrm = 0.0;
    if (valid)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < N1; ++jj) s += Vb[jj] * sH[le][c][jj * N1 + a];
            double shift = 0.0;
            if (mass_fix) {
                double mean = 0.0, quad = 0.0;
#pragma unroll
                for (int jj = 0; jj < N1; ++jj)
#pragma unroll
                    for (int ii = 0; ii < N1; ++ii) {
                        const double v = sT[le][c][jj * N1 + ii];
                        mean += v;
                        quad += A.R.wnc[ii] * A.R.wnc[jj] * v;
                    }
                shift = quad - mean / NP;
            }
            const double v = s - shift;
            U[c * N + e * NP + nd] = v;
            nrm += v * v;
        }
    if (red.partials) put_partial<NTH>(red, nrm);
}

template <int N1>
__global__ void __launch_bounds__(256) subgrid_map_kernel(DgArgs A, int nxf, int* __restrict__ out)
{
    constexpr int NP = N1 * N1;
    const long n = A.ne * NP;
    const long g = (long)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    const long e = g / NP;
    const int nd = (int)(g - e * NP);
    const int ez = (int)(e / A.nx), ex = (int)(e - (long)ez * A.nx);
    out[subcell_index(ex, ez, nd % N1, nd / N1, N1, nxf)] = (int)g;
}

int transfer_grid(int k, long ne)
{
    const int epb = k == 1 ? TrShape<2>::EPB : k == 2 ? TrShape<3>::EPB : TrShape<4>::EPB;
    return (int)((ne + epb - 1) / epb);
}

template <int N1, typename T, bool RG>
static void transfer_T_n(dim3 g, const DgArgs& A, int mass_fix, const double* U, T* u, int nxf, hipStream_t st,
                         const double* snrm2, double* Us, const Mb& mb, const ZeroStage<T>& z0, double sgn)
{
    timed_launch(transfer_T_kernel<N1, T, RG>, g, dim3(TrShape<N1>::NTH), st, A, mb.tab, mass_fix, U, u, nxf, snrm2,
                 Us, z0.x1, z0.slots, z0.alpha, z0.red, mb.ms, sgn);
}

template <int N1, typename T>
static void transfer_T_k(dim3 g, const DgArgs& A, int mass_fix, const double* U, T* u, int nxf, hipStream_t st,
                         const double* snrm2, double* Us, const Mb& mb, const ZeroStage<T>& z0, double sgn)
{
    if (mb.tab) transfer_T_n<N1, T, true>(g, A, mass_fix, U, u, nxf, st, snrm2, Us, mb, z0, sgn);
    else transfer_T_n<N1, T, false>(g, A, mass_fix, U, u, nxf, st, snrm2, Us, mb, z0, sgn);
}

template <typename T>
int launch_transfer_T(int k, const DgArgs& A, int mass_fix, const double* U, T* u, int nxf, hipStream_t st,
                      const double* snrm2, double* Us, const Mb& mb, const ZeroStage<T>& z0, double sgn)
{
    const dim3 g(transfer_grid(k, A.ne), 1, mb.n);
    if (k == 1) transfer_T_k<2, T>(g, A, mass_fix, U, u, nxf, st, snrm2, Us, mb, z0, sgn);
    else if (k == 2) transfer_T_k<3, T>(g, A, mass_fix, U, u, nxf, st, snrm2, Us, mb, z0, sgn);
    else transfer_T_k<4, T>(g, A, mass_fix, U, u, nxf, st, snrm2, Us, mb, z0, sgn);
    return (int)g.x;
}

template <int N1, typename T>
static void transfer_Tinv_k(dim3 g, const DgArgs& A, int mass_fix, const T* u, double* U, int nxf, Red red,
                            hipStream_t st, const Mb& mb)
{
    if (mb.tab)
        timed_launch(transfer_Tinv_kernel<N1, T, true>, g, dim3(TrShape<N1>::NTH), st, A, mb.tab, mass_fix, u, U, nxf,
                     red, mb.ms);
    else
        timed_launch(transfer_Tinv_kernel<N1, T, false>, g, dim3(TrShape<N1>::NTH), st, A, mb.tab, mass_fix, u, U,
                     nxf, red, mb.ms);
}

template <typename T>
void launch_transfer_Tinv(int k, const DgArgs& A, int mass_fix, const T* u, double* U, int nxf, Red red, hipStream_t st,
                          const Mb& mb)
{
    const dim3 g(transfer_grid(k, A.ne), 1, mb.n);
    if (k == 1) transfer_Tinv_k<2, T>(g, A, mass_fix, u, U, nxf, red, st, mb);
    else if (k == 2) transfer_Tinv_k<3, T>(g, A, mass_fix, u, U, nxf, red, st, mb);
    else transfer_Tinv_k<4, T>(g, A, mass_fix, u, U, nxf, red, st, mb);
    if (red.out) launch_finalize(red.partials, (int)g.x, 1, red.out, st, Gate{}, mb);
}

template int launch_transfer_T<double>(int, const DgArgs&, int, const double*, double*, int, hipStream_t,
                                       const double*, double*, const Mb&, const ZeroStage<double>&, double);
template int launch_transfer_T<float>(int, const DgArgs&, int, const double*, float*, int, hipStream_t,
                                      const double*, double*, const Mb&, const ZeroStage<float>&, double);
template void launch_transfer_Tinv<double>(int, const DgArgs&, int, const double*, double*, int, Red, hipStream_t,
                                           const Mb&);
template void launch_transfer_Tinv<float>(int, const DgArgs&, int, const float*, double*, int, Red, hipStream_t,
                                          const Mb&);

void launch_subgrid_map(int k, const DgArgs& A, int nxf, int* out, hipStream_t st)
{
    const long n = A.ne * (k + 1) * (k + 1);
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (k == 1) subgrid_map_kernel<2><<<grid, block, 0, st>>>(A, nxf, out);
    else if (k == 2) subgrid_map_kernel<3><<<grid, block, 0, st>>>(A, nxf, out);
    else subgrid_map_kernel<4><<<grid, block, 0, st>>>(A, nxf, out);
}

}  // namespace jfmg
