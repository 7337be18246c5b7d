// Internal interface between the host driver and the kernel launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "jfmg.h"
#include "jfmg_dev.h"

namespace jfmg {

// Kernel timing by the dispatch packet itself (start/stop events of
// hipExtLaunchKernel): when `start` is set, the next launch that goes through
// timed_launch() records into these events and marks them used.  Event pairs
// around a launch would include host gaps when the GPU waits for the host.
struct LaunchTimer {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
extern thread_local LaunchTimer g_launch_timer;

template <typename K, typename... Args>
inline void timed_launch(K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    if (g_launch_timer.start && !g_launch_timer.used) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, g_launch_timer.start, g_launch_timer.stop, 0, args...);
        g_launch_timer.used = true;
    } else {
        kernel<<<grid, block, 0, st>>>(args...);
    }
}

constexpr int MAXN1 = 4;      // k + 1 <= 4
constexpr int MAXLEV = 8;

// Reference-element tables (host-built, passed by value).
struct RefTab {
    double xi[MAXN1], w[MAXN1], D[MAXN1][MAXN1], em[MAXN1], ep[MAXN1], dm[MAXN1], dp[MAXN1];
    double V[MAXN1][MAXN1], Vinv[MAXN1][MAXN1], wnc[MAXN1];
};

// ---------------------------------------------------------------------------
// Background atmospheres (paper test cases): neutral theta = theta0 with
// T = theta0 - g z / cp, p = p0 (T/theta0)^(cp/R); or constant N with
// theta = T0 e^{z/H}, T = T0 (a - (a-1) e^{z/H}), p = p0 exp(cp/R (ln(T/T0) - z/H)),
// H = g/N^2, a = g H/(cp T0), T0 = theta0.  rho theta = p0^{R/cp} p^{1/gamma}/R.
// Host code builds the problem tables with it; the allocation-free residual
// evaluates the same formula on the device.
// ---------------------------------------------------------------------------
struct BgPoint {
    double U[4], dU[4], theta;
};

__host__ __device__ inline BgPoint background_at(const jfmg_config& c, double z)
{
    const double cp = c.gamma * c.R / (c.gamma - 1.0);
    double th, dth, p, dp;
    if (c.background == 0) {
        th = c.theta0;
        dth = 0.0;
        const double T = c.theta0 - c.g * z / cp;
        p = c.p0 * ::pow(T / c.theta0, cp / c.R);
        dp = -(c.g * c.p0 / (c.R * c.theta0)) * ::pow(T / c.theta0, cp / c.R - 1.0);
    } else {
        const double H = c.g / (c.N * c.N);
        const double a = c.g * H / (cp * c.theta0);
        const double ez = ::exp(z / H);
        th = c.theta0 * ez;
        dth = th / H;
        const double T = c.theta0 * (a - (a - 1.0) * ez);
        const double dT = -c.theta0 * (a - 1.0) * ez / H;
        p = c.p0 * ::exp((cp / c.R) * (::log(T / c.theta0) - z / H));
        dp = p * (cp / c.R) * (dT / T - 1.0 / H);
    }
    const double C = ::pow(c.p0, c.R / cp) / c.R;
    const double rt = C * ::pow(p, 1.0 / c.gamma);
    const double drt = C * (1.0 / c.gamma) * ::pow(p, 1.0 / c.gamma - 1.0) * dp;
    const double rho = rt / th;
    const double drho = (drt - rho * dth) / th;
    BgPoint b;
    b.U[0] = rho; b.U[1] = rho * c.u_mean; b.U[2] = 0.0; b.U[3] = rt;
    b.dU[0] = drho; b.dU[1] = drho * c.u_mean; b.dU[2] = 0.0; b.dU[3] = drt;
    b.theta = th;
    return b;
}

// background pressure p0 (R rho_theta / p0)^gamma of the potential-temperature equation of state
__host__ __device__ inline double bg_pressure(const jfmg_config& c, double rt)
{
    return c.p0 * ::pow(c.R * rt / c.p0, c.gamma);
}

// Host helpers of the driver used by other translation units: the reference
// element tables, the configuration check (EINVAL with a message) and the gas
// constants of the DG kernels.
bool build_reftab(int k, int transfer, RefTab& R);
jfmg_status check_config(const jfmg_config& c, const char** msg);
Gas<double> gas_of(const jfmg_config& c);
// message returned by jfmg_last_error(NULL) for calls without a problem
void set_create_error(const std::string& msg);

// Everything a DG kernel needs about the grid, the gas and the background.
struct DgArgs {
    long ne;
    int nx, nz, bc, physics;
    double dx, dz, J, g, mu, c_ip;
    // set by the launcher from dx, dz and c_ip: 2/dx, 2/dz and the interior
    // penalty factors c_ip (k+1)^2 / h of x- and z-faces
    double rdx2, rdz2, eta_x, eta_z;
    Gas<double> gas;
    const double* bg_node;   // [nz*(k+1)][4] background at the z of each node row
    const double* dbg_node;  // [nz*(k+1)][4] d/dz of it
    const double* th_node;   // [nz*(k+1)]    background theta
    const double* bg_face;   // [nz+1][4]     background at element z-faces
    const double* dbg_face;  // [nz+1][4]
    const double* pb_node;   // [nz*(k+1)]    background pressure and 1/(rho theta) at node rows
    const double* irt_node;
    const double* pb_face;   // [nz+1]        the same at element z-faces
    const double* irt_face;
    // fluxes of the linearization state U', written once per linearization (mode 5)
    // and read by every product with it (mode 3): the volume fluxes F^x, F^z per
    // node, [8][ne (k+1)^2], then the face terms per face point of every element,
    // [8][ne 4 (k+1)] (flux, then the symmetric term's jump); lin_doubles() long
    double* lin0 = nullptr;
    RefTab R;
};

// One FV level in precision T.
template <typename T> struct FvArgs {
    int nxl, nzl, bc, physics;
    long nc;
    T hx, hz, area, iarea, g, mu;
    int tile;        // jfmg_tile shape of the operator kernels on this level (host side)
    int lev;         // level index (the entry of a ragged batch's member table)
    Gas<T> gas;
    const T* bgc;    // [nzl][4]   background at cell-centre z
    const T* bgf;    // [nzl+1][4] background at z-faces
    const T* dbgf;   // [nzl+1][4] d/dz background at z-faces
    const T* pc;     // [nzl][2]   background pressure, 1/(rho theta) at cell-centre z
    const T* pf;     // [nzl+1][2] the same at z-faces
};

// device scalar slots of one FV level (doubles)
enum { LV_UTOT = 0, LV_LAM = 1, LV_DTAU = 2, LV_IUTOT = 3, LV_NSLOT = 4 };   // LV_IUTOT = 1/||u + Ubar||

// Kernel arguments of one member of a ragged batch (members of different grid
// sizes and domains in one problem): device resident, one entry per member.  Each
// kernel of a ragged launch reads its member's entry (blockIdx.z), takes its
// extents from it and leaves the blocks beyond them idle (writing zero partial
// sums), so every member computes exactly what it computes alone; table pointers
// are absolute (into the member's own workspace region).
struct MemberArgs {
    DgArgs dg;
    long N;                        // DG vector length 4 ne (k+1)^2
    int live;                      // 0: the member sits out (kernels skip it, zero partials)
    FvArgs<double> f64[MAXLEV];    // FV levels (the entries of the problem's precision are set)
    FvArgs<float> f32[MAXLEV];
};

// Members of a lock-step batch: n members, member m at byte offset m * ms from
// member 0 in every per-member buffer (device workspace regions of equal layout).
// tab: the member table of a ragged batch (null for a single problem and for a
// batch of equal members).
struct Mb {
    int n = 1;
    long ms = 0;
    const MemberArgs* tab = nullptr;
};

// The arguments a kernel works with: its own (RG false) or its member's entry.
template <bool RG> __device__ __forceinline__ const DgArgs& dg_of(const DgArgs& a, const MemberArgs* t)
{
    if constexpr (RG) return t[blockIdx.z].dg;
    else return a;
}
template <typename T> __device__ __forceinline__ const FvArgs<T>& fv_entry(const MemberArgs* t, int lev)
{
    if constexpr (std::is_same_v<T, float>) return t[blockIdx.z].f32[lev];
    else return t[blockIdx.z].f64[lev];
}
template <typename T, bool RG> __device__ __forceinline__ const FvArgs<T>& fv_of(const FvArgs<T>& a, const MemberArgs* t)
{
    if constexpr (RG) return fv_entry<T>(t, a.lev);
    else return a;
}
// a vector length of the member (ragged batch; 0 while it sits out) or the given one
__device__ __forceinline__ long len_of(long n, const MemberArgs* t)
{
    return t ? (t[blockIdx.z].live ? t[blockIdx.z].N : 0) : n;
}
// a ragged member that sits out (converged while others iterate)
__device__ __forceinline__ bool sits_out(const MemberArgs* t) { return t && !t[blockIdx.z].live; }
// live[m] = 1 for the members m in `bits` (at most MAXMEMBERS), by a kernel
constexpr int MAXMEMBERS = 4096;
struct LiveBits {
    unsigned long long w[MAXMEMBERS / 64];
};
void launch_set_live(MemberArgs* tab, int n, const LiveBits& bits, hipStream_t st);

// ---- DG kernels (dg.hip) ----
// mode 0: <psi,L>  1: M^-1 L  2: G = U - adt M^-1 L - Ubar (+ ||G||^2 into red.out)
// mode 3: JVP out = Y - adt/eps M^-1 (L(U+eps Y) - L(U)), eps from the device scalars
//         yn2 = ||Y||^2 and ut2 = ||U + Ubar||^2 (eps_mode 1)
// mode 4: explicit Runge-Kutta stage out = ex.a0 Ubar + ex.a1 U + ex.c M^-1 L(U)
//         (out must not alias U: neighbour traces are read from U by other blocks)
// mode 5: the fluxes of U into A.lin0 (the linearization state of mode 3's products)
struct ExStage {
    double a0 = 0.0, a1 = 1.0, c = 0.0;
};
// mode 3 (JVP): ||y||^2 is yn2[0], or with ycount > 0 the sum of ycount block partials at yn2
void launch_dg(int k, bool ns, int mode, const DgArgs& A, const double* U, const double* Y,
               const double* Ubar, double* out, const double* yn2, const double* ut2, int eps_mode,
               double adt, Red red, hipStream_t st, const Mb& mb = Mb{}, const ExStage& ex = ExStage{},
               int ycount = 0);
// doubles of DgArgs::lin0 for degree k and ne elements
inline long lin_doubles(int k, long ne) { return 8 * ne * (k + 1) * (k + 1) + 8 * ne * 4 * (k + 1); }
int transfer_grid(int k, long ne);
int dg_grid(int k, long ne);
void launch_initial_state(int k, const DgArgs& A, int shape, double amp, double xc, double zc,
                          double xr, double zr, double a, double Z, double x0, double z0,
                          double u_mean, double* U, hipStream_t st, const Mb& mb = Mb{});
// sum over nodes of (U + Ubar)^2
void launch_norm2_total(int k, const DgArgs& A, const double* U, Red red, hipStream_t st, const Mb& mb = Mb{});
int norm_total_grid(long n);

// ---- transfers (transfer.hip) ----
// The first RK stage of the finest level from x = 0, x1 = alpha dtau u (dtau in
// slots[LV_DTAU]) with ||x1||^2 block partials into red.partials, can be produced
// by the same kernel (x1 != nullptr); the return value is the number of blocks.
template <typename T> struct ZeroStage {
    T* x1 = nullptr;
    const double* slots = nullptr;
    double alpha = 0.0;
    Red red{nullptr, nullptr};
};
// u = T U; with snrm2 the input is first scaled, sgn U / sqrt(snrm2[0]), and written to Us
template <typename T>
int launch_transfer_T(int k, const DgArgs& A, int mass_fix, const double* U, T* u, int nxf, hipStream_t st,
                      const double* snrm2 = nullptr, double* Us = nullptr, const Mb& mb = Mb{},
                      const ZeroStage<T>& z0 = ZeroStage<T>{}, double sgn = 1.0);
template <typename T>
void launch_transfer_Tinv(int k, const DgArgs& A, int mass_fix, const T* u, double* U, int nxf, Red red,
                          hipStream_t st, const Mb& mb = Mb{});
void launch_subgrid_map(int k, const DgArgs& A, int nxf, int* out, hipStream_t st);

// ---- FV kernels (fv.hip) ----
// default tile shape of the FV operator kernels on a level nxl cells wide, and
// whether a shape is one of the wide ones (one wave per 64-cell row)
int fv_default_tile(long nxl);
bool fv_wide_tile(int tile);
// FV partial-sum blocks needed by the largest launch on a level of nxl x nzl cells
long fv_partial_blocks(long nxl, long nzl);

// The FV -> DG transfer applied by the last smoother stage of a cycle on the finest
// level (FvLaunch::stage_tinv): output vector, k + 1, the mass-fix flag and the tables
// of transfer_Tinv_kernel.
struct TinvOut {
    double* z = nullptr;
    int n1 = 0, mass_fix = 0;
    double Vinv[MAXN1][MAXN1] = {};
    double wnc[MAXN1] = {};
};
// whether stage_tinv serves this tile shape and k + 1 (tiles of whole elements, k + 1 = 2 or 4)
bool fv_tile_fits_elements(int tile, int n1);

// per level of a linearization: number of LIN partials and cell widths
struct LinLevels {
    int nb[MAXLEV];
    double hx[MAXLEV], hz[MAXLEV];
};

template <typename T> struct FvLaunch {
    // F0 = f~(u) and the block partials of ||u + Ubar||^2 and max |v| + c (2 x the returned
    // count at red.partials); with uc != nullptr also uc = R u, the next coarser level's state
    static int lin_level(const FvArgs<T>& A, const T* u, T* F0, T* uc, Red red, double adt, hipStream_t st,
                         const Mb& mb = Mb{});
    // the slots of levels 0..nlev-1 (||u + Ubar||, max |v| + c, dtau at slots + 4 l) from
    // their LIN partials at partials + l * pstride, one launch for all levels
    static void lin_finalize(const double* partials, long pstride, const LinLevels& lv, int nlev, double* slots,
                             double mu, double adt, double cfl, hipStream_t st, const Mb& mb = Mb{});
    // one RK stage; ||x_p||^2 is the sum of xcount partials at xpart; writes the
    // ||xo||^2 partials to red.partials and returns their count
    static int stage(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b, T* xo,
                     const double* xpart, int xcount, const double* slots, double alpha_j, double adt, int zero,
                     Red red, hipStream_t st, const Mb& mb = Mb{});
    // the same stage without storing its result v: the next finer level's x (xf, level
    // dimensions twice those of A) becomes xf - P v (-P v when fine_zero), with the
    // ||xf||^2 partials into red.partials; returns their count
    static int stage_prolong(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b,
                             T* xf, bool fine_zero, const double* xpart, int xcount, const double* slots,
                             double alpha_j, double adt, Red red, hipStream_t st, const Mb& mb = Mb{});
    // the same stage on the finest level without storing its result v: z = T^-1 v into
    // tv.z (tiles of whole elements), with the ||z||^2 partials into red.partials;
    // returns their count
    static int stage_tinv(const FvArgs<T>& A, const T* u, const T* F0, const T* xp, const T* x0, const T* b,
                          const TinvOut& tv, const double* xpart, int xcount, const double* slots, double alpha_j,
                          double adt, Red red, hipStream_t st, const Mb& mb = Mb{});
    static void matvec(const FvArgs<T>& A, const T* u, const T* F0, const T* x, T* out, const double* xpart,
                       int xcount, const double* slots, double adt, hipStream_t st, const Mb& mb = Mb{});
    // coarse defect rc = R(g'x - b) (x = 0: R(-b)); with z0.x1 the first RK stage of the
    // coarse level from x = 0 as well (z0.slots = the coarse level's slots); returns the
    // number of ||x1||^2 partials (0 when z0.x1 is null or x = 0)
    static int defect_restrict(const FvArgs<T>& A, const T* u, const T* F0, const T* x, const T* b, T* rc,
                               const double* xpart, int xcount, const double* slots, double adt, int zero,
                               hipStream_t st, const Mb& mb = Mb{}, const ZeroStage<T>& z0 = ZeroStage<T>{});
    static int prolong_correct(const FvArgs<T>& Af, T* x, const T* v, Red red, hipStream_t st, const Mb& mb = Mb{});
    static void restrict_(const FvArgs<T>& Af, const T* f, T* c, hipStream_t st, const Mb& mb = Mb{});
    static void prolong(const FvArgs<T>& Af, const T* c, T* f, hipStream_t st, const Mb& mb = Mb{});
    static void norm2(const T* x, long n, Red red, hipStream_t st, const Mb& mb = Mb{});
    static int norm_blocks(long n);
};

// ---- linear algebra (la.hip) ----
int la_blocks(long n);
// out[q] = sum over nb block partials [q][nb], fixed order (one block)
// Gate of the Arnoldi re-orthogonalization pass.  h holds the first Gram-Schmidt
// pass's coefficients h[0..nv) and ||w||^2 before the pass in h[nv]; ||w||^2 after
// it is, by Pythagoras, h[nv] - sum_i h[i]^2 (gate_after: accurate to a few
// hundred ulps where the gate stays closed, i.e. where the pass kept more than
// sqrt(tau2) of ||w||; nv <= 64, the FGMRES restart length).  The gated kernels work only where gate_after < tau2 h[nv];
// h == nullptr means always open.
struct Gate {
    const double* h = nullptr;
    int nv = 0;
    double tau2 = 0.0;
};
// every wave evaluates it with one load per lane and a butterfly sum (nv <= 64): the
// same fixed order, so the same value, in every wave and every kernel.  All 64 lanes
// of the wave must call it (no divergent branch around the call).
__device__ __forceinline__ double gate_after(const Gate& g)
{
    const int l = threadIdx.x & 63;
    const double hl = l < g.nv ? g.h[l] : 0.0;
    return g.h[g.nv] - wave_sum(hl * hl);
}
__device__ __forceinline__ bool gate_open(const Gate& g) { return !g.h || gate_after(g) < g.tau2 * g.h[g.nv]; }

void launch_finalize(const double* partials, int nb, int nq, double* out, hipStream_t st, Gate gate = Gate{},
                     const Mb& mb = Mb{});
void launch_norm2(const double* x, long n, Red red, hipStream_t st, const Mb& mb = Mb{});
// device scalar slots <-> coherent pinned host memory (count values per member)
void launch_gather(const double* src, int count, double* host, hipStream_t st, const Mb& mb);
void launch_scatter(double* dst, int count, const double* host, long hstride, hipStream_t st, const Mb& mb);
// the finalize into red.out is launched only when red.out != nullptr
void launch_multidot(const double* w, const double* V, long ld, int nv, int self, long n, Gate gate, Red red,
                     hipStream_t st, const Mb& mb = Mb{});
struct Publish;
// w -= sum_i h[i] V_i; optional ||w||^2 into red.out when red.out != nullptr.  With dots (g2.h
// set), where gate g2 opens, the multi-dot <w_new, v_i> (i < nv) of the updated w follows in the
// same kernel, its block partials at dots (la_blocks(n) per entry, as launch_multidot stores
// them); where it stays closed, the kernel publishes (pub) with ||w_new||^2 by Pythagoras.
void launch_update(double* w, const double* V, long ld, int nv, long n, const double* h, Red red, hipStream_t st,
                   Gate gate, const Mb& mb, Gate g2, double* dots, const Publish& pub);
// Publication of an FGMRES iteration's scalars: src[0..ns) to host-visible pinned memory
// (host, member m at host + m * host_stride), entry idx replaced by ||w||^2 (also stored to
// out[0]), entries zoff .. zoff+zn by 0 where the second pass was skipped, entry fidx by 1
// where it ran and 0 where it was skipped; cnt: a counter in device memory, zero between
// launches.
struct Publish {
    double* out = nullptr;
    const double* src = nullptr;
    int ns = 0, idx = 0;
    double* host = nullptr;
    long host_stride = 0;
    int zoff = 0, zn = 0, fidx = -1;
    unsigned long long* cnt = nullptr;
};
// The gated second Gram-Schmidt pass (coefficients summed from the multi-dot's partials at
// hpart, la_blocks(n) per entry, stored to hout; ||w||^2 partials at wpart) and, where it runs,
// the iteration's publication, in one launch (where the gate stays closed the first pass's
// update kernel publishes).  gate.h must be set.
void launch_update2_publish(double* w, const double* V, long ld, int nv, long n, Gate gate, const double* hpart,
                            double* hout, double* wpart, const Publish& pub, hipStream_t st, const Mb& mb);
void launch_scale(double* out, const double* in, long n, const double* nrm2, hipStream_t st, double sgn = 1.0,
                  const Mb& mb = Mb{});
// out = base + sum_i y[i] Z_i   (base may alias out)
void launch_lincomb(double* out, const double* base, const double* Z, long ld, int nv, long n, const double* y,
                    hipStream_t st, const Mb& mb = Mb{});
// zero `bytes` (a multiple of 4) with a kernel (graph-capture safe, unlike a memset node)
void launch_zero(void* ptr, size_t bytes, hipStream_t st, const Mb& mb = Mb{});
template <typename T> void launch_fill_pattern(T* x, long n, hipStream_t st, const Mb& mb = Mb{});
// DG-level smoother stage out = x0 + s (r - t), s = alpha dtau[0] (alpha when dtau is null),
// x0 / t null meaning 0; out may alias x0 or t (elementwise); ||out||^2 into red.out
// (when red.out is set)
void launch_dg_smooth(double* out, const double* x0, const double* r, const double* t, double alpha,
                      const double* dtau, long n, Red red, hipStream_t st, const Mb& mb = Mb{});
// out[0] = cfl / (1 + adt (lam[0] (1/hx + 1/hz) + 2 mu (1/hx^2 + 1/hz^2)))
void launch_dg_dtau(const double* lam, double* out, double hx, double hz, double mu, double adt, double cfl,
                    hipStream_t st, const Mb& mb = Mb{});
// out = a*x + b*y
void launch_axpby(double* out, double a, const double* x, double b, const double* y, long n, hipStream_t st,
                  const Mb& mb = Mb{});

}  // namespace jfmg
