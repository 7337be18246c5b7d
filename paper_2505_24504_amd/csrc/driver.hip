// Host side of the library: configuration checks, reference-element and
// background tables, workspace carving, the stage solver (inexact Newton with
// Eisenstat-Walker forcing, right-preconditioned FGMRES, the FV multigrid
// V/W-cycle) and the C-ABI of include/jfmg.h.  All vector work runs in the
// kernels of dg.hip, transfer.hip, fv.hip and la.hip on the problem's stream;
// the host keeps only the small Hessenberg least-squares problem.
#include "jfmg.h"
#include "jfmg_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace jfmg;

namespace jfmg {
thread_local LaunchTimer g_launch_timer;
}

namespace {

thread_local std::string g_create_error;

// ---------------------------------------------------------------------------
// Reference element: Gauss-Legendre nodes (Newton on P_{k+1}), barycentric
// Lagrange evaluation, the GL differentiation matrix, the subcell-centre
// interpolation matrix and its inverse, the modified Newton-Cotes weights.
// ---------------------------------------------------------------------------
void legendre_pd(int n, double x, double& p, double& d)
{
    double pm = 1.0, pc = x;
    for (int m = 1; m < n; ++m) {
        const double pn = ((2 * m + 1) * x * pc - m * pm) / (m + 1);
        pm = pc;
        pc = pn;
    }
    p = (n == 0) ? 1.0 : pc;
    d = (n == 0) ? 0.0 : n * (pm - x * pc) / (1.0 - x * x);
}

void gl_rule(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double r = std::cos(M_PI * (4.0 * (n - 1 - i) + 3.0) / (4.0 * n + 2.0));
        for (int it = 0; it < 60; ++it) {
            double p, d;
            legendre_pd(n, r, p, d);
            const double step = p / d;
            r -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double p, d;
        legendre_pd(n, r, p, d);
        x[i] = r;
        w[i] = 2.0 / ((1.0 - r * r) * d * d);
    }
}

struct Bary {
    int n;
    double x[MAXN1], bw[MAXN1];
    void init(int n_, const double* xs)
    {
        n = n_;
        for (int j = 0; j < n; ++j) {
            x[j] = xs[j];
            double p = 1.0;
            for (int m = 0; m < n; ++m)
                if (m != j) p *= (xs[j] - xs[m]);
            bw[j] = 1.0 / p;
        }
    }
    void eval(double t, double* l) const   // all basis values at t
    {
        for (int j = 0; j < n; ++j)
            if (t == x[j]) {
                for (int m = 0; m < n; ++m) l[m] = (m == j) ? 1.0 : 0.0;
                return;
            }
        double den = 0.0;
        for (int j = 0; j < n; ++j) den += bw[j] / (t - x[j]);
        for (int j = 0; j < n; ++j) l[j] = (bw[j] / (t - x[j])) / den;
    }
    void deriv(double t, double* d) const   // all basis derivatives at a non-node t
    {
        double l[MAXN1];
        eval(t, l);
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int m = 0; m < n; ++m)
                if (m != j) s += 1.0 / (t - x[m]);
            d[j] = l[j] * s;
        }
    }
};

bool invert(int n, const double A[MAXN1][MAXN1], double Ai[MAXN1][MAXN1])
{
    double M[MAXN1][2 * MAXN1];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) M[i][j] = j < n ? A[i][j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return false;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(M[p][j], M[c][j]);
        const double inv = 1.0 / M[c][c];
        for (int j = 0; j < 2 * n; ++j) M[c][j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c || M[r][c] == 0.0) continue;
            const double f = M[r][c];
            for (int j = 0; j < 2 * n; ++j) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ai[i][j] = M[i][n + j];
    return true;
}

// Monomial coefficients (lowest degree first) of the Lagrange polynomial l_j
// through the nodes x[0..n).
void lagrange_coefs(int n, const double* x, int j, double* coef)
{
    for (int d = 0; d <= n; ++d) coef[d] = 0.0;
    coef[0] = 1.0;
    int deg = 0;
    for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        const double s = 1.0 / (x[j] - x[m]);
        for (int d = deg + 1; d >= 0; --d) {
            const double lower = d > 0 ? coef[d - 1] : 0.0;
            coef[d] = (lower - x[m] * coef[d]) * s;
        }
        ++deg;
    }
}

// transfer 0: the subcell-centre values of the nodal polynomial (V) and the inverse
// map; transfer 1: its subcell averages (L2 projection onto the subcells), in 1D
// P_ia = (1/h) int over [s_i, s_i + h] of l_a, h = 2/(k+1), integrated term by term.
bool reftab(int k, int transfer, RefTab& R)
{
    const int n = k + 1;
    std::memset(&R, 0, sizeof(R));
    gl_rule(n, R.xi, R.w);
    Bary B;
    B.init(n, R.xi);
    // differentiation matrix D_ij = l_j'(xi_i) (barycentric form)
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            R.D[i][j] = (B.bw[j] / B.bw[i]) / (R.xi[i] - R.xi[j]);
            diag -= R.D[i][j];
        }
        R.D[i][i] = diag;
    }
    B.eval(-1.0, R.em);
    B.eval(1.0, R.ep);
    B.deriv(-1.0, R.dm);
    B.deriv(1.0, R.dp);
    if (transfer == 1) {
        const double h = 2.0 / n;
        for (int a = 0; a < n; ++a) {
            double coef[MAXN1 + 1];
            lagrange_coefs(n, R.xi, a, coef);
            for (int i = 0; i < n; ++i) {
                const double lo = -1.0 + i * h, hi = lo + h;
                double integ = 0.0, plo = lo, phi = hi;   // lo^(d+1), hi^(d+1)
                for (int d = 0; d < n; ++d) {
                    integ += coef[d] * (phi - plo) / (d + 1);
                    plo *= lo;
                    phi *= hi;
                }
                R.V[i][a] = integ / h;
            }
        }
    } else {
        for (int i = 0; i < n; ++i) B.eval(-1.0 + (2.0 * i + 1.0) / n, R.V[i]);
    }
    if (!invert(n, R.V, R.Vinv)) return false;
    // interpolatory rule on the subcell centres of [0,1]: w_i = int_0^1 of the
    // Lagrange polynomial through G_m = (2m+1)/(2(k+1)), integrated term by term
    double G[MAXN1];
    for (int m = 0; m < n; ++m) G[m] = (2.0 * m + 1.0) / (2.0 * n);
    for (int i = 0; i < n; ++i) {
        double coef[MAXN1 + 1] = {1.0};   // polynomial coefficients, lowest degree first
        int deg = 0;
        for (int m = 0; m < n; ++m) {
            if (m == i) continue;
            const double s = 1.0 / (G[i] - G[m]);
            for (int d = deg + 1; d >= 0; --d) {
                const double lower = d > 0 ? coef[d - 1] : 0.0;
                coef[d] = (lower - G[m] * coef[d]) * s;
            }
            ++deg;
        }
        double integ = 0.0;
        for (int d = deg; d >= 0; --d) integ += coef[d] / (d + 1);
        R.wnc[i] = integ;
    }
    return true;
}

struct Key {
    int a, b, c, d, e, f, cycle;
};

bool parse_key(const char* s, Key& k)
{
    if (std::strlen(s) != 9 || s[0] != 'm' || s[1] != 'g') return false;
    int v[6];
    for (int i = 0; i < 6; ++i) {
        if (s[2 + i] < '0' || s[2 + i] > '9') return false;
        v[i] = s[2 + i] - '0';
    }
    if (s[8] != 'V' && s[8] != 'W') return false;
    k = {v[0], v[1], v[2], v[3], v[4], v[5], s[8] == 'V' ? 1 : 2};
    return true;
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
constexpr int NSCAL = 1024;
// scalar slots
enum {
    S_G = 0,        // ||G||^2
    S_UTOT = 1,     // ||U + Ubar||^2 (DG)
    S_Y = 2,        // ||y||^2 for jvp
    S_Z = 3,        // ||z_j||^2
    S_W = 258,      // ||w||^2 after orthogonalization (right after h2: one readback)
    S_R = 5,        // restart residual norm^2
    S_TMP = 6,
    S_CNT = 7,      // counter of the gated pass's work-groups (64-bit, zero between launches)
    S_DGZ = 9,      // ||z||^2 and ||z_j||^2 of the DG-level smoother (key a, b)
    S_DGX = 10,
    S_DGC = 11,     // ||T^-1 x||^2 of a coarse correction that is added to z
    S_DTDG = 12,    // pseudo time step of the DG-level smoother
    S_LEV = 16,     // + 4*level: LV_* slots
    S_H1 = 128,     // 65 entries: h of the first pass, then ||w||^2 before it
    S_H2 = 193,     // 65 entries
    S_RF = 259,     // 1 where the second Gram-Schmidt pass ran, else 0 (published only)
    S_HB = 132,     // doubles from S_H1 through S_RF
    S_Yc = 384,     // 65 entries: FGMRES coefficients
    HSCAL = 8       // scalars per member the host reads at once
};

struct Carve {
    size_t off = 0;
    char* base = nullptr;
    void* take(size_t bytes)
    {
        off = (off + 255) & ~size_t(255);
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// partial-sum regions per FV level: one per iterate buffer
constexpr int FVP_PER_LEVEL = 3;

struct Level {
    int nx, nz;
    long nc;
    int tile;   // jfmg_tile of the FV operator kernels
    double hx, hz;
    void* u;
    void* F0;
    void* buf[3];
    void* b;
    void* bgc;
    void* bgf;
    void* dbgf;
    void* pc;
    void* pf;
};

}  // namespace

// v = sgn src / sqrt(nrm2[0]), formed by the preconditioner's first kernel
struct Norm {
    const double* src = nullptr;
    const double* nrm2 = nullptr;
    double sgn = 1.0;
};

struct jfmg_problem {
    jfmg_config cfg;
    Key key;
    int n1, np;
    long ne, N;
    double dx, dz;
    int nlev;
    Level lev[MAXLEV];
    int prec;          // 64 or 32
    hipStream_t st;        // stream the internal functions issue to (user_st or cs)
    hipStream_t user_st;   // the caller's stream
    hipStream_t cs;        // private stream of jfmg_implicit_step (graph capture and replay)
    RefTab R;
    DgArgs A;
    // device memory (in the caller's workspace)
    double* scal;
    double* partials;   // block partials of reductions that are finalized right away
    size_t npartials;
    double* fvpart;     // block partials of ||x||^2 of each FV buffer, [level][FVP_PER_LEVEL][FVP]
    size_t fvp;
    int xcnt[MAXLEV][3];
    double* bg_node; double* dbg_node; double* th_node; double* bg_face; double* dbg_face;
    double* pb_node; double* pb_face;   // [.][2]: background pressure, 1/(rho theta)
    double *Un, *Ubar, *Uk, *G, *delta, *tmp1, *tmp2, *Ulin, *lin0;
    double *V, *Z;
    int m;
    Mb mb;   // members of a lock-step batch (1 for a single problem) and their byte stride
    // ragged batch: members of different grid sizes, each in an envelope-sized region;
    // DG length and offset of each member in the caller's (packed) state vectors
    bool ragged = false;
    std::vector<long> mlen, moff;
    MemberArgs* tab = nullptr;   // device member table (in the workspace, after the members)
    // kernel-class timing (HIP events on st), used by the benchmark
    struct Pend { int cls; hipEvent_t a, b; double bytes; };
    struct Prof {
        unsigned mask = 0;
        std::vector<hipEvent_t> pool;
        std::vector<Pend> pend;
        double ms[JFMG_K_NCLASS] = {};
        long long cnt[JFMG_K_NCLASS] = {};
        double bytes[JFMG_K_NCLASS] = {};
    } prof;
    // one captured HIP graph per FGMRES iteration index j
    struct IterGraph {
        hipGraphExec_t exec = nullptr;
        int mv[MAXLEV] = {};
        int jvps = 0;
    };
    std::vector<IterGraph> graphs;
    double graph_adt = 0.0;
    bool use_graphs = false;
    bool fuse_tinv = true;   // the last finest-level stage applies T^-1 (JFMG_NO_FUSED_TINV=1: off)
    bool reorth_always = false;   // the second Gram-Schmidt pass on every iteration (JFMG_REORTH_ALWAYS=1)
    Norm v0;   // set by a cycle start: v_0 formed by iteration 0's first kernel (eager launches only)
    IterGraph* capturing = nullptr;
    double* hpin = nullptr;            // coherent pinned host copies of the Arnoldi scalars, per iteration
    double* hscal = nullptr;           // coherent pinned: scalars read by the host, [member][HSCAL]
    double* ycoef = nullptr;           // coherent pinned: FGMRES coefficients, [member][m]
    std::vector<hipEvent_t> hev;       // completion of each copy
    // host side
    int have_lin;
    double adt;
    std::string err;
    jfmg_stats* stats;
    int mv_count[MAXLEV];
    int lh_count, jvp_count, syncs;
    int reorths;   // FGMRES iterations (per member) whose second Gram-Schmidt pass ran
    std::vector<double> hbuf;
};

namespace {

jfmg_status fail(jfmg_problem* p, jfmg_status s, const std::string& msg)
{
    if (p) p->err = msg;
    else g_create_error = msg;
    return s;
}

#define HIPCHK(p, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail((p), JFMG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t ev_get(jfmg_problem* p)
{
    hipEvent_t e = nullptr;
    if (!p->prof.pool.empty()) {
        e = p->prof.pool.back();
        p->prof.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Times the next launch of kernel class `cls` (when that class is being
// profiled) with the start/stop events of its own dispatch; `bytes` is the
// launch's algorithmic HBM traffic.  Not used while a graph is captured.
struct ProfScope {
    jfmg_problem* p;
    int cls;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(jfmg_problem* p_, int c, double by) : p(p_), cls(c), bytes(by)
    {
        if (!(p->prof.mask & (1u << cls)) || p->capturing) return;
        a = ev_get(p);
        b = ev_get(p);
        if (!a || !b) return;
        g_launch_timer = LaunchTimer{a, b, false};
    }
    ~ProfScope()
    {
        if (!a || !b) return;
        if (g_launch_timer.used) p->prof.pend.push_back({cls, a, b, bytes});
        else { p->prof.pool.push_back(a); p->prof.pool.push_back(b); }
        g_launch_timer = LaunchTimer{};
    }
};

void prof_flush(jfmg_problem* p)
{
    for (auto& q : p->prof.pend) {
        float ms = 0.f;
        if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            p->prof.ms[q.cls] += ms;
            p->prof.cnt[q.cls] += 1;
            p->prof.bytes[q.cls] += q.bytes;
        }
        p->prof.pool.push_back(q.a);
        p->prof.pool.push_back(q.b);
    }
    p->prof.pend.clear();
}

jfmg_status check_launch(jfmg_problem* p)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(p, JFMG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return JFMG_OK;
}

int members_of(const jfmg_config& c) { return c.batch > 1 ? c.batch : 1; }

jfmg_status validate(const jfmg_config& c, Key& key, std::string& msg)
{
    if (c.batch < 0 || c.batch > 4096) { msg = "batch must be in 0..4096"; return JFMG_EINVAL; }
    if (c.k < 1 || c.k > 3) { msg = "k must be 1, 2 or 3"; return JFMG_EINVAL; }
    if (c.nx < 1 || c.nz < 1) { msg = "nx, nz must be positive"; return JFMG_EINVAL; }
    // node arrays are addressed with 32-bit byte offsets per component (far above
    // what a workspace of 288 GB can hold)
    if ((long)c.nx * c.nz * (c.k + 1) * (c.k + 1) > (1L << 28)) { msg = "grid too large"; return JFMG_EINVAL; }
    if (!(c.x1 > c.x0) || !(c.z1 > c.z0)) { msg = "empty domain"; return JFMG_EINVAL; }
    if (c.physics < 0 || c.physics > 1 || c.background < 0 || c.background > 1 || c.bc < 0 || c.bc > 1 ||
        c.scheme < 0 || c.scheme > 1) { msg = "physics/background/bc/scheme out of range"; return JFMG_EINVAL; }
    if (c.background == 1 && !(c.N > 0)) { msg = "constant-N background needs N > 0"; return JFMG_EINVAL; }
    if (c.gmres_m < 1 || c.gmres_m > 64) { msg = "gmres_m must be in 1..64"; return JFMG_EINVAL; }
    if (c.rk_stages < 1 || c.rk_stages > 4) { msg = "rk_stages must be in 1..4"; return JFMG_EINVAL; }
    if (c.mg_levels < 1 || c.mg_levels > MAXLEV) { msg = "mg_levels must be in 1..8"; return JFMG_EINVAL; }
    if (c.mg_precision != 32 && c.mg_precision != 64) { msg = "mg_precision must be 32 or 64"; return JFMG_EINVAL; }
    if (c.transfer != 0 && c.transfer != 1) { msg = "transfer must be 0 (interpolation) or 1 (L2 projection)"; return JFMG_EINVAL; }
    if (c.newton_maxit < 1 || c.gmres_max_restarts < 0) { msg = "bad iteration caps"; return JFMG_EINVAL; }
    if (!(c.newton_stall >= 0.0 && c.newton_stall < 1.0)) { msg = "newton_stall must be in [0, 1)"; return JFMG_EINVAL; }
    if (!(c.dt > 0) || !(c.gamma > 1) || !(c.R > 0) || !(c.p0 > 0) || !(c.theta0 > 0) || c.mu < 0) {
        msg = "bad physical constants"; return JFMG_EINVAL;
    }
    char ks[16];
    std::memcpy(ks, c.mg_key, 16);
    ks[15] = 0;
    if (!parse_key(ks, key)) { msg = "bad multigrid key (expected mgabcdefV or mgabcdefW)"; return JFMG_EINVAL; }
    if ((key.a || key.b) && !(c.pseudo_cfl_dg > 0)) { msg = "pseudo_cfl_dg must be > 0"; return JFMG_EINVAL; }
    int nxl = (c.k + 1) * c.nx, nzl = (c.k + 1) * c.nz;
    for (int l = 1; l < c.mg_levels; ++l) {
        if ((nxl & 1) || (nzl & 1)) { msg = "an FV level dimension is odd before the coarsest level"; return JFMG_EINVAL; }
        nxl /= 2;
        nzl /= 2;
    }
    return JFMG_OK;
}

// Layout of the workspace; with base == nullptr it only measures.
template <typename F>
size_t layout(const jfmg_config& c, char* base, F&& bind)
{
    Carve cv;
    cv.base = base;
    const int n1 = c.k + 1, np = n1 * n1;
    const long ne = (long)c.nx * c.nz, N = 4 * ne * np;
    const size_t ts = c.mg_precision == 32 ? 4 : 8;
    const int m = c.gmres_m;
    const long la = (N + 1023) / 1024;
    long nfv = (long)n1 * c.nx * n1 * c.nz;
    const long fvblk = fv_partial_blocks((long)n1 * c.nx, (long)n1 * c.nz);   // blocks of the finest FV level
    const long dgblk = ne;   // at most one block per element
    size_t npart = (size_t)std::max<long>({la * (m + 2), 2 * fvblk, dgblk, 2048, 4096});
    bind("scal", cv.take(NSCAL * 8), 0);
    bind("partials", cv.take(npart * 8), npart);
    const size_t fvp = (size_t)std::max<long>(fvblk, transfer_grid(c.k, ne));   // FV stages, fused transfer
    bind("fvpart", cv.take(fvp * FVP_PER_LEVEL * c.mg_levels * 8), fvp);
    bind("bg_node", cv.take((size_t)c.nz * n1 * 4 * 8), 0);
    bind("dbg_node", cv.take((size_t)c.nz * n1 * 4 * 8), 0);
    bind("th_node", cv.take((size_t)c.nz * n1 * 8), 0);
    bind("bg_face", cv.take((size_t)(c.nz + 1) * 4 * 8), 0);
    bind("dbg_face", cv.take((size_t)(c.nz + 1) * 4 * 8), 0);
    bind("pb_node", cv.take((size_t)c.nz * n1 * 2 * 8), 0);
    bind("pb_face", cv.take((size_t)(c.nz + 1) * 2 * 8), 0);
    const char* dgn[] = {"Un", "Ubar", "Uk", "G", "delta", "tmp1", "tmp2", "Ulin"};
    for (const char* s : dgn) bind(s, cv.take((size_t)N * 8), 0);
    bind("lin0", cv.take((size_t)lin_doubles(c.k, ne) * 8), 0);
    bind("V", cv.take((size_t)N * 8 * (m + 1)), 0);
    bind("Z", cv.take((size_t)N * 8 * m), 0);
    int nxl = n1 * c.nx, nzl = n1 * c.nz;
    for (int l = 0; l < c.mg_levels; ++l) {
        const long nc = (long)nxl * nzl;
        const char* fvn[] = {"u", "F0", "x0", "x1", "x2", "b"};
        for (const char* s : fvn) bind(s, cv.take((size_t)4 * nc * ts), l);
        bind("bgc", cv.take((size_t)nzl * 4 * ts), l);
        bind("bgf", cv.take((size_t)(nzl + 1) * 4 * ts), l);
        bind("dbgf", cv.take((size_t)(nzl + 1) * 4 * ts), l);
        bind("pc", cv.take((size_t)nzl * 2 * ts), l);
        bind("pf", cv.take((size_t)(nzl + 1) * 2 * ts), l);
        nxl /= 2;
        nzl /= 2;
    }
    (void)nfv;
    return (cv.off + 255) & ~size_t(255);   // bytes of one member
}

Red red_at(jfmg_problem* p, int slot) { return Red{p->partials, p->scal + slot}; }

// copy `bytes` of every member from src to dst (both inside the members' workspaces)
hipError_t copy_members(jfmg_problem* p, void* dst, const void* src, size_t bytes)
{
    if (p->mb.n == 1) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, p->st);
    return hipMemcpy2DAsync(dst, (size_t)p->mb.ms, src, (size_t)p->mb.ms, bytes, (size_t)p->mb.n,
                            hipMemcpyDeviceToDevice, p->st);
}
// the caller's state vectors hold the members back to back (each its own length);
// in the workspace member m starts m * ms bytes after member 0
hipError_t members_in(jfmg_problem* p, double* ws, const double* user)
{
    const size_t vb = sizeof(double) * p->N;
    if (p->mb.n == 1) return hipMemcpyAsync(ws, user, vb, hipMemcpyDeviceToDevice, p->st);
    if (!p->ragged)
        return hipMemcpy2DAsync(ws, (size_t)p->mb.ms, user, vb, vb, (size_t)p->mb.n, hipMemcpyDeviceToDevice, p->st);
    hipError_t e = hipSuccess;
    for (int m = 0; m < p->mb.n && !e; ++m)
        e = hipMemcpyAsync((char*)ws + (size_t)m * p->mb.ms, user + p->moff[m], sizeof(double) * p->mlen[m],
                           hipMemcpyDeviceToDevice, p->st);
    return e;
}
hipError_t members_out(jfmg_problem* p, double* user, const double* ws)
{
    const size_t vb = sizeof(double) * p->N;
    if (p->mb.n == 1) return hipMemcpyAsync(user, ws, vb, hipMemcpyDeviceToDevice, p->st);
    if (!p->ragged)
        return hipMemcpy2DAsync(user, vb, ws, (size_t)p->mb.ms, vb, (size_t)p->mb.n, hipMemcpyDeviceToDevice, p->st);
    hipError_t e = hipSuccess;
    for (int m = 0; m < p->mb.n && !e; ++m)
        e = hipMemcpyAsync(user + p->moff[m], (const char*)ws + (size_t)m * p->mb.ms, sizeof(double) * p->mlen[m],
                           hipMemcpyDeviceToDevice, p->st);
    return e;
}

Red no_red() { return Red{nullptr, nullptr}; }
// the mass fix corrects the interpolation transfer only (the L2 projection conserves mass)
int mass_fix_of(const jfmg_problem* p) { return p->cfg.transfer == 0 ? p->cfg.mass_fix : 0; }
double* fvpart(jfmg_problem* p, int l, int bi) { return p->fvpart + (FVP_PER_LEVEL * l + bi) * p->fvp; }

// read `count` device scalars starting at `slot` of every member into
// out[member * count + i] (synchronizes the stream)
jfmg_status read_scalars(jfmg_problem* p, int slot, int count, double* out)
{
    if (count > HSCAL) return fail(p, JFMG_EINVAL, "too many scalars");
    launch_gather(p->scal + slot, count, p->hscal, p->st, p->mb);
    HIPCHK(p, hipStreamSynchronize(p->st));
    std::memcpy(out, p->hscal, sizeof(double) * count * p->mb.n);
    p->syncs++;
    prof_flush(p);
    return JFMG_OK;
}

// gas constants and the binomial coefficients C(gamma, k) of (1 + s)^gamma
template <typename T> Gas<T> make_gas(const jfmg_config& c)
{
    Gas<T> g;
    g.gamma = (T)c.gamma;
    g.R = (T)c.R;
    g.p0 = (T)c.p0;
    double ck = 1.0;
    for (int k = 0; k < GAS_NCOEF; ++k) {
        g.cg[k] = (T)ck;
        ck *= (c.gamma - k) / (k + 1.0);
    }
    return g;
}

// background pressure p0 (R rho_theta / p0)^gamma of the potential-temperature equation of state

}  // namespace

bool jfmg::build_reftab(int k, int transfer, RefTab& R) { return reftab(k, transfer, R); }

jfmg_status jfmg::check_config(const jfmg_config& c, const char** msg)
{
    thread_local std::string m;
    Key key;
    const jfmg_status s = validate(c, key, m);
    if (msg) *msg = m.c_str();
    return s;
}

Gas<double> jfmg::gas_of(const jfmg_config& c) { return make_gas<double>(c); }

void jfmg::set_create_error(const std::string& msg) { g_create_error = msg; }

namespace {

template <typename T> FvArgs<T> fv_args(const jfmg_problem* p, int l)
{
    FvArgs<T> A;
    const Level& L = p->lev[l];
    A.nxl = L.nx; A.nzl = L.nz; A.bc = p->cfg.bc; A.physics = p->cfg.physics; A.nc = L.nc;
    A.hx = (T)L.hx; A.hz = (T)L.hz; A.area = (T)(L.hx * L.hz); A.iarea = (T)(1.0 / (L.hx * L.hz)); A.g = (T)p->cfg.g; A.mu = (T)p->cfg.mu;
    A.gas = make_gas<T>(p->cfg);
    A.bgc = (const T*)L.bgc; A.bgf = (const T*)L.bgf; A.dbgf = (const T*)L.dbgf;
    A.pc = (const T*)L.pc; A.pf = (const T*)L.pf;
    A.tile = L.tile;
    A.lev = l;
    return A;
}

// ---------------------------------------------------------------------------
// Linearization: ||U + Ubar||, u_0 = T^mf U, u_{l+1} = R u_l, f~(u_l), dtau_l
// ---------------------------------------------------------------------------
template <typename T> jfmg_status linearize_t(jfmg_problem* p, const double* U, double adt)
{
    hipStream_t st = p->st;
    if (U != p->Ulin) HIPCHK(p, copy_members(p, p->Ulin, U, sizeof(double) * p->N));
    p->adt = adt;
    launch_norm2_total(p->cfg.k, p->A, p->Ulin, red_at(p, S_UTOT), st, p->mb);
    {
        // the volume fluxes and face terms of U' that every product with this state differences against
        ProfScope ps(p, JFMG_K_DG_LINEARIZE, (double)p->N * 8 + 8.0 * lin_doubles(p->cfg.k, p->ne));
        launch_dg(p->cfg.k, p->cfg.physics == 1, 5, p->A, p->Ulin, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0.0,
                  no_red(), st, p->mb);
    }
    launch_transfer_T<T>(p->cfg.k, p->A, mass_fix_of(p), p->Ulin, (T*)p->lev[0].u, p->lev[0].nx, st, nullptr, nullptr,
                         p->mb);
    // level by level: F0 = f~(u_l), its partials, and u_{l+1} = R u_l from the same tiles;
    // then the slots of all levels in one launch
    LinLevels lv{};
    for (int l = 0; l < p->nlev; ++l) {
        const bool coarser = l + 1 < p->nlev;
        ProfScope ps(p, JFMG_K_FV_LINEARIZE, (2.0 + (coarser ? 0.25 : 0.0)) * 4.0 * p->lev[l].nc * sizeof(T));
        const FvArgs<T> A = fv_args<T>(p, l);
        lv.nb[l] = FvLaunch<T>::lin_level(A, (const T*)p->lev[l].u, (T*)p->lev[l].F0,
                                          coarser ? (T*)p->lev[l + 1].u : nullptr, Red{fvpart(p, l, 0), nullptr}, adt,
                                          st, p->mb);
        lv.hx[l] = (double)A.hx;
        lv.hz[l] = (double)A.hz;
    }
    FvLaunch<T>::lin_finalize(fvpart(p, 0, 0), (long)FVP_PER_LEVEL * p->fvp, lv, p->nlev, p->scal + S_LEV,
                              (double)fv_args<T>(p, 0).mu, adt, p->cfg.pseudo_cfl, st, p->mb);
    if (p->key.a || p->key.b) {
        // DG-level pseudo time step: the level formula with the element widths over
        // 2k+1 (the explicit DG step scale) and the finest FV level's wave speed
        const double kk = 2.0 * p->cfg.k + 1.0;
        launch_dg_dtau(p->scal + S_LEV + LV_LAM, p->scal + S_DTDG, p->A.dx / kk, p->A.dz / kk, p->cfg.mu, adt,
                       p->cfg.pseudo_cfl_dg, st, p->mb);
    }
    p->have_lin = 1;
    return check_launch(p);
}

jfmg_status linearize(jfmg_problem* p, const double* U, double adt)
{
    return p->prec == 32 ? linearize_t<float>(p, U, adt) : linearize_t<double>(p, U, adt);
}

// ---------------------------------------------------------------------------
// Multigrid MG_l(x, b; u): smoother = s-stage low-storage explicit RK in
// pseudo time with one uniform dtau per level; a zero flag replaces the
// matvec with the zero vector.  Level 0 is the finest.
// ---------------------------------------------------------------------------
struct MgState {
    int xi[MAXLEV];      // buffer holding x on each level
    bool xzero[MAXLEV];  // x is the zero vector (buffer content not valid)
    int pre[MAXLEV];     // > 0: the first stage from x = 0 is already in buffer 1 (made by the
                         // kernel that wrote b), with this many ||x||^2 partials
};

// coefficient alpha_j of the s-stage low-storage pseudo-time smoother (j from 0):
// the configured one, else 1/(s - j)
double smoother_alpha(const jfmg_problem* p, int j)
{
    return p->cfg.rk_alpha[j] > 0 ? p->cfg.rk_alpha[j] : 1.0 / (p->cfg.rk_stages - j);
}

template <typename T> struct Mg {
    jfmg_problem* p;
    MgState s;
    double alpha[4];
    // set by mg_apply_t: the last stage of the cycle on the finest level applies the
    // FV -> DG transfer itself (FvLaunch::stage_tinv), ||z||^2 into tinv_red.out
    const TinvOut* tinv = nullptr;
    Red tinv_red{};   // without .out the partials are left for the consumer
    bool tinv_done = false;
    int tinv_count = 0;   // number of ||z||^2 partials

    void init()
    {
        for (int j = 0; j < 4; ++j) alpha[j] = smoother_alpha(p, j);
        for (int l = 0; l < MAXLEV; ++l) s.pre[l] = 0;
    }
    // the first stage of level l from x = 0 can be fused into the kernel that writes b
    ZeroStage<T> zero_stage(int l, int nu_pre)
    {
        ZeroStage<T> z;
        if (nu_pre > 0 && p->cfg.rk_stages >= 1) {
            z.x1 = (T*)p->lev[l].buf[1];
            z.slots = p->scal + S_LEV + 4 * l;
            z.alpha = alpha[0];
            z.red = Red{fvpart(p, l, 1), nullptr};
        }
        return z;
    }

    // nu sweeps on level l.  With pc >= 0 (the next finer level) the last stage of the
    // last sweep does not store its result v but applies the coarse-grid correction
    // x_pc -= P v itself (FvLaunch::stage_prolong); returns whether it did.
    // With post set on the finest level (the cycle's final sweeps) the very last stage
    // may apply the FV -> DG transfer instead (tinv).
    bool smooth(int l, int nu, int pc = -1, bool post = false)
    {
        const FvArgs<T> A = fv_args<T>(p, l);
        Level& L = p->lev[l];
        const int S = p->cfg.rk_stages;
        bool fused = false;
        for (int sw = 0; sw < nu; ++sw) {
            const int i0 = s.xi[l];
            const int oth[2] = {(i0 + 1) % 3, (i0 + 2) % 3};
            int prev = i0;
            for (int j = 0; j < S; ++j) {
                const int out = oth[j & 1];
                const int zero = (j == 0 && s.xzero[l]) ? 1 : 0;
                if (zero && s.pre[l] > 0 && out == 1) {   // made by the producer of b
                    p->xcnt[l][out] = s.pre[l];
                    s.pre[l] = 0;
                    prev = out;
                    continue;
                }
                const T* x0 = s.xzero[l] ? nullptr : (const T*)L.buf[i0];   // null: x^(0) = 0
                const double vb = 4.0 * L.nc * sizeof(T);
                if (pc >= 0 && sw == nu - 1 && j == S - 1 && !zero) {
                    Level& F = p->lev[pc];
                    const bool fz = s.xzero[pc];
                    const int cls = fv_wide_tile(L.tile) ? JFMG_K_FV_STAGE : JFMG_K_FV_STAGE_SMALL;
                    // the stage's reads (no write of v), x_f read unless zero and written: four
                    // vectors of this level each
                    ProfScope ps(p, cls, ((x0 && prev != i0 ? 5 : 4) + (fz ? 4 : 8)) * vb);
                    p->xcnt[pc][s.xi[pc]] = FvLaunch<T>::stage_prolong(
                        A, (const T*)L.u, (const T*)L.F0, (const T*)L.buf[prev], x0, (const T*)L.b,
                        (T*)F.buf[s.xi[pc]], fz, fvpart(p, l, prev), p->xcnt[l][prev], p->scal + S_LEV + 4 * l,
                        alpha[j], p->adt, Red{fvpart(p, pc, s.xi[pc]), nullptr}, p->st, p->mb);
                    p->mv_count[l]++;
                    s.xzero[pc] = false;
                    fused = true;
                    prev = out;   // v itself is not needed any more
                    continue;
                }
                if (tinv && post && l == 0 && pc < 0 && sw == nu - 1 && j == S - 1 && !zero) {
                    int nb;
                    {   // reads u, F0, x^(j-1), x^(0) (when not x^(j-1)), b; writes the DG vector z
                        ProfScope ps(p, fv_wide_tile(L.tile) ? JFMG_K_FV_STAGE : JFMG_K_FV_STAGE_SMALL,
                                     (x0 && prev != i0 ? 5 : 4) * vb + 4.0 * L.nc * 8.0);
                        nb = FvLaunch<T>::stage_tinv(A, (const T*)L.u, (const T*)L.F0, (const T*)L.buf[prev], x0,
                                                     (const T*)L.b, *tinv, fvpart(p, l, prev), p->xcnt[l][prev],
                                                     p->scal + S_LEV + 4 * l, alpha[j], p->adt, tinv_red, p->st,
                                                     p->mb);
                    }
                    if (tinv_red.out) launch_finalize(tinv_red.partials, nb, 1, tinv_red.out, p->st, Gate{}, p->mb);
                    p->mv_count[l]++;
                    tinv_done = true;
                    tinv_count = nb;
                    prev = out;
                    continue;
                }
                // algorithmic bytes: reads u, F0, x^(j-1), x^(0), b, writes x^(j) (x^(0) not when it is 0
                // or when it is x^(j-1), the first stage of a sweep); the zero-start stage reads b and
                // writes x^(1)
                const int cls = zero ? JFMG_K_FV_STAGE_ZERO
                                     : (fv_wide_tile(L.tile) ? JFMG_K_FV_STAGE : JFMG_K_FV_STAGE_SMALL);
                ProfScope ps(p, cls, zero ? 2 * vb : (x0 && prev != i0 ? 6 : 5) * vb);
                p->xcnt[l][out] = FvLaunch<T>::stage(
                    A, (const T*)L.u, (const T*)L.F0, (const T*)L.buf[prev], x0, (const T*)L.b, (T*)L.buf[out],
                    fvpart(p, l, prev), p->xcnt[l][prev], p->scal + S_LEV + 4 * l, alpha[j], p->adt, zero,
                    Red{fvpart(p, l, out), nullptr}, p->st, p->mb);
                if (!zero) p->mv_count[l]++;
                prev = out;
            }
            s.xi[l] = prev;
            s.xzero[l] = false;
        }
        return fused;
    }

    // MG_l; with pc >= 0 the final smoother stage applies the correction of level pc
    // (see smooth); returns whether it did
    bool cycle(int l, int pc = -1)
    {
        const Key& k = p->key;
        const bool fine = (l == 0);
        smooth(l, fine ? k.c : k.e);
        if (l + 1 < p->nlev) {
            const FvArgs<T> A = fv_args<T>(p, l);
            Level& L = p->lev[l];
            Level& C = p->lev[l + 1];
            // reads u, F0, x, b and writes the quarter-size coarse defect (x = 0: reads b only),
            // and with x != 0 the coarse level's first stage from zero as well
            const ZeroStage<T> z0 = s.xzero[l] ? ZeroStage<T>{} : zero_stage(l + 1, k.e);
            int nb;
            {   // the scope ends before the coarse cycle, whose own scopes would reset the timer
                ProfScope ps(p, JFMG_K_FV_DEFECT, (s.xzero[l] ? 1.25 : (z0.x1 ? 4.5 : 4.25)) * 4.0 * L.nc * sizeof(T));
                nb = FvLaunch<T>::defect_restrict(A, (const T*)L.u, (const T*)L.F0, (const T*)L.buf[s.xi[l]],
                                                  (const T*)L.b, (T*)C.b, fvpart(p, l, s.xi[l]),
                                                  p->xcnt[l][s.xi[l]], p->scal + S_LEV + 4 * l, p->adt,
                                                  s.xzero[l] ? 1 : 0, p->st, p->mb, z0);
            }
            if (!s.xzero[l]) p->mv_count[l]++;
            s.xzero[l + 1] = true;
            s.xi[l + 1] = 0;
            s.pre[l + 1] = nb;
            bool fused = false;
            for (int cyc = 0; cyc < k.cycle; ++cyc) fused = cycle(l + 1, cyc == k.cycle - 1 ? l : -1);
            if (!fused && !s.xzero[l + 1]) {
                if (s.xzero[l]) {
                    // x = 0 - P v: materialize the zero vector first
                    launch_zero(L.buf[s.xi[l]], sizeof(T) * 4 * L.nc, p->st, p->mb);
                }
                ProfScope ps2(p, JFMG_K_FV_PROLONG, 2.25 * 4.0 * L.nc * sizeof(T));
                p->xcnt[l][s.xi[l]] = FvLaunch<T>::prolong_correct(A, (T*)L.buf[s.xi[l]], (const T*)C.buf[s.xi[l + 1]],
                                                                   Red{fvpart(p, l, s.xi[l]), nullptr}, p->st, p->mb);
                s.xzero[l] = false;
            }
        }
        return smooth(l, fine ? k.d : k.f, pc, fine);
    }

    // x = MG(0, b) on the finest level; b must be in lev[0].b; result pointer returned
    T* run()
    {
        s.xi[0] = 0;
        s.xzero[0] = true;
        cycle(0);
        if (tinv_done) return nullptr;   // z has been written by the last stage
        Level& L = p->lev[0];
        if (s.xzero[0]) launch_zero(L.buf[s.xi[0]], sizeof(T) * 4 * L.nc, p->st, p->mb);
        return (T*)L.buf[s.xi[0]];
    }
};

// z = Q^-1 r, ||z||^2 into slot zslot; with nm != nullptr r is first formed as
// nm->sgn nm->src / sqrt(nm->nrm2[0]) (in place when src == r) by the DG -> FV transfer.
// With zcount != nullptr the ||z||^2 block partials are left in p->partials instead
// (*zcount of them, for a consumer that sums them itself) and the slot is not written.
template <typename T>
jfmg_status mg_apply_t(jfmg_problem* p, double* r, double* z, int zslot, const Norm* nm, int* zcount = nullptr)
{
    Level& L = p->lev[0];
    Mg<T> mg{p};
    mg.init();
    {
        // b = T r, and the finest level's first stage from zero in the same kernel
        const ZeroStage<T> z0 = mg.zero_stage(0, p->key.c);
        ProfScope ps(p, JFMG_K_TRANSFER_T,
                     (double)p->N * (8 + (z0.x1 ? 2 : 1) * sizeof(T)) + (nm ? 8.0 * p->N : 0.0));
        const int nb = launch_transfer_T<T>(p->cfg.k, p->A, mass_fix_of(p), nm ? nm->src : r, (T*)L.b, L.nx, p->st,
                                            nm ? nm->nrm2 : nullptr, nm ? r : nullptr, p->mb, z0, nm ? nm->sgn : 1.0);
        if (z0.x1) mg.s.pre[0] = nb;
    }
    TinvOut tv;
    if (p->fuse_tinv && fv_tile_fits_elements(L.tile, p->n1)) {   // the last finest-level stage transfers back itself
        tv.z = z;
        tv.n1 = p->n1;
        tv.mass_fix = mass_fix_of(p);
        std::memcpy(tv.Vinv, p->A.R.Vinv, sizeof(tv.Vinv));
        std::memcpy(tv.wnc, p->A.R.wnc, sizeof(tv.wnc));
        mg.tinv = &tv;
        mg.tinv_red = zcount ? Red{p->partials, nullptr} : red_at(p, zslot);
    }
    T* x = mg.run();
    if (!x) {
        if (zcount) *zcount = mg.tinv_count;
        return check_launch(p);
    }
    ProfScope ps(p, JFMG_K_TRANSFER_TINV, (double)p->N * (8 + sizeof(T)));
    launch_transfer_Tinv<T>(p->cfg.k, p->A, mass_fix_of(p), x, z, L.nx,
                            zcount ? Red{p->partials, nullptr} : red_at(p, zslot), p->st, p->mb);
    if (zcount) *zcount = transfer_grid(p->cfg.k, p->A.ne);
    return check_launch(p);
}

// out = G'(U_lin) y with ||y||^2 already in slot yslot, or (ycount > 0) as ycount
// block partials in p->partials
void jvp_slot(jfmg_problem* p, const double* y, double* out, int yslot, int ycount = 0)
{
    ProfScope ps(p, JFMG_K_DG_JVP, 3.0 * p->N * 8 + 8.0 * lin_doubles(p->cfg.k, p->ne));
    launch_dg(p->cfg.k, p->cfg.physics == 1, 3, p->A, p->Ulin, y, nullptr, out,
              ycount > 0 ? p->partials : p->scal + yslot, p->scal + S_UTOT, p->cfg.fd_eps_mode, p->adt, no_red(),
              p->st, p->mb, ExStage{}, ycount);
    p->jvp_count++;
}

// nu sweeps of the DG-level smoother on G'(U) z = r, z_j = z_0 + alpha_j dtau_dg (r - G' z_{j-1})
// (G' 0 skipped while z is zero).  ||z||^2 is in S_DGZ on entry (z nonzero) and on exit,
// except that the very last stage writes it into slot `last` instead.  The stages
// alternate between z (the last stage of a sweep, in place over z_0) and tmp1; tmp2
// holds the products.
void dg_smooth(jfmg_problem* p, double* z, const double* r, int nu, bool& zzero, int last)
{
    const int S = p->cfg.rk_stages;
    double* xs = p->tmp1;
    double* t = p->tmp2;
    const double* dtau = p->scal + S_DTDG;
    for (int sw = 0; sw < nu; ++sw) {
        for (int j = 0; j < S; ++j) {
            const bool lastst = j == S - 1;
            double* out = lastst ? z : xs;
            const double* prev = j == 0 ? z : xs;
            const int slot = lastst ? (sw == nu - 1 ? last : S_DGZ) : S_DGX;
            if (j == 0 && zzero) {   // reads r, writes z_1
                ProfScope ps(p, JFMG_K_DG_SMOOTH, 2.0 * p->N * 8);
                launch_dg_smooth(out, nullptr, r, nullptr, smoother_alpha(p, j), dtau, p->N, red_at(p, slot), p->st,
                                 p->mb);
            } else {                 // reads r, G' z_{j-1} and z_0 (when nonzero), writes z_j
                jvp_slot(p, prev, t, j == 0 ? S_DGZ : S_DGX);
                ProfScope ps(p, JFMG_K_DG_SMOOTH, (zzero ? 3.0 : 4.0) * p->N * 8);
                launch_dg_smooth(out, zzero ? nullptr : z, r, t, smoother_alpha(p, j), dtau, p->N, red_at(p, slot),
                                 p->st, p->mb);
            }
        }
        zzero = false;
    }
}

// z = Q^-1 r with the DG data as the finest level of the cycle (key a, b > 0): a DG
// sweeps from z = 0, z += T^-1 q^-1 T (r - G' z), b DG sweeps; ||z||^2 into zslot
template <typename T> jfmg_status mg_apply_dg_t(jfmg_problem* p, double* r, double* z, int zslot, const Norm* nm)
{
    const Key& k = p->key;
    if (nm) launch_scale(r, nm->src, p->N, nm->nrm2, p->st, nm->sgn, p->mb);
    bool zzero = true;
    dg_smooth(p, z, r, k.a, zzero, S_DGZ);
    const int cslot = k.b ? S_DGZ : zslot;
    jfmg_status s;
    if (zzero) {
        s = mg_apply_t<T>(p, r, z, cslot, nullptr);
    } else {
        // defect d = r - G' z in tmp2, correction into tmp1, z += it
        jvp_slot(p, z, p->tmp2, S_DGZ);
        {
            ProfScope ps(p, JFMG_K_DG_SMOOTH, 3.0 * p->N * 8);
            launch_dg_smooth(p->tmp2, nullptr, r, p->tmp2, 1.0, nullptr, p->N, Red{nullptr, nullptr}, p->st, p->mb);
        }
        s = mg_apply_t<T>(p, p->tmp2, p->tmp1, S_DGC, nullptr);
        if (s) return s;
        ProfScope ps(p, JFMG_K_DG_SMOOTH, 3.0 * p->N * 8);
        launch_dg_smooth(z, z, p->tmp1, nullptr, 1.0, nullptr, p->N, red_at(p, cslot), p->st, p->mb);
    }
    if (s) return s;
    zzero = false;
    dg_smooth(p, z, r, k.b, zzero, zslot);
    return check_launch(p);
}

// z = Q^-1 r, ||z||^2 into slot zslot; with nm != nullptr r is first formed as
// nm->sgn nm->src / ||nm->src|| (the Arnoldi v_j = w / ||w||, v_0 = -G / ||G||).  With
// zcount != nullptr the FV multigrid form may leave the ||z||^2 partials in
// p->partials instead (*zcount > 0 then; 0 means the slot was written).
jfmg_status precond(jfmg_problem* p, double* r, double* z, int zslot, const Norm* nm = nullptr,
                    int* zcount = nullptr)
{
    if (zcount) *zcount = 0;
    if (!p->cfg.precond) {
        if (nm) launch_scale(r, nm->src, p->N, nm->nrm2, p->st, nm->sgn, p->mb);
        HIPCHK(p, copy_members(p, z, r, sizeof(double) * p->N));
        launch_norm2(z, p->N, red_at(p, zslot), p->st, p->mb);
        return check_launch(p);
    }
    if (p->key.a || p->key.b)
        return p->prec == 32 ? mg_apply_dg_t<float>(p, r, z, zslot, nm) : mg_apply_dg_t<double>(p, r, z, zslot, nm);
    return p->prec == 32 ? mg_apply_t<float>(p, r, z, zslot, nm, zcount)
                         : mg_apply_t<double>(p, r, z, zslot, nm, zcount);
}

// G = U - adt f(U) - Ubar and its norm (host)
jfmg_status stage_residual(jfmg_problem* p, const double* U, const double* Ubar, double adt, double* G, double* nrm)
{
    {
        ProfScope ps(p, JFMG_K_DG_RESIDUAL, 3.0 * p->N * 8);
        launch_dg(p->cfg.k, p->cfg.physics == 1, 2, p->A, U, nullptr, Ubar, G, nullptr, nullptr, 0, adt, red_at(p, S_G),
                  p->st, p->mb);
    }
    p->lh_count++;
    jfmg_status s = check_launch(p);
    if (s) return s;
    if (nrm) {   // one norm per member
        s = read_scalars(p, S_G, 1, nrm);
        if (s) return s;
        for (int b = 0; b < p->mb.n; ++b) nrm[b] = std::sqrt(nrm[b]);
    }
    return JFMG_OK;
}

// ---------------------------------------------------------------------------
// Right-preconditioned FGMRES(m) for G'(U) delta = -G, CGS2 Arnoldi on device,
// Givens rotations on the host; U += delta on success.
// ---------------------------------------------------------------------------
// One FGMRES iteration on the device: v_j = w_{j-1}/||w_{j-1}|| (j > 0),
// z_j = Q^-1 v_j, w = G'(U) z_j, classical Gram-Schmidt against v_0..v_j with a
// re-orthogonalization pass where needed; leaves h1, h2 (0 without the second
// pass) and ||w||^2 in the scalar slots and in pinned host memory.  No host
// synchronization.
// Re-orthogonalize when the first Gram-Schmidt pass leaves less than this
// fraction of ||w|| (Kahan's "twice is enough" test with kappa = 10).
constexpr double REORTH_TAU = 0.1;

jfmg_status iter_ops(jfmg_problem* p, int j)
{
    const long N = p->N;
    hipStream_t st = p->st;
    double* vj = p->V + (long)j * N;
    double* zj = p->Z + (long)j * N;
    double* w = p->V + (long)(j + 1) * N;
    // v_j = w_{j-1} / ||w_{j-1}|| (j > 0), and v_0 where the cycle left it to this
    // iteration (p->v0), is formed by the preconditioner's first kernel
    int zc = 0;   // > 0: ||z_j||^2 is left as block partials, summed by the JVP itself
    const Norm nw{vj, p->scal + S_W, 1.0};
    const Norm* nm = j > 0 ? &nw : (p->v0.src ? &p->v0 : nullptr);
    jfmg_status s = precond(p, vj, zj, S_Z, nm, &zc);
    if (s) return s;
    jvp_slot(p, zj, w, S_Z, zc);
    // Classical Gram-Schmidt; the second (re-orthogonalization) pass runs only
    // where the first one cancelled more than 1 - REORTH_TAU of ||w||, decided
    // on the device (the gated kernels return at once otherwise).
    const int nv = j + 1;
    const double md = (j + 2.0) * N * 8, up = (j + 3.0) * N * 8;
    // ||w||^2 after the first pass is taken by Pythagoras from its coefficients and
    // ||w||^2 before it (Gate), so the first update needs no norm of its own
    const Gate reorth{p->scal + S_H1, nv, p->reorth_always ? 1e300 : REORTH_TAU * REORTH_TAU};
    // the gated second pass: its multi-dot is taken by the first update kernel (from the w
    // it has formed), its coefficients are summed by its own update kernel, and its ||w||^2
    // partials go after the multi-dot's.  The scalar block h1, h2 (0 where the second pass
    // did not run), ||w||^2 (of the second pass where it ran, else the first pass's by
    // Pythagoras) of iteration j goes to pinned host memory from the first update kernel
    // where the pass is skipped, else from the second
    Publish pub;
    pub.out = p->scal + S_W;
    pub.src = p->scal + S_H1;
    pub.ns = S_HB;
    pub.idx = S_W - S_H1;
    pub.host = p->hpin + (size_t)j * S_HB;
    pub.host_stride = (long)S_HB * p->m;
    pub.zoff = S_H2 - S_H1;
    pub.zn = nv;
    pub.fidx = S_RF - S_H1;
    pub.cnt = (unsigned long long*)(p->scal + S_CNT);
    { ProfScope ps(p, JFMG_K_MULTIDOT, md); launch_multidot(w, p->V, N, nv, 1, N, Gate{}, red_at(p, S_H1), st, p->mb); }
    { ProfScope ps(p, JFMG_K_UPDATE, up);
      launch_update(w, p->V, N, nv, N, p->scal + S_H1, Red{nullptr, nullptr}, st, Gate{}, p->mb, reorth,
                    p->partials, pub); }
    double* wpart = p->partials + (long)(p->m + 1) * la_blocks(N);
    launch_update2_publish(w, p->V, N, nv, N, reorth, p->partials, p->scal + S_H2, wpart, pub, st, p->mb);
    return check_launch(p);
}

void invalidate_graphs(jfmg_problem* p)
{
    for (auto& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
    }
}

// Run iteration j, from its captured graph when graphs are on (captured on
// first use; the multigrid schedule and all pointers are fixed per problem,
// every varying scalar lives in device memory).
jfmg_status run_iter(jfmg_problem* p, int j)
{
    if (!p->use_graphs || p->prof.mask) return iter_ops(p, j);   // profiling times eager launches
    if ((int)p->graphs.size() < p->m) p->graphs.resize(p->m);
    if (p->graph_adt != p->adt) {
        invalidate_graphs(p);
        p->graph_adt = p->adt;
    }
    auto& G = p->graphs[j];
    if (!G.exec) {
        int mv0[MAXLEV];
        std::memcpy(mv0, p->mv_count, sizeof(mv0));
        const int j0 = p->jvp_count;
        HIPCHK(p, hipStreamBeginCapture(p->st, hipStreamCaptureModeThreadLocal));
        p->capturing = &G;
        jfmg_status s = iter_ops(p, j);
        p->capturing = nullptr;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(p->st, &graph);
        if (s) {
            if (!e && graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (!e) {
            e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
        }
        if (e) {   // graphs unavailable here: run this problem eagerly from now on
            G.exec = nullptr;
            (void)hipGetLastError();
            std::memcpy(p->mv_count, mv0, sizeof(mv0));
            p->jvp_count = j0;
            p->use_graphs = false;
            return iter_ops(p, j);
        }
        for (int l = 0; l < MAXLEV; ++l) {
            G.mv[l] = p->mv_count[l] - mv0[l];
            p->mv_count[l] = mv0[l];
        }
        G.jvps = p->jvp_count - j0;
        p->jvp_count = j0;
    }
    HIPCHK(p, hipGraphLaunch(G.exec, p->st));
    for (int l = 0; l < MAXLEV; ++l) p->mv_count[l] += G.mv[l];
    p->jvp_count += G.jvps;
    return JFMG_OK;
}

// ---------------------------------------------------------------------------
// Right-preconditioned FGMRES(m) for G'(U) delta = -G, CGS2 Arnoldi on device,
// Givens rotations on the host; U += delta on success.
// ---------------------------------------------------------------------------
// Members of a lock-step batch run the same iterations; each member's
// Hessenberg column is read from its own pinned block and a member stops
// taking part (its coefficients stay 0, so its delta is no longer changed)
// once it has converged.  `active` marks the members that solve at all.
// ragged batch: live flags of the members (1 for those that pred selects) in the device table
template <typename F> void set_live(jfmg_problem* p, F&& pred)
{
    if (!p->ragged) return;
    LiveBits bits{};
    for (int b = 0; b < p->mb.n; ++b)
        if (pred(b)) bits.w[b >> 6] |= 1ull << (b & 63);
    launch_set_live(p->tab, p->mb.n, bits, p->st);
}

jfmg_status fgmres_cycles(jfmg_problem* p, const double* G, const std::vector<double>& gnorm, const std::vector<double>& tol,
                   const std::vector<char>& active, double* U, int* its_out)
{
    const long N = p->N;
    const int m = p->m, B = p->mb.n;
    hipStream_t st = p->st;
    struct Member {
        std::vector<double> H, cs, sn, g, y;
        std::vector<double> res;   // residual estimate |g_j| after iteration j-1 (res[0] = beta)
        double beta = 0.0;
        bool done = false, conv = false;
        int jend = 0;
    };
    std::vector<Member> M(B);
    int left = 0;
    for (int b = 0; b < B; ++b) {
        Member& x = M[b];
        x.H.assign((size_t)(m + 1) * m, 0.0);
        x.cs.assign(m, 0.0);
        x.sn.assign(m, 0.0);
        x.g.assign(m + 1, 0.0);
        x.y.assign(m, 0.0);
        x.res.assign(m + 1, 0.0);
        x.beta = gnorm[b];
        x.done = !active[b];
        left += !x.done;
    }
    int its = 0;
    // V_0 = -G / ||G|| (||G||^2 of each member in slot S_G), formed by iteration 0's first
    // kernel (a separate launch where iterations are replayed from graphs)
    auto set_v0 = [&](const double* src, int slot, double sgn) {
        if (p->use_graphs) launch_scale(p->V, src, N, p->scal + slot, st, sgn, p->mb);
        else p->v0 = Norm{src, p->scal + slot, sgn};
    };
    set_v0(G, S_G, -1.0);
    bool delta_zero = true;   // delta = 0 until the first cycle's combination writes it
    std::vector<double> ybuf((size_t)B * m), r2(B);
    jfmg_status status = left ? JFMG_ENOCONV : JFMG_OK;
    std::vector<char> part(B);   // members that take part in the current cycle
    for (int cyc = 0; left && cyc <= p->cfg.gmres_max_restarts; ++cyc) {
        for (Member& x : M) {
            std::fill(x.g.begin(), x.g.end(), 0.0);
            x.g[0] = x.beta;
            x.res[0] = std::fabs(x.beta);
            x.jend = 0;
            x.conv = false;
        }
        // in a ragged batch the members that are done, and later those that converge
        // within the cycle, sit out the iterations' kernels
        for (int b = 0; b < B; ++b) part[b] = !M[b].done;
        set_live(p, [&](int b) { return part[b] != 0; });
        // Iteration j+1 is issued before the host looks at iteration j's
        // Hessenberg columns, so the readback round trip overlaps GPU work, except
        // where iteration j is likely to end the cycle: a speculative iteration
        // issued in vain costs a whole iteration of the device, one issued after
        // the readback only the host's turnaround (≈15 us).  "Likely": every active
        // member's residual estimate, extrapolated by its fastest recent reduction
        // factor (1/4 before the first iteration), is within SPEC_MARGIN of its
        // tolerance.
        constexpr double SPEC_MARGIN = 4.0;
        auto likely_end = [&](int j) {
            bool any = false;
            for (int mb = 0; mb < B; ++mb) {
                const Member& x = M[mb];
                if (x.done || x.conv) continue;
                any = true;
                double rho = 0.25;
                if (j >= 1 && x.res[j - 1] > 0.0) rho = x.res[j] / x.res[j - 1];
                if (j >= 2 && x.res[j - 2] > 0.0) rho = std::min(rho, x.res[j - 1] / x.res[j - 2]);
                if (!(x.res[j] * rho <= SPEC_MARGIN * tol[mb])) return false;
            }
            return any;
        };
        auto issue = [&](int j) -> jfmg_status {
            jfmg_status s = run_iter(p, j);   // ends by publishing its scalars to hpin
            if (s) return s;
            HIPCHK(p, hipEventRecord(p->hev[j], st));
            return JFMG_OK;
        };
        jfmg_status s0 = issue(0);
        p->v0 = Norm{};
        if (s0) return s0;
        int next = 1;   // next iteration to issue
        for (int j = 0; j < m; ++j) {
            if (next == j + 1 && j + 1 < m && !likely_end(j)) {
                jfmg_status s = issue(j + 1);
                if (s) return s;
                ++next;
            }
            HIPCHK(p, hipEventSynchronize(p->hev[j]));
            p->syncs++;
            ++its;
            bool all_conv = true, conv_now = false;
            for (int mb = 0; mb < B; ++mb) {
                Member& x = M[mb];
                if (x.done || x.conv) continue;
                std::vector<double>& H = x.H;
                const double* hb = p->hpin + ((size_t)mb * m + j) * S_HB;
                for (int i = 0; i <= j; ++i) H[i * m + j] = hb[i] + hb[(S_H2 - S_H1) + i];
                p->reorths += hb[S_RF - S_H1] != 0.0;
                const double hn = std::sqrt(hb[S_W - S_H1]);
                H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double a = H[i * m + j], b = H[(i + 1) * m + j];
                    H[i * m + j] = x.cs[i] * a + x.sn[i] * b;
                    H[(i + 1) * m + j] = -x.sn[i] * a + x.cs[i] * b;
                }
                const double a = H[j * m + j], b = H[(j + 1) * m + j];
                const double rr = std::sqrt(a * a + b * b);
                x.cs[j] = a / rr;
                x.sn[j] = b / rr;
                H[j * m + j] = rr;
                H[(j + 1) * m + j] = 0.0;
                x.g[j + 1] = -x.sn[j] * x.g[j];
                x.g[j] = x.cs[j] * x.g[j];
                x.res[j + 1] = std::fabs(x.g[j + 1]);
                x.jend = j + 1;
                if (!std::isfinite(x.g[j + 1]) || !std::isfinite(hn)) {
                    *its_out = its;
                    return fail(p, JFMG_ENONFINITE, "non-finite value in the Arnoldi process");
                }
                if (std::fabs(x.g[j + 1]) <= tol[mb] || hn == 0.0) x.conv = conv_now = true;
                else all_conv = false;
            }
            if (all_conv) break;
            if (p->ragged && conv_now) set_live(p, [&](int b) { return part[b] && !M[b].conv; });
            if (next == j + 1 && j + 1 < m) {   // not issued speculatively
                jfmg_status s = issue(j + 1);
                if (s) return s;
                ++next;
            }
        }
        set_live(p, [&](int b) { return part[b] != 0; });   // the cycle's update, restart residual
        int jmax = 0;
        std::fill(ybuf.begin(), ybuf.end(), 0.0);
        for (int mb = 0; mb < B; ++mb) {
            Member& x = M[mb];
            if (x.done) continue;
            for (int i = x.jend - 1; i >= 0; --i) {
                double s = x.g[i];
                for (int t = i + 1; t < x.jend; ++t) s -= x.H[i * m + t] * x.y[t];
                x.y[i] = s / x.H[i * m + i];
            }
            std::copy(x.y.begin(), x.y.begin() + x.jend, ybuf.begin() + (size_t)mb * m);
            jmax = std::max(jmax, x.jend);
        }
        if (jmax > 0) {
            // the previous cycle's scatter has finished reading ycoef (its lincomb was
            // followed by a synchronizing read or this cycle's event waits)
            std::copy(ybuf.begin(), ybuf.end(), p->ycoef);
            launch_scatter(p->scal + S_Yc, jmax, p->ycoef, m, st, p->mb);
            // the first combination starts from zero (delta = Z y); a ragged member that sits it
            // out needs its delta cleared first
            if (delta_zero && p->ragged && std::find(part.begin(), part.end(), 0) != part.end())
                launch_zero(p->delta, sizeof(double) * N, st, p->mb), delta_zero = false;
            launch_lincomb(p->delta, delta_zero ? nullptr : p->delta, p->Z, N, jmax, N, p->scal + S_Yc, st, p->mb);
            delta_zero = false;
        }
        prof_flush(p);
        for (Member& x : M)
            if (!x.done && x.conv) { x.done = true; --left; }
        if (!left) { status = JFMG_OK; break; }
        if (cyc == p->cfg.gmres_max_restarts) break;
        // restart the others from the true residual r = -G - G' delta
        launch_norm2(p->delta, N, red_at(p, S_Y), st, p->mb);
        jvp_slot(p, p->delta, p->tmp2, S_Y);
        launch_axpby(p->tmp2, -1.0, G, -1.0, p->tmp2, N, st, p->mb);
        launch_norm2(p->tmp2, N, red_at(p, S_R), st, p->mb);
        jfmg_status s = read_scalars(p, S_R, 1, r2.data());
        if (s) return s;
        for (int mb = 0; mb < B; ++mb) {
            Member& x = M[mb];
            if (x.done) continue;
            x.beta = std::sqrt(r2[mb]);
            if (!std::isfinite(x.beta)) return fail(p, JFMG_ENONFINITE, "non-finite restart residual");
            if (x.beta <= tol[mb]) { x.done = true; --left; }
        }
        if (!left) { status = JFMG_OK; break; }
        set_v0(p->tmp2, S_R, 1.0);   // V_0 = r / ||r||
    }
    *its_out = its;
    if (status != JFMG_OK) return fail(p, JFMG_ENOCONV, "FGMRES did not reach its tolerance");
    set_live(p, [](int) { return true; });   // every member's delta, from all cycles
    if (!delta_zero) launch_axpby(U, 1.0, U, 1.0, p->delta, N, st, p->mb);
    return check_launch(p);
}

jfmg_status fgmres(jfmg_problem* p, const double* G, const std::vector<double>& gnorm, const std::vector<double>& tol,
                   const std::vector<char>& active, double* U, int* its_out)
{
    const jfmg_status s = fgmres_cycles(p, G, gnorm, tol, active, U, its_out);
    p->v0 = Norm{};
    set_live(p, [](int) { return true; });   // every member takes part in the Newton-level work
    return s;
}

// Inexact Newton for G(U) = U - adt f(U) - Ubar = 0 from U^0 = Ubar; result in
// p->Uk.  The members of a batch iterate in lock step; a member whose test is
// met takes no further part (its updates are zero).
jfmg_status newton_stage(jfmg_problem* p, const double* Ubar, double adt, jfmg_stats* st)
{
    const jfmg_config& c = p->cfg;
    const int B = p->mb.n;
    HIPCHK(p, copy_members(p, p->Uk, Ubar, sizeof(double) * p->N));
    std::vector<double> g0(B), gk(B), gprev(B), eta(B, c.ew_eta0), tol(B);
    std::vector<char> active(B, 1);
    jfmg_status s = stage_residual(p, p->Uk, Ubar, adt, p->G, g0.data());
    if (s) return s;
    int left = 0;
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(g0[b])) return fail(p, JFMG_ENONFINITE, "non-finite initial stage residual");
        if (g0[b] == 0.0) active[b] = 0;
        left += active[b];
    }
    if (st) {
        st->g0_norm = *std::max_element(g0.begin(), g0.end());
        st->g_norm = 0.0;
    }
    gk = g0;
    gprev = g0;
    for (int it = 0; left && it < c.newton_maxit; ++it) {
        for (int b = 0; b < B; ++b) {
            if (it > 0 && active[b]) {
                double en = c.ew_gamma * std::pow(gk[b] / gprev[b], c.ew_alpha);
                const double safe = c.ew_gamma * std::pow(eta[b], c.ew_alpha);
                if (safe > 0.1 && safe > en) en = safe;
                eta[b] = std::min(en, c.ew_eta_max);
            }
            tol[b] = eta[b] * gk[b];
        }
        s = linearize(p, p->Uk, adt);
        if (s) return s;
        int its = 0;
        s = fgmres(p, p->G, gk, tol, active, p->Uk, &its);
        if (st) { st->gmres_its += its; st->newton_its++; }
        if (s) return s;
        gprev = gk;
        s = stage_residual(p, p->Uk, Ubar, adt, p->G, gk.data());
        if (s) return s;
        double gmax = 0.0;
        for (int b = 0; b < B; ++b) {
            if (!active[b]) continue;
            if (!std::isfinite(gk[b])) return fail(p, JFMG_ENONFINITE, "non-finite stage residual");
            gmax = std::max(gmax, gk[b]);
            bool stop = gk[b] < c.newton_rtol * g0[b];
            // rounding floor of G: no halving any more although already below newton_stall ||G^0||
            if (!stop && c.newton_stall > 0.0 && gk[b] <= c.newton_stall * g0[b] && gk[b] > 0.5 * gprev[b]) {
                if (st) st->stall_stops++;
                stop = true;
            }
            if (stop) {
                active[b] = 0;
                --left;
                if (st) st->reached_rtol = std::max(st->reached_rtol, gk[b] / g0[b]);
            }
        }
        if (st) st->g_norm = gmax;
    }
    if (left) return fail(p, JFMG_ENOCONV, "Newton did not converge within newton_maxit");
    return JFMG_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
namespace {
// Time the smoother stage kernel of every level in every tile shape (see jfmg_autotune).
template <typename T> jfmg_status autotune_t(jfmg_problem* p, int reps, int* shapes, double* times_us)
{
    hipStream_t st = p->st;
    hipEvent_t e0, e1;
    HIPCHK(p, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(p, JFMG_EDEVICE, "hipEventCreate failed");
    }
    jfmg_status res = JFMG_OK;
    for (int l = 0; l < p->nlev && res == JFMG_OK; ++l) {
        Level& L = p->lev[l];
        const long n = 4 * L.nc;
        // test vector in buffer 0 (fixed pattern of O(1) values) and its norm partials
        launch_fill_pattern((T*)L.buf[0], n, st, p->mb);
        FvLaunch<T>::norm2((const T*)L.buf[0], n, Red{fvpart(p, l, 0), nullptr}, st, p->mb);
        const int xc = FvLaunch<T>::norm_blocks(n);
        int best = L.tile;
        float best_ms = 0.0f;
        for (int sh = 0; sh < JFMG_TILE_NSHAPE; ++sh) {
            FvArgs<T> A = fv_args<T>(p, l);
            A.tile = sh;
            auto launch = [&]() {
                FvLaunch<T>::stage(A, (const T*)L.u, (const T*)L.F0, (const T*)L.buf[0], (const T*)L.buf[0],
                                   (const T*)L.buf[0], (T*)L.buf[1], fvpart(p, l, 0), xc, p->scal + S_LEV + 4 * l,
                                   1.0, p->adt, 0, Red{fvpart(p, l, 1), nullptr}, st, p->mb);
            };
            launch();
            if (hipEventRecord(e0, st) != hipSuccess) { res = fail(p, JFMG_EDEVICE, "hipEventRecord failed"); break; }
            for (int r = 0; r < reps; ++r) launch();
            float ms = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                res = fail(p, JFMG_EDEVICE, "event timing failed");
                break;
            }
            if (times_us) times_us[l * JFMG_TILE_NSHAPE + sh] = 1e3 * ms / reps;
            if (sh == 0 || ms < best_ms) { best = sh; best_ms = ms; }
        }
        if (res == JFMG_OK) {
            L.tile = best;
            if (shapes) shapes[l] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    invalidate_graphs(p);
    if (res) return res;
    return check_launch(p);
}
}  // namespace

extern "C" {

jfmg_status jfmg_config_default(jfmg_config* c)
{
    if (!c) return JFMG_EINVAL;
    std::memset(c, 0, sizeof(*c));
    c->nx = 16; c->nz = 16; c->k = 1;
    c->physics = 0; c->background = 0; c->bc = 0; c->scheme = 1;
    c->newton_maxit = 20; c->gmres_m = 30; c->gmres_max_restarts = 10; c->fd_eps_mode = 1;
    c->mg_levels = 3; c->rk_stages = 3; c->mass_fix = 1; c->mg_precision = 64; c->precond = 1;
    std::strcpy(c->mg_key, "mg002222V");
    c->x0 = 0; c->x1 = 1000; c->z0 = 0; c->z1 = 1000;
    c->g = 9.81; c->gamma = 1.4; c->R = 287.0; c->p0 = 1e5;
    c->theta0 = 300.0; c->N = 0.0; c->u_mean = 0.0; c->mu = 0.0; c->c_ip = 2.0;
    c->dt = 1.0; c->newton_rtol = 1e-8;
    c->ew_gamma = 0.1; c->ew_alpha = 1.0; c->ew_eta0 = 0.1; c->ew_eta_max = 0.9;
    c->pseudo_cfl = 1.0;
    c->pseudo_cfl_dg = 1.0;
    return JFMG_OK;
}

}  // extern "C"

namespace {

// Members of a ragged batch may differ in these fields only.
bool same_but_grid(const jfmg_config& a, const jfmg_config& b)
{
    static_assert(sizeof(jfmg_config) == 14 * 4 + 16 + 26 * 8 + 2 * 4 + 8, "jfmg_config has no padding");
    jfmg_config x = a, y = b;
    for (jfmg_config* c : {&x, &y}) {
        c->nx = c->nz = 0;
        c->x0 = c->x1 = c->z0 = c->z1 = 0.0;
        c->batch = 0;
    }
    return std::memcmp(&x, &y, sizeof(x)) == 0;
}

// The configuration whose workspace layout every member of a ragged batch uses:
// the largest grid in each direction.
jfmg_config envelope(const jfmg_config* cfgs, int n)
{
    jfmg_config e = cfgs[0];
    for (int m = 1; m < n; ++m) {
        e.nx = std::max(e.nx, cfgs[m].nx);
        e.nz = std::max(e.nz, cfgs[m].nz);
    }
    e.batch = n;
    return e;
}

size_t table_bytes(int n) { return ((sizeof(MemberArgs) * (size_t)n + 255) & ~size_t(255)); }

jfmg_status validate_ensemble(const jfmg_config* cfgs, int n, Key& key, std::string& msg)
{
    if (!cfgs || n < 1 || n > 4096) { msg = "an ensemble has 1..4096 members"; return JFMG_EINVAL; }
    for (int m = 0; m < n; ++m) {
        jfmg_config c = cfgs[m];
        if (c.batch > 1) { msg = "ensemble members are single problems (batch 0 or 1)"; return JFMG_EINVAL; }
        c.batch = 0;
        jfmg_status s = validate(c, key, msg);
        if (s) { msg = "member " + std::to_string(m) + ": " + msg; return s; }
        if (!same_but_grid(cfgs[0], c)) {
            msg = "ensemble members may differ only in nx, nz and the domain";
            return JFMG_EINVAL;
        }
    }
    if (key.a || key.b) { msg = "DG-level smoothing (key a, b) is not available in a ragged batch"; return JFMG_EINVAL; }
    const jfmg_config e = envelope(cfgs, n);
    return validate(e, key, msg);
}

// Background tables of configuration c (its own grid and domain) into the member
// region that starts `off` bytes after member 0.  The host arrays are kept in
// `keep` until the stream is synchronized.
hipError_t upload_tables(jfmg_problem* p, const jfmg_config& c, size_t off, std::vector<std::vector<char>>& keep)
{
    auto at = [off](void* ptr) { return (void*)((char*)ptr + off); };
    hipStream_t st = p->st;
    auto up = [&](void* dst, const std::vector<double>& v, bool single) {
        std::vector<char> b(v.size() * (single ? 4 : 8));
        if (single) { for (size_t i = 0; i < v.size(); ++i) ((float*)b.data())[i] = (float)v[i]; }
        else std::memcpy(b.data(), v.data(), b.size());
        keep.push_back(std::move(b));
        return hipMemcpyAsync(at(dst), keep.back().data(), keep.back().size(), hipMemcpyHostToDevice, st);
    };
    const int n1 = p->n1;
    const double dz = (c.z1 - c.z0) / c.nz;
    std::vector<double> bgn((size_t)c.nz * n1 * 4), dbgn(bgn.size()), thn((size_t)c.nz * n1);
    std::vector<double> bgf((size_t)(c.nz + 1) * 4), dbgf(bgf.size());
    std::vector<double> pbn((size_t)c.nz * n1 * 2), pbfc((size_t)(c.nz + 1) * 2);   // [pb | 1/rt]
    for (int ez = 0; ez < c.nz; ++ez)
        for (int b = 0; b < n1; ++b) {
            const double z = c.z0 + (ez + 0.5 * (1.0 + p->R.xi[b])) * dz;
            const BgPoint bp = background_at(c, z);
            const int zi = ez * n1 + b;
            for (int k = 0; k < 4; ++k) { bgn[zi * 4 + k] = bp.U[k]; dbgn[zi * 4 + k] = bp.dU[k]; }
            thn[zi] = bp.theta;
            pbn[zi] = bg_pressure(c, bp.U[3]);
            pbn[(size_t)c.nz * n1 + zi] = 1.0 / bp.U[3];
        }
    for (int f = 0; f <= c.nz; ++f) {
        const BgPoint bp = background_at(c, c.z0 + f * dz);
        for (int k = 0; k < 4; ++k) { bgf[f * 4 + k] = bp.U[k]; dbgf[f * 4 + k] = bp.dU[k]; }
        pbfc[f] = bg_pressure(c, bp.U[3]);
        pbfc[c.nz + 1 + f] = 1.0 / bp.U[3];
    }
    hipError_t e = hipSuccess;
    e = e ? e : up(p->bg_node, bgn, false);
    e = e ? e : up(p->dbg_node, dbgn, false);
    e = e ? e : up(p->th_node, thn, false);
    e = e ? e : up(p->bg_face, bgf, false);
    e = e ? e : up(p->dbg_face, dbgf, false);
    e = e ? e : up(p->pb_node, pbn, false);
    e = e ? e : up(p->pb_face, pbfc, false);
    int nzl = n1 * c.nz;
    for (int l = 0; l < p->nlev && !e; ++l, nzl /= 2) {
        const Level& L = p->lev[l];
        const double hz = (c.z1 - c.z0) / nzl;
        std::vector<double> c4((size_t)nzl * 4), f4((size_t)(nzl + 1) * 4), df4(f4.size());
        std::vector<double> pc2((size_t)nzl * 2), pf2((size_t)(nzl + 1) * 2);
        for (int J = 0; J < nzl; ++J) {
            const BgPoint bp = background_at(c, c.z0 + (J + 0.5) * hz);
            for (int k = 0; k < 4; ++k) c4[J * 4 + k] = bp.U[k];
            pc2[2 * J] = bg_pressure(c, bp.U[3]);
            pc2[2 * J + 1] = 1.0 / bp.U[3];
        }
        for (int J = 0; J <= nzl; ++J) {
            const BgPoint bp = background_at(c, c.z0 + J * hz);
            for (int k = 0; k < 4; ++k) { f4[J * 4 + k] = bp.U[k]; df4[J * 4 + k] = bp.dU[k]; }
            pf2[2 * J] = bg_pressure(c, bp.U[3]);
            pf2[2 * J + 1] = 1.0 / bp.U[3];
        }
        const std::vector<double>* src[5] = {&c4, &f4, &df4, &pc2, &pf2};
        void* dst[5] = {L.bgc, L.bgf, L.dbgf, L.pc, L.pf};
        for (int t = 0; t < 5 && !e; ++t) e = up(dst[t], *src[t], p->prec == 32);
    }
    return e;
}

// DG kernel arguments of configuration c whose tables start `off` bytes after member 0's
DgArgs dg_args_of(const jfmg_problem* p, const jfmg_config& c, size_t off)
{
    auto at = [off](const double* ptr) { return (const double*)((const char*)ptr + off); };
    DgArgs A;
    A.ne = (long)c.nx * c.nz; A.nx = c.nx; A.nz = c.nz; A.bc = c.bc; A.physics = c.physics;
    A.dx = (c.x1 - c.x0) / c.nx; A.dz = (c.z1 - c.z0) / c.nz;
    A.J = A.dx * A.dz / 4.0; A.g = c.g; A.mu = c.mu; A.c_ip = c.c_ip;
    A.rdx2 = 2.0 / A.dx;
    A.rdz2 = 2.0 / A.dz;
    A.eta_x = A.c_ip * (double)(p->n1 * p->n1) / A.dx;
    A.eta_z = A.c_ip * (double)(p->n1 * p->n1) / A.dz;
    A.gas = make_gas<double>(c);
    A.bg_node = at(p->bg_node); A.dbg_node = at(p->dbg_node); A.th_node = at(p->th_node);
    A.bg_face = at(p->bg_face); A.dbg_face = at(p->dbg_face);
    A.pb_node = at(p->pb_node); A.irt_node = at(p->pb_node + (size_t)c.nz * p->n1);
    A.pb_face = at(p->pb_face); A.irt_face = at(p->pb_face + (c.nz + 1));
    A.R = p->R;
    A.lin0 = (double*)((char*)p->lin0 + off);
    return A;
}

// FV level l of configuration c whose tables start `off` bytes after member 0's
template <typename T> FvArgs<T> fv_args_of(const jfmg_problem* p, const jfmg_config& c, int l, size_t off)
{
    auto at = [off](const void* ptr) { return (const T*)((const char*)ptr + off); };
    const Level& L = p->lev[l];
    FvArgs<T> A;
    A.nxl = (p->n1 * c.nx) >> l; A.nzl = (p->n1 * c.nz) >> l; A.bc = c.bc; A.physics = c.physics;
    A.nc = (long)A.nxl * A.nzl;
    const double hx = (c.x1 - c.x0) / A.nxl, hz = (c.z1 - c.z0) / A.nzl;
    A.hx = (T)hx; A.hz = (T)hz; A.area = (T)(hx * hz); A.iarea = (T)(1.0 / (hx * hz)); A.g = (T)c.g; A.mu = (T)c.mu;
    A.gas = make_gas<T>(c);
    A.bgc = at(L.bgc); A.bgf = at(L.bgf); A.dbgf = at(L.dbgf); A.pc = at(L.pc); A.pf = at(L.pf);
    A.tile = L.tile;
    A.lev = l;
    return A;
}

// One problem: a single one (n = 1), a lock-step batch of equal members
// (cfgs[0].batch members) or a ragged batch of the n configurations.
jfmg_status create_impl(const jfmg_config* cfgs, int n, bool ragged, void* workspace, size_t ws_bytes,
                        void* hip_stream, jfmg_problem** out)
{
    if (!cfgs || !out) return fail(nullptr, JFMG_EINVAL, "null argument");
    *out = nullptr;
    Key key;
    std::string msg;
    jfmg_status s = ragged ? validate_ensemble(cfgs, n, key, msg) : validate(cfgs[0], key, msg);
    if (s) return fail(nullptr, s, msg);
    const jfmg_config env = ragged ? envelope(cfgs, n) : cfgs[0];
    const jfmg_config* cfg = &env;
    const int members = members_of(env);
    const size_t member_bytes = layout(env, nullptr, [](const char*, void*, size_t) {});
    const size_t need = member_bytes * (size_t)members + (ragged ? table_bytes(members) : 0);
    if (!workspace || ws_bytes < need) return fail(nullptr, JFMG_ENOMEM, "workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, JFMG_EINVAL, "workspace must be 256-byte aligned");

    jfmg_problem* p = new jfmg_problem();
    p->cfg = env;
    p->key = key;
    p->n1 = cfg->k + 1;
    p->np = p->n1 * p->n1;
    p->ne = (long)cfg->nx * cfg->nz;
    p->N = 4 * p->ne * p->np;
    p->dx = (cfg->x1 - cfg->x0) / cfg->nx;
    p->dz = (cfg->z1 - cfg->z0) / cfg->nz;
    p->nlev = cfg->mg_levels;
    p->prec = cfg->mg_precision;
    p->m = cfg->gmres_m;
    p->mb = Mb{members, (long)member_bytes};
    p->ragged = ragged;
    p->st = (hipStream_t)hip_stream;
    p->user_st = p->st;
    p->cs = nullptr;
    {   // FGMRES iterations run eagerly unless JFMG_GRAPH=1 asks for graph replay
        const char* g = std::getenv("JFMG_GRAPH");
        p->use_graphs = g && g[0] == '1';
        const char* f = std::getenv("JFMG_NO_FUSED_TINV");
        p->fuse_tinv = !(f && f[0] == '1');
        const char* ra = std::getenv("JFMG_REORTH_ALWAYS");
        p->reorth_always = ra && ra[0] == '1';
    }
    if (!reftab(cfg->k, cfg->transfer, p->R)) {
        delete p;
        return fail(nullptr, JFMG_EINVAL, "singular subcell transfer");
    }
    layout(*cfg, (char*)workspace, [&](const char* name, void* ptr, size_t nn) {
        const std::string nm(name);
        if (nm == "scal") p->scal = (double*)ptr;
        else if (nm == "fvpart") { p->fvpart = (double*)ptr; p->fvp = nn; }
        else if (nm == "partials") { p->partials = (double*)ptr; p->npartials = nn; }
        else if (nm == "bg_node") p->bg_node = (double*)ptr;
        else if (nm == "dbg_node") p->dbg_node = (double*)ptr;
        else if (nm == "th_node") p->th_node = (double*)ptr;
        else if (nm == "bg_face") p->bg_face = (double*)ptr;
        else if (nm == "dbg_face") p->dbg_face = (double*)ptr;
        else if (nm == "pb_node") p->pb_node = (double*)ptr;
        else if (nm == "pb_face") p->pb_face = (double*)ptr;
        else if (nm == "Un") p->Un = (double*)ptr;
        else if (nm == "Ubar") p->Ubar = (double*)ptr;
        else if (nm == "Uk") p->Uk = (double*)ptr;
        else if (nm == "G") p->G = (double*)ptr;
        else if (nm == "delta") p->delta = (double*)ptr;
        else if (nm == "tmp1") p->tmp1 = (double*)ptr;
        else if (nm == "tmp2") p->tmp2 = (double*)ptr;
        else if (nm == "Ulin") p->Ulin = (double*)ptr;
        else if (nm == "lin0") p->lin0 = (double*)ptr;
        else if (nm == "V") p->V = (double*)ptr;
        else if (nm == "Z") p->Z = (double*)ptr;
        else {
            Level& L = p->lev[nn];
            if (nm == "u") L.u = ptr;
            else if (nm == "F0") L.F0 = ptr;
            else if (nm == "x0") L.buf[0] = ptr;
            else if (nm == "x1") L.buf[1] = ptr;
            else if (nm == "x2") L.buf[2] = ptr;
            else if (nm == "b") L.b = ptr;
            else if (nm == "bgc") L.bgc = ptr;
            else if (nm == "bgf") L.bgf = ptr;
            else if (nm == "dbgf") L.dbgf = ptr;
            else if (nm == "pc") L.pc = ptr;
            else if (nm == "pf") L.pf = ptr;
        }
    });
    // level geometry (the envelope's for a ragged batch: launch shapes)
    int nxl = p->n1 * cfg->nx, nzl = p->n1 * cfg->nz;
    for (int l = 0; l < p->nlev; ++l) {
        Level& L = p->lev[l];
        L.nx = nxl; L.nz = nzl; L.nc = (long)nxl * nzl;
        L.tile = fv_default_tile(nxl);
        L.hx = (cfg->x1 - cfg->x0) / nxl;
        L.hz = (cfg->z1 - cfg->z0) / nzl;
        nxl /= 2;
        nzl /= 2;
    }
    hipStream_t st = p->st;
    std::vector<std::vector<char>> keep;
    std::vector<MemberArgs> tab;
    hipError_t e = hipSuccess;
    if (!ragged) {
        // one set of tables (member 0's; the members of a lock-step batch share them)
        e = upload_tables(p, *cfg, 0, keep);
    } else {
        tab.resize(members);
        long off = 0;
        for (int m = 0; m < members && !e; ++m) {
            const jfmg_config& c = cfgs[m];
            const size_t ob = (size_t)m * member_bytes;
            e = upload_tables(p, c, ob, keep);
            MemberArgs& M = tab[m];
            std::memset(&M, 0, sizeof(M));
            M.dg = dg_args_of(p, c, ob);
            M.N = 4L * c.nx * c.nz * p->np;
            M.live = 1;
            for (int l = 0; l < p->nlev; ++l) {
                if (p->prec == 32) M.f32[l] = fv_args_of<float>(p, c, l, ob);
                else M.f64[l] = fv_args_of<double>(p, c, l, ob);
            }
            p->mlen.push_back(M.N);
            p->moff.push_back(off);
            off += M.N;
        }
        p->tab = (MemberArgs*)((char*)workspace + (size_t)members * member_bytes);
        if (!e) e = hipMemcpyAsync(p->tab, tab.data(), sizeof(MemberArgs) * members, hipMemcpyHostToDevice, st);
        p->mb.tab = p->tab;
    }
    for (int b = 0; b < p->mb.n && !e; ++b) e = hipMemsetAsync((char*)p->scal + (size_t)b * p->mb.ms, 0, NSCAL * 8, st);
    e = e ? e : hipStreamSynchronize(st);
    e = e ? e : hipStreamCreateWithFlags(&p->cs, hipStreamNonBlocking);
    // coherent pinned memory: the last kernel of each FGMRES iteration stores its scalars here
    e = e ? e : hipHostMalloc((void**)&p->hpin, sizeof(double) * S_HB * cfg->gmres_m * p->mb.n, hipHostMallocCoherent);
    e = e ? e : hipHostMalloc((void**)&p->hscal, sizeof(double) * HSCAL * p->mb.n, hipHostMallocCoherent);
    e = e ? e : hipHostMalloc((void**)&p->ycoef, sizeof(double) * cfg->gmres_m * p->mb.n, hipHostMallocCoherent);
    for (int j = 0; j < cfg->gmres_m && !e; ++j) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (!e) p->hev.push_back(ev);
    }
    if (e) {
        const std::string m2 = std::string("table upload: ") + hipGetErrorString(e);
        delete p;
        return fail(nullptr, JFMG_EDEVICE, m2);
    }
    // DG kernel arguments (the envelope's for a ragged batch: launch shapes)
    p->A = dg_args_of(p, *cfg, 0);
    *out = p;
    return JFMG_OK;
}

}  // namespace

extern "C" {

jfmg_status jfmg_workspace_bytes(const jfmg_config* cfg, size_t* bytes)
{
    if (!cfg || !bytes) return fail(nullptr, JFMG_EINVAL, "null argument");
    Key key;
    std::string msg;
    jfmg_status s = validate(*cfg, key, msg);
    if (s) return fail(nullptr, s, msg);
    *bytes = layout(*cfg, nullptr, [](const char*, void*, size_t) {}) * (size_t)members_of(*cfg);
    return JFMG_OK;
}

jfmg_status jfmg_create_problem(const jfmg_config* cfg, void* workspace, size_t ws_bytes, void* hip_stream,
                                jfmg_problem** out)
{
    return create_impl(cfg, 1, false, workspace, ws_bytes, hip_stream, out);
}

jfmg_status jfmg_ensemble_workspace_bytes(const jfmg_config* cfgs, int n, size_t* bytes)
{
    if (!cfgs || !bytes) return fail(nullptr, JFMG_EINVAL, "null argument");
    Key key;
    std::string msg;
    jfmg_status s = validate_ensemble(cfgs, n, key, msg);
    if (s) return fail(nullptr, s, msg);
    const jfmg_config env = envelope(cfgs, n);
    *bytes = layout(env, nullptr, [](const char*, void*, size_t) {}) * (size_t)n + table_bytes(n);
    return JFMG_OK;
}

jfmg_status jfmg_create_ensemble(const jfmg_config* cfgs, int n, void* workspace, size_t ws_bytes, void* hip_stream,
                                 jfmg_problem** out)
{
    return create_impl(cfgs, n, true, workspace, ws_bytes, hip_stream, out);
}

jfmg_status jfmg_destroy_problem(jfmg_problem* p)
{
    if (p) {
        if (p->cs) (void)hipStreamSynchronize(p->cs);
        prof_flush(p);
        invalidate_graphs(p);
        for (hipEvent_t e : p->prof.pool) (void)hipEventDestroy(e);
        if (p->cs) (void)hipStreamDestroy(p->cs);
        for (hipEvent_t e : p->hev) (void)hipEventDestroy(e);
        if (p->hpin) (void)hipHostFree(p->hpin);
        if (p->hscal) (void)hipHostFree(p->hscal);
        if (p->ycoef) (void)hipHostFree(p->ycoef);
    }
    delete p;
    return JFMG_OK;
}

size_t jfmg_num_dofs(const jfmg_problem* p) { return p ? (size_t)p->N : 0; }

size_t jfmg_member_dofs(const jfmg_problem* p, int member)
{
    if (!p || member < 0 || member >= p->mb.n) return 0;
    return p->ragged ? (size_t)p->mlen[member] : (size_t)p->N;
}

size_t jfmg_fv_size(const jfmg_problem* p, int level)
{
    if (!p || level < 0 || level >= p->nlev) return 0;
    return (size_t)(4 * p->lev[level].nc);
}

jfmg_status jfmg_initial_state(jfmg_problem* p, const jfmg_perturbation* q, double* U)
{
    if (!p || !q || !U) return fail(p, JFMG_EINVAL, "null argument");
    if (q->shape < 0 || q->shape > 1) return fail(p, JFMG_EINVAL, "unknown perturbation shape");
    if (p->ragged) return fail(p, JFMG_EINVAL, "a ragged batch takes its members' initial states from single problems");
    // every member of a batch gets the same state ([members][N] back to back)
    launch_initial_state(p->cfg.k, p->A, q->shape, q->amp, q->xc, q->zc, q->xr, q->zr, q->a, q->Z, p->cfg.x0,
                         p->cfg.z0, p->cfg.u_mean, U, p->st, Mb{p->mb.n, (long)(sizeof(double) * p->N)});
    return check_launch(p);
}

jfmg_status jfmg_residual(jfmg_problem* p, const double* U, double* out, int apply_minv)
{
    if (!p || !U || !out) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    launch_dg(p->cfg.k, p->cfg.physics == 1, apply_minv ? 1 : 0, p->A, U, nullptr, nullptr, out, nullptr, nullptr, 0,
              0.0, no_red(), p->st);
    return check_launch(p);
}

jfmg_status jfmg_stage_residual(jfmg_problem* p, const double* U, const double* Ubar, double alpha_dt, double* G,
                                double* norm)
{
    if (!p || !U || !Ubar || !G) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    return stage_residual(p, U, Ubar, alpha_dt, G, norm);
}

jfmg_status jfmg_linearize(jfmg_problem* p, const double* U, double alpha_dt)
{
    if (!p || !U) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) {   // caller's members back to back -> member-strided workspace
        HIPCHK(p, members_in(p, p->Ulin, U));
        return linearize(p, p->Ulin, alpha_dt);
    }
    return linearize(p, U, alpha_dt);
}

jfmg_status jfmg_jvp(jfmg_problem* p, const double* y, double* out)
{
    if (!p || !y || !out) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "jfmg_jvp needs jfmg_linearize first");
    launch_norm2(y, p->N, red_at(p, S_Y), p->st);
    jvp_slot(p, y, out, S_Y);
    return check_launch(p);
}

jfmg_status jfmg_mg_apply(jfmg_problem* p, const double* r, double* z)
{
    if (!p || !r || !z) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "jfmg_mg_apply needs jfmg_linearize first");
    return precond(p, const_cast<double*>(r), z, S_TMP);   // r is written only when normalizing
}

static jfmg_status implicit_step_body(jfmg_problem* p, double* U, jfmg_stats* stats)
{
    const auto t0 = std::chrono::steady_clock::now();
    jfmg_stats st;
    std::memset(&st, 0, sizeof(st));
    std::memset(p->mv_count, 0, sizeof(p->mv_count));
    p->lh_count = 0;
    p->jvp_count = 0;
    p->syncs = 0;
    p->reorths = 0;
    const jfmg_config& c = p->cfg;
    jfmg_status s;
    // the caller's U holds the members back to back
    hipError_t e = members_in(p, p->Un, U);
    if (e) return fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    if (c.scheme == 0) {
        s = newton_stage(p, p->Un, c.dt, &st);
    } else {
        const double a = 1.0 - std::sqrt(2.0) / 2.0;
        s = newton_stage(p, p->Un, a * c.dt, &st);
        if (s == JFMG_OK) {
            // Ubar_2 = U^n + (1 - a) dt f(U_1)
            launch_dg(c.k, c.physics == 1, 1, p->A, p->Uk, nullptr, nullptr, p->tmp1, nullptr, nullptr, 0, 0.0, no_red(),
                      p->st, p->mb);
            p->lh_count++;
            launch_axpby(p->Ubar, 1.0, p->Un, (1.0 - a) * c.dt, p->tmp1, p->N, p->st, p->mb);
            s = check_launch(p);
            if (s == JFMG_OK) s = newton_stage(p, p->Ubar, a * c.dt, &st);
        }
    }
    if (s == JFMG_OK) {
        e = members_out(p, U, p->Uk);
        if (!e) e = hipStreamSynchronize(p->st);
        if (e) s = fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    } else {
        (void)hipStreamSynchronize(p->st);
    }
    prof_flush(p);
    st.status = s;
    st.lh_evals = p->lh_count;
    st.jvps = p->jvp_count;
    st.host_syncs = p->syncs;
    st.reorth_its = p->reorths;
    for (int l = 0; l < MAXLEV && l < 8; ++l) st.fv_matvecs[l] = p->mv_count[l];
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return s;
}

jfmg_status jfmg_implicit_step(jfmg_problem* p, double* U, jfmg_stats* stats)
{
    if (!p || !U) return fail(p, JFMG_EINVAL, "null argument");
    // host-synchronous: order after the caller's stream, then work on the private
    // stream (HIP graphs cannot be captured on the legacy default stream)
    hipError_t e = hipStreamSynchronize(p->user_st);
    if (e) return fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    p->st = p->cs;
    jfmg_status s = implicit_step_body(p, U, stats);
    (void)hipStreamSynchronize(p->cs);
    p->st = p->user_st;
    return s;
}

jfmg_status jfmg_newton_stage(jfmg_problem* p, const double* Ubar, double alpha_dt, double* U, jfmg_stats* stats)
{
    if (!p || !Ubar || !U) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!(alpha_dt > 0.0) || !std::isfinite(alpha_dt)) return fail(p, JFMG_EINVAL, "alpha_dt must be positive and finite");
    hipError_t e = hipStreamSynchronize(p->user_st);
    if (e) return fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    p->st = p->cs;
    const auto t0 = std::chrono::steady_clock::now();
    jfmg_stats st;
    std::memset(&st, 0, sizeof(st));
    std::memset(p->mv_count, 0, sizeof(p->mv_count));
    p->lh_count = 0;
    p->jvp_count = 0;
    p->syncs = 0;
    p->reorths = 0;
    const size_t vb = sizeof(double) * p->N;
    jfmg_status s = JFMG_OK;
    e = hipMemcpyAsync(p->Ubar, Ubar, vb, hipMemcpyDeviceToDevice, p->st);
    if (e) s = fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    if (s == JFMG_OK) s = newton_stage(p, p->Ubar, alpha_dt, &st);
    if (s == JFMG_OK) {
        e = hipMemcpyAsync(U, p->Uk, vb, hipMemcpyDeviceToDevice, p->st);
        if (!e) e = hipStreamSynchronize(p->st);
        if (e) s = fail(p, JFMG_EDEVICE, hipGetErrorString(e));
    } else {
        (void)hipStreamSynchronize(p->st);
    }
    prof_flush(p);
    p->st = p->user_st;
    st.status = s;
    st.lh_evals = p->lh_count;
    st.jvps = p->jvp_count;
    st.host_syncs = p->syncs;
    st.reorth_its = p->reorths;
    for (int l = 0; l < MAXLEV; ++l) st.fv_matvecs[l] = p->mv_count[l];
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return s;
}

jfmg_status jfmg_explicit_steps(jfmg_problem* p, double* U, double dt, int nsteps)
{
    if (!p || !U) return fail(p, JFMG_EINVAL, "null argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!(std::isfinite(dt)) || nsteps < 0) return fail(p, JFMG_EINVAL, "dt must be finite and nsteps >= 0");
    // SSP RK(4,3): four stages of size dt/2 with the convex combination
    // 2/3 U^n + 1/3 U^(2) before the third; every stage is one DG launch with
    // the combination fused into its output (the input is never the output)
    const int k = p->cfg.k;
    const bool ns = p->cfg.physics == 1;
    const ExStage half{0.0, 1.0, 0.5 * dt}, third{2.0 / 3.0, 1.0 / 3.0, dt / 6.0};
    for (int it = 0; it < nsteps; ++it) {
        launch_dg(k, ns, 4, p->A, U, nullptr, nullptr, p->Uk, nullptr, nullptr, 0, 0.0, no_red(), p->st, Mb{}, half);
        launch_dg(k, ns, 4, p->A, p->Uk, nullptr, nullptr, p->tmp2, nullptr, nullptr, 0, 0.0, no_red(), p->st, Mb{},
                  half);
        launch_dg(k, ns, 4, p->A, p->tmp2, nullptr, U, p->Uk, nullptr, nullptr, 0, 0.0, no_red(), p->st, Mb{}, third);
        launch_dg(k, ns, 4, p->A, p->Uk, nullptr, nullptr, U, nullptr, nullptr, 0, 0.0, no_red(), p->st, Mb{}, half);
    }
    return check_launch(p);
}

jfmg_status jfmg_transfer(jfmg_problem* p, int dir, const void* in, void* out)
{
    if (!p || !in || !out || (dir != 0 && dir != 1)) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    const int nxf = p->lev[0].nx;
    if (dir == 0) {
        if (p->prec == 32) launch_transfer_T<float>(p->cfg.k, p->A, mass_fix_of(p), (const double*)in, (float*)out, nxf, p->st);
        else launch_transfer_T<double>(p->cfg.k, p->A, mass_fix_of(p), (const double*)in, (double*)out, nxf, p->st);
    } else {
        if (p->prec == 32) launch_transfer_Tinv<float>(p->cfg.k, p->A, mass_fix_of(p), (const float*)in, (double*)out, nxf, no_red(), p->st);
        else launch_transfer_Tinv<double>(p->cfg.k, p->A, mass_fix_of(p), (const double*)in, (double*)out, nxf, no_red(), p->st);
    }
    return check_launch(p);
}

jfmg_status jfmg_restrict(jfmg_problem* p, int fine_level, const void* fine, void* coarse)
{
    if (!p || !fine || !coarse || fine_level < 0 || fine_level + 1 >= p->nlev) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (p->prec == 32) FvLaunch<float>::restrict_(fv_args<float>(p, fine_level), (const float*)fine, (float*)coarse, p->st);
    else FvLaunch<double>::restrict_(fv_args<double>(p, fine_level), (const double*)fine, (double*)coarse, p->st);
    return check_launch(p);
}

jfmg_status jfmg_prolong(jfmg_problem* p, int coarse_level, const void* coarse, void* fine)
{
    if (!p || !fine || !coarse || coarse_level < 1 || coarse_level >= p->nlev) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (p->prec == 32) FvLaunch<float>::prolong(fv_args<float>(p, coarse_level - 1), (const float*)coarse, (float*)fine, p->st);
    else FvLaunch<double>::prolong(fv_args<double>(p, coarse_level - 1), (const double*)coarse, (double*)fine, p->st);
    return check_launch(p);
}

jfmg_status jfmg_fv_level_state(jfmg_problem* p, int level, void* u)
{
    if (!p || !u || level < 0 || level >= p->nlev) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    const size_t ts = p->prec == 32 ? 4 : 8;
    HIPCHK(p, hipMemcpyAsync(u, p->lev[level].u, ts * 4 * p->lev[level].nc, hipMemcpyDeviceToDevice, p->st));
    return JFMG_OK;
}

jfmg_status jfmg_fv_dtau(jfmg_problem* p, int level, double* dtau)
{
    if (!p || !dtau || level < 0 || level >= p->nlev) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    return read_scalars(p, S_LEV + 4 * level + LV_DTAU, 1, dtau);
}

jfmg_status jfmg_dg_dtau(jfmg_problem* p, double* dtau)
{
    if (!p || !dtau) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->key.a && !p->key.b) return fail(p, JFMG_EINVAL, "no DG-level smoothing in mg_key");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    return read_scalars(p, S_DTDG, 1, dtau);
}

jfmg_status jfmg_fv_matvec(jfmg_problem* p, int level, const void* x, void* out)
{
    if (!p || !x || !out || level < 0 || level >= p->nlev) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    const Level& L = p->lev[level];
    if (p->prec == 32) {
        FvLaunch<float>::norm2((const float*)x, 4 * L.nc, red_at(p, S_TMP), p->st);
        FvLaunch<float>::matvec(fv_args<float>(p, level), (const float*)L.u, (const float*)L.F0, (const float*)x,
                                (float*)out, p->scal + S_TMP, 1, p->scal + S_LEV + 4 * level, p->adt, p->st);
    } else {
        FvLaunch<double>::norm2((const double*)x, 4 * L.nc, red_at(p, S_TMP), p->st);
        FvLaunch<double>::matvec(fv_args<double>(p, level), (const double*)L.u, (const double*)L.F0, (const double*)x,
                                 (double*)out, p->scal + S_TMP, 1, p->scal + S_LEV + 4 * level, p->adt, p->st);
    }
    return check_launch(p);
}

jfmg_status jfmg_mg_fv(jfmg_problem* p, const void* b, void* x)
{
    if (!p || !b || !x) return fail(p, JFMG_EINVAL, "bad argument");
    if (p->mb.n > 1) return fail(p, JFMG_EINVAL, "a batched problem supports jfmg_implicit_step, jfmg_initial_state, jfmg_linearize and the tile calls");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    const Level& L = p->lev[0];
    const size_t bytes = (p->prec == 32 ? 4 : 8) * 4 * L.nc;
    HIPCHK(p, hipMemcpyAsync(L.b, b, bytes, hipMemcpyDeviceToDevice, p->st));
    void* r;
    if (p->prec == 32) { Mg<float> mg{p}; mg.init(); r = mg.run(); }
    else { Mg<double> mg{p}; mg.init(); r = mg.run(); }
    HIPCHK(p, hipMemcpyAsync(x, r, bytes, hipMemcpyDeviceToDevice, p->st));
    return check_launch(p);
}

jfmg_status jfmg_subgrid_map(jfmg_problem* p, int* fv_to_dg)
{
    if (!p || !fv_to_dg) return fail(p, JFMG_EINVAL, "null argument");
    launch_subgrid_map(p->cfg.k, p->A, p->lev[0].nx, fv_to_dg, p->st);
    return check_launch(p);
}

jfmg_status jfmg_get_tiles(const jfmg_problem* p, int* shapes)
{
    if (!p || !shapes) return JFMG_EINVAL;
    for (int l = 0; l < p->nlev; ++l) shapes[l] = p->lev[l].tile;
    return JFMG_OK;
}

jfmg_status jfmg_set_tiles(jfmg_problem* p, const int* shapes)
{
    if (!p || !shapes) return fail(p, JFMG_EINVAL, "bad argument");
    for (int l = 0; l < p->nlev; ++l)
        if (shapes[l] < 0 || shapes[l] >= JFMG_TILE_NSHAPE) return fail(p, JFMG_EINVAL, "unknown tile shape");
    for (int l = 0; l < p->nlev; ++l) p->lev[l].tile = shapes[l];
    invalidate_graphs(p);
    return JFMG_OK;
}


jfmg_status jfmg_autotune(jfmg_problem* p, int reps, int* shapes, double* times_us)
{
    if (!p || reps < 1 || reps > 1000) return fail(p, JFMG_EINVAL, "bad argument");
    if (!p->have_lin) return fail(p, JFMG_ESTATE, "needs jfmg_linearize first");
    return p->prec == 32 ? autotune_t<float>(p, reps, shapes, times_us) : autotune_t<double>(p, reps, shapes, times_us);
}

jfmg_status jfmg_profile_enable(jfmg_problem* p, unsigned class_mask)
{
    if (!p) return fail(p, JFMG_EINVAL, "null argument");
    HIPCHK(p, hipStreamSynchronize(p->st));
    prof_flush(p);
    p->prof.mask = class_mask;
    for (int i = 0; i < JFMG_K_NCLASS; ++i) { p->prof.ms[i] = 0; p->prof.cnt[i] = 0; p->prof.bytes[i] = 0; }
    return JFMG_OK;
}

jfmg_status jfmg_profile_read(jfmg_problem* p, double* ms, long long* launches, double* bytes)
{
    if (!p || !ms || !launches || !bytes) return fail(p, JFMG_EINVAL, "null argument");
    HIPCHK(p, hipStreamSynchronize(p->st));
    prof_flush(p);
    for (int i = 0; i < JFMG_K_NCLASS; ++i) { ms[i] = p->prof.ms[i]; launches[i] = p->prof.cnt[i]; bytes[i] = p->prof.bytes[i]; }
    return JFMG_OK;
}

const char* jfmg_last_error(const jfmg_problem* p)
{
    return p ? p->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
