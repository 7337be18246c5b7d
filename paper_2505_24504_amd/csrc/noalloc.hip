// Allocation-free stage residual G = U - alpha dt M^-1 L_h(U) - Ubar and
// ||G||^2 (eq. newton with the DG operator of eqs. convDiscr, elementint,
// surfaceint, perturbed-euler), without a problem handle and without a
// workspace argument: the background tables of the DG kernel and the block
// partials of the norm live in one file-scope device array per GPU.  For
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array's host-side name is not a device address.  The first call on a
// device resolves that device's copy with hipGetSymbolAddress and keeps the
// pointer; every launch uses the resolved pointer.  Every call on a GPU shares
// that GPU's copy: calls that overlap on one GPU (two streams, two threads)
// race on it.  Every value a call reads from the array is written earlier in
// the same call (tables by their kernel, partials by the DG kernel), so nothing
// has to start at zero.
#include "jfmg_internal.h"

#include <cmath>
#include <mutex>
#include <string>

namespace {

constexpr size_t SCRATCH_BYTES = JFMG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void* g_scratch[MAX_DEVICES];   // resolved address of `scratch` on each device

struct TableParams {
    jfmg_config c;
    double xi[jfmg::MAXN1];
    int n1;
    double dz;
};

// Byte layout of one call inside the array (256-byte aligned regions).
struct Layout {
    size_t bg_node, dbg_node, th_node, bg_face, dbg_face, pb_node, pb_face, partials, end;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout_of(const jfmg_config& c)
{
    const size_t rows = (size_t)c.nz * (c.k + 1), faces = (size_t)c.nz + 1;
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
    L.bg_node = take(rows * 4 * 8);
    L.dbg_node = take(rows * 4 * 8);
    L.th_node = take(rows * 8);
    L.bg_face = take(faces * 4 * 8);
    L.dbg_face = take(faces * 4 * 8);
    L.pb_node = take(rows * 2 * 8);
    L.pb_face = take(faces * 2 * 8);
    L.partials = take((size_t)jfmg::dg_grid(c.k, (long)c.nx * c.nz) * 8);
    L.end = o;
    return L;
}

// The background tables of the DG kernel (the layout jfmg_create_problem
// uploads): node rows i = ez (k+1) + b at z = z0 + (ez + (1 + xi_b)/2) dz, then
// element z-faces f at z = z0 + f dz.  Pressure and 1/(rho theta) arrays hold
// all rows' pressures first, then all reciprocals.
__global__ void __launch_bounds__(256)
bg_tables_kernel(TableParams P, double* __restrict__ bg_node, double* __restrict__ dbg_node,
                 double* __restrict__ th_node, double* __restrict__ bg_face, double* __restrict__ dbg_face,
                 double* __restrict__ pb_node, double* __restrict__ pb_face)
{
    const int rows = P.c.nz * P.n1, faces = P.c.nz + 1;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < rows) {
        const int ez = i / P.n1, b = i - ez * P.n1;
        const jfmg::BgPoint bp = jfmg::background_at(P.c, P.c.z0 + (ez + 0.5 * (1.0 + P.xi[b])) * P.dz);
        for (int c = 0; c < 4; ++c) {
            bg_node[i * 4 + c] = bp.U[c];
            dbg_node[i * 4 + c] = bp.dU[c];
        }
        th_node[i] = bp.theta;
        pb_node[i] = jfmg::bg_pressure(P.c, bp.U[3]);
        pb_node[rows + i] = 1.0 / bp.U[3];
    } else if (i < rows + faces) {
        const int f = i - rows;
        const jfmg::BgPoint bp = jfmg::background_at(P.c, P.c.z0 + f * P.dz);
        for (int c = 0; c < 4; ++c) {
            bg_face[f * 4 + c] = bp.U[c];
            dbg_face[f * 4 + c] = bp.dU[c];
        }
        pb_face[f] = jfmg::bg_pressure(P.c, bp.U[3]);
        pb_face[faces + f] = 1.0 / bp.U[3];
    }
}

jfmg_status report(jfmg_status s, const std::string& msg)
{
    jfmg::set_create_error(msg);
    return s;
}

// This device's copy of the array, resolved once per device.
jfmg_status scratch_of_current_device(unsigned char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(JFMG_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return report(JFMG_EDEVICE, "device index beyond the supported range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return report(JFMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = (unsigned char*)g_scratch[dev];
    return JFMG_OK;
}

}  // namespace

extern "C" jfmg_status jfmg_stage_residual_noalloc(const jfmg_config* cfg, const double* U, const double* Ubar,
                                                   double alpha_dt, double* G, double* norm2, void* hip_stream)
{
    if (!cfg || !U || !Ubar || !G) return report(JFMG_EINVAL, "null argument");
    const char* msg = nullptr;
    const jfmg_status s = jfmg::check_config(*cfg, &msg);
    if (s) return report(s, msg ? msg : "invalid configuration");
    if (cfg->batch > 1) return report(JFMG_EINVAL, "the allocation-free residual takes a single problem (batch 0 or 1)");
    if (!std::isfinite(alpha_dt)) return report(JFMG_EINVAL, "alpha_dt must be finite");
    const Layout L = layout_of(*cfg);
    if (L.end > SCRATCH_BYTES)
        return report(JFMG_ENOMEM, "problem needs " + std::to_string(L.end) + " bytes of the " +
                                       std::to_string(SCRATCH_BYTES) + "-byte static scratch");
    jfmg::RefTab R;
    if (!jfmg::build_reftab(cfg->k, cfg->transfer, R)) return report(JFMG_EINVAL, "singular subcell transfer");
    unsigned char* base = nullptr;
    const jfmg_status ss = scratch_of_current_device(&base);
    if (ss) return ss;
    hipStream_t st = (hipStream_t)hip_stream;

    const int n1 = cfg->k + 1;
    const double dx = (cfg->x1 - cfg->x0) / cfg->nx, dz = (cfg->z1 - cfg->z0) / cfg->nz;
    TableParams P;
    P.c = *cfg;
    for (int i = 0; i < jfmg::MAXN1; ++i) P.xi[i] = R.xi[i];
    P.n1 = n1;
    P.dz = dz;
    double* bg_node = (double*)(base + L.bg_node);
    double* dbg_node = (double*)(base + L.dbg_node);
    double* th_node = (double*)(base + L.th_node);
    double* bg_face = (double*)(base + L.bg_face);
    double* dbg_face = (double*)(base + L.dbg_face);
    double* pb_node = (double*)(base + L.pb_node);
    double* pb_face = (double*)(base + L.pb_face);
    const int entries = cfg->nz * n1 + cfg->nz + 1;
    bg_tables_kernel<<<dim3((entries + 255) / 256), dim3(256), 0, st>>>(P, bg_node, dbg_node, th_node, bg_face,
                                                                        dbg_face, pb_node, pb_face);

    jfmg::DgArgs A;
    A.ne = (long)cfg->nx * cfg->nz;
    A.nx = cfg->nx; A.nz = cfg->nz; A.bc = cfg->bc; A.physics = cfg->physics;
    A.dx = dx; A.dz = dz; A.J = dx * dz / 4.0; A.g = cfg->g; A.mu = cfg->mu; A.c_ip = cfg->c_ip;
    A.gas = jfmg::gas_of(*cfg);
    A.bg_node = bg_node; A.dbg_node = dbg_node; A.th_node = th_node;
    A.bg_face = bg_face; A.dbg_face = dbg_face;
    A.pb_node = pb_node; A.irt_node = pb_node + (size_t)cfg->nz * n1;
    A.pb_face = pb_face; A.irt_face = pb_face + (cfg->nz + 1);
    A.R = R;
    // G and its block partials; with norm2 the one-block finalize sums them into norm2[0]
    jfmg::launch_dg(cfg->k, cfg->physics == 1, 2, A, U, nullptr, Ubar, G, nullptr, nullptr, 0, alpha_dt,
                    jfmg::Red{(double*)(base + L.partials), norm2}, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report(JFMG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return JFMG_OK;
}
