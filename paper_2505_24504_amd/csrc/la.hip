// FP64 vector kernels of the FGMRES Arnoldi process (classical Gram-Schmidt,
// re-orthogonalized where the first pass cancels most of w): multi-dot products <w, v_i> of one vector
// against the whole basis in a single pass, the basis update w -= V h, scaling,
// and the final combination delta = Z y.  Streaming, HBM bound; every
// reduction is two-level with a fixed summation order (run-to-run identical).
#include "jfmg_internal.h"

namespace jfmg {

constexpr int LA_NTH = 256, LA_EL = 4;   // threads per block, elements per thread

int la_blocks(long n)
{
    return (int)((n + (long)LA_NTH * LA_EL - 1) / ((long)LA_NTH * LA_EL));
}

// out[q] = sum_b p[q * nb + b], one block per q, fixed order (0 where the gate is closed)
__global__ void __launch_bounds__(256) finalize_kernel(const double* __restrict__ p, int nb, double* __restrict__ out,
                                                       Gate gate, long ms)
{
    p = mbr(p, ms);
    out = mbr(out, ms);
    gate.h = mbr(gate.h, ms);
    __shared__ double sh[4];
    const int q = blockIdx.x;
    if (!gate_open(gate)) {
        if (threadIdx.x == 0) out[q] = 0.0;
        return;
    }
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) a += p[(long)q * nb + i];
    a = block_sum<256>(a, sh);
    if (threadIdx.x == 0) out[q] = a;
}

void launch_finalize(const double* partials, int nb, int nq, double* out, hipStream_t st, Gate gate, const Mb& mb)
{
    finalize_kernel<<<dim3(nq, 1, mb.n), dim3(256), 0, st>>>(partials, nb, out, gate, mb.ms);
}

// Scalars between the device slots of every member and coherent pinned host
// memory, by kernels (no copy engine): gather host[m * count + i] = slot_m[i],
// scatter slot_m[i] = host[m * hstride + i].
__global__ void __launch_bounds__(64) gather_kernel(const double* __restrict__ src, int count, double* __restrict__ host,
                                                    long ms)
{
    src = mbr(src, ms);
    host += (long)blockIdx.z * count;
    for (int i = threadIdx.x; i < count; i += 64) host[i] = src[i];
}

__global__ void __launch_bounds__(64) scatter_kernel(double* __restrict__ dst, int count, const double* __restrict__ host,
                                                     long hstride, long ms)
{
    dst = mbr(dst, ms);
    host += (long)blockIdx.z * hstride;
    for (int i = threadIdx.x; i < count; i += 64) dst[i] = host[i];
}

void launch_gather(const double* src, int count, double* host, hipStream_t st, const Mb& mb)
{
    gather_kernel<<<dim3(1, 1, mb.n), dim3(64), 0, st>>>(src, count, host, mb.ms);
}

void launch_scatter(double* dst, int count, const double* host, long hstride, hipStream_t st, const Mb& mb)
{
    scatter_kernel<<<dim3(1, 1, mb.n), dim3(64), 0, st>>>(dst, count, host, hstride, mb.ms);
}

__global__ void __launch_bounds__(256)
norm2_kernel(const double* __restrict__ x, long n, Red red, long ms, const MemberArgs* __restrict__ mt)
{
    x = mbr(x, ms);
    red = mbr(red, ms);
    n = len_of(n, mt);
    const long nb = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;   // this member's work-groups
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) s += x[i] * x[i];
    put_partial<256>(red, s);
}

void launch_norm2(const double* x, long n, Red red, hipStream_t st, const Mb& mb)
{
    long b = (n + 255) / 256;
    const int nb = (int)(b < 1024 ? b : 1024);
    norm2_kernel<<<dim3(nb, 1, mb.n), dim3(256), 0, st>>>(x, n, red, mb.ms, mb.tab);
    if (red.out) launch_finalize(red.partials, nb, 1, red.out, st, Gate{}, mb);
}

// <w, v_i> for i < nv (and <w, w> as entry nv when self is set): the entries are
// split into groups of MAXV consecutive ones, one group per grid row (blockIdx.y),
// so every thread keeps MAXV accumulators in registers whatever nv is (w is read
// once per group); each wave reduces them with butterflies and one LDS exchange
// combines the waves (a single barrier per block); the block partials [v][block]
// are summed by the finalize kernel.  Nothing is computed where the gate is closed.
template <int MAXV>
__global__ void __launch_bounds__(LA_NTH)
multidot_kernel(const double* __restrict__ w, const double* __restrict__ V, long ld, int nv, int self, long n, Gate gate,
                Red red, long ms, const MemberArgs* __restrict__ mt)
{
    constexpr int NW = LA_NTH / 64;
    n = len_of(n, mt);   // a ragged member's length: blocks beyond it store zero partials
    __shared__ double sh[NW][MAXV];
    w = mbr(w, ms);
    V = mbr(V, ms);
    gate.h = mbr(gate.h, ms);
    red = mbr(red, ms);
    if (!gate_open(gate)) return;
    const int nt = nv + self;
    const int v0 = blockIdx.y * MAXV;   // first entry of this block's group
    const long base = (long)blockIdx.x * LA_NTH * LA_EL + threadIdx.x;
    double acc[MAXV];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) acc[q] = 0.0;
    if (base - threadIdx.x + LA_NTH * LA_EL <= n && v0 + MAXV <= nv) {
        // a whole block of basis vectors: every load issued before the first product
        // (the same products in the same order as below)
        double wv[LA_EL], vv[LA_EL][MAXV];
#pragma unroll
        for (int k = 0; k < LA_EL; ++k) {
            const long i = base + (long)k * LA_NTH;
            wv[k] = w[i];
#pragma unroll
            for (int q = 0; q < MAXV; ++q) vv[k][q] = V[(long)(v0 + q) * ld + i];
        }
#pragma unroll
        for (int k = 0; k < LA_EL; ++k)
#pragma unroll
            for (int q = 0; q < MAXV; ++q) acc[q] += wv[k] * vv[k][q];
    } else {
#pragma unroll
        for (int k = 0; k < LA_EL; ++k) {
            const long i = base + (long)k * LA_NTH;
            if (i < n) {
                const double wi = w[i];
#pragma unroll
                for (int q = 0; q < MAXV; ++q) {
                    const int v = v0 + q;
                    if (v < nv) acc[q] += wi * V[(long)v * ld + i];
                    else if (v == nv && self) acc[q] += wi * wi;
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < MAXV; ++q) {
        if (v0 + q < nt) {
            const double s = wave_sum(acc[q]);
            if (lane == 0) sh[wid][q] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < MAXV && v0 + (int)threadIdx.x < nt) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NW; ++r) s += sh[r][threadIdx.x];
        red.partials[(long)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
}

void launch_multidot(const double* w, const double* V, long ld, int nv, int self, long n, Gate gate, Red red,
                     hipStream_t st, const Mb& mb)
{
    // groups of 4 entries: measured at the density-current size (nv up to 30), the mean
    // first-pass launch takes 23.5 us with groups of 4, 25.7 with 8, 33.5 with 16 and 41.8
    // with all entries in one group (w is re-read once per group, V once)
    const int nt = nv + self;
    const dim3 g(la_blocks(n), (nt + 3) / 4, mb.n);
    timed_launch(multidot_kernel<4>, g, dim3(LA_NTH), st, w, V, ld, nv, self, n, gate, red, mb.ms, mb.tab);
    if (red.out) launch_finalize(red.partials, la_blocks(n), nt, red.out, st, gate, mb);
}

// w -= sum_v h[v] V_v.
// With dots (the first pass) the gate g2 of the second pass decides: where it opens, the
// kernel goes on to that pass's multi-dot <w, v_q> of the w it has just formed, still in
// registers: the block partials at dots[q * gridDim.x + blockIdx.x], with the multi-dot
// kernel's products, order and partial layout (its launch, one kernel per iteration, is
// saved); where it stays closed, work-group 0 stores ||w||^2 after this pass, by Pythagoras,
// to pub.out and publishes (first thing, so that its loads and host stores overlap the update).
// SELF: the gated second Gram-Schmidt pass together with the iteration's last reduction and
// its publication (pub), in one launch:
//  * gate closed (the pass is skipped): every work-group returns at once;
//  * gate open: h is not given but formed by every work-group from the multi-dot's hnb block
//    partials per entry at hpart (lane-strided sums and the wave's butterfly, a fixed order;
//    work-group 0 stores it to hout), each work-group updates its part of w and stores its
//    ||w||^2 partial in red; the last work-group to finish (a release fence and a counter in
//    device memory, so no work-group waits for another) sums the partials in a fixed order into
//    pub.out, publishes, and clears the counter for the next launch.
// Publishing stores the scalar block pub.src[0..ns) to host-visible pinned memory, entry idx
// replaced by pub.out's value, entry fidx by 1 where the second pass ran (else 0) and, where
// the gate is closed, entries zoff .. zoff+zn (the skipped pass's coefficients) by 0, so the
// host reads the Hessenberg column after the iteration's completion event without a separate
// copy.
template <bool SELF>
__global__ void __launch_bounds__(LA_NTH)
update_kernel(double* __restrict__ w, const double* __restrict__ V, long ld, int nv, long n,
              const double* __restrict__ h, Gate gate, Red red, long ms, const MemberArgs* __restrict__ mt,
              const double* __restrict__ hpart, int hnb, double* __restrict__ hout, Gate g2,
              double* __restrict__ dots, Publish pub)
{
    n = len_of(n, mt);
    gate.h = mbr(gate.h, ms);
    g2.h = mbr(g2.h, ms);
    pub.out = mbr(pub.out, ms);
    pub.src = mbr(pub.src, ms);
    pub.cnt = mbr(pub.cnt, ms);
    pub.host += (long)blockIdx.z * pub.host_stride;
    bool dots2 = false;
    if constexpr (SELF) {
        if (!gate_open(gate)) return;   // every lane takes part in the gate's wave sum
    } else {
        if (!gate_open(gate)) return;
        if (dots) {
            const double after = gate_after(g2);   // every lane, as above
            dots2 = after < g2.tau2 * g2.h[g2.nv];   // gate_open's decision
            if (!dots2 && blockIdx.x == 0) {
                if (threadIdx.x == 0) pub.out[0] = after;
                for (int i = threadIdx.x; i < pub.ns; i += LA_NTH)
                    pub.host[i] = (i == pub.idx)                             ? after
                                  : (i == pub.fidx)                          ? 0.0
                                  : (i >= pub.zoff && i < pub.zoff + pub.zn) ? 0.0
                                                                             : pub.src[i];
            }
        }
    }
    w = mbr(w, ms);
    V = mbr(V, ms);
    red = mbr(red, ms);
    __shared__ double hs[SELF ? 64 : 1];
    if constexpr (SELF) {
        hpart = mbr(hpart, ms);
        const int lane = threadIdx.x & 63;
        for (int q = threadIdx.x >> 6; q < nv; q += LA_NTH / 64) {
            double a = 0.0;
            for (int i = lane; i < hnb; i += 64) a += hpart[(long)q * hnb + i];
            a = wave_sum(a);
            if (lane == 0) hs[q] = a;
        }
        __syncthreads();
        if (blockIdx.x == 0 && (int)threadIdx.x < nv) mbr(hout, ms)[threadIdx.x] = hs[threadIdx.x];
    } else {
        h = mbr(h, ms);
    }
    auto coef = [&](int v) { if constexpr (SELF) return hs[v]; else return h[v]; };
    const long base = (long)blockIdx.x * LA_NTH * LA_EL + threadIdx.x;
    double acc[LA_EL];
#pragma unroll
    for (int k = 0; k < LA_EL; ++k) {
        const long i = base + (long)k * LA_NTH;
        acc[k] = i < n ? w[i] : 0.0;
    }
    int v = 0;
    if (base - threadIdx.x + LA_NTH * LA_EL <= n) {
        // whole block: four basis vectors at a time, every load issued before the
        // products (the same products in the same order as below)
        for (; v + 4 <= nv; v += 4) {
            double vv[4][LA_EL];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int k = 0; k < LA_EL; ++k) vv[r][k] = V[(long)(v + r) * ld + base + (long)k * LA_NTH];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double hv = coef(v + r);
#pragma unroll
                for (int k = 0; k < LA_EL; ++k) acc[k] -= hv * vv[r][k];
            }
        }
    }
    for (; v < nv; ++v) {
        const double hv = coef(v);
        const double* Vi = V + (long)v * ld;
#pragma unroll
        for (int k = 0; k < LA_EL; ++k) {
            const long i = base + (long)k * LA_NTH;
            if (i < n) acc[k] -= hv * Vi[i];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < LA_EL; ++k) {
        const long i = base + (long)k * LA_NTH;
        if (i < n) {
            w[i] = acc[k];
            s += acc[k] * acc[k];
        }
    }
    if (red.partials) put_partial<LA_NTH>(red, s);
    if constexpr (SELF) {
        __shared__ bool last;
        __shared__ double sh[LA_NTH / 64], total;
        if (threadIdx.x == 0) {
            // release: this work-group's partial (and work-group 0's hout) before its count
            // (no cache invalidation, which the other work-groups' reads of hpart would pay)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            last = atomicAdd(pub.cnt, 1ull) == (unsigned long long)(gridDim.x - 1);
        }
        __syncthreads();
        if (!last) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every work-group's partial after its count
        double a = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += LA_NTH) a += red.partials[i];
        a = block_sum<LA_NTH>(a, sh);   // in thread 0
        if (threadIdx.x == 0) {
            pub.out[0] = a;
            total = a;
            atomicExch(pub.cnt, 0ull);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < pub.ns; i += LA_NTH)
            pub.host[i] = (i == pub.idx) ? total : (i == pub.fidx) ? 1.0 : pub.src[i];
        return;
    }
    if (!dots2) return;
    dots = mbr(dots, ms);
    constexpr int NW = LA_NTH / 64, G = 4;
    __shared__ double sd[NW][G];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool whole = base - threadIdx.x + LA_NTH * LA_EL <= n;
    for (int v0 = 0; v0 < nv; v0 += G) {
        double a[G];
#pragma unroll
        for (int q = 0; q < G; ++q) a[q] = 0.0;
        if (whole && v0 + G <= nv) {
            double vv[LA_EL][G];
#pragma unroll
            for (int k = 0; k < LA_EL; ++k)
#pragma unroll
                for (int q = 0; q < G; ++q) vv[k][q] = V[(long)(v0 + q) * ld + base + (long)k * LA_NTH];
#pragma unroll
            for (int k = 0; k < LA_EL; ++k)
#pragma unroll
                for (int q = 0; q < G; ++q) a[q] += acc[k] * vv[k][q];
        } else {
#pragma unroll
            for (int k = 0; k < LA_EL; ++k) {
                const long i = base + (long)k * LA_NTH;
                if (i < n) {
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        if (v0 + q < nv) a[q] += acc[k] * V[(long)(v0 + q) * ld + i];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (v0 + q < nv) {
                const double t = wave_sum(a[q]);
                if (lane == 0) sd[wid][q] = t;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < G && v0 + (int)threadIdx.x < nv) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < NW; ++r) t += sd[r][threadIdx.x];
            dots[(long)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

void launch_update(double* w, const double* V, long ld, int nv, long n, const double* h, Red red, hipStream_t st,
                   Gate gate, const Mb& mb, Gate g2, double* dots, const Publish& pub)
{
    timed_launch(update_kernel<false>, dim3(la_blocks(n), 1, mb.n), dim3(LA_NTH), st, w, V, ld, nv, n, h, gate,
                 red, mb.ms, mb.tab, (const double*)nullptr, 0, (double*)nullptr, g2, dots, pub);
    if (red.out) launch_finalize(red.partials, la_blocks(n), 1, red.out, st, Gate{}, mb);
}

void launch_update2_publish(double* w, const double* V, long ld, int nv, long n, Gate gate, const double* hpart,
                            double* hout, double* wpart, const Publish& pub, hipStream_t st, const Mb& mb)
{
    timed_launch(update_kernel<true>, dim3(la_blocks(n), 1, mb.n), dim3(LA_NTH), st, w, V, ld, nv, n,
                 (const double*)nullptr, gate, Red{wpart, nullptr}, mb.ms, mb.tab, hpart, la_blocks(n), hout, Gate{},
                 (double*)nullptr, pub);
}

__global__ void __launch_bounds__(256)
scale_kernel(double* __restrict__ out, const double* __restrict__ in, long n, const double* __restrict__ nrm2,
             double sgn, long ms, const MemberArgs* __restrict__ mt)
{
    n = len_of(n, mt);
    out = mbr(out, ms);
    in = mbr(in, ms);
    nrm2 = mbr(nrm2, ms);
    const double s = sgn / sqrt(nrm2[0]);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) out[i] = in[i] * s;
}

// out = sgn * in / sqrt(nrm2[0]) (per member)
void launch_scale(double* out, const double* in, long n, const double* nrm2, hipStream_t st, double sgn,
                  const Mb& mb)
{
    long b = (n + 255) / 256;
    scale_kernel<<<dim3((unsigned)(b < 4096 ? b : 4096), 1, mb.n), dim3(256), 0, st>>>(out, in, n, nrm2, sgn, mb.ms,
                                                                                       mb.tab);
}

__global__ void __launch_bounds__(LA_NTH)
lincomb_kernel(double* out, const double* base_, const double* __restrict__ Z, long ld, int nv, long n,
               const double* __restrict__ y, long ms, const MemberArgs* __restrict__ mt)
{
    n = len_of(n, mt);
    out = mbr(out, ms);
    base_ = mbr(base_, ms);
    Z = mbr(Z, ms);
    y = mbr(y, ms);
    const long base = (long)blockIdx.x * LA_NTH * LA_EL + threadIdx.x;
    double acc[LA_EL];
#pragma unroll
    for (int k = 0; k < LA_EL; ++k) {
        const long i = base + (long)k * LA_NTH;
        acc[k] = (i < n && base_) ? base_[i] : 0.0;
    }
    for (int v = 0; v < nv; ++v) {
        const double yv = y[v];
        if (yv == 0.0) continue;   // a zero coefficient adds nothing (its column may be unset)
        const double* Zi = Z + (long)v * ld;
#pragma unroll
        for (int k = 0; k < LA_EL; ++k) {
            const long i = base + (long)k * LA_NTH;
            if (i < n) acc[k] += yv * Zi[i];
        }
    }
#pragma unroll
    for (int k = 0; k < LA_EL; ++k) {
        const long i = base + (long)k * LA_NTH;
        if (i < n) out[i] = acc[k];
    }
}

void launch_lincomb(double* out, const double* base, const double* Z, long ld, int nv, long n, const double* y,
                    hipStream_t st, const Mb& mb)
{
    lincomb_kernel<<<dim3(la_blocks(n), 1, mb.n), dim3(LA_NTH), 0, st>>>(out, base, Z, ld, nv, n, y, mb.ms, mb.tab);
}

__global__ void __launch_bounds__(256)
axpby_kernel(double* out, double a, const double* x, double b, const double* y,
             long n, long ms, const MemberArgs* __restrict__ mt)
{
    n = len_of(n, mt);
    out = mbr(out, ms);
    x = mbr(x, ms);
    y = mbr(y, ms);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) out[i] = a * x[i] + b * y[i];
}

void launch_axpby(double* out, double a, const double* x, double b, const double* y, long n, hipStream_t st,
                  const Mb& mb)
{
    long blk = (n + 255) / 256;
    axpby_kernel<<<dim3((unsigned)(blk < 4096 ? blk : 4096), 1, mb.n), dim3(256), 0, st>>>(out, a, x, b, y, n, mb.ms,
                                                                                           mb.tab);
}

// Stage of the DG-level pseudo-time smoother; out may alias x0 or t (no restrict):
// every element is read and written by the same thread.
__global__ void __launch_bounds__(256)
dg_smooth_kernel(double* out, const double* x0, const double* __restrict__ r, const double* t, double alpha,
                 const double* __restrict__ dtau, long n, Red red, long ms)
{
    out = mbr(out, ms);
    x0 = mbr(x0, ms);
    r = mbr(r, ms);
    t = mbr(t, ms);
    dtau = mbr(dtau, ms);
    red = mbr(red, ms);
    const double s = dtau ? alpha * dtau[0] : alpha;
    double a = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double d = t ? r[i] - t[i] : r[i];
        const double v = x0 ? x0[i] + s * d : s * d;
        out[i] = v;
        a += v * v;
    }
    if (red.partials) put_partial<256>(red, a);
}

void launch_dg_smooth(double* out, const double* x0, const double* r, const double* t, double alpha,
                      const double* dtau, long n, Red red, hipStream_t st, const Mb& mb)
{
    long b = (n + 255) / 256;
    const int nb = (int)(b < 1024 ? b : 1024);
    if (!red.out) red.partials = nullptr;
    timed_launch(dg_smooth_kernel, dim3(nb, 1, mb.n), dim3(256), st, out, x0, r, t, alpha, dtau, n, red, mb.ms);
    if (red.out) launch_finalize(red.partials, nb, 1, red.out, st, Gate{}, mb);
}

__global__ void __launch_bounds__(64) dg_dtau_kernel(const double* __restrict__ lam, double* __restrict__ out,
                                                     double hx, double hz, double mu, double adt, double cfl,
                                                     long ms)
{
    lam = mbr(lam, ms);
    out = mbr(out, ms);
    if (threadIdx.x == 0)
        out[0] = cfl / (1.0 + adt * (lam[0] * (1.0 / hx + 1.0 / hz) + 2.0 * mu * (1.0 / (hx * hx) + 1.0 / (hz * hz))));
}

void launch_dg_dtau(const double* lam, double* out, double hx, double hz, double mu, double adt, double cfl,
                    hipStream_t st, const Mb& mb)
{
    dg_dtau_kernel<<<dim3(1, 1, mb.n), dim3(64), 0, st>>>(lam, out, hx, hz, mu, adt, cfl, mb.ms);
}

__global__ void __launch_bounds__(256) zero_kernel(unsigned* __restrict__ x, long n, long ms)
{
    x = mbr(x, ms);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) x[i] = 0u;
}

// x[i] = a fixed pattern of values in [-1/2, 1/2) (test vectors of the autotuner)
template <typename T> __global__ void __launch_bounds__(256) fill_pattern_kernel(T* __restrict__ x, long n, long ms)
{
    x = mbr(x, ms);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        x[i] = (T)((double)(((unsigned long)i * 2654435761UL) & 0xffffUL) * (1.0 / 65536.0) - 0.5);
}

template <typename T> void launch_fill_pattern(T* x, long n, hipStream_t st, const Mb& mb)
{
    const long nb = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
    fill_pattern_kernel<T><<<dim3((unsigned)nb, 1, mb.n), dim3(256), 0, st>>>(x, n, mb.ms);
}
template void launch_fill_pattern<double>(double*, long, hipStream_t, const Mb&);
template void launch_fill_pattern<float>(float*, long, hipStream_t, const Mb&);

void launch_zero(void* ptr, size_t bytes, hipStream_t st, const Mb& mb)
{
    const long n = (long)(bytes / 4);
    long blk = (n + 255) / 256;
    zero_kernel<<<dim3((unsigned)(blk < 4096 ? blk : 4096), 1, mb.n), dim3(256), 0, st>>>((unsigned*)ptr, n, mb.ms);
}

__global__ void __launch_bounds__(256) set_live_kernel(MemberArgs* __restrict__ tab, int n, LiveBits bits)
{
    for (int m = blockIdx.x * 256 + threadIdx.x; m < n; m += gridDim.x * 256)
        tab[m].live = (int)((bits.w[m >> 6] >> (m & 63)) & 1ull);
}

void launch_set_live(MemberArgs* tab, int n, const LiveBits& bits, hipStream_t st)
{
    set_live_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(tab, n, bits);
}

}  // namespace jfmg
