// Device helpers shared by the gfx950 kernels: gas physics, the HLLC flux,
// the viscous flux and wave64 / block / multi-block reductions (fixed
// summation order everywhere, no float atomics).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace jfmg {

// sqrt of the unit roundoff used in finite-difference steps: 2^-26 (FP64), 2^-11.5 (FP32)
template <typename T> struct FdEps;
template <> struct FdEps<double> {
    static constexpr double sqrt_eps = 1.4901161193847656e-08;
    static constexpr double inv_sqrt_eps = 1.0 / sqrt_eps;
};
template <> struct FdEps<float> {
    static constexpr double sqrt_eps = 3.4526698300124393e-04;
    static constexpr double inv_sqrt_eps = 1.0 / sqrt_eps;
};

// Gas constants plus the binomial coefficients C(gamma, k) used to evaluate
// the equation of state around the background pressure (see pert_pressure).
constexpr int GAS_NCOEF = 12;
template <typename T> struct Gas {
    T gamma, R, p0;
    T cg[GAS_NCOEF];   // C(gamma, k), k = 0 .. GAS_NCOEF-1
};

template <typename T> __device__ __forceinline__ T dpow(T a, T b)
{
    if constexpr (std::is_same_v<T, float>) return powf(a, b);
    else return pow(a, b);
}
template <typename T> __device__ __forceinline__ T dsqrt(T a)
{
    if constexpr (std::is_same_v<T, float>) return sqrtf(a);
    else return sqrt(a);
}
// Square root of a positive normal number (sound speeds): hardware 1/sqrt
// estimate, one coupled Goldschmidt step for g ~ sqrt(a), h ~ 1/(2 sqrt(a)),
// then two Newton corrections g += h (a - g^2).  Without the rescaling of
// denormal, zero and infinite arguments that the library square root carries.
template <typename T> __device__ __forceinline__ T psqrt(T a)
{
    if constexpr (std::is_same_v<T, float>) {
        return sqrtf(a);
    } else {
        const double y = __builtin_amdgcn_rsq(a);
        double g = a * y, h = 0.5 * y;
        const double r = fma(-h, g, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        double d = fma(-g, g, a);
        g = fma(d, h, g);
        d = fma(-g, g, a);
        return fma(d, h, g);
    }
}
template <typename T> __device__ __forceinline__ T dabs(T a)
{
    if constexpr (std::is_same_v<T, float>) return fabsf(a);
    else return fabs(a);
}

// Element i of an array addressed by a 32-bit byte offset from its base (usually
// wave-uniform, in scalar registers): one vector register per address instead of
// two.  Arrays must be smaller than 4 GiB.
template <typename T> __device__ __forceinline__ T ld(const T* base, unsigned i)
{
    return *(const T*)((const char*)base + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ void st(T* base, unsigned i, T v)
{
    *(T*)((char*)base + i * (unsigned)sizeof(T)) = v;
}

// The same (wave-uniform) pointer, opaque to the optimizer: loads through it are
// issued again instead of being merged with earlier loads of the same address,
// whose values would otherwise be held in registers in between.
template <typename T> __device__ __forceinline__ T* opaque(T* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// A value that is the same in every lane of the wave, moved to scalar registers
// (keeps it out of the vector register budget).
__device__ __forceinline__ double uniform(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Reciprocal from the hardware estimate refined by Newton's iteration for 1/a,
// r <- r + r (1 - a r): the FP64 estimate (relative error ~5e-8) needs two steps
// to reach the accuracy of a correctly rounded division (measured: within one ulp,
// equal to it for >99.9 % of inputs); the FP32 estimate is accurate to one ulp.
// Shorter dependency chain than the IEEE division sequence.  a must be a finite,
// nonzero normal number (densities and HLLC wave-speed differences are).
template <typename T> __device__ __forceinline__ T frcp(T a)
{
    if constexpr (std::is_same_v<T, float>) {
        return __builtin_amdgcn_rcpf(a);
    } else {
        double r = __builtin_amdgcn_rcp(a);
        double e = fma(-a, r, 1.0);
        r = fma(r, e, r);
        e = fma(-a, r, 1.0);
        return fma(r, e, r);
    }
}

// Equation of state of the potential-temperature form, p = p0 (R rho theta / p0)^gamma,
// evaluated at the total state rho theta = rtb (1 + s), s = (rho theta)' / rtb, as
// p = pb (1 + s)^gamma with the background pressure pb = p0 (R rtb / p0)^gamma.
// (1 + s)^gamma is the binomial series in Horner form, truncated below the unit
// roundoff for 1 < gamma <= 5/3: 6 terms for |s| <= 2^-10 (atmospheric pressure
// perturbations; truncation <= 6e-21) and 12 for |s| <= 1/20 (<= 3e-19) in FP64,
// 4 and 7 terms in FP32; pow beyond.  s = 0 returns pb exactly, so background and
// perturbed evaluations agree bitwise.
template <typename T> __device__ __forceinline__ T pert_pressure(const Gas<T>& G, T rt1, T irtb, T pb)
{
    constexpr bool F32 = std::is_same_v<T, float>;
    const T s = rt1 * irtb;
    const T as = dabs<T>(s);
    T f;
    if (as <= T(1.0 / 1024.0)) {
        constexpr int n = F32 ? 4 : 6;
        f = G.cg[n - 1];
#pragma unroll
        for (int k = n - 2; k >= 0; --k) f = f * s + G.cg[k];
    } else if (as <= T(0.05)) {
        constexpr int n = F32 ? 7 : GAS_NCOEF;
        f = G.cg[n - 1];
#pragma unroll
        for (int k = n - 2; k >= 0; --k) f = f * s + G.cg[k];
    } else {
        f = dpow<T>(T(1) + s, G.gamma);
    }
    return pb * f;
}

// The pressure's deviation from the background, p - pb = pb ((1 + s)^gamma - 1): the
// series of pert_pressure without its constant term, so that it is accurate to the
// unit roundoff of p - pb rather than of p (FP32 FV operators, whose values enter only
// differences of two evaluations, carry p - pb where the pressure enters additively).
template <typename T> __device__ __forceinline__ T pert_dpress(const Gas<T>& G, T rt1, T irtb, T pb)
{
    constexpr bool F32 = std::is_same_v<T, float>;
    const T s = rt1 * irtb;
    const T as = dabs<T>(s);
    T f;
    if (as <= T(1.0 / 1024.0)) {
        constexpr int n = F32 ? 4 : 6;
        f = G.cg[n - 1];
#pragma unroll
        for (int k = n - 2; k >= 1; --k) f = f * s + G.cg[k];
        f = f * s;
    } else if (as <= T(0.05)) {
        constexpr int n = F32 ? 7 : GAS_NCOEF;
        f = G.cg[n - 1];
#pragma unroll
        for (int k = n - 2; k >= 1; --k) f = f * s + G.cg[k];
        f = f * s;
    } else {
        f = dpow<T>(T(1) + s, G.gamma) - T(1);
    }
    return pb * f;
}

// Convective flux F_c(U) . n for an axis-aligned unit normal (nx, nz), pressure p given.
template <typename T>
__device__ __forceinline__ void conv_flux(const T* U, T p, T nx, T nz, T* F)
{
    const T ir = frcp<T>(U[0]);
    const T q = (U[1] * nx + U[2] * nz) * ir;
    F[0] = U[1] * nx + U[2] * nz;
    F[1] = U[1] * q + p * nx;
    F[2] = U[2] * q + p * nz;
    F[3] = U[3] * q;
}

// Both Cartesian convective fluxes F_c^x(U) and F_c^z(U) (pressure given) with one
// reciprocal of rho; the same numbers as conv_flux with (1, 0) and (0, 1).
template <typename T>
__device__ __forceinline__ void conv_flux_xz(const T* U, T p, T* Fx, T* Fz)
{
    const T ir = frcp<T>(U[0]);
    const T u = U[1] * ir, w = U[2] * ir;
    Fx[0] = U[1];
    Fx[1] = U[1] * u + p;
    Fx[2] = U[2] * u;
    Fx[3] = U[3] * u;
    Fz[0] = U[2];
    Fz[1] = U[1] * w;
    Fz[2] = U[2] * w + p;
    Fz[3] = U[3] * w;
}

// HLLC flux (Toro) with Davis wave speeds S_L = min(q_L - c_L, q_R - c_R),
// S_R = max(q_L + c_L, q_R + c_R); star flux in the S*-factored form
// (S*(S_K U_K - F_K) + S_K p*_K D*) / (S_K - S*), p*_K = p_K + rho_K (S_K - q_K)(S* - q_K).
// Pressures of both states are given.
template <typename T>
__device__ __forceinline__ void hllc(const Gas<T>& G, const T* UL, const T* UR, T pL, T pR, T nx, T nz, T* F)
{
    const T rL = UL[0], rR = UR[0];
    const T irL = frcp<T>(rL), irR = frcp<T>(rR);
    const T qL = (UL[1] * nx + UL[2] * nz) * irL, qR = (UR[1] * nx + UR[2] * nz) * irR;
    const T cL = dsqrt<T>(G.gamma * pL * irL), cR = dsqrt<T>(G.gamma * pR * irR);
    const T SL = fmin(qL - cL, qR - cR);
    const T SR = fmax(qL + cL, qR + cR);
    if (SL >= T(0)) {
        F[0] = UL[1] * nx + UL[2] * nz;
        F[1] = UL[1] * qL + pL * nx;
        F[2] = UL[2] * qL + pL * nz;
        F[3] = UL[3] * qL;
        return;
    }
    const T Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) * frcp<T>(rL * (SL - qL) - rR * (SR - qR));
    const T* UK;
    T SK, rK, qK, pK;
    if (Ss >= T(0)) { UK = UL; SK = SL; rK = rL; qK = qL; pK = pL; }
    else if (SR > T(0)) { UK = UR; SK = SR; rK = rR; qK = qR; pK = pR; }
    else {
        F[0] = UR[1] * nx + UR[2] * nz;
        F[1] = UR[1] * qR + pR * nx;
        F[2] = UR[2] * qR + pR * nz;
        F[3] = UR[3] * qR;
        return;
    }
    const T FK0 = UK[1] * nx + UK[2] * nz;
    const T FK1 = UK[1] * qK + pK * nx;
    const T FK2 = UK[2] * qK + pK * nz;
    const T FK3 = UK[3] * qK;
    const T pst = pK + rK * (SK - qK) * (Ss - qK);
    const T iden = frcp<T>(SK - Ss);
    F[0] = (Ss * (SK * UK[0] - FK0)) * iden;
    F[1] = (Ss * (SK * UK[1] - FK1) + SK * pst * nx) * iden;
    F[2] = (Ss * (SK * UK[2] - FK2) + SK * pst * nz) * iden;
    F[3] = (Ss * (SK * UK[3] - FK3)) * iden;
}

// The same HLLC flux for the normal +e_D of a Cartesian face (D = 1: x, D = 2: z),
// with 1/rho of both states given (the callers reuse them).  A face with normal
// -e_D is the mirror case, H(a, b; -e) = -H(b, a; +e), so every Cartesian face
// (slip walls included, via a mirrored ghost state) needs only this form.
template <typename T, int D>
__device__ __forceinline__ void hllc_ax(const Gas<T>& G, const T* UL, const T* UR, T pL, T pR, T irL, T irR, T* F)
{
    constexpr int E = 3 - D;   // tangential momentum
    const T rL = UL[0], rR = UR[0];
    const T qL = UL[D] * irL, qR = UR[D] * irR;
    const T cL = psqrt<T>(G.gamma * pL * irL), cR = psqrt<T>(G.gamma * pR * irR);
    const T SL = fmin(qL - cL, qR - cR);
    const T SR = fmax(qL + cL, qR + cR);
    if (SL >= T(0)) {
        F[0] = UL[D];
        F[D] = UL[D] * qL + pL;
        F[E] = UL[E] * qL;
        F[3] = UL[3] * qL;
        return;
    }
    if (SR <= T(0)) {
        F[0] = UR[D];
        F[D] = UR[D] * qR + pR;
        F[E] = UR[E] * qR;
        F[3] = UR[3] * qR;
        return;
    }
    const T Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) * frcp<T>(rL * (SL - qL) - rR * (SR - qR));
    const bool lk = Ss >= T(0);
    const T SK = lk ? SL : SR, rK = lk ? rL : rR, qK = lk ? qL : qR, pK = lk ? pL : pR;
    const T uD = lk ? UL[D] : UR[D], uE = lk ? UL[E] : UR[E], u3 = lk ? UL[3] : UR[3];
    const T pst = pK + rK * (SK - qK) * (Ss - qK);
    const T iden = frcp<T>(SK - Ss);
    F[0] = (Ss * (SK * rK - uD)) * iden;
    F[D] = (Ss * (SK * uD - (uD * qK + pK)) + SK * pst) * iden;
    F[E] = (Ss * (SK * uE - uE * qK)) * iden;
    F[3] = (Ss * (SK * u3 - u3 * qK)) * iden;
}

// HLLC flux F . n on a Cartesian face whose normal n = side e_D (side = +-1) has
// its axis chosen per thread (xf: D = 1, else D = 2), so that the lanes of a wave
// working on x- and z-faces take one path: both states are rotated into the face
// frame (normal momentum side U_D, tangential U_E), the one-dimensional form above
// is evaluated there and its normal-momentum component rotated back (F_D = side
// times it).  Multiplication by +-1 and the component swap are exact.
template <typename T>
__device__ __forceinline__ void hllc_face(const Gas<T>& G, const T* UL, const T* UR, T pL, T pR, T irL, T irR,
                                          bool xf, T side, T* F)
{
    const T a[4] = {UL[0], side * (xf ? UL[1] : UL[2]), xf ? UL[2] : UL[1], UL[3]};
    const T b[4] = {UR[0], side * (xf ? UR[1] : UR[2]), xf ? UR[2] : UR[1], UR[3]};
    T Fn[4];
    hllc_ax<T, 1>(G, a, b, pL, pR, irL, irR, Fn);
    const T fd = side * Fn[1];
    F[0] = Fn[0];
    F[1] = xf ? fd : Fn[2];
    F[2] = xf ? Fn[2] : fd;
    F[3] = Fn[3];
}

// The same HLLC flux less pb e_D (pb: the background pressure of the face, the same on
// both sides): p (full) sets the sound speeds, dp = p - pb enters wherever the pressure
// is added (the physical fluxes, the star pressure, p_R - p_L).  Algebraically
// F - pb e_D, since the star flux (S*(S_K U_K - F_K) + S_K p*_K e_D) / (S_K - S*) is
// affine in the pressure with weight one.
template <typename T, int D>
__device__ __forceinline__ void hllc_ax_dp(const Gas<T>& G, const T* UL, const T* UR, T pL, T pR, T dpL, T dpR, T irL,
                                           T irR, T* F)
{
    constexpr int E = 3 - D;   // tangential momentum
    const T rL = UL[0], rR = UR[0];
    const T qL = UL[D] * irL, qR = UR[D] * irR;
    const T cL = psqrt<T>(G.gamma * pL * irL), cR = psqrt<T>(G.gamma * pR * irR);
    const T SL = fmin(qL - cL, qR - cR);
    const T SR = fmax(qL + cL, qR + cR);
    if (SL >= T(0)) {
        F[0] = UL[D];
        F[D] = UL[D] * qL + dpL;
        F[E] = UL[E] * qL;
        F[3] = UL[3] * qL;
        return;
    }
    if (SR <= T(0)) {
        F[0] = UR[D];
        F[D] = UR[D] * qR + dpR;
        F[E] = UR[E] * qR;
        F[3] = UR[3] * qR;
        return;
    }
    const T Ss = (dpR - dpL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) * frcp<T>(rL * (SL - qL) - rR * (SR - qR));
    const bool lk = Ss >= T(0);
    const T SK = lk ? SL : SR, rK = lk ? rL : rR, qK = lk ? qL : qR, dpK = lk ? dpL : dpR;
    const T uD = lk ? UL[D] : UR[D], uE = lk ? UL[E] : UR[E], u3 = lk ? UL[3] : UR[3];
    const T pst = dpK + rK * (SK - qK) * (Ss - qK);
    const T iden = frcp<T>(SK - Ss);
    F[0] = (Ss * (SK * rK - uD)) * iden;
    F[D] = (Ss * (SK * uD - (uD * qK + dpK)) + SK * pst) * iden;
    F[E] = (Ss * (SK * uE - uE * qK)) * iden;
    F[3] = (Ss * (SK * u3 - u3 * qK)) * iden;
}

// Viscous flux F_v(U, G) . n = mu rho grad(U_c / rho) . n written with the
// conserved-variable gradient G = (Gx, Gz): mu (G_c - (U_c/rho) G_rho), c = 1..3.
template <typename T>
__device__ __forceinline__ void visc_flux(T mu, const T* U, const T* Gx, const T* Gz, T nx, T nz, T* F)
{
    F[0] = T(0);
    const T ir = frcp<T>(U[0]);
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        T r = U[c] * ir;
        F[c] = mu * ((Gx[c] - r * Gx[0]) * nx + (Gz[c] - r * Gz[0]) * nz);
    }
}

// ---------------------------------------------------------------------------
// Reductions.  Wave64 butterfly, then waves combined by thread 0 in wave order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block sum over NTH threads (a multiple of 64); result valid in thread 0.
template <int NTH> __device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NTH / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}
template <int NTH> __device__ __forceinline__ double block_max(double v, double* sh)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NTH / 64; ++i) s = fmax(s, sh[i]);
    __syncthreads();
    return s;
}

// Multi-block reductions without tickets or fences: every block writes its
// partial with a plain store; the partials are summed in a fixed order either
// by a one-block finalize kernel launched right after the producer (scalars the
// host or a later kernel reads) or by each block of the consuming kernel
// itself (sum_partials).  Kernel boundaries make the partials visible; no
// agent-scope fence is executed per block.
struct Red {
    double* partials;   // [nq][number of blocks]
    double* out;        // if non-null the launcher finalizes into out[0..nq)
};

__device__ __forceinline__ unsigned block_linear() { return blockIdx.y * gridDim.x + blockIdx.x; }

// The dispatcher hands work-groups to the 8 XCDs of the chip round-robin by
// linear id, and each XCD has its own L2.  Stencil kernels therefore renumber
// their tiles so that XCD x works on one contiguous range of tiles (rows of
// neighbouring tiles share halo cache lines inside one L2).  Bijective on [0, nb).
constexpr unsigned NUM_XCD = 8;
__device__ __forceinline__ unsigned xcd_tile(unsigned w, unsigned nb)
{
    const unsigned x = w % NUM_XCD, i = w / NUM_XCD, q = nb / NUM_XCD, r = nb % NUM_XCD;
    return x * q + (x < r ? x : r) + i;
}

template <int NTH> __device__ __forceinline__ void put_partial(const Red& r, double v)
{
    __shared__ double sh[NTH / 64];
    const double s = block_sum<NTH>(v, sh);
    if (threadIdx.x == 0) r.partials[block_linear()] = s;
}

// Lock-step batches: member m of a batched problem lives m * ms bytes after
// member 0 (identical layouts); kernels run with gridDim.z = members and shift
// every per-member pointer by blockIdx.z * ms (ms = 0 for a single problem).
template <typename P> __device__ __forceinline__ P* mbr(P* p, long ms)
{
    return p ? (P*)((char*)p + (long)blockIdx.z * ms) : p;
}
__device__ __forceinline__ Red mbr(Red r, long ms) { return Red{mbr(r.partials, ms), mbr(r.out, ms)}; }

// deterministic sum of n partials, returned to every thread of the block
template <int NTH> __device__ __forceinline__ double sum_partials(const double* p, int n)
{
    __shared__ double sh[NTH / 64];
    __shared__ double res;
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += NTH) a += p[i];
    a = block_sum<NTH>(a, sh);
    if (threadIdx.x == 0) res = a;
    __syncthreads();
    return res;
}

}  // namespace jfmg
