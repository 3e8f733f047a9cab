// device.h -- device-side helpers shared by the gfx950 kernels of libmts:
// complex arithmetic on interleaved (re, im) pairs, precision-generic math
// wrappers, the link phasor and plaquette angle, and the deterministic
// block reduction into FP64 partials.
#pragma once
#include <math.h>

#include "kernels.h"

namespace mts {

// Complex products with their fused multiply-adds written out (and no other
// contraction), so every kernel that uses them rounds identically.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
#pragma clang fp contract(off)
    return {fma_t(a.re, b.re, -(a.im * b.im)), fma_t(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // conj(a) * b
#pragma clang fp contract(off)
    return {fma_t(a.re, b.re, a.im * b.im), fma_t(a.re, b.im, -(a.im * b.re))};
}
template <typename T>
__device__ __forceinline__ T imc(cx<T> a, cx<T> b) {  // Im(conj(a) * b)
#pragma clang fp contract(off)
    return fma_t(a.re, b.im, -(a.im * b.re));
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) {
#pragma clang fp contract(off)
    return fma_t(a.re, a.re, a.im * a.im);
}

// sin and cos in FP32 for the link phasors: Cody-Waite reduction by pi/2
// (three-part split of pi/2, fused multiply-adds: exact far beyond the link
// angles a run produces), then odd and even polynomials on [-pi/4, pi/4]
// whose coefficients were fitted to sin and cos (relative error 4e-9 and
// absolute error 2e-9 before rounding).  Absolute error <= 1e-7 for
// |x| < 1e5 (about 1.5 ulp of results of order one), 24 instructions on
// its path against 33 for the library's sincosf; larger |x| goes to the
// library routine.
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) {
#pragma clang fp contract(off)
    if (!(fabsf(x) < 1.0e5f)) {
        sincosf(x, s, c);
        return;
    }
    constexpr float TWO_OVER_PI = 0.636619772367581f;
    constexpr float C1 = 1.57079637050628662e+00f;    // fl(pi/2)
    constexpr float C2 = -4.37113882867379289e-08f;   // fl(pi/2 - C1)
    constexpr float C3 = -1.77635683940025046e-15f;   // fl(pi/2 - C1 - C2)
    const float j = rintf(x * TWO_OVER_PI);
    const int q = (int)j;
    float r = __builtin_fmaf(-j, C1, x);
    r = __builtin_fmaf(-j, C2, r);
    r = __builtin_fmaf(-j, C3, r);
    const float r2 = r * r;
    float ps = __builtin_fmaf(r2, -1.951456361e-04f, 8.332156576e-03f);
    ps = __builtin_fmaf(r2, ps, -1.666665524e-01f);
    const float sr = __builtin_fmaf(r2 * r, ps, r);
    float pc = __builtin_fmaf(r2, 2.502162715e-05f, -1.389301848e-03f);
    pc = __builtin_fmaf(r2, pc, 4.166677594e-02f);
    const float cr = __builtin_fmaf(r2 * r2, pc, __builtin_fmaf(r2, -0.5f, 1.0f));
    // quadrant q: (sin, cos) of x = (sr, cr), (cr, -sr), (-sr, -cr), (-cr, sr)
    const bool swap = (q & 1) != 0;
    float sv = swap ? cr : sr, cv = swap ? sr : cr;
    if (q & 2) sv = -sv;
    if ((q + 1) & 2) cv = -cv;
    *s = sv;
    *c = cv;
}
// The same in FP64: three-part split of pi/2 (to 160 bits), then the Taylor
// series of sin to x^15 and cos to x^16 on [-pi/4, pi/4] (truncation below
// 1e-16); within 1 ulp for |x| < 1e5 in an exact-arithmetic emulation.
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) {
#pragma clang fp contract(off)
    if (!(fabs(x) < 1.0e5)) {
        sincos(x, s, c);
        return;
    }
    constexpr double TWO_OVER_PI = 0.6366197723675814;
    constexpr double C1 = 1.5707963267948966;        // fl(pi/2)
    constexpr double C2 = 6.123233995736766e-17;     // fl(pi/2 - C1)
    constexpr double C3 = -1.4973849048591698e-33;   // fl(pi/2 - C1 - C2)
    const double j = rint(x * TWO_OVER_PI);
    const int q = (int)j;
    double r = __builtin_fma(-j, C1, x);
    r = __builtin_fma(-j, C2, r);
    r = __builtin_fma(-j, C3, r);
    const double r2 = r * r;
    // sin r = r + r^3 (-1/3! + r^2 (1/5! - ...)), cos r = 1 - r^2/2 + r^4 (1/4! - r^2 (1/6! - ...))
    double ps = __builtin_fma(r2, -7.647163731819816e-13, 1.6059043836821613e-10);
    ps = __builtin_fma(r2, ps, -2.505210838544172e-08);
    ps = __builtin_fma(r2, ps, 2.7557319223985893e-06);
    ps = __builtin_fma(r2, ps, -0.0001984126984126984);
    ps = __builtin_fma(r2, ps, 0.008333333333333333);
    ps = __builtin_fma(r2, ps, -0.16666666666666666);
    const double sr = __builtin_fma(r2 * r, ps, r);
    double pc = __builtin_fma(r2, 4.779477332387385e-14, -1.1470745597729725e-11);
    pc = __builtin_fma(r2, pc, 2.08767569878681e-09);
    pc = __builtin_fma(r2, pc, -2.755731922398589e-07);
    pc = __builtin_fma(r2, pc, 2.48015873015873e-05);
    pc = __builtin_fma(r2, pc, -0.001388888888888889);
    pc = __builtin_fma(r2, pc, 0.041666666666666664);
    const double cr = __builtin_fma(r2 * r2, pc, __builtin_fma(r2, -0.5, 1.0));
    const bool swap = (q & 1) != 0;
    double sv = swap ? cr : sr, cv = swap ? sr : cr;
    if (q & 2) sv = -sv;
    if ((q + 1) & 2) cv = -cv;
    *s = sv;
    *c = cv;
}

// sin and cos alone, through the same reduction and polynomials (the
// compiler shares the work where both are taken of one angle)
template <typename T>
__device__ __forceinline__ T sin_t(T x) {
    T s, c;
    sincos_t(x, &s, &c);
    return s;
}
template <typename T>
__device__ __forceinline__ T cos_t(T x) {
    T s, c;
    sincos_t(x, &s, &c);
    return c;
}

// Two-argument arctangent in FP32, for the phases alpha = arg(phi) of the
// winding stage: the octant reduction a = min(|x|, |y|) / max(|x|, |y|) in
// [0, 1], atan(a) from an odd polynomial a q(a^2) of degree 15, then the
// octant's reflections (pi/2 - r, pi - r, sign of y).  The coefficients are
// a fit of atan on [0, 1] made for this function: Lawson's iteratively
// reweighted least squares (minimax in the limit) on 4000 Chebyshev points,
// rounded to FP32; evaluated in FP32 (Horner), atan(a) is within 1.4e-7 of
// the true value on all of [0, 1], and the result within 4e-7 rad with the
// reflections' rounding: far inside the 1e-4 rad margin the winding guard
// keeps from the branch cut, so windings do not depend on it.  About 20
// instructions against about 50 for the library's atan2f.  NaN for a NaN
// argument; (0, 0) is the caller's case (phase_of).
__device__ __forceinline__ float atan2_fast(float y, float x) {
#pragma clang fp contract(fast)
    constexpr float C0 = 0.9999993443489075f, C1 = -0.33329859375953674f, C2 = 0.19946566224098206f,
                    C3 = -0.1390862911939621f, C4 = 0.09642194956541061f, C5 = -0.05591228976845741f,
                    C6 = 0.021862929686903954f, C7 = -0.004054558929055929f;
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float a = mn * __builtin_amdgcn_rcpf(mx);
    const float s = a * a;
    float q = C7;
    q = q * s + C6;
    q = q * s + C5;
    q = q * s + C4;
    q = q * s + C3;
    q = q * s + C2;
    q = q * s + C1;
    q = q * s + C0;
    float r = a * q;
    if (ay > ax) r = 1.57079637f - r;
    if (x < 0.0f) r = 3.14159274f - r;
    r = copysignf(r, y);
    return (x != x || y != y) ? x + y : r;
}

__device__ __forceinline__ float atan2_t(float y, float x) { return atan2_fast(y, x); }
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float rint_t(float x) { return rintf(x); }
__device__ __forceinline__ double rint_t(double x) { return rint(x); }

template <typename T>
struct Pi;
template <>
struct Pi<float> {
    static constexpr float v = 3.14159265358979323846f;
};
template <>
struct Pi<double> {
    static constexpr double v = 3.14159265358979323846;
};

// ---- link phases for the plaquette windings (Sec. III.A)
//
// With alpha(x) = arg phi(x), the covariant link phase
//   chi_mu(x) = arg(conj(phi(x)) U_mu(x) phi(x+mu)) = wrap(alpha(x+mu) - alpha(x) - h A_mu(x))
// takes no transcendental function per link.  A link whose chi lies within
// Guard::cut of the branch cut, has an endpoint with phi = 0 or |h A| above
// Guard::big is recomputed in FP64 from the complex product, so the windings
// equal an FP64 evaluation of the same inputs bit for bit.

template <typename T>
struct Guard;
template <>
struct Guard<float> {
    static constexpr float cut = 1e-4f, big = 1e3f;
};
template <>
struct Guard<double> {
    static constexpr double cut = 1e-9, big = 1e6;
};

template <typename T>
__device__ __forceinline__ T wrap_pi(T v) {   // into [-pi, pi], +pi for the cut itself
    const T two_pi = T(2) * Pi<T>::v;
    T r = v - two_pi * rint_t(v * (T(0.5) / Pi<T>::v));
    return r <= -Pi<T>::v ? Pi<T>::v : r;
}

// FP64 link phase from the complex product, -pi mapped to +pi.
__device__ __forceinline__ double exact_link_phase_body(double are, double aim, double bre, double bim, double hA) {
    double s, c;
    sincos(hA, &s, &c);
    const double ure = c, uim = -s;
    // (conj(a) * U) * b
    const double tre = are * ure + aim * uim, tim = are * uim - aim * ure;
    const double zre = tre * bre - tim * bim, zim = tre * bim + tim * bre;
    double ang = atan2(zim, zre);
    return ang <= -Pi<double>::v ? Pi<double>::v : ang;
}
static __device__ __noinline__ double exact_link_phase(double are, double aim, double bre, double bim, double hA) {
    return exact_link_phase_body(are, aim, bre, bim, hA);
}

// The fast link phase from the two phases; `need` is set where the guard
// asks for the FP64 product instead.
template <typename T>
__device__ __forceinline__ T link_chi_fast(T aa, T ab, T hA, bool &need) {
    const T chi = wrap_pi((ab - aa) - hA);
    need = isnan(aa) || isnan(ab) || fabs(chi) > Pi<T>::v - Guard<T>::cut || fabs(hA) > Guard<T>::big;
    return chi;
}

// The guarded link phase from the field values at the two ends (0 if either
// vanishes), FP64.
template <typename T>
__device__ __forceinline__ T link_chi_exact(cx<T> a, cx<T> b, T hA) {
    const bool z0 = (a.re == T(0) && a.im == T(0)) || (b.re == T(0) && b.im == T(0));
    return z0 ? T(0) : (T)exact_link_phase(a.re, a.im, b.re, b.im, (double)hA);
}

// Wrap count of a link for the fused windings: with v = (ab - aa) - h A,
// n = rint(v / 2 pi) and chi = v - 2 pi n.  Around a plaquette the phase
// differences telescope and the h A terms make up the plaquette angle, so the
// winding through a face is minus the oriented sum of its four links' wrap
// counts.  `flag` where the guard asks for FP64 instead (|chi| within
// Guard::cut of the branch cut, |h A| above Guard::big, or a NaN phase at a
// zero of the field); an unflagged count has |n| < 256.
template <typename T>
__device__ __forceinline__ int link_wrap(T aa, T ab, T hA, bool &flag) {
#pragma clang fp contract(off)
    const T v = (ab - aa) - hA;
    const T n = rint_t(v * (T(0.5) / Pi<T>::v));
    const T chi = v - (T(2) * Pi<T>::v) * n;
    flag = !(fabs(chi) <= Pi<T>::v - Guard<T>::cut && fabs(hA) <= Guard<T>::big);
    return flag ? 0 : (int)n;
}

// h A of a link, rounded on its own (the same value wherever it is formed)
template <typename T>
__device__ __forceinline__ T link_angle(T h, T A) {
#pragma clang fp contract(off)
    return h * A;
}

// Packed wrap counts of a site's three links (x, y, z: 9-bit fields, two's
// complement) and their guard flags (bits 27, 28, 29).
__device__ __forceinline__ int wrap_word(int nx, int ny, int nz, bool fx, bool fy, bool fz) {
    return (nx & 0x1FF) | ((ny & 0x1FF) << 9) | ((nz & 0x1FF) << 18) | ((int)fx << 27) | ((int)fy << 28) |
           ((int)fz << 29);
}
template <int K>
__device__ __forceinline__ int wrap_n(int w) {
    return (int)((uint32_t)w << (23 - 9 * K)) >> 23;
}
// the flag bits a face reads from the words of its corner sites: all three
// at the site, y and z at +x, x and z at +y, x and y at +z
constexpr int WRAP_F_XYZ = 7 << 27, WRAP_F_YZ = 6 << 27, WRAP_F_XZ = 5 << 27, WRAP_F_XY = 3 << 27;

// chi + h A of a link for the fused diagnostics, or NaN where the guard asks
// for the FP64 product (near the branch cut or |h A| above Guard::big; a NaN
// phase, phi = 0 at an end, gives NaN by itself).
template <typename T>
__device__ __forceinline__ T link_value_or_nan(T aa, T ab, T hA) {
#pragma clang fp contract(off)
    const T chi = wrap_pi((ab - aa) - hA);
    const bool ok = fabs(chi) <= Pi<T>::v - Guard<T>::cut && fabs(hA) <= Guard<T>::big;
    return ok ? chi + hA : T(NAN);
}

// chi of the link from site a to site b (phases aa, ab; link hA), guarded.
template <typename T>
__device__ __forceinline__ T link_chi(T aa, T ab, T hA, const cx<T> *phi, uint32_t sa, uint32_t sb) {
    bool need;
    T chi = link_chi_fast(aa, ab, hA, need);
    if (need) {
        const cx<T> a = phi[sa], b = phi[sb];
        const bool z0 = (a.re == T(0) && a.im == T(0)) || (b.re == T(0) && b.im == T(0));
        chi = z0 ? T(0) : (T)exact_link_phase(a.re, a.im, b.re, b.im, (double)hA);
    }
    return chi;
}

// arg phi, NaN where phi = 0 (the winding kernels' phase)
template <typename T>
__device__ __forceinline__ T phase_of(cx<T> p) {
    return (p.re == T(0) && p.im == T(0)) ? T(NAN) : atan2_t(p.im, p.re);
}

// Gauss law at n + 1/2 (Sec. II; reading R9): the divergence of E from its
// values at the site and at x - i, the charge term g Im[conj(phi^n) Pi^{n+1/2}],
// and their accumulation into |C| and the scale |div E| + |g rho|.  One
// definition for every kernel that evaluates it, contraction off, so the
// per-site terms agree bit for bit.
template <typename T>
__device__ __forceinline__ T gauss_div(T ex, T ex_m, T ey, T ey_m, T ez, T ez_m, T inv_h) {
#pragma clang fp contract(off)
    return (((ex - ex_m) + (ey - ey_m)) + (ez - ez_m)) * inv_h;
}
template <typename T>
__device__ __forceinline__ T gauss_charge(T g, cx<T> f, cx<T> p) {
#pragma clang fp contract(off)
    return g * imc(f, p);
}
template <typename T>
__device__ __forceinline__ void gauss_accumulate(T div, T grho, double &abs_acc, double &scale_acc) {
#pragma clang fp contract(off)
    abs_acc += (double)fabs(div - grho);
    scale_acc += (double)fabs(div) + (double)fabs(grho);
}

// Stores of data written once per step and not re-read by this launch.
// With NT they are streaming (non-temporal) stores that bypass L2
// allocation, leaving L2 to the halo rows neighbouring tiles share; the
// gain depends on the launch (measured 1-3 %), so it is tunable.
// A pointer known to address global memory.  Pointers read from a table in
// device memory are generic to the compiler, which then emits FLAT accesses
// (counted against the LDS wait counter as well, so every LDS wait also
// drains outstanding HBM loads); the round trip through the global address
// space lets it emit global loads and stores instead.
template <typename P>
__device__ __forceinline__ P *as_global(P *p) {
    auto *g = (__attribute__((address_space(1))) P *)(uintptr_t)p;
    return (P *)g;
}

template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(cx<T> *p, cx<T> v) {
    if constexpr (NT) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        v2 w = {v.re, v.im};
        __builtin_nontemporal_store(w, reinterpret_cast<v2 *>(p));
    } else {
        *p = v;
    }
}

// XCD-contiguous numbering of a 1-D grid of nblk workgroups: the blocks the
// hardware deals to XCD k (k, k + 8, ...) become one contiguous run, so
// neighbouring tiles (which share halo rows) run under one L2.
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t nblk) {
    constexpr uint32_t NXCD = 8;
    const uint32_t xcd = b % NXCD, slot = b / NXCD;
    const uint32_t per = nblk / NXCD, extra = nblk % NXCD;
    return xcd * per + min(xcd, extra) + slot;
}

// link phasor exp(-i h A)
template <typename T>
__device__ __forceinline__ cx<T> phasor(T hA) {
    T s, c;
    sincos_t(hA, &s, &c);
    return {c, -s};
}
// The same from h and A, the product rounded on its own (never fused into
// the caller's arithmetic), so every kernel gets the same phasor bits.
template <typename T>
__device__ __forceinline__ cx<T> phasor(T h, T A) {
#pragma clang fp contract(off)
    const T hA = h * A;
    return phasor<T>(hA);
}

// plaquette angle from its four links, in the order
// A_i(x) + A_j(x+i) - A_i(x+j) - A_j(x)
template <typename T>
__device__ __forceinline__ T plaq(T h, T a1, T a2, T a3, T a4) {
    return h * (((a1 + a2) - a3) - a4);
}

// Deterministic block sum of NV doubles: wave64 shuffles, then the waves in
// order through LDS; thread 0 writes partial[slot0 + v][blk].
template <int NV, int NWAVES>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], Partials part, int slot0, uint32_t blk) {
    __shared__ double red[NWAVES][NV];
    const int lane = threadIdx.x + blockDim.x * threadIdx.y;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double t = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        v[q] = t;
    }
    const int wave = lane >> 6;
    if ((lane & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) red[wave][q] = v[q];
    }
    __syncthreads();
    if (lane < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NWAVES; w++) t += red[w][lane];
        part.base[(size_t)(slot0 + lane) * part.maxblk + blk] = t;
    }
}

}  // namespace mts
