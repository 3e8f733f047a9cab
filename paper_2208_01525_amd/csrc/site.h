// site.h -- the per-site arithmetic of one leapfrog step (Correia & Martins,
// arXiv:2208.01525, Sec. III: the Pi/Psi kick, the E/H kick and the drift),
// shared by the single-step and the two-step tiled kernels so that both
// evaluate every site with the same operations in the same order.  The fused
// multiply-adds are written out and no other contraction is allowed, so the
// two kernels' results are bitwise identical.
#pragma once
#include "device.h"

namespace mts {

// Own plaquette phasors of a site,
//   P_ij(x) = U_i(x) U_j(x+i) conj(U_i(x+j)) conj(U_j(x)) = exp(-i theta_ij(x)),
// so sin theta = -Im P and cos theta = Re P, in the order xy, xz, yz.
// u: the site's links; uy_px = U_y(x+x), ux_py = U_x(x+y), uz_px = U_z(x+x),
// uz_py = U_z(x+y), ux_pz = U_x(x+z), uy_pz = U_y(x+z).
template <typename T>
__device__ __forceinline__ void own_plaquettes(cx<T> ux, cx<T> uy, cx<T> uz, cx<T> uy_px, cx<T> ux_py, cx<T> uz_px,
                                               cx<T> uz_py, cx<T> ux_pz, cx<T> uy_pz, T (&sn)[3], T (&cs)[3]) {
#pragma clang fp contract(off)
    const cx<T> axy = cmul(ux, uy_px), bxy = cmul(ux_py, uy);
    const cx<T> Pxy = cmulc(bxy, axy);     // conj(b) a
    const cx<T> axz = cmul(ux, uz_px), bxz = cmul(ux_pz, uz);
    const cx<T> Pxz = cmulc(bxz, axz);
    const cx<T> ayz = cmul(uy, uz_py), byz = cmul(uy_pz, uz);
    const cx<T> Pyz = cmulc(byz, ayz);
    sn[0] = -Pxy.im;
    sn[1] = -Pxz.im;
    sn[2] = -Pyz.im;
    cs[0] = Pxy.re;
    cs[1] = Pxz.re;
    cs[2] = Pyz.re;
}

// Inputs of one sector's update at a site: the scalar at x and its six
// neighbours, the other sector's scalar at x, the links at x and at x - i,
// the plaquette sines around the links of x, the momenta at n - 1/2 and the
// link angles at n.
template <typename T>
struct SiteIn {
    cx<T> f, o;                        // phi_sigma(x), phi_other(x)
    cx<T> fxp, fxm, fyp, fym, fzp, fzm;
    cx<T> ux, uy, uz, ux_m, uy_m, uz_m;
    T sxy, sxz, syz;                   // own plaquettes
    T sxy_my, sxy_mx, sxz_mx, syz_my, sxz_mz, syz_mz;   // neighbours' (x - j)
    cx<T> p0;                          // Pi^{n-1/2}
    T e0[3];                           // E^{n-1/2}
    T a[3];                            // A^n (h A is the link angle)
};

// Magnetic force on a link, -h^-3 [(s1 - s2) + (s3 - s4)] from the sines of
// the two plaquettes at the link's site and the two at x - j (Sec. III E
// kick, the divergence form of reading R3).
template <typename T>
__device__ __forceinline__ T mag_force(const StepCoef<T> &c, T s1, T s2, T s3, T s4) {
#pragma clang fp contract(off)
    return -c.inv_h3 * ((s1 - s2) + (s3 - s4));
}

// The current 2 e^2 a^{2s} h^-1 Im[conj(phi) U phi(x+i)] (w = U phi(x+i)).
template <typename T>
__device__ __forceinline__ T current(const StepCoef<T> &c, int sec, cx<T> f, cx<T> w) {
#pragma clang fp contract(off)
    return c.cur[sec] * imc(f, w);
}

// The damped gauge kick of one link: (1+omega) E' = (1-omega) E + k (M + J).
template <typename T>
__device__ __forceinline__ T e_kick(const StepCoef<T> &c, T e0, T M, T J) {
#pragma clang fp contract(off)
    return fma_t(c.cE, e0, c.kE * (M + J));
}

template <typename T>
struct SiteOut {
    cx<T> p1;                          // Pi^{n+1/2}   (COOL: the force)
    cx<T> fn;                          // phi^{n+1}
    T e1[3];                           // E^{n+1/2}    (COOL: the force)
    T an[3];                           // A^{n+1}
    cx<T> wx, wy, wz;                  // U_i(x) phi(x+i)
    T m2;                              // |phi(x)|^2
};

// One sector of one step at a site: covariant Laplacian, potential force,
// scalar kick, plaquette (magnetic) force and current, gauge kick, drift.
// With COOL the fields move along their forces (forward Euler of the cooling
// flow; momenta neither read nor produced).
template <typename T, bool COOL>
__device__ __forceinline__ SiteOut<T> site_update(const StepCoef<T> &c, int sec, const SiteIn<T> &q) {
#pragma clang fp contract(off)
    SiteOut<T> r;
    const cx<T> f = q.f;
    r.wx = cmul(q.ux, q.fxp);
    r.wy = cmul(q.uy, q.fyp);
    r.wz = cmul(q.uz, q.fzp);
    const cx<T> vx = cmulc(q.ux_m, q.fxm), vy = cmulc(q.uy_m, q.fym), vz = cmulc(q.uz_m, q.fzm);
    cx<T> lap;
    lap.re = fma_t(T(-6), f.re, ((r.wx.re + vx.re) + (r.wy.re + vy.re)) + (r.wz.re + vz.re));
    lap.im = fma_t(T(-6), f.im, ((r.wx.im + vx.im) + (r.wy.im + vy.im)) + (r.wz.im + vz.im));
    r.m2 = norm2(f);
    const T o2 = norm2(q.o);
    const T br = fma_t(c.lamh[sec], r.m2 - c.sig2[sec], -(c.kap * (o2 - c.sig2[1 - sec])));
    cx<T> F;
    F.re = fma_t(c.inv_h2, lap.re, -(br * f.re));
    F.im = fma_t(c.inv_h2, lap.im, -(br * f.im));
    if constexpr (COOL) {
        r.p1 = F;
    } else {
        r.p1.re = fma_t(c.cpi, q.p0.re, c.kpi * F.re);
        r.p1.im = fma_t(c.cpi, q.p0.im, c.kpi * F.im);
    }
    r.fn.re = fma_t(c.k, r.p1.re, f.re);
    r.fn.im = fma_t(c.k, r.p1.im, f.im);

    const T Mx = mag_force(c, q.sxy, q.sxy_my, q.sxz, q.sxz_mz);
    const T My = mag_force(c, q.sxy_mx, q.sxy, q.syz, q.syz_mz);
    const T Mz = mag_force(c, q.sxz_mx, q.sxz, q.syz_my, q.syz);
    const T Jx = current(c, sec, f, r.wx), Jy = current(c, sec, f, r.wy), Jz = current(c, sec, f, r.wz);
    if constexpr (COOL) {
        r.e1[0] = Mx + Jx;
        r.e1[1] = My + Jy;
        r.e1[2] = Mz + Jz;
    } else {
        r.e1[0] = e_kick(c, q.e0[0], Mx, Jx);
        r.e1[1] = e_kick(c, q.e0[1], My, Jy);
        r.e1[2] = e_kick(c, q.e0[2], Mz, Jz);
    }
#pragma unroll
    for (int i = 0; i < 3; i++) r.an[i] = fma_t(c.k, r.e1[i], q.a[i]);
    return r;
}

}  // namespace mts
