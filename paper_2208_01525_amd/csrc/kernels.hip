// kernels.hip -- gfx950 kernels of the U(1)xU(1) multitension-string lattice
// update (Correia & Martins, arXiv:2208.01525, Sec. III) and its fused
// network diagnostics (Sec. III.A-B).
//
// Lattice operators (compact links, A carries the gauge coupling):
//   U_i(x)      = exp(-i h A_i(x))
//   D^-D^+ phi  = h^-2 sum_i [U_i(x) phi(x+i) - 2 phi(x) + conj(U_i(x-i)) phi(x-i)]
//   theta_ij(x) = h [A_i(x) + A_j(x+i) - A_i(x+j) - A_j(x)]
//   d_j^- F_ij -> h^-3 [sin theta_ij(x) - sin theta_ij(x-j)]
//   Im[phi* D_i^+ phi] = h^-1 Im[conj(phi(x)) U_i(x) phi(x+i)]
// One thread per site; neighbours come straight from global memory (the
// x-neighbours from the same cache lines, y/z-neighbours from L2).
#include "device.h"
#include "kernels.h"

namespace mts {

// ------------------------------------------------------------ per-site helpers

struct Site {
    uint32_t s, xm, xp, ym, yp, zm, zp;        // x +- 1 etc.
    uint32_t xp_ym, xm_yp, xp_zm, xm_zp, yp_zm, ym_zp;
};

__device__ __forceinline__ Site site_of(const Geom &g, int x, int y, int z) {
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z + 1 == g.nz ? 0 : z + 1;
    const uint32_t nx = g.nx, nxy = g.nxy;
    const uint32_t ry = nx * y, rym = nx * ym, ryp = nx * yp;
    const uint32_t rz = nxy * z, rzm = nxy * zm, rzp = nxy * zp;
    Site q;
    q.s = x + ry + rz;
    q.xm = xm + ry + rz;
    q.xp = xp + ry + rz;
    q.ym = x + rym + rz;
    q.yp = x + ryp + rz;
    q.zm = x + ry + rzm;
    q.zp = x + ry + rzp;
    q.xp_ym = xp + rym + rz;
    q.xm_yp = xm + ryp + rz;
    q.xp_zm = xp + ry + rzm;
    q.xm_zp = xm + ry + rzp;
    q.yp_zm = x + ryp + rzm;
    q.ym_zp = x + rym + rzp;
    return q;
}

constexpr int BX = 64, BY = 4;  // block of the per-site kernels: one x-row of 64 per wave

uint32_t site_blocks(const Geom &g) {
    return (uint32_t)((g.nx + BX - 1) / BX) * (uint32_t)((g.ny + BY - 1) / BY) * (uint32_t)g.nz;
}

// ------------------------------------------------------------ the update

// MODE 0: leapfrog step; 1: step with the integer-time sums; 2: one
// forward-Euler step of the diffusive cooling flow (fields move along their
// forces, momenta untouched; the host passes kappa = 0, a = 1, k = d eta).
template <typename T, int MODE>
__global__ __launch_bounds__(BX *BY) void step_site_kernel(Geom g, Fields<T> in, Fields<T> out, Moms<T> mom,
                                                           StepCoef<T> c, Partials part) {
    constexpr bool DIAG = MODE == 1, COOL = MODE == 2;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    const bool active = x < g.nx && y < g.ny;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    if (active) {
        const Site q = site_of(g, x, y, z);
        T Kd = 0, Gd = 0, Kg = 0, Bg = 0;        // diagnostic pieces, both sectors
        T mod2[2];

#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            const cx<T> *P = in.phi[sec];
            const cx<T> *O = in.phi[1 - sec];
            const T *Ax = in.A[sec][0], *Ay = in.A[sec][1], *Az = in.A[sec][2];

            const cx<T> f = P[q.s];
            const cx<T> fxp = P[q.xp], fxm = P[q.xm], fyp = P[q.yp], fym = P[q.ym], fzp = P[q.zp], fzm = P[q.zm];
            const cx<T> o = O[q.s];

            const T ax = Ax[q.s], ay = Ay[q.s], az = Az[q.s];
            const T ax_mx = Ax[q.xm], ay_my = Ay[q.ym], az_mz = Az[q.zm];

            // links and covariant hops
            const cx<T> ux = phasor<T>(c.h * ax), uy = phasor<T>(c.h * ay), uz = phasor<T>(c.h * az);
            const cx<T> ux_m = phasor<T>(c.h * ax_mx), uy_m = phasor<T>(c.h * ay_my), uz_m = phasor<T>(c.h * az_mz);
            const cx<T> wx = cmul(ux, fxp), wy = cmul(uy, fyp), wz = cmul(uz, fzp);   // U_i(x) phi(x+i)
            const cx<T> vx = cmulc(ux_m, fxm), vy = cmulc(uy_m, fym), vz = cmulc(uz_m, fzm);  // conj(U_i(x-i)) phi(x-i)

            // covariant Laplacian and potential force
            cx<T> lap;
            lap.re = (((wx.re + vx.re) + (wy.re + vy.re)) + (wz.re + vz.re)) - T(6) * f.re;
            lap.im = (((wx.im + vx.im) + (wy.im + vy.im)) + (wz.im + vz.im)) - T(6) * f.im;
            const T m2 = norm2(f), o2 = norm2(o);
            const T br = c.lamh[sec] * (m2 - c.sig2[sec]) - c.kap * (o2 - c.sig2[1 - sec]);
            cx<T> F;
            F.re = c.inv_h2 * lap.re - br * f.re;
            F.im = c.inv_h2 * lap.im - br * f.im;

            // scalar kick (in place) and drift; cooling moves phi along F
            cx<T> p0{T(0), T(0)}, p1{T(0), T(0)}, fn;
            if constexpr (COOL) {
                fn.re = f.re + c.k * F.re;
                fn.im = f.im + c.k * F.im;
            } else {
                p0 = mom.pi[sec][q.s];
                p1.re = c.cpi * p0.re + c.kpi * F.re;
                p1.im = c.cpi * p0.im + c.kpi * F.im;
                mom.pi[sec][q.s] = p1;
                fn.re = f.re + c.k * p1.re;
                fn.im = f.im + c.k * p1.im;
            }
            out.phi[sec][q.s] = fn;

            // plaquettes around the three links of x
            const T sxy = sin_t(plaq(c.h, ax, Ay[q.xp], Ax[q.yp], ay));
            const T sxy_my = sin_t(plaq(c.h, Ax[q.ym], Ay[q.xp_ym], ax, ay_my));
            const T sxy_mx = sin_t(plaq(c.h, ax_mx, ay, Ax[q.xm_yp], Ay[q.xm]));
            const T sxz = sin_t(plaq(c.h, ax, Az[q.xp], Ax[q.zp], az));
            const T sxz_mz = sin_t(plaq(c.h, Ax[q.zm], Az[q.xp_zm], ax, az_mz));
            const T sxz_mx = sin_t(plaq(c.h, ax_mx, az, Ax[q.xm_zp], Az[q.xm]));
            const T syz = sin_t(plaq(c.h, ay, Az[q.yp], Ay[q.zp], az));
            const T syz_mz = sin_t(plaq(c.h, Ay[q.zm], Az[q.yp_zm], ay, az_mz));
            const T syz_my = sin_t(plaq(c.h, ay_my, az, Ay[q.ym_zp], Az[q.ym]));

            // -sum_j d_j^- F_ij (compact) + current
            const T Mx = -c.inv_h3 * ((sxy - sxy_my) + (sxz - sxz_mz));
            const T My = -c.inv_h3 * ((sxy_mx - sxy) + (syz - syz_mz));
            const T Mz = -c.inv_h3 * ((sxz_mx - sxz) + (syz_my - syz));
            const T Jx = c.cur[sec] * imc(f, wx), Jy = c.cur[sec] * imc(f, wy), Jz = c.cur[sec] * imc(f, wz);

            T e0x = 0, e0y = 0, e0z = 0, e1x, e1y, e1z;
            if constexpr (COOL) {
                e1x = Mx + Jx;          // the links flow along their force
                e1y = My + Jy;
                e1z = Mz + Jz;
            } else {
                T *Ex = mom.E[sec][0], *Ey = mom.E[sec][1], *Ez = mom.E[sec][2];
                e0x = Ex[q.s];
                e0y = Ey[q.s];
                e0z = Ez[q.s];
                e1x = c.cE * e0x + c.kE * (Mx + Jx);
                e1y = c.cE * e0y + c.kE * (My + Jy);
                e1z = c.cE * e0z + c.kE * (Mz + Jz);
                Ex[q.s] = e1x;
                Ey[q.s] = e1y;
                Ez[q.s] = e1z;
            }
            out.A[sec][0][q.s] = ax + c.k * e1x;
            out.A[sec][1][q.s] = ay + c.k * e1y;
            out.A[sec][2][q.s] = az + c.k * e1z;

            if constexpr (DIAG) {
                cx<T> pb;                                  // (Pi^{n-1/2} + Pi^{n+1/2}) / 2
                pb.re = T(0.5) * (p0.re + p1.re);
                pb.im = T(0.5) * (p0.im + p1.im);
                Kd += norm2(pb);
                cx<T> dx_, dy_, dz_;                       // h D_i^+ phi
                dx_.re = wx.re - f.re; dx_.im = wx.im - f.im;
                dy_.re = wy.re - f.re; dy_.im = wy.im - f.im;
                dz_.re = wz.re - f.re; dz_.im = wz.im - f.im;
                Gd += c.inv_h2 * ((norm2(dx_) + norm2(dy_)) + norm2(dz_));
                const T ebx = T(0.5) * (e0x + e1x), eby = T(0.5) * (e0y + e1y), ebz = T(0.5) * (e0z + e1z);
                Kg += c.inv_2e2[sec] * ((ebx * ebx + eby * eby) + ebz * ebz);
                const T cxy = cos_t(plaq(c.h, ax, Ay[q.xp], Ax[q.yp], ay));
                const T cxz = cos_t(plaq(c.h, ax, Az[q.xp], Ax[q.zp], az));
                const T cyz = cos_t(plaq(c.h, ay, Az[q.yp], Ay[q.zp], az));
                Bg += c.inv_e2h4[sec] * (((T(1) - cxy) + (T(1) - cxz)) + (T(1) - cyz));
                mod2[sec] = m2;
            }
        }

        if constexpr (DIAG) {
            const T dp = mod2[0] - c.sig2[0], dq = mod2[1] - c.sig2[1];
            const T Vint = c.kap0 * dp * dq;
            const T V = (c.lam4[0] * dp * dp + c.lam4[1] * dq * dq) - Vint;
            const T eps = (Kd + Gd) + c.am2s * (Kg + Bg) + c.a2s * V;
            const T lag = (Kd - Gd) + c.am2s * (Kg - Bg) - c.a2s * V;
            const double K = Kd, G = Gd, L = lag, Vi = Vint;
            acc[0] = (double)eps;
            acc[1] = L;
            acc[2] = K * L;
            acc[3] = G * L;
            acc[4] = K * Vi;
            acc[5] = G * Vi;
        }
    }
    if constexpr (DIAG) {
        const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum_store<6, (BX * BY) / 64>(acc, part, SL_EPS, blk);
    }
}

template <typename T>
hipError_t launch_step(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, const StepCoef<T> &c, bool diag,
                       Partials part, hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    if (diag)
        step_site_kernel<T, 1><<<grid, block, 0, st>>>(g, in, out, mom, c, part);
    else
        step_site_kernel<T, 0><<<grid, block, 0, st>>>(g, in, out, mom, c, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cool(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, const StepCoef<T> &c, hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    step_site_kernel<T, 2><<<grid, block, 0, st>>>(g, in, out, mom, c, Partials{nullptr, 0});
    return hipGetLastError();
}

// ------------------------------------------------------------ initial conditions

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output `counter` of the
// stream started at `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(BX *BY) void init_kernel(Geom g, Fields<T> f, Moms<T> mom, uint64_t seed, double sig_p,
                                                      double sig_q) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t s = x + g.nx * y + g.nxy * z;
    const uint64_t S = (uint64_t)g.nxy * (uint64_t)g.nz;
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        const uint64_t r = splitmix64(seed, (uint64_t)sec * S + s);
        const double phase = 2.0 * Pi<double>::v * ((double)(r >> 11) * 0x1.0p-53);
        double sn, cs;
        sincos(phase, &sn, &cs);
        const double sig = sec == 0 ? sig_p : sig_q;
        f.phi[sec][s] = cx<T>{(T)(sig * cs), (T)(sig * sn)};
        mom.pi[sec][s] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 3; i++) {
            f.A[sec][i][s] = T(0);
            mom.E[sec][i][s] = T(0);
        }
    }
}

template <typename T>
hipError_t launch_init(const Geom &g, Fields<T> f, Moms<T> mom, uint64_t seed, double sig_p, double sig_q,
                       hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    init_kernel<T><<<grid, block, 0, st>>>(g, f, mom, seed, sig_p, sig_q);
    return hipGetLastError();
}

// ------------------------------------------------------------ spot reads

template <typename T>
__global__ void gather_kernel(Fields<T> f, Moms<T> mom, const uint64_t *sites, int n, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t s = sites[i];
    double *o = out + (size_t)i * 20;
    for (int sec = 0; sec < 2; sec++) {
        const cx<T> p = f.phi[sec][s], q = mom.pi[sec][s];
        o[2 * sec] = p.re;
        o[2 * sec + 1] = p.im;
        o[4 + 2 * sec] = q.re;
        o[5 + 2 * sec] = q.im;
        for (int k = 0; k < 3; k++) {
            o[8 + 3 * sec + k] = f.A[sec][k][s];
            o[14 + 3 * sec + k] = mom.E[sec][k][s];
        }
    }
}

template <typename T>
hipError_t launch_gather(Fields<T> f, Moms<T> mom, const uint64_t *sites, int n, double *out, hipStream_t st) {
    gather_kernel<T><<<(n + 255) / 256, 256, 0, st>>>(f, mom, sites, n, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ instantiations

template hipError_t launch_step<float>(const Geom &, Fields<float>, Fields<float>, Moms<float>,
                                       const StepCoef<float> &, bool, Partials, hipStream_t);
template hipError_t launch_step<double>(const Geom &, Fields<double>, Fields<double>, Moms<double>,
                                        const StepCoef<double> &, bool, Partials, hipStream_t);
template hipError_t launch_cool<float>(const Geom &, Fields<float>, Fields<float>, Moms<float>,
                                       const StepCoef<float> &, hipStream_t);
template hipError_t launch_cool<double>(const Geom &, Fields<double>, Fields<double>, Moms<double>,
                                        const StepCoef<double> &, hipStream_t);
template hipError_t launch_gather<float>(Fields<float>, Moms<float>, const uint64_t *, int, double *, hipStream_t);
template hipError_t launch_gather<double>(Fields<double>, Moms<double>, const uint64_t *, int, double *, hipStream_t);
template hipError_t launch_init<float>(const Geom &, Fields<float>, Moms<float>, uint64_t, double, double,
                                       hipStream_t);
template hipError_t launch_init<double>(const Geom &, Fields<double>, Moms<double>, uint64_t, double, double,
                                        hipStream_t);

}  // namespace mts
