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

template <typename T, bool DIAG>
__global__ __launch_bounds__(BX *BY) void step_site_kernel(Geom g, Fields<T> in, Fields<T> out, Moms<T> mom,
                                                           StepCoef<T> c, Partials part) {
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

            // scalar kick (in place) and drift
            const cx<T> p0 = mom.pi[sec][q.s];
            cx<T> p1;
            p1.re = c.cpi * p0.re + c.kpi * F.re;
            p1.im = c.cpi * p0.im + c.kpi * F.im;
            mom.pi[sec][q.s] = p1;
            cx<T> fn;
            fn.re = f.re + c.k * p1.re;
            fn.im = f.im + c.k * p1.im;
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

            T *Ex = mom.E[sec][0], *Ey = mom.E[sec][1], *Ez = mom.E[sec][2];
            const T e0x = Ex[q.s], e0y = Ey[q.s], e0z = Ez[q.s];
            const T e1x = c.cE * e0x + c.kE * (Mx + Jx);
            const T e1y = c.cE * e0y + c.kE * (My + Jy);
            const T e1z = c.cE * e0z + c.kE * (Mz + Jz);
            Ex[q.s] = e1x;
            Ey[q.s] = e1y;
            Ez[q.s] = e1z;
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
        step_site_kernel<T, true><<<grid, block, 0, st>>>(g, in, out, mom, c, part);
    else
        step_site_kernel<T, false><<<grid, block, 0, st>>>(g, in, out, mom, c, part);
    return hipGetLastError();
}

// ------------------------------------------------------------ windings and Gauss

// chi = arg(conj(a) exp(-i h A) b) in (-pi, pi].  Near the branch cut
// (Re z < 0, |Im z| < 1e-4 |z|) a float link is recomputed in double so that
// the side of the cut, and hence the winding, matches an FP64 evaluation of
// the same float inputs.
template <typename T>
__device__ __forceinline__ T link_phase(cx<T> a, cx<T> b, T A, T h) {
    const cx<T> z = cmul(cmulc(a, phasor<T>(h * A)), b);
    T ang;
    if constexpr (sizeof(T) == 4) {
        if (z.re < 0.0f && fabsf(z.im) < 1e-4f * (fabsf(z.re) + fabsf(z.im))) {
            const cx<double> ad{a.re, a.im}, bd{b.re, b.im};
            const cx<double> zd = cmul(cmulc(ad, phasor<double>((double)h * (double)A)), bd);
            double ad_ang = atan2(zd.im, zd.re);
            if (ad_ang <= -Pi<double>::v) ad_ang = Pi<double>::v;
            return (float)ad_ang;
        }
    }
    ang = atan2_t(z.im, z.re);
    if (ang <= -Pi<T>::v) ang = Pi<T>::v;
    return ang;
}

template <typename T>
__global__ __launch_bounds__(BX *BY) void wind_gauss_kernel(Geom g, Fields<T> f, Moms<T> mom, T h, double g_p,
                                                            double g_q, uint8_t *wabs, uint32_t plane,
                                                            int8_t *signed_out, Partials part) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    double acc[6] = {0, 0, 0, 0, 0, 0};   // gauss_abs p,q; gauss_scale p,q; wind p,q
    if (x < g.nx && y < g.ny) {
        const Site q = site_of(g, x, y, z);
        // second neighbours for the links of the neighbouring sites
        const int xp = x + 1 == g.nx ? 0 : x + 1, yp = y + 1 == g.ny ? 0 : y + 1, zp = z + 1 == g.nz ? 0 : z + 1;
        const uint32_t xp_yp = xp + g.nx * yp + g.nxy * z;
        const uint32_t xp_zp = xp + g.nx * y + g.nxy * zp;
        const uint32_t yp_zp = x + g.nx * yp + g.nxy * zp;
        const T two_pi_inv = T(0.5) / Pi<T>::v;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            const cx<T> *P = f.phi[sec];
            const T *Ax = f.A[sec][0], *Ay = f.A[sec][1], *Az = f.A[sec][2];
            const cx<T> p0 = P[q.s], pxp = P[q.xp], pyp = P[q.yp], pzp = P[q.zp];
            const T ax = Ax[q.s], ay = Ay[q.s], az = Az[q.s];
            const T chx = link_phase(p0, pxp, ax, h);
            const T chy = link_phase(p0, pyp, ay, h);
            const T chz = link_phase(p0, pzp, az, h);
            const T chy_px = link_phase(pxp, P[xp_yp], Ay[q.xp], h);
            const T chz_px = link_phase(pxp, P[xp_zp], Az[q.xp], h);
            const T chx_py = link_phase(pyp, P[xp_yp], Ax[q.yp], h);
            const T chz_py = link_phase(pyp, P[yp_zp], Az[q.yp], h);
            const T chx_pz = link_phase(pzp, P[xp_zp], Ax[q.zp], h);
            const T chy_pz = link_phase(pzp, P[yp_zp], Ay[q.zp], h);
            const T txy = plaq(h, ax, Ay[q.xp], Ax[q.yp], ay);
            const T tyz = plaq(h, ay, Az[q.yp], Ay[q.zp], az);
            const T tzx = plaq(h, az, Ax[q.zp], Az[q.xp], ax);
            const int Wz = (int)rint_t(((((chx + chy_px) - chx_py) - chy) + txy) * two_pi_inv);
            const int Wx = (int)rint_t(((((chy + chz_py) - chy_pz) - chz) + tyz) * two_pi_inv);
            const int Wy = (int)rint_t(((((chz + chx_pz) - chz_px) - chx) + tzx) * two_pi_inv);
            if (signed_out) {
                auto cl = [](int w) { return (int8_t)(w > 127 ? 127 : (w < -127 ? -127 : w)); };
                signed_out[(size_t)(3 * sec + 0) * plane + q.s] = cl(Wx);
                signed_out[(size_t)(3 * sec + 1) * plane + q.s] = cl(Wy);
                signed_out[(size_t)(3 * sec + 2) * plane + q.s] = cl(Wz);
                continue;
            }
            const int aWx = abs(Wx), aWy = abs(Wy), aWz = abs(Wz);
            wabs[(size_t)sec * plane + q.s] =
                (uint8_t)(min(aWx, 3) | (min(aWy, 3) << 2) | (min(aWz, 3) << 4));
            acc[4 + sec] = (double)(aWx + aWy + aWz);

            // Gauss residual at n+1/2: div E^{n+1/2} - g Im[conj(phi^n) Pi^{n+1/2}]
            const T *Ex = mom.E[sec][0], *Ey = mom.E[sec][1], *Ez = mom.E[sec][2];
            const T div = (((Ex[q.s] - Ex[q.xm]) + (Ey[q.s] - Ey[q.ym])) + (Ez[q.s] - Ez[q.zm])) / h;
            const T gs = (T)(sec == 0 ? g_p : g_q);
            const T grho = gs * imc(p0, mom.pi[sec][q.s]);
            const T C = div - grho;
            acc[sec] = (double)fabs(C);
            acc[2 + sec] = (double)fabs(div) + (double)fabs(grho);
        }
    }
    if (!signed_out) {
        const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum_store<6, (BX * BY) / 64>(acc, part, SL_GAUSS_ABS_P, blk);
    }
}

template <typename T>
hipError_t launch_wind_gauss(const Geom &g, Fields<T> f, Moms<T> mom, T h, const double gcoef[2], uint8_t *wabs,
                             uint32_t plane, int8_t *signed_out, Partials part, hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    wind_gauss_kernel<T><<<grid, block, 0, st>>>(g, f, mom, h, gcoef[0], gcoef[1], wabs, plane, signed_out, part);
    return hipGetLastError();
}

// ------------------------------------------------------------ cells and overlap

__global__ __launch_bounds__(BX *BY) void cells_kernel(Geom g, const uint8_t *wabs, uint8_t *cells, uint32_t plane) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Site q = site_of(g, x, y, z);
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        const uint8_t *w = wabs + (size_t)sec * plane;
        const uint32_t w0 = w[q.s];
        const uint32_t n = (w0 & 3) + (w[q.xp] & 3) + ((w0 >> 2) & 3) + ((w[q.yp] >> 2) & 3) + ((w0 >> 4) & 3) +
                           ((w[q.zp] >> 4) & 3);
        cells[(size_t)sec * plane + q.s] = (uint8_t)n;
    }
}

hipError_t launch_cells(const Geom &g, const uint8_t *wabs, uint8_t *cells, uint32_t plane, hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    cells_kernel<<<grid, block, 0, st>>>(g, wabs, cells, plane);
    return hipGetLastError();
}

__global__ __launch_bounds__(BX *BY) void overlap_kernel(Geom g, const uint8_t *cells, uint32_t plane, int radius,
                                                         Partials part) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    double acc[2] = {0, 0};
    if (x < g.nx && y < g.ny) {
        const uint32_t s = x + g.nx * y + g.nxy * z;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            if (cells[(size_t)sec * plane + s] == 0) continue;
            const uint8_t *o = cells + (size_t)(1 - sec) * plane;
            bool hit = false;
            for (int dz = -radius; dz <= radius && !hit; dz++) {
                int zz = z + dz;
                zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
                for (int dy = -radius; dy <= radius && !hit; dy++) {
                    int yy = y + dy;
                    yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
                    for (int dx = -radius; dx <= radius && !hit; dx++) {
                        int xx = x + dx;
                        xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
                        hit = o[xx + g.nx * yy + g.nxy * zz] != 0;
                    }
                }
            }
            acc[sec] = hit ? 1.0 : 0.0;
        }
    }
    const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum_store<2, (BX * BY) / 64>(acc, part, SL_OV_P, blk);
}

hipError_t launch_overlap(const Geom &g, const uint8_t *cells, uint32_t plane, int radius, Partials part,
                          hipStream_t st) {
    dim3 block(BX, BY, 1);
    dim3 grid((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
    overlap_kernel<<<grid, block, 0, st>>>(g, cells, plane, radius, part);
    return hipGetLastError();
}

// ------------------------------------------------------------ final reduce

// One block per slot; thread t sums partials t, t+256, ... in order, then a
// fixed tree over the 256 threads.
__global__ __launch_bounds__(256) void reduce_kernel(Partials part, const uint32_t *nblk, double *rec) {
    __shared__ double red[256];
    const int slot = blockIdx.x;
    const uint32_t n = nblk[slot];
    const double *p = part.base + (size_t)slot * part.maxblk;
    double t = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += 256) t += p[i];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rec[slot] = red[0];
}

hipError_t launch_reduce(Partials part, const uint32_t *nblk_per_slot_dev, double *rec, hipStream_t st) {
    reduce_kernel<<<NSLOT, 256, 0, st>>>(part, nblk_per_slot_dev, rec);
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

// ------------------------------------------------------------ instantiations

template hipError_t launch_step<float>(const Geom &, Fields<float>, Fields<float>, Moms<float>,
                                       const StepCoef<float> &, bool, Partials, hipStream_t);
template hipError_t launch_step<double>(const Geom &, Fields<double>, Fields<double>, Moms<double>,
                                        const StepCoef<double> &, bool, Partials, hipStream_t);
template hipError_t launch_wind_gauss<float>(const Geom &, Fields<float>, Moms<float>, float, const double[2],
                                             uint8_t *, uint32_t, int8_t *, Partials, hipStream_t);
template hipError_t launch_wind_gauss<double>(const Geom &, Fields<double>, Moms<double>, double, const double[2],
                                              uint8_t *, uint32_t, int8_t *, Partials, hipStream_t);
template hipError_t launch_init<float>(const Geom &, Fields<float>, Moms<float>, uint64_t, double, double,
                                       hipStream_t);
template hipError_t launch_init<double>(const Geom &, Fields<double>, Moms<double>, uint64_t, double, double,
                                        hipStream_t);

}  // namespace mts
