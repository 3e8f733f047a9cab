// diag.hip -- post-step diagnostic kernels of the U(1)xU(1) lattice update
// (Correia & Martins, arXiv:2208.01525, Sec. III.A-B and the Gauss law of
// Sec. II): plaquette windings, the Gauss residual, cell values, the
// fast-method bound-state overlap, and the final fixed-order reduction.
//
// Windings.  With alpha(x) = arg phi(x), the covariant link phase is
//   chi_mu(x) = arg(conj(phi(x)) U_mu(x) phi(x+mu)) = wrap(alpha(x+mu) - alpha(x) - h A_mu(x)),
// wrap into (-pi, pi], so one atan2 per site replaces a sincos and an atan2
// per link (guarded near the branch cut: link_chi in device.h).  The winding
// through the face normal to rho, (mu, nu, rho) cyclic, is
//   W_rho(x) = rint([chi_mu(x) + chi_nu(x+mu) - chi_mu(x+nu) - chi_nu(x) + theta_mu,nu(x)] / 2 pi).
//
// Overlap.  When nx is a multiple of 64, the cell kernel also packs "cell
// pierced" into 64-bit words along x with a wave ballot; a cell of one sector
// counts when the 3x3x3 dilation of the other sector's mask covers it, which
// is shifts and ORs of 27 words and a popcount per 64 cells.  Other boxes use
// a direct scan of the 27 neighbouring cell bytes.
#include "device.h"
#include "kernels.h"
#include "post.h"

namespace mts {

namespace {

constexpr int DX = 64, DY = 4, DZ = 4;   // wind/Gauss blocks: 64 x 4 columns, DZ planes per thread

}  // namespace

// ---------------------------------------------------------------- phases

template <typename T>
__global__ __launch_bounds__(256) void phase_kernel(Fields<T> f, T *alpha, uint32_t plane, uint32_t S) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        const cx<T> p = f.phi[sec][s];
        alpha[(size_t)sec * plane + s] = phase_of(p);
    }
}

template <typename T>
hipError_t launch_phase(const Geom &g, Fields<T> f, T *alpha, uint32_t plane, hipStream_t st) {
    const uint32_t S = g.nxy * (uint32_t)g.nz;
    phase_kernel<T><<<(S + 255) / 256, 256, 0, st>>>(f, alpha, plane, S);
    return hipGetLastError();
}

// ---------------------------------------------------------------- windings and Gauss

uint32_t wind_blocks(const Geom &g) {
    return (uint32_t)((g.nx + DX - 1) / DX) * (uint32_t)((g.ny + DY - 1) / DY) * (uint32_t)((g.nz + DZ - 1) / DZ);
}

template <typename T>
__global__ __launch_bounds__(DX *DY) void wind_gauss_kernel(Geom g, Fields<T> f, Moms<T> mom, const T *alpha, T h,
                                                            T inv_h, double g_p, double g_q, uint8_t *wabs,
                                                            uint32_t plane, int8_t *signed_out, Partials part) {
    const int x = blockIdx.x * DX + threadIdx.x;
    const int y = blockIdx.y * DY + threadIdx.y;
    double acc[6] = {0, 0, 0, 0, 0, 0};   // gauss_abs p,q; gauss_scale p,q; wind p,q
    if (x < g.nx && y < g.ny) {
        const int xp = wrap1(x + 1, g.nx), xm = wrap1(x - 1, g.nx);
        const int yp = wrap1(y + 1, g.ny), ym = wrap1(y - 1, g.ny);
        const uint32_t nx = g.nx, nxy = g.nxy;
        const int zb = blockIdx.z * DZ, z1 = min(zb + DZ, g.nz);
        // Values of plane z+1 that plane z reads are those plane z+1 reads at
        // its own site and its x and y neighbours: they are carried over in
        // registers (phases, A_x, A_y) instead of being loaded again, and so
        // is E_z of plane z for the divergence at plane z+1.
        T c_a0[2], c_ax[2], c_ay[2], c_Ax[2], c_Ay[2], c_Ez[2];
        {
            const uint32_t s = x + nx * y + nxy * zb;
            const uint32_t s_x = xp + nx * y + nxy * zb, s_y = x + nx * yp + nxy * zb;
            const uint32_t s_mz = x + nx * y + nxy * wrap1(zb - 1, g.nz);
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const T *al = alpha + (size_t)sec * plane;
                c_a0[sec] = al[s];
                c_ax[sec] = al[s_x];
                c_ay[sec] = al[s_y];
                c_Ax[sec] = f.A[sec][0][s];
                c_Ay[sec] = f.A[sec][1][s];
                c_Ez[sec] = signed_out ? T(0) : mom.E[sec][2][s_mz];
            }
        }
        for (int z = zb; z < z1; z++) {
            const int zp = wrap1(z + 1, g.nz);
            const uint32_t s = x + nx * y + nxy * z;
            const uint32_t s_x = xp + nx * y + nxy * z, s_y = x + nx * yp + nxy * z, s_z = x + nx * y + nxy * zp;
            const uint32_t s_xy = xp + nx * yp + nxy * z, s_xz = xp + nx * y + nxy * zp, s_yz = x + nx * yp + nxy * zp;
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const T *al = alpha + (size_t)sec * plane;
                const cx<T> *P = f.phi[sec];
                const T *Ax = f.A[sec][0], *Ay = f.A[sec][1], *Az = f.A[sec][2];
                const T a0 = c_a0[sec], ax = c_ax[sec], ay = c_ay[sec], az = al[s_z];
                const T axy = al[s_xy], axz = al[s_xz], ayz = al[s_yz];
                const T Ax0 = c_Ax[sec], Ay0 = c_Ay[sec], Az0 = Az[s];
                const T Ax_z = Ax[s_z], Ay_z = Ay[s_z];
                c_a0[sec] = az;
                c_ax[sec] = axz;
                c_ay[sec] = ayz;
                c_Ax[sec] = Ax_z;
                c_Ay[sec] = Ay_z;
                int Wx, Wy, Wz;
                face_windings(h, P, a0, ax, ay, az, axy, axz, ayz, Ax0, Ay0, Az0, Ay[s_x], Az[s_x], Ax[s_y], Az[s_y],
                              Ax_z, Ay_z, s, s_x, s_y, s_z, s_xy, s_xz, s_yz, Wx, Wy, Wz);
                if (signed_out) {
                    auto cl = [](int w) { return (int8_t)(w > 127 ? 127 : (w < -127 ? -127 : w)); };
                    signed_out[(size_t)(3 * sec + 0) * plane + s] = cl(Wx);
                    signed_out[(size_t)(3 * sec + 1) * plane + s] = cl(Wy);
                    signed_out[(size_t)(3 * sec + 2) * plane + s] = cl(Wz);
                    continue;
                }
                wabs[(size_t)sec * plane + s] = pack_wabs(Wx, Wy, Wz);
                acc[4 + sec] += (double)(abs(Wx) + abs(Wy) + abs(Wz));

                // Gauss residual at n+1/2: div E^{n+1/2} - g Im[conj(phi^n) Pi^{n+1/2}]
                const T *Ex = mom.E[sec][0], *Ey = mom.E[sec][1], *Ez = mom.E[sec][2];
                const uint32_t s_mx = xm + nx * y + nxy * z, s_my = x + nx * ym + nxy * z;
                const T ez0 = Ez[s], ezm = c_Ez[sec];
                c_Ez[sec] = ez0;
                const T div = gauss_div(Ex[s], Ex[s_mx], Ey[s], Ey[s_my], ez0, ezm, inv_h);
                const T gs = (T)(sec == 0 ? g_p : g_q);
                gauss_accumulate(div, gauss_charge(gs, P[s], mom.pi[sec][s]), acc[sec], acc[2 + sec]);
            }
        }
    }
    if (!signed_out) {
        const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum_store<6, (DX * DY) / 64>(acc, part, SL_GAUSS_ABS_P, blk);
    }
}

template <typename T>
hipError_t launch_wind_gauss(const Geom &g, Fields<T> f, Moms<T> mom, const T *alpha, T h, T inv_h,
                             const double gcoef[2], uint8_t *wabs, uint32_t plane, int8_t *signed_out, Partials part,
                             hipStream_t st) {
    dim3 block(DX, DY, 1);
    dim3 grid((g.nx + DX - 1) / DX, (g.ny + DY - 1) / DY, (g.nz + DZ - 1) / DZ);
    wind_gauss_kernel<T><<<grid, block, 0, st>>>(g, f, mom, alpha, h, inv_h, gcoef[0], gcoef[1], wabs, plane,
                                                 signed_out, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------- windings and Gauss, tiled
//
// The windings and Gauss residual of a diagnostic step that is not fused
// (FP64, whose update tile has no registers left to do it in place; FP32
// with fusion off, on the per-site kernel, or where no second momentum copy
// fits) in one z-marching pass over 64 x WG_TY tiles with a one-site halo,
// as the fused FP32 diagnostic tile forms them: each site's phase alpha of
// plane z+1 and the new E_x, E_y of plane z go through LDS; each link's wrap
// count is formed once and packed with its site's others; the winding
// through a face is minus the oriented sum of its four links' counts; a
// flagged link (guard, or a count beyond the packed field) marks the site
// WABS_FIX for the FP64 fix-up passes.  It reads phi, A, E and Pi once per
// site (the halo rows from L2), each plane's loads issued one plane ahead so
// that they are in flight across the previous plane's barriers.
//
// The Gauss residual is summed in FP64 from the per-site terms of the
// fields' own precision, as in the fused tile.
//
// For FP32 fields the phases and wrap counts are the fused tile's (the FP32
// guard).  For FP64 fields the phases are FP32 (atan2_fast of the FP64 phi,
// both components first scaled by one power of two, which is exact), the
// wrap decision FP64:
// v = (alpha_b - alpha_a) - h A in double from the widened phases.  Each
// phase is within 5e-7 rad of the FP64 one (4e-7 from atan2_fast, 6e-8
// from rounding the scaled components), so v is within about 1e-6 of its
// FP64 value, and a link with |chi| <= pi - MIXED_CUT has the same count as
// in FP64; every other link, and every link with a zero, NaN or infinite
// phi at an end, is flagged and its faces evaluated in FP64 by the fix-up.
// The windings are therefore those of the FP64 evaluation bit for bit.

namespace {

constexpr int WG_TY = 8;    // interior rows of a tile (WG_TY + 3 waves: rows, two halo rows, halo columns)
constexpr int WG_TZ = 32;   // planes per tile
constexpr int WG_LW = 66;   // LDS row width: 64 + the -x and +x halo columns
constexpr double MIXED_CUT = 1e-4;   // rad kept from the branch cut by FP32 phases

__device__ __forceinline__ int wrapn(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// FP32 phase of an FP64 phi; NaN for phi = 0 or a non-finite component.
__device__ __forceinline__ float phase_f32(cx<double> p) {
    const double mx = fmax(fabs(p.re), fabs(p.im));
    if (!(mx > 0.0 && mx <= 1.7976931348623157e308)) return __builtin_nanf("");
    int e;
    (void)frexp(mx, &e);
    return atan2_fast((float)ldexp(p.im, -e), (float)ldexp(p.re, -e));
}

// Wrap count of a link from FP32 phases and the FP64 h A (see above); a
// count beyond the 9-bit field is left to the fix-up as well.
__device__ __forceinline__ int link_wrap_mixed(float aa, float ab, double hA, bool &flag) {
#pragma clang fp contract(off)
    const double v = ((double)ab - (double)aa) - hA;
    const double n = rint(v * (0.5 / Pi<double>::v));
    const double chi = v - (2.0 * Pi<double>::v) * n;
    flag = !(fabs(chi) <= Pi<double>::v - MIXED_CUT && fabs(hA) <= Guard<double>::big && fabs(n) <= 255.0);
    return flag ? 0 : (int)n;
}

// The pass's phase and wrap count per precision: FP64 fields as above; FP32
// fields exactly as the fused FP32 tile forms them (atan2_fast, the FP32
// guard, whose |h A| bound keeps every unflagged count inside the field).
__device__ __forceinline__ float tile_phase(cx<double> p) { return phase_f32(p); }
__device__ __forceinline__ float tile_phase(cx<float> p) { return phase_of(p); }
__device__ __forceinline__ int tile_wrap(float aa, float ab, double hA, bool &flag) {
    return link_wrap_mixed(aa, ab, hA, flag);
}
__device__ __forceinline__ int tile_wrap(float aa, float ab, float hA, bool &flag) {
    return link_wrap(aa, ab, hA, flag);
}

}  // namespace

uint32_t wind_tile_blocks(const Geom &g) {
    return (uint32_t)((g.nx + 63) / 64) * (uint32_t)((g.ny + WG_TY - 1) / WG_TY) *
           (uint32_t)((g.nz + WG_TZ - 1) / WG_TZ);
}

// FP32: two workgroups per CU (at most 80 VGPRs); FP64 keeps its 3 waves per SIMD
template <typename T>
constexpr int wind_tile_waves() {
    return sizeof(T) == 4 ? 6 : 3;
}

template <typename T>
__global__ __launch_bounds__(64 * (WG_TY + 3)) __attribute__((amdgpu_waves_per_eu(wind_tile_waves<T>())))
void wind_gauss_tile_kernel(Geom g, Fields<T> f, Moms<T> mom, T h,
                                                                            T inv_h, double g_p, double g_q,
                                                                            uint8_t *wabs, uint32_t plane,
                                                                            Partials part) {
    constexpr int TY = WG_TY, R = TY + 2, LW = WG_LW;
    // two buffers by plane parity, so that a plane's stores never meet the
    // previous plane's loads and the plane ends without a barrier
    __shared__ float s_al[2][2][R * LW];                 // alpha of plane z+1
    __shared__ T s_ex[2][2][R * LW], s_ey[2][2][R * LW]; // E_x, E_y (n + 1/2) of plane z
    __shared__ int s_w[2][2][R * LW];                    // packed wrap counts of plane z
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + WG_TZ - 1) / WG_TZ;
    const uint32_t t = xcd_order(blockIdx.x, (uint32_t)(ntx * nty * ntz));
    const int X0 = (int)(t % ntx) * 64, Y0 = (int)((t / ntx) % nty) * TY, Z0 = (int)(t / (ntx * nty)) * WG_TZ;

    // which site of the tile this thread holds (as the update tile does)
    const int lx = threadIdx.x, w = threadIdx.y;
    int row, col;
    bool owner = true;
    if (w < TY) {
        row = w + 1;
        col = lx + 1;
    } else if (w == TY) {
        row = 0;
        col = lx + 1;
    } else if (w == TY + 1) {
        row = R - 1;
        col = lx + 1;
    } else if (lx < R) {
        row = lx;
        col = 0;
    } else if (lx < 2 * R) {
        row = lx - R;
        col = LW - 1;
    } else {
        row = 0;
        col = 0;
        owner = false;
    }
    const int gx = X0 - 1 + col, gy = Y0 - 1 + row;
    const int x = wrapn(gx, g.nx), y = wrapn(gy, g.ny);
    const bool interior = w < TY && gx < g.nx && gy < g.ny;
    const bool need_ex = owner && (interior || (col == 0 && row >= 1 && row <= TY));   // E_x at x - 1
    const bool need_ey = owner && (interior || (row == 0 && col >= 1 && col <= LW - 2)); // E_y at y - 1
    // the faces read phases and wrap counts at the site and at +x and +y
    // only: the row y0 - 1 and the column x0 - 1 form neither
    const bool wraps = owner && row > 0 && col > 0;
    const uint32_t colidx = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const int li = row * LW + col;
    const int lxp = row * LW + min(col + 1, LW - 1), lyp = min(row + 1, R - 1) * LW + col;
    const int lxm = row * LW + max(col - 1, 0), lym = max(row - 1, 0) * LW + col;
    const int zbeg = Z0, zend = min(Z0 + WG_TZ, g.nz);
    const T gs[2] = {(T)g_p, (T)g_q};

    cx<T> cf[2];    // phi of plane z
    float alc[2];   // its phases
    T caz[2], ezp[2] = {T(0), T(0)};
    int wxy[2] = {0, 0};
    // loaded one plane ahead: phi and A of plane z+1, E and Pi of plane z
    cx<T> pf[2], ppi[2];
    T pax[2], pay[2], paz[2], pex[2], pey[2], pez[2];
    {
        const uint32_t s = colidx + g.nxy * (uint32_t)wrapn(zbeg - 1, g.nz);
        const uint32_t sn = colidx + g.nxy * (uint32_t)zbeg;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            cf[sec] = pf[sec] = cx<T>{T(0), T(0)};
            alc[sec] = 0.f;
            caz[sec] = pax[sec] = pay[sec] = paz[sec] = T(0);
            if (wraps) {   // phi and A only where wrap counts are formed (interior sites among them)
                cf[sec] = f.phi[sec][s];
                alc[sec] = tile_phase(cf[sec]);
                caz[sec] = f.A[sec][2][s];
                pf[sec] = f.phi[sec][sn];
                pax[sec] = f.A[sec][0][sn];
                pay[sec] = f.A[sec][1][sn];
                paz[sec] = f.A[sec][2][sn];
            }
            if (interior) ezp[sec] = mom.E[sec][2][s];
            pex[sec] = pey[sec] = pez[sec] = T(0);
            ppi[sec] = cx<T>{T(0), T(0)};
        }
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};   // gauss |C| p, q; scale p, q; wind p, q
    for (int z = zbeg - 1; z < zend; z++) {
        const bool upd = interior && z >= zbeg;
        const int pb = (z - zbeg + 1) & 1;   // this plane's LDS buffers
        const uint32_t s = colidx + g.nxy * (uint32_t)wrapn(z, g.nz);
        cx<T> nf[2], pic[2];
        T nax[2], nay[2], naz[2], exc[2], eyc[2], ezc[2];
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            nf[sec] = pf[sec];
            nax[sec] = pax[sec];
            nay[sec] = pay[sec];
            naz[sec] = paz[sec];
            exc[sec] = pex[sec];
            eyc[sec] = pey[sec];
            ezc[sec] = pez[sec];
            pic[sec] = ppi[sec];
        }
        if (z + 1 < zend) {   // the next plane's loads (z+1 < nz; z+2 wraps at the box's end)
            const uint32_t s1 = colidx + g.nxy * (uint32_t)(z + 1);
            const uint32_t s2 = colidx + g.nxy * (uint32_t)wrapn(z + 2, g.nz);
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                if (wraps) {
                    pf[sec] = f.phi[sec][s2];
                    pax[sec] = f.A[sec][0][s2];
                    pay[sec] = f.A[sec][1][s2];
                    paz[sec] = f.A[sec][2][s2];
                }
                if (need_ex) pex[sec] = mom.E[sec][0][s1];
                if (need_ey) pey[sec] = mom.E[sec][1][s1];
                if (interior) {
                    pez[sec] = mom.E[sec][2][s1];
                    ppi[sec] = mom.pi[sec][s1];
                }
            }
        }
        float aln[2] = {0.f, 0.f};
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            if (wraps) {
                aln[sec] = tile_phase(nf[sec]);
                s_al[pb][sec][li] = aln[sec];
            }
            if (z >= zbeg) {
                if (need_ex) s_ex[pb][sec][li] = exc[sec];
                if (need_ey) s_ey[pb][sec][li] = eyc[sec];
            }
        }
        __syncthreads();
        // wrap counts of the x and y links of plane z+1 and of the z link of
        // plane z (garbage where the neighbour lies outside the tile: no face
        // reads those); the word of plane z staged
        int wnext[2] = {0, 0}, wown[2] = {0, 0};
        if (wraps) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                bool fx, fy, fz;
                const int nx_ = tile_wrap(aln[sec], s_al[pb][sec][lxp], link_angle(h, nax[sec]), fx);
                const int ny_ = tile_wrap(aln[sec], s_al[pb][sec][lyp], link_angle(h, nay[sec]), fy);
                const int nz_ = tile_wrap(alc[sec], aln[sec], link_angle(h, caz[sec]), fz);
                wnext[sec] = wrap_word(nx_, ny_, 0, fx, fy, false);
                wown[sec] = wxy[sec] | wrap_word(0, 0, nz_, false, false, fz);
                s_w[pb][sec][li] = wown[sec];
            }
        }
        __syncthreads();
        if (upd) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                // windings through the three faces at the site (lower corner x)
                const int o = wown[sec], xp = s_w[pb][sec][lxp], yp = s_w[pb][sec][lyp], zp = wnext[sec];
                const int Wz = -(((wrap_n<0>(o) + wrap_n<1>(xp)) - wrap_n<0>(yp)) - wrap_n<1>(o));
                const int Wx = -(((wrap_n<1>(o) + wrap_n<2>(yp)) - wrap_n<1>(zp)) - wrap_n<2>(o));
                const int Wy = -(((wrap_n<2>(o) + wrap_n<0>(zp)) - wrap_n<2>(xp)) - wrap_n<0>(o));
                const int flagged = (o & WRAP_F_XYZ) | (xp & WRAP_F_YZ) | (yp & WRAP_F_XZ) | (zp & WRAP_F_XY);
                uint8_t byte = WABS_FIX;
                if (!flagged) {
                    byte = pack_wabs(Wx, Wy, Wz);
                    acc[4 + sec] += (double)(abs(Wx) + abs(Wy) + abs(Wz));
                }
                wabs[(size_t)sec * plane + s] = byte;
                // Gauss residual at n + 1/2: div E^{n+1/2} - g Im[conj(phi^n) Pi^{n+1/2}]
                const T div = gauss_div(s_ex[pb][sec][li], s_ex[pb][sec][lxm], s_ey[pb][sec][li],
                                        s_ey[pb][sec][lym], ezc[sec], ezp[sec], inv_h);
                gauss_accumulate(div, gauss_charge(gs[sec], cf[sec], pic[sec]), acc[sec], acc[2 + sec]);
                ezp[sec] = ezc[sec];
            }
        }
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            cf[sec] = nf[sec];
            alc[sec] = aln[sec];
            caz[sec] = naz[sec];
            wxy[sec] = wnext[sec];
        }
    }
    block_sum_store<6, TY + 3>(acc, part, SL_GAUSS_ABS_P, blockIdx.x);
}

template <typename T>
hipError_t launch_wind_gauss_tile(const Geom &g, Fields<T> f, Moms<T> mom, T h, T inv_h, const double gcoef[2],
                                  uint8_t *wabs, uint32_t plane, Partials part, hipStream_t st) {
    wind_gauss_tile_kernel<T><<<wind_tile_blocks(g), dim3(64, WG_TY + 3, 1), 0, st>>>(
        g, f, mom, h, inv_h, gcoef[0], gcoef[1], wabs, plane, part);
    return hipGetLastError();
}

template hipError_t launch_wind_gauss_tile<float>(const Geom &, Fields<float>, Moms<float>, float, float,
                                                  const double[2], uint8_t *, uint32_t, Partials, hipStream_t);
template hipError_t launch_wind_gauss_tile<double>(const Geom &, Fields<double>, Moms<double>, double, double,
                                                   const double[2], uint8_t *, uint32_t, Partials, hipStream_t);

// ---------------------------------------------------------------- fix-up of the fused windings

uint32_t wind_fix_scan_blocks(const Geom &g) { return fix_blocks_of(g.nxy * (uint32_t)g.nz); }
uint32_t wind_fix_blocks(const Geom &g) { return wind_fix_scan_blocks(g) + FIX_PROC_BLOCKS; }

// The fused diagnostic step marks (WABS_FIX) the sites whose windings used a
// link the guard sends to FP64; here each marked site's three faces are
// evaluated as the post-step kernel does, its byte rewritten and its sum |W|
// added to the SL_FIX_P / SL_FIX_Q partials (the fused kernel counted nothing
// for it): a scan that lists the marked sites (16 per thread and pass, one
// 16-byte load per sector; the sector's byte plane is padded to a multiple
// of 64 sites), then a pass that evaluates the list with every lane busy.

template <typename T>
__global__ __launch_bounds__(256) void wind_fix_scan_kernel(Geom g, Fields<T> f, T h, uint8_t *wabs, uint32_t plane,
                                                            Partials part, uint32_t *list) {
    fix_scan_block(g, f, h, wabs, plane, part, blockIdx.x, gridDim.x, threadIdx.x, list);
}

template <typename T>
__global__ __launch_bounds__(256) void wind_fix_proc_kernel(Geom g, Fields<T> f, T h, uint8_t *wabs, uint32_t plane,
                                                            Partials part, const uint32_t *list, uint32_t nscan) {
    fix_proc_block(g, f, h, wabs, plane, part, nscan, nscan, blockIdx.x, gridDim.x, threadIdx.x, list);
}

template <typename T>
hipError_t launch_wind_fix(const Geom &g, Fields<T> f, T h, uint8_t *wabs, uint32_t plane, Partials part,
                           uint32_t *list, hipStream_t st) {
    const uint32_t nscan = wind_fix_scan_blocks(g);
    wind_fix_scan_kernel<T><<<nscan, 256, 0, st>>>(g, f, h, wabs, plane, part, list);
    wind_fix_proc_kernel<T><<<FIX_PROC_BLOCKS, 256, 0, st>>>(g, f, h, wabs, plane, part, list, nscan);
    return hipGetLastError();
}

template hipError_t launch_wind_fix<float>(const Geom &, Fields<float>, float, uint8_t *, uint32_t, Partials,
                                           uint32_t *, hipStream_t);
template hipError_t launch_wind_fix<double>(const Geom &, Fields<double>, double, uint8_t *, uint32_t, Partials,
                                            uint32_t *, hipStream_t);

// ---------------------------------------------------------------- cells

bool overlap_uses_bits(const Geom &g) { return g.nx % 64 == 0; }

uint32_t overlap_words(const Geom &g) { return (uint32_t)(g.nx / 64) * (uint32_t)g.ny * (uint32_t)g.nz; }

// Cell value = sum of |W| over the six faces of the cell [x, x+1]^3; with
// `bits`, also the 64-cell occupancy words of each sector.  A block holds
// 64 x 4 columns and walks CZ planes, carrying the packed |W| byte of the
// next plane (the upper z face) over to the following iteration.  Blocks
// are dealt to the XCDs in contiguous runs (x fastest, then y, then z), so
// the neighbouring column and row bytes a block reads come from its own
// XCD's L2 (512^3: 344 against 402 us, a third of the fetched bytes).  The
// wind/Gauss kernel keeps the hardware's round-robin order: the same
// remapping made it slower (2.89 against 2.77 ms) although it fetched 11 %
// less.
__global__ __launch_bounds__(256) void cells_kernel(Geom g, const uint8_t *wabs, uint8_t *cells, uint64_t *bits,
                                                    uint32_t plane, uint32_t nwords) {
    const uint32_t blk = xcd_order(blockIdx.x, gridDim.x);
    if (cells_by_words(g)) cells4_block(g, wabs, cells, bits, plane, nwords, blk, threadIdx.x, threadIdx.y);
    else cells_block(g, wabs, cells, bits, plane, nwords, blk, threadIdx.x, threadIdx.y);
}

hipError_t launch_cells(const Geom &g, const uint8_t *wabs, uint8_t *cells, uint64_t *bits, uint32_t plane,
                        hipStream_t st) {
    dim3 block(64, 4, 1);
    cells_kernel<<<cells_blocks(g), block, 0, st>>>(g, wabs, cells, overlap_uses_bits(g) ? bits : nullptr, plane,
                                         overlap_words(g));
    return hipGetLastError();
}

// ---------------------------------------------------------------- overlap

uint32_t overlap_blocks(const Geom &g) {
    if (overlap_uses_bits(g)) return (overlap_words(g) + 255) / 256;
    return (uint32_t)((g.nx + 63) / 64) * (uint32_t)((g.ny + 3) / 4) * (uint32_t)g.nz;
}

__global__ __launch_bounds__(256) void overlap_bits_kernel(Geom g, const uint64_t *bits, uint32_t nwords, int radius,
                                                           Partials part) {
    overlap_bits_block(g, bits, nwords, radius, part, blockIdx.x, threadIdx.x);
}

__global__ __launch_bounds__(256) void overlap_bytes_kernel(Geom g, const uint8_t *cells, uint32_t plane, int radius,
                                                            Partials part) {
    overlap_bytes_block(g, cells, plane, radius, part, blockIdx.x, threadIdx.x & 63, threadIdx.x >> 6);
}

hipError_t launch_overlap(const Geom &g, const uint8_t *cells, const uint64_t *bits, uint32_t plane, int radius,
                          Partials part, hipStream_t st) {
    if (overlap_uses_bits(g)) {
        const uint32_t nw = overlap_words(g);
        overlap_bits_kernel<<<(nw + 255) / 256, 256, 0, st>>>(g, bits, nw, radius, part);
    } else {
        overlap_bytes_kernel<<<overlap_blocks(g), 256, 0, st>>>(g, cells, plane, radius, part);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- final reduce

// One block per slot; thread t sums partials t, t + 1024, ... in order (four
// independent running sums combined in a fixed order), then a fixed tree.
__global__ __launch_bounds__(1024) void reduce_kernel(Partials part, const uint32_t *nblk, double *rec) {
    reduce_lanes<1024>(part, nblk, rec, blockIdx.x);
}

hipError_t launch_reduce(Partials part, const uint32_t *nblk_per_slot_dev, double *rec, hipStream_t st) {
    reduce_kernel<<<NSLOT, 1024, 0, st>>>(part, nblk_per_slot_dev, rec);
    return hipGetLastError();
}

// ---------------------------------------------------------------- ensembles

// the last box whose first block (member `first`) is <= t
template <typename B>
__device__ __forceinline__ int box_of(const B *boxes, int nbox, uint32_t t, uint32_t B::*first) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].*first <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ Fields<T> fields_global(const Fields<T> &f) {
    Fields<T> r;
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        r.phi[sec] = as_global(f.phi[sec]);
#pragma unroll
        for (int i = 0; i < 3; i++) r.A[sec][i] = as_global(f.A[sec][i]);
    }
    return r;
}

__device__ __forceinline__ Partials part_global(Partials p) {
    p.base = as_global(p.base);
    return p;
}

template <typename T>
__global__ __launch_bounds__(256) void fix_scan_batch_kernel(const BatchPost<T> *boxes, int nbox, int parity) {
    const int k = box_of(boxes, nbox, blockIdx.x, &BatchPost<T>::blk_fix);
    const BatchPost<T> &b = boxes[k];
    fix_scan_block(b.g, fields_global(b.f[parity]), b.h, as_global(b.wabs), b.plane, part_global(b.part),
                   blockIdx.x - b.blk_fix, fix_blocks_of(b.g.nxy * (uint32_t)b.g.nz), threadIdx.x,
                   as_global(b.fixlist));
}

// FIX_PROC_BLOCKS blocks per box, box-major
template <typename T>
__global__ __launch_bounds__(256) void fix_proc_batch_kernel(const BatchPost<T> *boxes, int parity) {
    const BatchPost<T> &b = boxes[blockIdx.x / FIX_PROC_BLOCKS];
    const uint32_t nscan = fix_blocks_of(b.g.nxy * (uint32_t)b.g.nz);
    fix_proc_block(b.g, fields_global(b.f[parity]), b.h, as_global(b.wabs), b.plane, part_global(b.part), nscan,
                   nscan, blockIdx.x % FIX_PROC_BLOCKS, FIX_PROC_BLOCKS, threadIdx.x, as_global(b.fixlist));
}

template <typename T>
__global__ __launch_bounds__(256) void cells_batch_kernel(const BatchPost<T> *boxes, int nbox, uint32_t total) {
    const uint32_t t = xcd_order(blockIdx.x, total);
    const int k = box_of(boxes, nbox, t, &BatchPost<T>::blk_cells);
    const BatchPost<T> &b = boxes[k];
    if (cells_by_words(b.g))
        cells4_block(b.g, as_global(b.wabs), as_global(b.cells), b.bits ? as_global(b.bits) : nullptr, b.plane,
                     b.nwords, t - b.blk_cells, threadIdx.x & 63, threadIdx.x >> 6);
    else
        cells_block(b.g, as_global(b.wabs), as_global(b.cells), b.bits ? as_global(b.bits) : nullptr, b.plane,
                    b.nwords, t - b.blk_cells, threadIdx.x & 63, threadIdx.x >> 6);
}

template <typename T>
__global__ __launch_bounds__(256) void overlap_batch_kernel(const BatchPost<T> *boxes, int nbox) {
    const int k = box_of(boxes, nbox, blockIdx.x, &BatchPost<T>::blk_ov);
    const BatchPost<T> &b = boxes[k];
    const uint32_t l = blockIdx.x - b.blk_ov;
    if (b.bits)
        overlap_bits_block(b.g, as_global(b.bits), b.nwords, b.radius, part_global(b.part), l, threadIdx.x);
    else
        overlap_bytes_block(b.g, as_global(b.cells), b.plane, b.radius, part_global(b.part), l, threadIdx.x & 63,
                            threadIdx.x >> 6);
}

template <typename T>
__global__ __launch_bounds__(1024) void reduce_batch_kernel(const BatchPost<T> *boxes, uint32_t ring_idx) {
    const BatchPost<T> &b = boxes[blockIdx.y];
    reduce_lanes<1024>(part_global(b.part), as_global(b.nblk), as_global(b.ring) + (size_t)ring_idx * NSLOT,
                       blockIdx.x);
}

uint32_t cells_blocks(const Geom &g) {
    if (cells_by_words(g)) {
        const uint32_t rpw = (uint32_t)cells_rows_per_wave(g);
        const uint32_t gx = rpw == 2 ? 1u : (uint32_t)g.nx / 256;
        return gx * (((uint32_t)g.ny + 4 * rpw - 1) / (4 * rpw)) * (uint32_t)((g.nz + CZ - 1) / CZ);
    }
    return (uint32_t)((g.nx + 63) / 64) * (uint32_t)((g.ny + 3) / 4) * (uint32_t)((g.nz + CZ - 1) / CZ);
}

template <typename T>
hipError_t launch_post_batch(const BatchPost<T> *boxes_dev, int nbox, uint32_t nfix, uint32_t ncells, uint32_t nov,
                             int parity, uint32_t ring_idx, hipStream_t st) {
    fix_scan_batch_kernel<T><<<nfix, 256, 0, st>>>(boxes_dev, nbox, parity);
    fix_proc_batch_kernel<T><<<(uint32_t)nbox * FIX_PROC_BLOCKS, 256, 0, st>>>(boxes_dev, parity);
    cells_batch_kernel<T><<<ncells, 256, 0, st>>>(boxes_dev, nbox, ncells);
    overlap_batch_kernel<T><<<nov, 256, 0, st>>>(boxes_dev, nbox);
    reduce_batch_kernel<T><<<dim3(NSLOT, (unsigned)nbox, 1), 1024, 0, st>>>(boxes_dev, ring_idx);
    return hipGetLastError();
}

template hipError_t launch_post_batch<float>(const BatchPost<float> *, int, uint32_t, uint32_t, uint32_t, int,
                                             uint32_t, hipStream_t);
template hipError_t launch_post_batch<double>(const BatchPost<double> *, int, uint32_t, uint32_t, uint32_t, int,
                                              uint32_t, hipStream_t);

template hipError_t launch_phase<float>(const Geom &, Fields<float>, float *, uint32_t, hipStream_t);
template hipError_t launch_phase<double>(const Geom &, Fields<double>, double *, uint32_t, hipStream_t);
template hipError_t launch_wind_gauss<float>(const Geom &, Fields<float>, Moms<float>, const float *, float, float,
                                             const double[2], uint8_t *, uint32_t, int8_t *, Partials, hipStream_t);
template hipError_t launch_wind_gauss<double>(const Geom &, Fields<double>, Moms<double>, const double *, double,
                                              double, const double[2], uint8_t *, uint32_t, int8_t *, Partials,
                                              hipStream_t);

}  // namespace mts
