// step_pair.hip -- two leapfrog steps of the U(1)xU(1) lattice update per
// sweep through HBM (temporal blocking) for gfx950 (Correia & Martins,
// arXiv:2208.01525, Sec. III).
//
// A workgroup owns a 64 x TY column of sites and walks it through TZ planes
// along z, like the single-step tiled kernel, but evaluates steps n -> n+1
// and n+1 -> n+2 in one pass:
//   level 0  the fields at n on a (TY+4) x 68 region (two halo rows and
//            columns on each side), read from HBM;
//   level 1  step n on the (TY+2) x 66 region inside it (momenta n - 1/2
//            read from HBM); its fields stay in registers, its momenta in a
//            per-thread LDS ring;
//   level 2  step n+1 on the 64 x TY interior, one plane behind level 1;
//            fields n+2 and momenta n+3/2 are written to HBM.
// Waves 0..TY+3 hold the rows of the region (lanes -> columns 2..65), wave
// TY+4 its four halo columns.  The phasors, scalars and plaquette sines of
// one level and plane are staged in LDS for the x and y neighbours; the
// z neighbours stay in registers.  Every site is evaluated with the same
// per-site arithmetic as the single-step kernel (site.h), so two steps here
// give the same bits as two single steps.
//
// HBM traffic per site and pair of steps: the 20 reals of step n read and
// the 20 of step n+2 written (the halo re-reads come from L2), against
// twice that for two single steps.  The fields go to the other field copy
// and the momenta to the other momentum copy: neighbouring tiles read this
// tile's interior at n - 1/2 as their halo, so nothing may be updated in
// place.
#include "device.h"
#include "kernels.h"
#include "site.h"

namespace mts {

namespace {

constexpr int PW = 68;    // LDS row width: 64 + two halo columns on each side

__device__ __forceinline__ int wrapp(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

enum PQ { P_FR, P_FI, P_UXR, P_UXI, P_UYR, P_UYI, P_UZR, P_UZI, P_SXY, P_SXZ, P_SYZ, NPQ };

template <typename T, int R>
struct PairLds {
    T v[2][NPQ][R * PW];                   // one level's plane: scalars, phasors, sines
    T mom[2][10][64 * (R + 1)];            // level-1 momenta of two planes, one slot per thread
};

template <typename T, int R>
__device__ __forceinline__ cx<T> ldp(const PairLds<T, R> &L, int sec, int q, int i) {
    return cx<T>{L.v[sec][q][i], L.v[sec][q + 1][i]};
}

// Level-0 data of one plane for a thread's (x, y) column (the link angles
// are re-read where the drift needs them).
template <typename T>
struct Lev0 {
    cx<T> f[2];           // scalars
    cx<T> u[2][3];        // link phasors exp(-i h A)
};

// Level-1 data of one plane.
template <typename T>
struct Lev1 {
    cx<T> f[2];
    T a[2][3];            // link angles / h
    cx<T> u[2][3];
};

// What the next plane needs of the one below it.
template <typename T>
struct Below {
    cx<T> f[2], uz[2];
    T sxz[2], syz[2];
};

}  // namespace

template <typename T, int TY, bool NT>
__global__ __launch_bounds__(64 * (TY + 5)) void step_pair_kernel(Geom g, Fields<T> in, Fields<T> out, Moms<T> min_,
                                                                  Moms<T> mout, StepCoef<T> c1, StepCoef<T> c2,
                                                                  int TZ, int ntx, int nty, int ntz) {
    constexpr int R = TY + 4;
    constexpr int N = R * PW;
    __shared__ PairLds<T, R> L;
    const uint32_t t = xcd_order(blockIdx.x, (uint32_t)(ntx * nty * ntz));
    const int tx = t % ntx, ty_ = (t / ntx) % nty, tz = t / (ntx * nty);
    const int X0 = tx * 64, Y0 = ty_ * TY, Z0 = tz * TZ;

    // ---- which site of the region this thread holds
    const int lx = threadIdx.x, w = threadIdx.y;
    const int tid = lx + 64 * w;
    int row, col;
    bool valid = true;
    if (w < R) {
        row = w;
        col = lx + 2;
    } else {
        const int q = lx / R;
        row = lx - q * R;
        col = q == 0 ? 0 : (q == 1 ? 1 : (q == 2 ? PW - 2 : PW - 1));
        if (q >= 4) {
            valid = false;
            row = 0;
            col = 0;
        }
    }
    const int gx = X0 - 2 + col, gy = Y0 - 2 + row;
    const int x = wrapp(gx, g.nx), y = wrapp(gy, g.ny);
    const bool lev1 = valid && row >= 1 && row <= R - 2 && col >= 1 && col <= PW - 2;
    const bool lev2 = valid && row >= 2 && row <= R - 3 && col >= 2 && col <= PW - 3 && gx < g.nx && gy < g.ny;
    const uint32_t colidx = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const int li = row * PW + col;
    const int lxp = min(li + 1, N - 1), lxm = max(li - 1, 0);
    const int lyp = min(li + PW, N - 1), lym = max(li - PW, 0);
    const int zend = min(Z0 + TZ, g.nz);

    auto load0 = [&](int zz, Lev0<T> &v) {
        const uint32_t s = colidx + g.nxy * (uint32_t)zz;
        T a[2][3];
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            v.f[sec] = in.phi[sec][s];
#pragma unroll
            for (int i = 0; i < 3; i++) a[sec][i] = in.A[sec][i][s];
        }
#pragma unroll
        for (int sec = 0; sec < 2; sec++)
#pragma unroll
            for (int i = 0; i < 3; i++) v.u[sec][i] = phasor<T>(c1.h, a[sec][i]);
    };
    auto stage = [&](const cx<T> (&f)[2], const cx<T> (&u)[2][3]) {
        if (!valid) return;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            L.v[sec][P_FR][li] = f[sec].re;
            L.v[sec][P_FI][li] = f[sec].im;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                L.v[sec][P_UXR + 2 * i][li] = u[sec][i].re;
                L.v[sec][P_UXI + 2 * i][li] = u[sec][i].im;
            }
        }
    };
    // plaquette sines of the staged plane (nu: the level's links one plane up);
    // the site's own values are read back from LDS
    auto sines = [&](const cx<T> (&nu)[2][3]) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            T sn[3], cs[3];
            own_plaquettes(ldp(L, sec, P_UXR, li), ldp(L, sec, P_UYR, li), ldp(L, sec, P_UZR, li),
                           ldp(L, sec, P_UYR, lxp), ldp(L, sec, P_UXR, lyp), ldp(L, sec, P_UZR, lxp),
                           ldp(L, sec, P_UZR, lyp), nu[sec][0], nu[sec][1], sn, cs);
            if (valid) {
                L.v[sec][P_SXY][li] = sn[0];
                L.v[sec][P_SXZ][li] = sn[1];
                L.v[sec][P_SYZ][li] = sn[2];
            }
        }
    };
    // one sector's inputs: the staged plane, the planes above (nf) and below,
    // the momenta at the half step before and the link angles
    auto gather = [&](int sec, const cx<T> (&nf)[2], const Below<T> &below, cx<T> p0, const T (&e0)[3],
                      const T (&a)[3]) {
        SiteIn<T> q;
        q.f = ldp(L, sec, P_FR, li);
        q.o = ldp(L, 1 - sec, P_FR, li);
        q.fxp = ldp(L, sec, P_FR, lxp);
        q.fxm = ldp(L, sec, P_FR, lxm);
        q.fyp = ldp(L, sec, P_FR, lyp);
        q.fym = ldp(L, sec, P_FR, lym);
        q.fzp = nf[sec];
        q.fzm = below.f[sec];
        q.ux = ldp(L, sec, P_UXR, li);
        q.uy = ldp(L, sec, P_UYR, li);
        q.uz = ldp(L, sec, P_UZR, li);
        q.ux_m = ldp(L, sec, P_UXR, lxm);
        q.uy_m = ldp(L, sec, P_UYR, lym);
        q.uz_m = below.uz[sec];
        q.sxy = L.v[sec][P_SXY][li];
        q.sxz = L.v[sec][P_SXZ][li];
        q.syz = L.v[sec][P_SYZ][li];
        q.sxy_my = L.v[sec][P_SXY][lym];
        q.sxy_mx = L.v[sec][P_SXY][lxm];
        q.sxz_mx = L.v[sec][P_SXZ][lxm];
        q.syz_my = L.v[sec][P_SYZ][lym];
        q.sxz_mz = below.sxz[sec];
        q.syz_mz = below.syz[sec];
        q.p0 = p0;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            q.e0[i] = e0[i];
            q.a[i] = a[i];
        }
        return q;
    };
    // the staged plane's values the plane above needs (own LDS slot)
    auto keep_below = [&](Below<T> &b) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            b.f[sec] = ldp(L, sec, P_FR, li);
            b.uz[sec] = ldp(L, sec, P_UZR, li);
            b.sxz[sec] = L.v[sec][P_SXZ][li];
            b.syz[sec] = L.v[sec][P_SYZ][li];
        }
    };

    Lev0<T> c0, n0;        // level 0 at planes r, r + 1
    Below<T> b0;           // level 0 at plane r - 1
    Lev1<T> cl, nl;        // level 1 at planes r - 1, r (outside the level-1 region: unused zeros)
    Below<T> bl;           // level 1 at plane r - 2
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        nl.f[sec] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 3; i++) {
            nl.a[sec][i] = T(0);
            nl.u[sec][i] = cx<T>{T(0), T(0)};
        }
    }
    cl = nl;

    load0(wrapp(Z0 - 2, g.nz), c0);
    for (int r = Z0 - 2; r <= zend; r++) {
        load0(wrapp(r + 1, g.nz), n0);
        const bool do1 = r >= Z0 - 1;      // step n on plane r
        const bool do2 = r >= Z0;          // sines of level 1 on plane r - 1 (and step n+1 there)
        const bool out2 = r - 1 >= Z0;
        const int slot = r & 1;            // LDS momenta slot of plane r (plane r - 1: the other)
        cx<T> p0[2];
        T e0[2][3], a0[2][3];
        if (do1 && lev1) {
            const uint32_t s = colidx + g.nxy * (uint32_t)wrapp(r, g.nz);
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                p0[sec] = min_.pi[sec][s];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    e0[sec][i] = min_.E[sec][i][s];
                    a0[sec][i] = in.A[sec][i][s];
                }
            }
        }

        // level 0, plane r: stage, sines, step n
        stage(c0.f, c0.u);
        __syncthreads();
        sines(n0.u);
        __syncthreads();
        if (do1 && lev1) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const SiteOut<T> o = site_update<T, false>(c1, sec, gather(sec, n0.f, b0, p0[sec], e0[sec], a0[sec]));
                L.mom[slot][2 * sec][tid] = o.p1.re;
                L.mom[slot][2 * sec + 1][tid] = o.p1.im;
                nl.f[sec] = o.fn;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    L.mom[slot][4 + 3 * sec + i][tid] = o.e1[i];
                    nl.a[sec][i] = o.an[i];
                }
            }
#pragma unroll
            for (int sec = 0; sec < 2; sec++)
#pragma unroll
                for (int i = 0; i < 3; i++) nl.u[sec][i] = phasor<T>(c2.h, nl.a[sec][i]);
        }
        __syncthreads();
        keep_below(b0);
        c0 = n0;

        // level 1, plane r - 1: stage, sines, step n + 1
        if (do2) {
            stage(cl.f, cl.u);
            __syncthreads();
            sines(nl.u);
            __syncthreads();
            if (out2 && lev2) {
                const uint32_t s = colidx + g.nxy * (uint32_t)(r - 1);
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    const cx<T> pm{L.mom[1 - slot][2 * sec][tid], L.mom[1 - slot][2 * sec + 1][tid]};
                    T em[3];
#pragma unroll
                    for (int i = 0; i < 3; i++) em[i] = L.mom[1 - slot][4 + 3 * sec + i][tid];
                    const SiteOut<T> o = site_update<T, false>(c2, sec, gather(sec, nl.f, bl, pm, em, cl.a[sec]));
                    st_stream<NT>(&mout.pi[sec][s], o.p1);
                    st_stream<NT>(&out.phi[sec][s], o.fn);
#pragma unroll
                    for (int i = 0; i < 3; i++) {
                        st_stream<NT>(&mout.E[sec][i][s], o.e1[i]);
                        st_stream<NT>(&out.A[sec][i][s], o.an[i]);
                    }
                }
            }
            __syncthreads();
            keep_below(bl);
        }
        if (do1) cl = nl;
    }
}

bool pair_tile_supported(TileShape ts) { return (ts.ty == 3 || ts.ty == 7) && ts.tz >= 1; }

template <typename T, int TY>
static hipError_t launch_pair_ty(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> min_, Moms<T> mout,
                                 const StepCoef<T> &c1, const StepCoef<T> &c2, int tz, bool nt, hipStream_t st) {
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + tz - 1) / tz;
    const dim3 grid((unsigned)(ntx * nty * ntz), 1, 1), block(64, TY + 5, 1);
    if (nt)
        step_pair_kernel<T, TY, true><<<grid, block, 0, st>>>(g, in, out, min_, mout, c1, c2, tz, ntx, nty, ntz);
    else
        step_pair_kernel<T, TY, false><<<grid, block, 0, st>>>(g, in, out, min_, mout, c1, c2, tz, ntx, nty, ntz);
    return hipGetLastError();
}

template <>
hipError_t launch_step_pair<float>(const Geom &g, Fields<float> in, Fields<float> out, Moms<float> min_,
                                   Moms<float> mout, const StepCoef<float> &c1, const StepCoef<float> &c2,
                                   TileShape ts, bool nt, hipStream_t st) {
    switch (ts.ty) {
        case 3: return launch_pair_ty<float, 3>(g, in, out, min_, mout, c1, c2, ts.tz, nt, st);
        case 7: return launch_pair_ty<float, 7>(g, in, out, min_, mout, c1, c2, ts.tz, nt, st);
        default: return hipErrorInvalidValue;
    }
}

// FP64 keeps one step per sweep: its z-march state does not fit the
// registers of a two-level pipeline.
template <>
hipError_t launch_step_pair<double>(const Geom &, Fields<double>, Fields<double>, Moms<double>, Moms<double>,
                                    const StepCoef<double> &, const StepCoef<double> &, TileShape, bool,
                                    hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace mts
