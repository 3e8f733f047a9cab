// step_tile.hip -- z-marching, LDS-tiled leapfrog step of the U(1)xU(1)
// lattice update for gfx950 (Correia & Martins, arXiv:2208.01525, Sec. III).
//
// A workgroup owns a 64 x TY column of sites and walks it through TZ planes.
// Waves 0..TY-1 hold the 64-wide rows of the tile, wave TY the row below it,
// wave TY+1 the row above it, wave TY+2 the two halo columns (with corners).
// Per plane every thread loads its site's fields once, evaluates its three
// link phasors U_i = exp(-i h A_i) per sector (one sincos each) and stages
// phi and U in LDS; then it forms its own three plaquette phasors
//   P_ij(x) = U_i(x) U_j(x+i) conj(U_i(x+j)) conj(U_j(x)) = exp(-i theta_ij(x)),
// so sin theta = -Im P and cos theta = Re P without further transcendental
// work, and stages the sines.  The z-neighbours (phi(z-1), U_z(z-1), the
// sines of plane z-1, and phi, U_x, U_y of plane z+1) stay in registers.
// Interior threads then apply the kick and drift exactly as the per-site
// kernel does.  Each field value is read from HBM once per step (halo
// re-reads come from L2); momenta and fields are read and written once.
//
// Workgroups are numbered so that each XCD (workgroups are dealt round-robin
// to the 8 XCDs) processes one contiguous run of tiles, keeping the halo
// rows shared by neighbouring tiles inside one L2.
#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "site.h"

namespace mts {

namespace {

constexpr int LW = 66;    // LDS row width: 64 + two halo columns

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// LDS quantities per sector; the fused diagnostic variant adds the phase of
// the next plane and the new electric fields E_x, E_y (for the divergence at
// x + i)
enum Q { Q_FR, Q_FI, Q_UXR, Q_UXI, Q_UYR, Q_UYI, Q_UZR, Q_UZI, Q_SXY, Q_SXZ, Q_SYZ, NQ };
enum QF { Q_AN = NQ, Q_EX, Q_EY, NQF };

template <typename T, int TY, int NQX = NQ>
struct Lds {
    T v[2][NQX][(TY + 2) * LW];
};

template <typename T, int TY, int NQX>
__device__ __forceinline__ cx<T> ldc(const Lds<T, TY, NQX> &L, int sec, int q, int i) {
    return cx<T>{L.v[sec][q][i], L.v[sec][q + 1][i]};
}

// Per-thread LDS slots of the fused diagnostics (interior threads, index
// w * 64 + lane): the FP64 sums of the Gauss residual and of the windings,
// and the new E_z and charge term of the plane just updated, which the
// divergence reads after the plane's last barrier.  Kept out of registers.
template <typename T, int TY>
struct FusedLds {
    double acc[4][64 * TY];   // Gauss |C| p, q; scale p, q
    int wsum[2][64 * TY];     // sum |W| p, q
    T ez[2][64 * TY];
    T gr[2][64 * TY];
    int nw[2][(TY + 2) * LW]; // the plane's packed link wrap counts, every site of the tile
};

template <typename T, int TY>
struct NoFusedLds {};

// c = chi + h A, the sum rounded on its own
template <typename T>
__device__ __forceinline__ T link_value(T chi, T hA) {
#pragma clang fp contract(off)
    return chi + hA;
}

}  // namespace

// Accumulators of one thread's integer-time sums: the six of the update
// (energy, Lagrangian, the four velocity sums), then with the fused
// diagnostics the Gauss residual sums (|C| and scale, per sector) and the
// winding sums (per sector), in the order of the reduction slots.
constexpr int NACC_FUSED = SL_WIND_Q + 1;

// One tile (64 x TY columns, planes [Z0, Z0 + TZ)) of one box; accumulates the
// integer-time sums of its interior sites into acc when DIAG.  With COOL the
// fields move along their forces (one forward-Euler step of the cooling
// flow, coefficients set by the caller) and the momenta are neither read nor
// written.
//
// FUSE (with DIAG): the windings and the Gauss residual of the step's input
// fields are computed here as well, and no phase is stored.  Per plane z,
// every thread stages the phase alpha(z+1) of its site; then it forms the
// wrap counts n_mu of its links at z (n_z) and z+1 (n_x, n_y, carried to the
// next plane), stages those of z packed in one word, and the interior
// threads take the windings through the three faces at their site,
//   W_z = -(n_x(x) + n_y(x+x) - n_x(x+y) - n_y(x))  (and cyclic),
// the value rint of the post-step kernel's sum of link phases and plaquette
// angle takes when no link of the face is flagged by the guard; a face with
// a flagged link marks its site for the fix-up kernel.
// The Gauss residual C = div E^{n+1/2} - g Im[conj(phi^n) Pi^{n+1/2}]
// needs the new E at x - i: the interior threads stage their E_x, E_y; the
// halo column x0 - 1 and row y0 - 1 recompute theirs (E_x and E_y only, with
// the same arithmetic as their owning tile), and at the plane below the tile
// the interior threads recompute E_z.  Those recomputations read E^{n-1/2} of
// sites other tiles update, so FUSE needs the momenta written out of place
// (mom_out a different copy from mom).
template <typename T, bool DIAG, int TY, bool NT, bool COOL = false, int PF = 0, bool FUSE = false>
__device__ __forceinline__ void tile_step(const Geom &g, const Fields<T> &in, const Fields<T> &out,
                                          const Moms<T> &mom, const Moms<T> &mom_out,
                                          const StepCoef<T> &c, int X0, int Y0, int Z0, int TZ,
                                          Lds<T, TY, FUSE ? NQF : NQ> &L, double (&acc)[FUSE ? NACC_FUSED : 6],
                                          T *alpha, uint8_t *wabs, uint32_t plane,
                                          typename std::conditional<FUSE, FusedLds<T, TY>, NoFusedLds<T, TY>>::type &FL) {
    static_assert(!FUSE || (DIAG && !COOL), "fused diagnostics belong to diagnostic steps");
    constexpr int R = TY + 2;

    // ---- which site of the tile this thread holds
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
    const int x = wrapi(gx, g.nx), y = wrapi(gy, g.ny);
    const bool interior = w < TY && gx < g.nx && gy < g.ny;
    const uint32_t colidx = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const int li = row * LW + col;
    const int lxp = row * LW + min(col + 1, LW - 1), lyp = min(row + 1, R - 1) * LW + col;
    const int lxm = row * LW + max(col - 1, 0), lym = max(row - 1, 0) * LW + col;

    // fused diagnostics: the halo sites whose new E_x (column x0 - 1) or E_y
    // (row y0 - 1) the divergence of an interior site needs; the faces read
    // phases and wrap counts at the site and at +x and +y only, so the row
    // y0 - 1 and the column x0 - 1 form neither
    const bool edge_x = FUSE && owner && col == 0 && row >= 1 && row <= TY && gy < g.ny;
    const bool edge_y = FUSE && w == TY && gx < g.nx;
    const bool wraps = FUSE && owner && row > 0 && col > 0;

    const int zbeg = Z0, zend = min(Z0 + TZ, g.nz);

    // registers: plane z (cur), z+1 (nxt), z-1 (prv)
    cx<T> cf[2], nf[2], pf[2];
    T cA[2][3], nA[2][3];
    cx<T> cU[2][3], nU[2][3], pUz[2];
    T psxz[2], psyz[2];
    // fused: alpha(z); packed wrap counts of the x and y links at z; E_z^{n+1/2}(z-1)
    T alc[2], ezp[2];
    int wxy[2];
    const int it = w * 64 + lx;            // interior thread's slot in FL
    // FP64 diagnostic steps keep their six running sums in LDS, one slot per
    // interior thread (same operations, same order): in registers they would
    // push the z-march past 256 VGPRs.  So does the fused FP32 step with the
    // deeper load pipeline, whose registers go to the loads in flight.
    constexpr bool ACC_LDS = DIAG && (sizeof(T) == 8 || (FUSE && PF >= 1));
    __shared__ double accs[ACC_LDS ? 6 : 1][ACC_LDS ? 64 * TY : 1];
    if constexpr (ACC_LDS) {
        if (interior) {
#pragma unroll
            for (int q = 0; q < 6; q++) accs[q][it] = 0.0;
        }
    }
    auto load_raw = [&](int zz, cx<T> (&f)[2], T (&A)[2][3]) {
        const uint32_t s = colidx + g.nxy * (uint32_t)zz;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            f[sec] = in.phi[sec][s];
#pragma unroll
            for (int i = 0; i < 3; i++) A[sec][i] = in.A[sec][i][s];
        }
    };
    auto make_U = [&](const T (&A)[2][3], cx<T> (&U)[2][3]) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++)
#pragma unroll
            for (int i = 0; i < 3; i++) U[sec][i] = phasor<T>(c.h, A[sec][i]);
    };
    auto load_mom = [&](uint32_t sm, cx<T> (&p)[2], T (&e)[2][3]) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            p[sec] = mom.pi[sec][sm];
#pragma unroll
            for (int i = 0; i < 3; i++) e[sec][i] = mom.E[sec][i][sm];
        }
    };
    // PF >= 1: the raw fields of plane z+2 are loaded one iteration ahead, so
    // the phasors of plane z+1 do not wait on loads issued in the same
    // iteration; PF = 2: the momenta of plane z+1 as well
    cx<T> rf[2], rp[2];
    T rA[2][3], re[2][3];

    load_raw(wrapi(zbeg - 1, g.nz), cf, cA);
    make_U(cA, cU);
    if constexpr (FUSE) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            alc[sec] = phase_of(cf[sec]);
            wxy[sec] = 0;
            ezp[sec] = T(0);
        }
        if (interior) {
#pragma unroll
            for (int q = 0; q < 4; q++) FL.acc[q][it] = 0.0;
            FL.wsum[0][it] = 0;
            FL.wsum[1][it] = 0;
        }
    }
    if constexpr (PF >= 1) {
        load_raw(wrapi(zbeg, g.nz), rf, rA);
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {    // plane zbeg - 1 is not updated
            rp[sec] = cx<T>{T(0), T(0)};
#pragma unroll
            for (int i = 0; i < 3; i++) re[sec][i] = T(0);
        }
    }

    for (int z = zbeg - 1; z < zend; z++) {
        const bool upd = interior && z >= zbeg;
        const int zz = wrapi(z, g.nz);
        const int zn = wrapi(z + 1, g.nz);
        const uint32_t s = colidx + g.nxy * (uint32_t)zz;
        cx<T> p0[2];
        T e0[2][3];
        if constexpr (PF >= 1) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                nf[sec] = rf[sec];
#pragma unroll
                for (int i = 0; i < 3; i++) nA[sec][i] = rA[sec][i];
            }
            if (z + 2 <= zend) load_raw(wrapi(z + 2, g.nz), rf, rA);
            if constexpr (PF == 2) {
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    p0[sec] = rp[sec];
#pragma unroll
                    for (int i = 0; i < 3; i++) e0[sec][i] = re[sec][i];
                }
                if (interior && !COOL && z + 1 >= zbeg && z + 1 < zend)
                    load_mom(colidx + g.nxy * (uint32_t)wrapi(z + 1, g.nz), rp, re);
            } else if (upd && !COOL) {
                load_mom(s, p0, e0);
            }
            make_U(nA, nU);
        } else {
            load_raw(zn, nf, nA);
            make_U(nA, nU);
            if (upd && !COOL) load_mom(s, p0, e0);
        }
        // fused: E^{n-1/2} of the halo components this thread recomputes
        T eh[2] = {T(0), T(0)};
        if constexpr (FUSE) {
            // the component chosen among loaded pointer values (prvalues: a
            // conditional over the struct's lvalues, or a runtime index, would
            // select addresses inside it, per lane): for a single box each lane
            // then loaded its pointer from the argument block before loading E,
            // a dependent round trip every plane; in the ensemble kernel, whose
            // pointer table is a local value, the table became a per-thread
            // array (the compiler moved it to LDS, 64 B a thread)
            if ((edge_x || edge_y) && z >= zbeg) {
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    const T *ex = static_cast<const T *>(mom.E[sec][0]);
                    const T *ey = static_cast<const T *>(mom.E[sec][1]);
                    eh[sec] = (edge_x ? ex : ey)[s];
                }
            } else if (interior && z == zbeg - 1) {
#pragma unroll
                for (int sec = 0; sec < 2; sec++) eh[sec] = mom.E[sec][2][s];
            }
        }

        // stage phi and U of plane z (fused: and the phase of plane z+1; the
        // phase of plane z is the one this thread staged one plane before)
        T aln[2] = {T(0), T(0)};
        if constexpr (FUSE) {
            if (wraps && z > zbeg - 1) {
#pragma unroll
                for (int sec = 0; sec < 2; sec++) alc[sec] = L.v[sec][Q_AN][li];
            }
        }
        if (owner) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                L.v[sec][Q_FR][li] = cf[sec].re;
                L.v[sec][Q_FI][li] = cf[sec].im;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    L.v[sec][Q_UXR + 2 * i][li] = cU[sec][i].re;
                    L.v[sec][Q_UXI + 2 * i][li] = cU[sec][i].im;
                }
                if constexpr (FUSE) {
                    if (wraps) {
                        aln[sec] = phase_of(nf[sec]);
                        L.v[sec][Q_AN][li] = aln[sec];
                    }
                }
            }
        }
        __syncthreads();

        // own plaquette phasors of plane z (a non-fused diagnostic step folds
        // its magnetic term in here, in the same order, so the cosines need not
        // stay live through the update)
        constexpr bool EARLY_B = DIAG && !FUSE;
        T sn[2][3], cs[2][3];
        T Bg = 0;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            own_plaquettes(cU[sec][0], cU[sec][1], cU[sec][2], ldc(L, sec, Q_UYR, lxp), ldc(L, sec, Q_UXR, lyp),
                           ldc(L, sec, Q_UZR, lxp), ldc(L, sec, Q_UZR, lyp), nU[sec][0], nU[sec][1], sn[sec],
                           cs[sec]);
            if (owner) {
                L.v[sec][Q_SXY][li] = sn[sec][0];
                L.v[sec][Q_SXZ][li] = sn[sec][1];
                L.v[sec][Q_SYZ][li] = sn[sec][2];
            }
            if constexpr (EARLY_B)
                Bg += c.inv_e2h4[sec] * (((T(1) - cs[sec][0]) + (T(1) - cs[sec][1])) + (T(1) - cs[sec][2]));
        }
        // fused: wrap counts of the x and y links of plane z+1 and of the z
        // link of plane z (garbage where the neighbour lies outside the tile:
        // no face reads those); stage the word of plane z
        int wnext[2] = {0, 0}, wown[2] = {0, 0};
        if constexpr (FUSE) {
            if (wraps) {
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    bool fx, fy, fz;
                    const int nx_ = link_wrap(aln[sec], L.v[sec][Q_AN][lxp], link_angle(c.h, nA[sec][0]), fx);
                    const int ny_ = link_wrap(aln[sec], L.v[sec][Q_AN][lyp], link_angle(c.h, nA[sec][1]), fy);
                    const int nz_ = link_wrap(alc[sec], aln[sec], link_angle(c.h, cA[sec][2]), fz);
                    wnext[sec] = wrap_word(nx_, ny_, 0, fx, fy, false);
                    wown[sec] = wxy[sec] | wrap_word(0, 0, nz_, false, false, fz);
                    FL.nw[sec][li] = wown[sec];
                }
            }
        }
        __syncthreads();

        if constexpr (FUSE) {
            if (upd) {
                // windings through the three faces at the site (lower corner x)
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    const int o = wown[sec], xp = FL.nw[sec][lxp], yp = FL.nw[sec][lyp], zp = wnext[sec];
                    const int Wz = -(((wrap_n<0>(o) + wrap_n<1>(xp)) - wrap_n<0>(yp)) - wrap_n<1>(o));
                    const int Wx = -(((wrap_n<1>(o) + wrap_n<2>(yp)) - wrap_n<1>(zp)) - wrap_n<2>(o));
                    const int Wy = -(((wrap_n<2>(o) + wrap_n<0>(zp)) - wrap_n<2>(xp)) - wrap_n<0>(o));
                    const int flagged = (o & WRAP_F_XYZ) | (xp & WRAP_F_YZ) | (yp & WRAP_F_XZ) | (zp & WRAP_F_XY);
                    uint8_t byte = WABS_FIX;
                    if (!flagged) {
                        const int aWx = abs(Wx), aWy = abs(Wy), aWz = abs(Wz);
                        byte = (uint8_t)(min(aWx, 3) | (min(aWy, 3) << 2) | (min(aWz, 3) << 4));
                        FL.wsum[sec][it] += aWx + aWy + aWz;
                    }
                    st_stream<NT>(wabs + (size_t)sec * plane + s, byte);
                }
            } else if (edge_x || edge_y) {
                if (z >= zbeg) {
                    // the halo's new E_x (column x0 - 1) or E_y (row y0 - 1), as its own tile computes it
#pragma unroll
                    for (int sec = 0; sec < 2; sec++) {
                        T e;
                        if (edge_x) {
                            const T M = mag_force(c, sn[sec][0], L.v[sec][Q_SXY][lym], sn[sec][1], psxz[sec]);
                            e = e_kick(c, eh[sec], M, current(c, sec, cf[sec], cmul(cU[sec][0], ldc(L, sec, Q_FR, lxp))));
                            L.v[sec][Q_EX][li] = e;
                        } else {
                            const T M = mag_force(c, L.v[sec][Q_SXY][lxm], sn[sec][0], sn[sec][2], psyz[sec]);
                            e = e_kick(c, eh[sec], M, current(c, sec, cf[sec], cmul(cU[sec][1], ldc(L, sec, Q_FR, lyp))));
                            L.v[sec][Q_EY][li] = e;
                        }
                    }
                }
            } else if (interior && z == zbeg - 1) {
                // E_z^{n+1/2} of the plane below the tile, for the divergence at its first plane
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    const T M = mag_force(c, L.v[sec][Q_SXZ][lxm], sn[sec][1], L.v[sec][Q_SYZ][lym], sn[sec][2]);
                    ezp[sec] = e_kick(c, eh[sec], M, current(c, sec, cf[sec], cmul(cU[sec][2], nf[sec])));
                }
            }
        }

        if (upd) {
            T Kd = 0, Gd = 0, Kg = 0, mod2[2] = {0, 0};
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                SiteIn<T> q;
                q.f = cf[sec];
                q.o = cf[1 - sec];
                q.fxp = ldc(L, sec, Q_FR, lxp);
                q.fxm = ldc(L, sec, Q_FR, lxm);
                q.fyp = ldc(L, sec, Q_FR, lyp);
                q.fym = ldc(L, sec, Q_FR, lym);
                q.fzp = nf[sec];
                q.fzm = pf[sec];
                q.ux = cU[sec][0];
                q.uy = cU[sec][1];
                q.uz = cU[sec][2];
                q.ux_m = ldc(L, sec, Q_UXR, lxm);
                q.uy_m = ldc(L, sec, Q_UYR, lym);
                q.uz_m = pUz[sec];
                q.sxy = sn[sec][0];
                q.sxz = sn[sec][1];
                q.syz = sn[sec][2];
                q.sxy_my = L.v[sec][Q_SXY][lym];
                q.sxy_mx = L.v[sec][Q_SXY][lxm];
                q.sxz_mx = L.v[sec][Q_SXZ][lxm];
                q.syz_my = L.v[sec][Q_SYZ][lym];
                q.sxz_mz = psxz[sec];
                q.syz_mz = psyz[sec];
                if constexpr (!COOL) {
                    q.p0 = p0[sec];
#pragma unroll
                    for (int i = 0; i < 3; i++) q.e0[i] = e0[sec][i];
                }
#pragma unroll
                for (int i = 0; i < 3; i++) q.a[i] = cA[sec][i];
                const SiteOut<T> r = site_update<T, COOL>(c, sec, q);
                if constexpr (!COOL) {
                    st_stream<NT>(&mom_out.pi[sec][s], r.p1);
#pragma unroll
                    for (int i = 0; i < 3; i++) st_stream<NT>(&mom_out.E[sec][i][s], r.e1[i]);
                }
                st_stream<NT>(&out.phi[sec][s], r.fn);
#pragma unroll
                for (int i = 0; i < 3; i++) st_stream<NT>(&out.A[sec][i][s], r.an[i]);

                if constexpr (DIAG) {
                    const cx<T> f = cf[sec];
                    cx<T> pb;
                    pb.re = T(0.5) * (p0[sec].re + r.p1.re);
                    pb.im = T(0.5) * (p0[sec].im + r.p1.im);
                    Kd += norm2(pb);
                    cx<T> dx_, dy_, dz_;
                    dx_.re = r.wx.re - f.re; dx_.im = r.wx.im - f.im;
                    dy_.re = r.wy.re - f.re; dy_.im = r.wy.im - f.im;
                    dz_.re = r.wz.re - f.re; dz_.im = r.wz.im - f.im;
                    Gd += c.inv_h2 * ((norm2(dx_) + norm2(dy_)) + norm2(dz_));
                    const T ebx = T(0.5) * (e0[sec][0] + r.e1[0]), eby = T(0.5) * (e0[sec][1] + r.e1[1]),
                            ebz = T(0.5) * (e0[sec][2] + r.e1[2]);
                    Kg += c.inv_2e2[sec] * ((ebx * ebx + eby * eby) + ebz * ebz);
                    if constexpr (!EARLY_B)
                        Bg += c.inv_e2h4[sec] * (((T(1) - cs[sec][0]) + (T(1) - cs[sec][1])) + (T(1) - cs[sec][2]));
                    mod2[sec] = r.m2;
                }
                if constexpr (FUSE) {
                    L.v[sec][Q_EX][li] = r.e1[0];
                    L.v[sec][Q_EY][li] = r.e1[1];
                    FL.ez[sec][it] = r.e1[2];
                    FL.gr[sec][it] = gauss_charge(c.gsig[sec], cf[sec], r.p1);
                }
            }
            if constexpr (DIAG) {
                if constexpr (!FUSE && sizeof(T) == 4) {
                    // phase of phi^n for the per-column winding kernel (NaN where
                    // phi = 0), where that kernel runs (alpha non-null); in FP64
                    // its atan2 here would spill
                    if (alpha != nullptr) {
#pragma unroll
                        for (int sec = 0; sec < 2; sec++)
                            st_stream<NT>(alpha + (size_t)sec * plane + s, phase_of(cf[sec]));
                    }
                }
                const T dp = mod2[0] - c.sig2[0], dq = mod2[1] - c.sig2[1];
                const T Vint = c.kap0 * dp * dq;
                const T V = (c.lam4[0] * dp * dp + c.lam4[1] * dq * dq) - Vint;
                const T eps = (Kd + Gd) + c.am2s * (Kg + Bg) + c.a2s * V;
                const T lag = (Kd - Gd) + c.am2s * (Kg - Bg) - c.a2s * V;
                const double K = Kd, G = Gd, Lg = lag, Vi = Vint;
                double *a0 = ACC_LDS ? &accs[0][it] : &acc[0];
                constexpr int AS = ACC_LDS ? 64 * TY : 1;   // stride between the six sums
                a0[0] += (double)eps;
                a0[AS] += Lg;
                a0[2 * AS] += K * Lg;
                a0[3 * AS] += G * Lg;
                a0[4 * AS] += K * Vi;
                a0[5 * AS] += G * Vi;
            }
        }
        __syncthreads();   // LDS of plane z is reused by plane z+1

        if constexpr (FUSE) {
            if (upd) {
                // Gauss residual at n + 1/2: div E^{n+1/2} - g Im[conj(phi^n) Pi^{n+1/2}]
#pragma unroll
                for (int sec = 0; sec < 2; sec++) {
                    const T ez = FL.ez[sec][it];
                    const T div = gauss_div(L.v[sec][Q_EX][li], L.v[sec][Q_EX][lxm], L.v[sec][Q_EY][li],
                                            L.v[sec][Q_EY][lym], ez, ezp[sec], c.inv_h);
                    double ga = FL.acc[sec][it], gsc = FL.acc[2 + sec][it];
                    gauss_accumulate(div, FL.gr[sec][it], ga, gsc);
                    FL.acc[sec][it] = ga;
                    FL.acc[2 + sec][it] = gsc;
                    ezp[sec] = ez;
                }
            }
#pragma unroll
            for (int sec = 0; sec < 2; sec++) wxy[sec] = wnext[sec];
        }

        // rotate registers
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            pf[sec] = cf[sec];
            pUz[sec] = cU[sec][2];
            psxz[sec] = sn[sec][1];
            psyz[sec] = sn[sec][2];
            cf[sec] = nf[sec];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                cA[sec][i] = nA[sec][i];
                cU[sec][i] = nU[sec][i];
            }
        }
    }
    if constexpr (ACC_LDS) {
        if (interior) {
#pragma unroll
            for (int q = 0; q < 6; q++) acc[q] = accs[q][it];
        }
    }
    if constexpr (FUSE) {
#pragma unroll
        for (int q = 0; q < 4; q++) acc[SL_GAUSS_ABS_P + q] = interior ? FL.acc[q][it] : 0.0;
        acc[SL_WIND_P] = interior ? (double)FL.wsum[0][it] : 0.0;
        acc[SL_WIND_Q] = interior ? (double)FL.wsum[1][it] : 0.0;
    }
}

template <typename T, bool DIAG, int TY, bool NT, int PF, bool FUSE>
__global__ __launch_bounds__(64 * (TY + 3)) void step_tile_kernel(Geom g, Fields<T> in, Fields<T> out, Moms<T> mom,
                                                                  Moms<T> mom_out,
                                                                  StepCoef<T> c, Partials part, int TZ, int ntx,
                                                                  int nty, int ntz, T *alpha, uint8_t *wabs,
                                                                  uint32_t plane, int xcd) {
    __shared__ Lds<T, TY, FUSE ? NQF : NQ> L;
    __shared__ typename std::conditional<FUSE, FusedLds<T, TY>, NoFusedLds<T, TY>>::type FL;
    const uint32_t t = xcd ? xcd_order(blockIdx.x, (uint32_t)(ntx * nty * ntz)) : blockIdx.x;
    const int tx = t % ntx, ty_ = (t / ntx) % nty, tz = t / (ntx * nty);
    double acc[FUSE ? NACC_FUSED : 6] = {};
    tile_step<T, DIAG, TY, NT, false, PF, FUSE>(g, in, out, mom, mom_out, c, tx * 64, ty_ * TY, tz * TZ, TZ, L, acc,
                                                alpha, wabs, plane, FL);
    if constexpr (DIAG) block_sum_store<FUSE ? NACC_FUSED : 6, TY + 3>(acc, part, SL_EPS, t);
}

// Ensemble of boxes in one launch: the blocks of box k are [blk0[k], blk0[k+1])
// of the XCD-ordered grid; each box has its own fields, coefficients and
// partials (indexed by the box-local block).  FUSE as for single boxes.
template <typename T, bool DIAG, int TY, bool NT, bool FUSE = false>
__global__ __launch_bounds__(64 * (TY + 3)) void step_tile_batch_kernel(const BatchBox<T> *boxes, int nbox,
                                                                        int parity, int mpin, int mpout,
                                                                        const StepCoef<T> *coef, uint32_t nblk,
                                                                        int xcd) {
    __shared__ Lds<T, TY, FUSE ? NQF : NQ> L;
    __shared__ typename std::conditional<FUSE, FusedLds<T, TY>, NoFusedLds<T, TY>>::type FL;
    const uint32_t t = xcd ? xcd_order(blockIdx.x, nblk) : blockIdx.x;
    int lo = 0, hi = nbox - 1;             // last box with blk0 <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].blk0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const BatchBox<T> &bx = boxes[lo];
    const uint32_t lt = t - bx.blk0;
    const int tx = lt % bx.ntx, ty_ = (lt / bx.ntx) % bx.nty, tz = lt / (bx.ntx * bx.nty);
    // the box table's pointers all address global memory
    Fields<T> fin, fout;
    Moms<T> mom, mom_out;
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        fin.phi[sec] = as_global(bx.f[parity].phi[sec]);
        fout.phi[sec] = as_global(bx.f[1 - parity].phi[sec]);
        mom.pi[sec] = as_global(bx.mom[mpin].pi[sec]);
        mom_out.pi[sec] = as_global(bx.mom[mpout].pi[sec]);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            fin.A[sec][i] = as_global(bx.f[parity].A[sec][i]);
            fout.A[sec][i] = as_global(bx.f[1 - parity].A[sec][i]);
            mom.E[sec][i] = as_global(bx.mom[mpin].E[sec][i]);
            mom_out.E[sec][i] = as_global(bx.mom[mpout].E[sec][i]);
        }
    }
    double acc[FUSE ? NACC_FUSED : 6] = {};
    // (the fused step with the deeper load pipeline and its sums in LDS, as
    // for single boxes, measured 20.8 against 18.3 ms over the 64-box ensemble)
    tile_step<T, DIAG, TY, NT, false, 0, FUSE>(bx.g, fin, fout, mom, mom_out, coef[lo], tx * 64, ty_ * TY,
                                               tz * bx.tz, bx.tz, L, acc, as_global(bx.alpha),
                                               FUSE ? as_global(bx.wabs) : nullptr, bx.plane, FL);
    if constexpr (DIAG) {
        Partials part = bx.part;
        part.base = as_global(part.base);
        block_sum_store<FUSE ? NACC_FUSED : 6, TY + 3>(acc, part, SL_EPS, lt);
    }
}

// One step of the cooling flow with the tiled kernel (momenta untouched).
template <typename T, int TY>
__global__ __launch_bounds__(64 * (TY + 3)) void cool_tile_kernel(Geom g, Fields<T> in, Fields<T> out, StepCoef<T> c,
                                                                  int TZ, int ntx, int nty, int ntz) {
    __shared__ Lds<T, TY> L;
    const uint32_t t = xcd_order(blockIdx.x, (uint32_t)(ntx * nty * ntz));
    const int tx = t % ntx, ty_ = (t / ntx) % nty, tz = t / (ntx * nty);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const Moms<T> none{};
    NoFusedLds<T, TY> nf;
    tile_step<T, false, TY, true, true>(g, in, out, none, none, c, tx * 64, ty_ * TY, tz * TZ, TZ, L, acc, nullptr,
                                        nullptr, 0, nf);
}

template <typename T>
hipError_t launch_cool_tile(const Geom &g, Fields<T> in, Fields<T> out, const StepCoef<T> &c, TileShape ts,
                            hipStream_t st) {
    // the cooling kernel has 4, 8 and 12 rows; tile shapes do not change results
    const int cty = ts.ty == 5 ? 4 : ts.ty == 13 ? 12 : ts.ty;
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + cty - 1) / cty, ntz = (g.nz + ts.tz - 1) / ts.tz;
    const dim3 grid((unsigned)(ntx * nty * ntz), 1, 1);
    switch (cty) {
        case 4: cool_tile_kernel<T, 4><<<grid, dim3(64, 7, 1), 0, st>>>(g, in, out, c, ts.tz, ntx, nty, ntz); break;
        case 8: cool_tile_kernel<T, 8><<<grid, dim3(64, 11, 1), 0, st>>>(g, in, out, c, ts.tz, ntx, nty, ntz); break;
        case 12: cool_tile_kernel<T, 12><<<grid, dim3(64, 15, 1), 0, st>>>(g, in, out, c, ts.tz, ntx, nty, ntz); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_cool_tile<float>(const Geom &, Fields<float>, Fields<float>, const StepCoef<float> &,
                                            TileShape, hipStream_t);
template hipError_t launch_cool_tile<double>(const Geom &, Fields<double>, Fields<double>, const StepCoef<double> &,
                                             TileShape, hipStream_t);

// Rows per tile: 4, 5, 8 and 12 in both precisions, 13 in FP32 (whose
// workgroup of 16 waves fills a CU's wave slots at 128 registers; in FP64 its
// LDS does not fit).  5 rows make 8 waves, the two-per-SIMD that FP64's
// 240-256 registers allow.
bool tile_supported(TileShape ts, bool fp64) {
    const bool ok = ts.ty == 4 || ts.ty == 5 || ts.ty == 8 || ts.ty == 12 || (ts.ty == 13 && !fp64);
    return ok && ts.tz >= 1;
}

bool batch_tile_supported(TileShape ts, bool fp64) { return tile_supported(ts, fp64); }

uint32_t tile_blocks(const Geom &g, TileShape ts) {
    const uint32_t ntx = (g.nx + 63) / 64, nty = (g.ny + ts.ty - 1) / ts.ty, ntz = (g.nz + ts.tz - 1) / ts.tz;
    return ntx * nty * ntz;
}

template <typename T, int TY>
static hipError_t launch_ty(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, Moms<T> mom_out,
                            const StepCoef<T> &c, bool diag,
                            Partials part, int tz, T *alpha, uint8_t *wabs, uint32_t plane, bool nt, bool pf,
                            bool xcd, hipStream_t st) {
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + tz - 1) / tz;
    dim3 block(64, TY + 3, 1);
    dim3 grid((unsigned)(ntx * nty * ntz), 1, 1);
#define MTS_TILE_LAUNCH(D, N, F, FU) \
    step_tile_kernel<T, D, TY, N, F, FU><<<grid, block, 0, st>>>(g, in, out, mom, mom_out, c, part, tz, ntx, nty, \
                                                                 ntz, alpha, wabs, plane, xcd ? 1 : 0)
    if (diag) {
        // FP32 diagnostic steps always load the fields one plane further
        // ahead: at the row counts they run with it costs no occupancy and
        // saves about 5 % (512^3: 4.82 against 5.08 ms).  The FP64 variant
        // is at its register limit already.  Diagnostic steps run at most 8
        // rows in FP32 and 5 in FP64, so the shapes only plain steps use have
        // no diagnostic variant.  With wabs the windings and the Gauss
        // residual are fused in (FP32; momenta out of place).
        constexpr int DPF = sizeof(T) == 4 ? 1 : 0;
        if constexpr (TY == 13 || (TY > 5 && sizeof(T) == 8)) {
            return hipErrorNotSupported;
        } else {
            if (wabs) {
                if constexpr (sizeof(T) == 4 && TY != 12) {
                    if (mom.pi[0] == mom_out.pi[0]) return hipErrorInvalidValue;
                    // deeper load pipeline, running sums in LDS (512^3: 6.17
                    // against 6.33 ms per diagnostic step)
                    if (nt) MTS_TILE_LAUNCH(true, true, 1, true);
                    else MTS_TILE_LAUNCH(true, false, 1, true);
                } else {
                    return hipErrorNotSupported;
                }
            } else {
                if (nt) MTS_TILE_LAUNCH(true, true, DPF, false);
                else MTS_TILE_LAUNCH(true, false, DPF, false);
            }
        }
    } else if (pf) {
        if (nt) MTS_TILE_LAUNCH(false, true, 1, false);
        else MTS_TILE_LAUNCH(false, false, 1, false);
    } else {
        if (nt) MTS_TILE_LAUNCH(false, true, 0, false);
        else MTS_TILE_LAUNCH(false, false, 0, false);
    }
#undef MTS_TILE_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_tile(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, Moms<T> mom_out,
                            const StepCoef<T> &c, bool diag,
                            Partials part, TileShape ts, T *alpha, uint8_t *wabs, uint32_t plane, bool nt, bool pf,
                            bool xcd, hipStream_t st) {
#define MTS_TY(TYV) \
    launch_ty<T, TYV>(g, in, out, mom, mom_out, c, diag, part, ts.tz, alpha, wabs, plane, nt, pf, xcd, st)
    switch (ts.ty) {
        case 4: return MTS_TY(4);
        case 8: return MTS_TY(8);
        case 5: return MTS_TY(5);
        case 12: return MTS_TY(12);
        case 13:
            if constexpr (sizeof(T) == 4)
                return MTS_TY(13);
            else
                return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
#undef MTS_TY
}

template <typename T>
hipError_t launch_step_tile_batch(const BatchBox<T> *boxes_dev, int nbox, uint32_t nblk, int parity, int mpin,
                                  int mpout, const StepCoef<T> *coef_dev, bool diag, int ty, bool nt, bool xcd,
                                  bool fused, hipStream_t st) {
    dim3 grid(nblk, 1, 1);
#define MTS_BATCH_LAUNCH(TYV, D, N, FU)                                                                            \
    step_tile_batch_kernel<T, D, TYV, N, FU><<<grid, dim3(64, TYV + 3, 1), 0, st>>>(boxes_dev, nbox, parity, mpin, \
                                                                                     mpout, coef_dev, nblk,        \
                                                                                     xcd ? 1 : 0)
    if (diag && fused) {
        // fused diagnostics: FP32, 8 rows, momenta out of place
        if constexpr (sizeof(T) == 4) {
            if (ty != 8 || mpin == mpout) return hipErrorInvalidValue;
            if (nt) MTS_BATCH_LAUNCH(8, true, true, true);
            else MTS_BATCH_LAUNCH(8, true, false, true);
            return hipGetLastError();
        } else {
            return hipErrorNotSupported;
        }
    }
    // as for single boxes: no diagnostic variant for the shapes only plain steps use
#define MTS_BATCH_CASE(TYV)                                           \
    case TYV:                                                         \
        if (diag) {                                                   \
            if constexpr (TYV == 13 || (TYV > 5 && sizeof(T) == 8)) {   \
                return hipErrorNotSupported;                          \
            } else {                                                  \
                if (nt) MTS_BATCH_LAUNCH(TYV, true, true, false);     \
                else MTS_BATCH_LAUNCH(TYV, true, false, false);       \
            }                                                         \
        } else {                                                      \
            if (nt) MTS_BATCH_LAUNCH(TYV, false, true, false);        \
            else MTS_BATCH_LAUNCH(TYV, false, false, false);          \
        }                                                             \
        return hipGetLastError();
    switch (ty) {
        MTS_BATCH_CASE(4)
        MTS_BATCH_CASE(5)
        MTS_BATCH_CASE(8)
        MTS_BATCH_CASE(12)
        case 13:
            if constexpr (sizeof(T) == 4) {
                if (diag) return hipErrorNotSupported;
                if (nt) MTS_BATCH_LAUNCH(13, false, true, false);
                else MTS_BATCH_LAUNCH(13, false, false, false);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
#undef MTS_BATCH_CASE
#undef MTS_BATCH_LAUNCH
}

template hipError_t launch_step_tile_batch<float>(const BatchBox<float> *, int, uint32_t, int, int, int,
                                                  const StepCoef<float> *, bool, int, bool, bool, bool, hipStream_t);
template hipError_t launch_step_tile_batch<double>(const BatchBox<double> *, int, uint32_t, int, int, int,
                                                   const StepCoef<double> *, bool, int, bool, bool, bool,
                                                   hipStream_t);

template hipError_t launch_step_tile<float>(const Geom &, Fields<float>, Fields<float>, Moms<float>, Moms<float>,
                                            const StepCoef<float> &, bool, Partials, TileShape, float *, uint8_t *,
                                            uint32_t, bool, bool, bool, hipStream_t);
template hipError_t launch_step_tile<double>(const Geom &, Fields<double>, Fields<double>, Moms<double>, Moms<double>,
                                             const StepCoef<double> &, bool, Partials, TileShape, double *, uint8_t *,
                                             uint32_t, bool, bool, bool, hipStream_t);


// ===================================================================== persistent ensemble kernel
//
// A run of plain steps of every box of an ensemble in one launch: the
// workgroups stay resident and loop over the steps; in each step they claim
// the tiles of every box (the plain-step tile table) one at a time and then
// meet at a device-wide barrier before the next step reads what this one
// wrote.  The arithmetic is the per-step launches': the same tile function on
// the same tiles, so the fields come out bit for bit the same.  Diagnostic
// steps are not part of it (their fused tile needs every register a wave may
// hold; the loop state of this kernel would make it spill).

namespace {

// Wait until every workgroup of the grid has arrived.  The last one to arrive
// sets the arrival count back to zero and advances the generation.  A wait
// that outlasts limit_ticks (some workgroup never arrives: a grid larger than
// what stays resident) raises the error flag, and every workgroup then leaves
// at its next barrier instead of waiting for ever.  The agent-scope fences
// make each workgroup's stores visible to the other XCDs before it arrives,
// and theirs to it once it leaves.  Returns false once the flag is up.
__device__ __forceinline__ bool grid_sync(GridSync *gs, uint32_t nblocks, uint32_t &gen, uint64_t limit_ticks) {
    __shared__ int s_ok;
    __threadfence();   // every thread: its stores of this step, visible at agent scope
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        int ok = 1;
        const uint32_t g = gen;
        if (atomicAdd(&gs->count, 1u) == nblocks - 1) {
            atomicExch(&gs->count, 0u);
            __threadfence();
            atomicAdd(&gs->gen, 1u);
        } else {
            const uint64_t t0 = (uint64_t)wall_clock64();
            while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = 0;
                    break;
                }
                if ((uint64_t)wall_clock64() - t0 > limit_ticks) {
                    atomicExch(&gs->err, 1);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        if (__hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        s_ok = ok;
    }
    gen++;
    __syncthreads();
    __threadfence();   // every thread: the other workgroups' stores, visible from here on
    return s_ok != 0;
}

// A read of host-written tables (the box table, the coefficients) that no
// kernel writes: through the constant address space, so that the compiler
// takes the wave-uniform value into scalar registers (and may load it again
// rather than hold it) although the kernel stores elsewhere in its loops.
template <typename V>
__device__ __forceinline__ V ld_uniform(const V *p) {
    static_assert(sizeof(V) % 4 == 0, "whole words");
    const __attribute__((address_space(4))) uint32_t *s = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t w[sizeof(V) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(V) / 4); i++) w[i] = s[i];
    V v;
    __builtin_memcpy(&v, w, sizeof(V));
    return v;
}

template <typename T>
__device__ __forceinline__ Fields<T> fields_global(Fields<T> f) {
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        f.phi[sec] = as_global(f.phi[sec]);
#pragma unroll
        for (int i = 0; i < 3; i++) f.A[sec][i] = as_global(f.A[sec][i]);
    }
    return f;
}

template <typename T>
__device__ __forceinline__ Moms<T> moms_global(Moms<T> m) {
#pragma unroll
    for (int sec = 0; sec < 2; sec++) {
        m.pi[sec] = as_global(m.pi[sec]);
#pragma unroll
        for (int i = 0; i < 3; i++) m.E[sec][i] = as_global(m.E[sec][i]);
    }
    return m;
}

}  // namespace

// waves per SIMD the per-step launch of the same shape reaches; the loop state
// must not cost the persistent kernel any of them
template <typename T, int TY>
constexpr int persist_waves() {
    return sizeof(T) == 4 ? 4 : (TY <= 5 ? 2 : (TY == 8 ? 3 : 4));
}

// The next tile index for this workgroup (thread 0 claims it, all read it).
__device__ __forceinline__ unsigned long long persist_claim(GridSync *gs) {
    __shared__ unsigned long long s_idx;
    if (threadIdx.x == 0 && threadIdx.y == 0) s_idx = atomicAdd(&gs->next, 1ull);
    __syncthreads();
    const unsigned long long v = s_idx;
    __syncthreads();
    return v;
}

template <typename T, int TY, bool NT>
__global__ __launch_bounds__(64 * (TY + 3)) __attribute__((amdgpu_waves_per_eu(persist_waves<T, TY>())))
void persist_plain_kernel(PersistArgs<T> a) {
    __shared__ Lds<T, TY, NQ> L;
    NoFusedLds<T, TY> nofl;
    uint32_t gen = __hip_atomic_load(&a.sync->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Tiles are claimed one at a time from a counter that runs through every
    // step's tiles in turn (step j owns [j ntiles, (j + 1) ntiles)).  A
    // workgroup stops a step at its first claim past the step's range and
    // keeps that index for the step it belongs to, so every index is taken
    // exactly once and no tile waits for a slow neighbour's share.
    unsigned long long idx = persist_claim(a.sync);
    for (int j = 0; j < a.nsteps; j++) {
        if (j > 0 && !grid_sync(a.sync, gridDim.x, gen, a.limit_ticks)) return;
        const int parity = (a.parity0 + j) & 1;
        const int mpin = a.mpp ? (a.mcur0 + j) & 1 : a.mcur0, mpout = a.mpp ? 1 - mpin : mpin;
        const unsigned long long first = (unsigned long long)j * a.ntiles, end = first + a.ntiles;
        while (idx >= first && idx < end) {
            const uint32_t t = (uint32_t)(idx - first);
            int lo = 0, hi = a.nbox - 1;   // last box with blk0 <= t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (ld_uniform(&a.boxes[mid].blk0) <= t) lo = mid;
                else hi = mid - 1;
            }
            const BatchBox<T> *bx = a.boxes + lo;
            const Geom g = ld_uniform(&bx->g);
            const uint32_t lt = t - ld_uniform(&bx->blk0);
            const int ntx = ld_uniform(&bx->ntx), nty = ld_uniform(&bx->nty), TZ = ld_uniform(&bx->tz);
            const int tx = lt % ntx, ty_ = (lt / ntx) % nty, tz = lt / (ntx * nty);
            const Fields<T> fin = fields_global(ld_uniform(&bx->f[parity]));
            const Fields<T> fout = fields_global(ld_uniform(&bx->f[1 - parity]));
            const Moms<T> mom = moms_global(ld_uniform(&bx->mom[mpin]));
            const Moms<T> mom_out = moms_global(ld_uniform(&bx->mom[mpout]));
            const StepCoef<T> c = ld_uniform(&a.coef[(size_t)j * a.nbox + lo]);
            double acc[6] = {};
            tile_step<T, false, TY, NT>(g, fin, fout, mom, mom_out, c, tx * 64, ty_ * TY, tz * TZ, TZ, L, acc,
                                        nullptr, nullptr, ld_uniform(&bx->plane), nofl);
            idx = persist_claim(a.sync);
        }
    }
}

__global__ void persist_reset_kernel(GridSync *gs) {
    gs->count = 0u;
    gs->err = 0;
    gs->next = 0ull;
}

hipError_t launch_persist_reset(GridSync *sync, hipStream_t st) {
    persist_reset_kernel<<<1, 1, 0, st>>>(sync);
    return hipGetLastError();
}

namespace {

template <typename T, int TY, bool NT>
hipError_t persist_blocks_t(int *per) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, persist_plain_kernel<T, TY, NT>, 64 * (TY + 3), 0);
}

template <typename T, int TY>
hipError_t persist_launch_t(const PersistArgs<T> &a, bool nt, uint32_t grid, hipStream_t st) {
    const dim3 block(64, TY + 3, 1);
    if (nt) persist_plain_kernel<T, TY, true><<<grid, block, 0, st>>>(a);
    else persist_plain_kernel<T, TY, false><<<grid, block, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t persist_max_blocks(bool fp64, int ty, bool nt, int *blocks) {
    int dev = 0, cus = 0, per = 0;
    *blocks = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
#define MTS_PERSIST_Q(TV, TYV) (nt ? persist_blocks_t<TV, TYV, true>(&per) : persist_blocks_t<TV, TYV, false>(&per))
    if (fp64) {
        switch (ty) {
            case 4: e = MTS_PERSIST_Q(double, 4); break;
            case 5: e = MTS_PERSIST_Q(double, 5); break;
            case 8: e = MTS_PERSIST_Q(double, 8); break;
            case 12: e = MTS_PERSIST_Q(double, 12); break;
            default: return hipSuccess;
        }
    } else {
        switch (ty) {
            case 4: e = MTS_PERSIST_Q(float, 4); break;
            case 5: e = MTS_PERSIST_Q(float, 5); break;
            case 8: e = MTS_PERSIST_Q(float, 8); break;
            case 12: e = MTS_PERSIST_Q(float, 12); break;
            case 13: e = MTS_PERSIST_Q(float, 13); break;
            default: return hipSuccess;
        }
    }
#undef MTS_PERSIST_Q
    if (e != hipSuccess) return e;
    *blocks = cus * per;
    return hipSuccess;
}

template <typename T>
hipError_t launch_persist(const PersistArgs<T> &a, int ty, bool nt, uint32_t grid, hipStream_t st) {
    if (grid == 0) return hipErrorInvalidValue;
    switch (ty) {
        case 4: return persist_launch_t<T, 4>(a, nt, grid, st);
        case 5: return persist_launch_t<T, 5>(a, nt, grid, st);
        case 8: return persist_launch_t<T, 8>(a, nt, grid, st);
        case 12: return persist_launch_t<T, 12>(a, nt, grid, st);
        case 13:
            if constexpr (sizeof(T) == 4) return persist_launch_t<T, 13>(a, nt, grid, st);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_persist<float>(const PersistArgs<float> &, int, bool, uint32_t, hipStream_t);
template hipError_t launch_persist<double>(const PersistArgs<double> &, int, bool, uint32_t, hipStream_t);

}  // namespace mts
