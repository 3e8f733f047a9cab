// post.h -- per-block bodies of the post-step diagnostic kernels of the
// U(1)xU(1) lattice update (Correia & Martins, arXiv:2208.01525, Sec. III.A-B
// windings, cells and bound-state overlap), and the fixed-order final
// reduction, shared by the standalone launches, the batched launches over an
// ensemble and the persistent ensemble kernel.  A "block" here is 256
// threads (four waves): a larger workgroup runs several at once, one per
// group of four waves, and the partial sums come out the same.
#pragma once
#include "device.h"
#include "kernels.h"

namespace mts {

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Windings through the three faces whose lower corner is site s (W_x: the yz
// face, W_y: zx, W_z: xy) from the phases of the seven corners involved
// (a0 at s, ax at s + x, ..., ayz at s + y + z), the link angles / h of the
// nine links (A*0 at s, A*_p* at the neighbour), the guarded link phases and
// the unwrapped plaquette angles.
template <typename T>
__device__ __forceinline__ void face_windings(T h, const cx<T> *P, T a0, T ax, T ay, T az, T axy, T axz, T ayz, T Ax0,
                                              T Ay0, T Az0, T Ay_px, T Az_px, T Ax_py, T Az_py, T Ax_pz, T Ay_pz,
                                              uint32_t s, uint32_t s_x, uint32_t s_y, uint32_t s_z, uint32_t s_xy,
                                              uint32_t s_xz, uint32_t s_yz, int &Wx, int &Wy, int &Wz) {
    const T inv2pi = T(0.5) / Pi<T>::v;
    const T hx = h * Ax0, hy = h * Ay0, hz = h * Az0;
    const T hy_px = h * Ay_px, hz_px = h * Az_px;
    const T hx_py = h * Ax_py, hz_py = h * Az_py;
    const T hx_pz = h * Ax_pz, hy_pz = h * Ay_pz;
    const T chx = link_chi(a0, ax, hx, P, s, s_x);
    const T chy = link_chi(a0, ay, hy, P, s, s_y);
    const T chz = link_chi(a0, az, hz, P, s, s_z);
    const T chy_px = link_chi(ax, axy, hy_px, P, s_x, s_xy);
    const T chz_px = link_chi(ax, axz, hz_px, P, s_x, s_xz);
    const T chx_py = link_chi(ay, axy, hx_py, P, s_y, s_xy);
    const T chz_py = link_chi(ay, ayz, hz_py, P, s_y, s_yz);
    const T chx_pz = link_chi(az, axz, hx_pz, P, s_z, s_xz);
    const T chy_pz = link_chi(az, ayz, hy_pz, P, s_z, s_yz);
    // unwrapped plaquette angles h [A_mu(x) + A_nu(x+mu) - A_mu(x+nu) - A_nu(x)]
    const T txy = plaq(h, Ax0, Ay_px, Ax_py, Ay0);
    const T tyz = plaq(h, Ay0, Az_py, Ay_pz, Az0);
    const T tzx = plaq(h, Az0, Ax_pz, Az_px, Ax0);
    Wz = (int)rint_t(((((chx + chy_px) - chx_py) - chy) + txy) * inv2pi);
    Wx = (int)rint_t(((((chy + chz_py) - chy_pz) - chz) + tyz) * inv2pi);
    Wy = (int)rint_t(((((chz + chx_pz) - chz_px) - chx) + tzx) * inv2pi);
}

__device__ __forceinline__ uint8_t pack_wabs(int Wx, int Wy, int Wz) {
    return (uint8_t)(min(abs(Wx), 3) | (min(abs(Wy), 3) << 2) | (min(abs(Wz), 3) << 4));
}


// Deterministic sum of NV doubles over a group of four waves (one 256-thread
// block of the post-step kernels; a larger block holds several groups, each
// one virtual block): wave64 shuffles, then the group's waves in order through
// LDS; the group's first NV threads write partial[slot0 + v][blk] when valid.
// The same operations in the same order as block_sum_store over four waves.
// Every thread of the block takes part (two barriers).
template <int NV>
__device__ __forceinline__ void group_sum_store(double (&v)[NV], Partials part, int slot0, uint32_t blk, int group,
                                                bool valid) {
    __shared__ double red[16][NV];
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
    const int gl = lane - 256 * group;   // thread within the group
    if (valid && gl >= 0 && gl < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 4; w++) t += red[4 * group + w][gl];
        part.base[(size_t)(slot0 + gl) * part.maxblk + blk] = t;
    }
    __syncthreads();
}

constexpr int FIX_SITES = 16;   // sites per thread and pass of the fix-up scan (one 16-byte load per sector)
constexpr uint32_t FIX_CHUNK = 256 * FIX_SITES;   // sites per (virtual) block and pass
constexpr uint32_t FIX_MAX_BLOCKS = 1024;

// Blocks of the fix-up scan of a box of S sites: one pass each up to
// FIX_MAX_BLOCKS, then several passes per block.  Nearly every byte it reads
// is unmarked, so the scan is a stream of 16-byte loads.
__host__ __device__ inline uint32_t fix_blocks_of(uint32_t S) {
    const uint32_t chunks = (S + FIX_CHUNK - 1) / FIX_CHUNK;
    return chunks < FIX_MAX_BLOCKS ? chunks : FIX_MAX_BLOCKS;
}

// One of two values, both passed by value: the sector of a listed site is a
// per-lane value, and indexing the pointer table with it would take an
// address inside the table (a per-lane pointer load from the argument
// block, or, for a table built in the kernel, a per-thread copy in scratch).
template <typename V>
__device__ __forceinline__ V pick(bool second, V a, V b) {
    return second ? b : a;
}

// One marked site of one sector: its three faces evaluated as the post-step
// kernel does (FP64 from the complex products where the guard asks for it),
// its byte rewritten; returns |Wx| + |Wy| + |Wz|.
template <typename T>
__device__ __forceinline__ int fix_site(const Geom &g, const Fields<T> &f, T h, uint8_t *wabs, uint32_t plane, int sec,
                                        uint32_t s) {
    const bool q = sec != 0;
    const cx<T> *P = pick<const cx<T> *>(q, f.phi[0], f.phi[1]);
    const T *Ax = pick<const T *>(q, f.A[0][0], f.A[1][0]), *Ay = pick<const T *>(q, f.A[0][1], f.A[1][1]),
            *Az = pick<const T *>(q, f.A[0][2], f.A[1][2]);
    const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / g.nxy;
    const uint32_t nx = g.nx, nxy = g.nxy;
    const int xp = wrap1(x + 1, g.nx), yp = wrap1(y + 1, g.ny), zp = wrap1(z + 1, g.nz);
    const uint32_t s_x = xp + nx * y + nxy * z, s_y = x + nx * yp + nxy * z, s_z = x + nx * y + nxy * zp;
    const uint32_t s_xy = xp + nx * yp + nxy * z, s_xz = xp + nx * y + nxy * zp;
    const uint32_t s_yz = x + nx * yp + nxy * zp;
    int Wx, Wy, Wz;
    face_windings(h, P, phase_of(P[s]), phase_of(P[s_x]), phase_of(P[s_y]), phase_of(P[s_z]), phase_of(P[s_xy]),
                  phase_of(P[s_xz]), phase_of(P[s_yz]), Ax[s], Ay[s], Az[s], Ay[s_x], Az[s_x], Ax[s_y], Az[s_y],
                  Ax[s_z], Ay[s_z], s, s_x, s_y, s_z, s_xy, s_xz, s_yz, Wx, Wy, Wz);
    wabs[(size_t)sec * plane + s] = pack_wabs(Wx, Wy, Wz);
    return abs(Wx) + abs(Wy) + abs(Wz);
}

// The fix-up in two passes.  Marked sites are rare per wave but, at early
// times, not rare per box, and each costs a chain of FP64 work: evaluated by
// the scanning thread, one lane at a time, they held a wave for the sum of
// its sites' chains.  So the scan only lists them (entry: sector << 31 |
// site; the box has fewer than 2^31 sites), and a second pass evaluates the
// list with every lane busy.  Each scan block owns a segment of FIX_SEG
// entries and counts into LDS (one global counter for the whole box had
// serialised its atomics: 0.49 ms at 512^3); it writes its count at the end,
// so the list needs no clearing.  A block's entries past FIX_SEG are
// evaluated by the scan itself.  Both passes add integer |W| sums, so the
// partials do not depend on the order of the list.
//   list: counts[FIX_MAX_BLOCKS], then entries[FIX_MAX_BLOCKS][FIX_SEG]
constexpr uint32_t FIX_SEG = 1024;
static_assert(FIX_LIST_WORDS == FIX_MAX_BLOCKS + FIX_MAX_BLOCKS * FIX_SEG, "list layout");

// Scan: virtual block lblk of nblk walks the chunks lblk, lblk + nblk, ...
// (partials at lblk; zero unless its segment overflowed).  Every lane of
// each wave takes part (wave-wide prefix sum and ballot).
template <typename T>
__device__ __forceinline__ void fix_scan_block(const Geom &g, const Fields<T> &f, T h, uint8_t *wabs, uint32_t plane,
                                               Partials part, uint32_t lblk, uint32_t nblk, uint32_t tid,
                                               uint32_t *list, int group = 0, bool valid = true) {
    __shared__ uint32_t s_cnt[16];
    const uint32_t S = g.nxy * (uint32_t)g.nz;
    const int lane = tid & 63;
    if (tid == 0) s_cnt[group] = 0u;
    __syncthreads();
    uint32_t *seg = list + FIX_MAX_BLOCKS + (size_t)lblk * FIX_SEG;
    double acc[2] = {0, 0};
    for (uint32_t c = lblk; valid && c * FIX_CHUNK < S; c += nblk) {
        const uint32_t s0 = c * FIX_CHUNK + tid * FIX_SITES;
        uint32_t m[2] = {0, 0};   // bit k: site s0 + k is marked
        if (s0 < S) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const uint4 v = *reinterpret_cast<const uint4 *>(wabs + (size_t)sec * plane + s0);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        if ((w[q] >> (8 * b)) & WABS_FIX) m[sec] |= 1u << (4 * q + b);
                if (s0 + FIX_SITES > S) m[sec] &= (1u << (S - s0)) - 1u;   // the plane's padding
            }
        }
        const uint32_t n = (uint32_t)(__popc(m[0]) + __popc(m[1]));
        if (__ballot(n != 0) == 0) continue;   // the common case: nothing marked in the wave's sites
        uint32_t incl = n;                     // inclusive prefix sum over the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
            if (lane >= d) incl += t;
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
        uint32_t base = 0;
        if (lane == 63) base = atomicAdd(&s_cnt[group], total);
        base = (uint32_t)__shfl((int)base, 63, 64);
        uint32_t idx = base + incl - n;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            uint32_t mm = m[sec];
            while (mm) {
                const int k = __ffs(mm) - 1;
                mm &= mm - 1;
                const uint32_t s = s0 + (uint32_t)k;
                if (idx < FIX_SEG) seg[idx] = ((uint32_t)sec << 31) | s;
                else acc[sec] += (double)fix_site(g, f, h, wabs, plane, sec, s);
                idx++;
            }
        }
    }
    __syncthreads();
    if (tid == 0 && valid) list[lblk] = s_cnt[group];
    group_sum_store<2>(acc, part, SL_FIX_P, lblk, group, valid);
}

// Evaluation of the listed sites of a box whose scan had nscan blocks: block
// pblk of nproc (256 threads) deals the entries of all segments out evenly,
// by a prefix sum of the segment counts in LDS, so every lane holds an entry
// while entries remain (partials at pblk0 + pblk).
template <typename T>
__device__ __forceinline__ void fix_proc_block(const Geom &g, const Fields<T> &f, T h, uint8_t *wabs, uint32_t plane,
                                               Partials part, uint32_t nscan, uint32_t pblk0, uint32_t pblk,
                                               uint32_t nproc, uint32_t tid, const uint32_t *list) {
    __shared__ uint32_t s_pre[FIX_MAX_BLOCKS + 1];   // segment counts, then their exclusive prefix sums
    __shared__ uint32_t s_part[256];
    for (uint32_t i = tid; i < FIX_MAX_BLOCKS; i += 256) s_pre[i] = i < nscan ? min(list[i], FIX_SEG) : 0u;
    __syncthreads();
    uint32_t loc[4], sum = 0;   // thread tid holds segments 4 tid .. 4 tid + 3
#pragma unroll
    for (int k = 0; k < 4; k++) {
        loc[k] = sum;
        sum += s_pre[4 * tid + k];
    }
    s_part[tid] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < 256; d <<= 1) {   // inclusive scan of the 256 sums
        const uint32_t v = tid >= d ? s_part[tid - d] : 0u;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    const uint32_t base = s_part[tid] - sum, total = s_part[255];
#pragma unroll
    for (int k = 0; k < 4; k++) s_pre[4 * tid + k] = base + loc[k];
    if (tid == 0) s_pre[FIX_MAX_BLOCKS] = total;
    __syncthreads();
    double acc[2] = {0, 0};
    for (uint32_t e = pblk * 256 + tid; e < total; e += nproc * 256) {
        uint32_t lo = 0, hi = nscan - 1;   // last segment with s_pre[lo] <= e
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t entry = list[FIX_MAX_BLOCKS + (size_t)lo * FIX_SEG + (e - s_pre[lo])];
        const int sec = (int)(entry >> 31);
        acc[sec] += (double)fix_site(g, f, h, wabs, plane, sec, entry & 0x7FFFFFFFu);
    }
    group_sum_store<2>(acc, part, SL_FIX_P, pblk0 + pblk, 0, true);
}


constexpr int CZ = 16;


__device__ __forceinline__ void cells_block(const Geom &g, const uint8_t *wabs, uint8_t *cells, uint64_t *bits,
                                            uint32_t plane, uint32_t nwords, uint32_t blk, int tx, int ty) {
    const uint32_t gx = (g.nx + 63) / 64, gy = (g.ny + 3) / 4;
    const uint32_t bx = blk % gx, by = (blk / gx) % gy, bz = blk / (gx * gy);
    const int x = bx * 64 + tx;
    const int y = by * 4 + ty;
    const bool in = x < g.nx && y < g.ny;
    const int z0 = bz * CZ, z1 = min(z0 + CZ, g.nz);
    const uint32_t col = in ? (uint32_t)x + (uint32_t)g.nx * (uint32_t)y : 0u;
    const uint32_t colx = in ? (uint32_t)wrap1(x + 1, g.nx) + (uint32_t)g.nx * (uint32_t)y : 0u;
    const uint32_t coly = in ? (uint32_t)x + (uint32_t)g.nx * (uint32_t)wrap1(y + 1, g.ny) : 0u;
    uint32_t w0[2] = {0, 0};
    if (in) {
#pragma unroll
        for (int sec = 0; sec < 2; sec++) w0[sec] = wabs[(size_t)sec * plane + col + g.nxy * (uint32_t)z0];
    }
    for (int z = z0; z < z1; z++) {
        uint32_t n[2] = {0, 0};
        if (in) {
            const uint32_t off = g.nxy * (uint32_t)z, offz = g.nxy * (uint32_t)wrap1(z + 1, g.nz);
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const uint8_t *w = wabs + (size_t)sec * plane;
                const uint32_t wz = w[col + offz];
                n[sec] = (w0[sec] & 3) + (w[colx + off] & 3) + ((w0[sec] >> 2) & 3) + ((w[coly + off] >> 2) & 3) +
                         ((w0[sec] >> 4) & 3) + ((wz >> 4) & 3);
                cells[(size_t)sec * plane + col + off] = (uint8_t)n[sec];
                w0[sec] = wz;
            }
        }
        if (bits) {   // nx % 64 == 0: the wave is one 64-cell word of one row
            const uint64_t mp = __ballot(in && n[0] > 0), mq = __ballot(in && n[1] > 0);
            if (tx == 0 && in) {
                const uint32_t wi = (uint32_t)(x / 64) + (uint32_t)(g.nx / 64) * ((uint32_t)y + (uint32_t)g.ny * z);
                bits[wi] = mp;
                bits[(size_t)nwords + wi] = mq;
            }
        }
    }
}


// Rows whose width is a multiple of 256, or exactly 128, take four cells per
// lane: a wave covers 256 cells of one row (or two rows of 128, one per
// half-wave), a block of 64 x 4 lanes four such waves, and it walks CZ
// planes, reading the packed |W| bytes as 32-bit words and adding the six
// face fields of four cells at once (each field is at most 3, so no byte of
// the sum carries into the next).  The x neighbour of a lane's last cell is
// the next lane's first byte (a shuffle; a row's last lane reads it).  With
// bits, lane k < 4 assembles the 64-cell word k of the wave's 256 cells from
// four ballots.
__host__ __device__ inline bool cells_by_words(const Geom &g) { return g.nx % 256 == 0 || g.nx == 128; }
__host__ __device__ inline int cells_rows_per_wave(const Geom &g) { return g.nx == 128 ? 2 : 1; }

__device__ __forceinline__ uint64_t spread4(uint32_t v) {   // bit i of v (16 bits) to bit 4 i
    uint64_t x = v & 0xFFFFu;
    x = (x | (x << 24)) & 0x000000FF000000FFull;
    x = (x | (x << 12)) & 0x000F000F000F000Full;
    x = (x | (x << 6)) & 0x0303030303030303ull;
    x = (x | (x << 3)) & 0x1111111111111111ull;
    return x;
}

__device__ __forceinline__ void cells4_block(const Geom &g, const uint8_t *wabs, uint8_t *cells, uint64_t *bits,
                                             uint32_t plane, uint32_t nwords, uint32_t blk, int lane, int ty) {
    const int rpw = cells_rows_per_wave(g), lpr = 64 / rpw;          // rows per wave, lanes per row
    const uint32_t gx = rpw == 2 ? 1u : (uint32_t)g.nx / 256, gy = (g.ny + 4 * rpw - 1) / (4 * rpw);
    const uint32_t bx = blk % gx, by = (blk / gx) % gy, bz = blk / (gx * gy);
    const int lx = lane % lpr;
    const int x = (int)bx * 256 + 4 * lx;
    const int y0 = ((int)by * 4 + ty) * rpw;   // the wave's first row
    if (y0 >= g.ny) return;                    // uniform per wave; no barrier below: the wave may leave
    const int yl = y0 + lane / lpr;
    const bool in = yl < g.ny;                 // a second row past the box: loads stay in the first, no stores
    const int y = in ? yl : y0;
    const int z0 = bz * CZ, z1 = min(z0 + CZ, g.nz);
    const uint32_t col = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const uint32_t colx4 = (uint32_t)wrap1(x + 4, g.nx) + (uint32_t)g.nx * (uint32_t)y;   // a row's last lane only
    const uint32_t coly = (uint32_t)x + (uint32_t)g.nx * (uint32_t)wrap1(y + 1, g.ny);
    constexpr uint32_t M = 0x03030303u;
    uint32_t w0[2];
#pragma unroll
    for (int sec = 0; sec < 2; sec++)
        w0[sec] = *reinterpret_cast<const uint32_t *>(wabs + (size_t)sec * plane + col + g.nxy * (uint32_t)z0);
    for (int z = z0; z < z1; z++) {
        const uint32_t off = g.nxy * (uint32_t)z, offz = g.nxy * (uint32_t)wrap1(z + 1, g.nz);
        uint32_t n[2];
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            const uint8_t *w = wabs + (size_t)sec * plane;
            const uint32_t o = w0[sec];
            const uint32_t wz = *reinterpret_cast<const uint32_t *>(w + col + offz);
            const uint32_t wy = *reinterpret_cast<const uint32_t *>(w + coly + off);
            uint32_t nb = (uint32_t)__shfl_down((int)o, 1, 64) & 0xFFu;   // next lane's first cell
            if (lx == lpr - 1) nb = w[colx4 + off];
            const uint32_t wx = (o >> 8) | (nb << 24);
            n[sec] = (o & M) + (wx & M) + ((o >> 2) & M) + ((wy >> 2) & M) + ((o >> 4) & M) + ((wz >> 4) & M);
            if (in) *reinterpret_cast<uint32_t *>(cells + (size_t)sec * plane + col + off) = n[sec];
            w0[sec] = wz;
        }
        if (bits) {
#pragma unroll
            for (int sec = 0; sec < 2; sec++) {
                const uint32_t v = n[sec];
                uint64_t word = 0;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint64_t b = __ballot(((v >> (8 * j)) & 0xFFu) != 0);
                    word |= spread4((uint32_t)(b >> (16 * (lane & 3)))) << j;
                }
                const int wrow = y0 + lane * rpw / 4;   // word k < 4: row of the wave's k-th 64 cells
                if (lane < 4 && wrow < g.ny) {
                    const uint32_t xw = bx * 4 + (uint32_t)(lane % (4 / rpw));   // word index within the row
                    const uint32_t wi = xw + (uint32_t)(g.nx / 64) * ((uint32_t)wrow + (uint32_t)g.ny * (uint32_t)z);
                    bits[(size_t)sec * nwords + wi] = word;
                }
            }
        }
    }
}

// x-dilation of the word at (xw, y, z) by one cell with periodic wrap
__device__ __forceinline__ uint64_t dilate_x(const uint64_t *m, uint32_t row, int xw, int nw) {
    const uint64_t w = m[row + xw];
    const uint64_t l = m[row + (xw == 0 ? nw - 1 : xw - 1)], r = m[row + (xw + 1 == nw ? 0 : xw + 1)];
    return w | (w << 1) | (w >> 1) | (l >> 63) | (r << 63);
}

__device__ __forceinline__ void overlap_bits_block(const Geom &g, const uint64_t *bits, uint32_t nwords, int radius,
                                                   Partials part, uint32_t lblk, uint32_t tid, int group = 0,
                                                   bool valid = true) {
    const uint32_t i = lblk * 256 + tid;
    double acc[2] = {0, 0};
    if (valid && i < nwords) {
        const int nw = g.nx / 64;
        const int xw = i % nw, y = (i / nw) % g.ny, z = i / (nw * g.ny);
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            const uint64_t *own = bits + (size_t)sec * nwords, *oth = bits + (size_t)(1 - sec) * nwords;
            uint64_t d = 0;
            if (radius == 0) {
                d = oth[i];
            } else {
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++) {
                        const uint32_t row =
                            (uint32_t)nw * ((uint32_t)wrap1(y + dy, g.ny) + (uint32_t)g.ny * (uint32_t)wrap1(z + dz, g.nz));
                        d |= dilate_x(oth, row, xw, nw);
                    }
            }
            acc[sec] = (double)__popcll(own[i] & d);
        }
    }
    group_sum_store<2>(acc, part, SL_OV_P, lblk, group, valid);
}

// lblk = bx + gx (by + gy z): 64 x 4 columns of one plane
__device__ __forceinline__ void overlap_bytes_block(const Geom &g, const uint8_t *cells, uint32_t plane, int radius,
                                                    Partials part, uint32_t lblk, int tx, int ty, int group = 0,
                                                    bool valid = true) {
    const uint32_t gx = (g.nx + 63) / 64, gy = (g.ny + 3) / 4;
    const int x = (lblk % gx) * 64 + tx;
    const int y = ((lblk / gx) % gy) * 4 + ty;
    const int z = lblk / (gx * gy);
    double acc[2] = {0, 0};
    if (valid && x < g.nx && y < g.ny) {
        const uint32_t s = x + g.nx * y + g.nxy * z;
#pragma unroll
        for (int sec = 0; sec < 2; sec++) {
            if (cells[(size_t)sec * plane + s] == 0) continue;
            const uint8_t *o = cells + (size_t)(1 - sec) * plane;
            bool hit = false;
            for (int dz = -radius; dz <= radius && !hit; dz++) {
                const int zz = wrap1(z + dz, g.nz);
                for (int dy = -radius; dy <= radius && !hit; dy++) {
                    const int yy = wrap1(y + dy, g.ny);
                    for (int dx = -radius; dx <= radius && !hit; dx++) {
                        const int xx = wrap1(x + dx, g.nx);
                        hit = o[xx + g.nx * yy + g.nxy * zz] != 0;
                    }
                }
            }
            acc[sec] = hit ? 1.0 : 0.0;
        }
    }
    group_sum_store<2>(acc, part, SL_OV_P, lblk, group, valid);
}


// Fixed-order FP64 sum of one slot's partials into rec[slot]: virtual lane v
// (0..1023) sums partials v, v + 1024, ... (four interleaved running sums
// combined in a fixed order), then a fixed tree over the 1024 lanes.  A block
// of NTHR threads (NTHR >= 512) takes lanes tid and tid + NTHR, so every block
// size gives the same bits.
template <int NTHR>
__device__ __forceinline__ void reduce_lanes(Partials part, const uint32_t *nblk, double *rec, int slot) {
    static_assert(NTHR >= 512 && NTHR <= 1024, "two lanes per thread at most, 512 tree threads");
    __shared__ double red[1024];
    const uint32_t n = nblk[slot];
    const double *p = part.base + (size_t)slot * part.maxblk;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    for (int v = tid; v < 1024; v += NTHR) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        uint32_t i = v;
        for (; i + 3 * 1024 < n; i += 4 * 1024) {
            t0 += p[i];
            t1 += p[i + 1024];
            t2 += p[i + 2 * 1024];
            t3 += p[i + 3 * 1024];
        }
        for (; i < n; i += 1024) t0 += p[i];
        red[v] = (t0 + t1) + (t2 + t3);
    }
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) rec[slot] = red[0];
    __syncthreads();
}

}  // namespace mts
