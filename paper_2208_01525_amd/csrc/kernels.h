// kernels.h -- internal interface between the host library (api.hip) and the
// gfx950 kernels (kernels.hip) of the U(1)xU(1) lattice update.
//
// Device state layout (one buffer owned by the caller), in units of
// `plane` elements of T (plane = sites rounded up to 64):
//   [ 0,10)  field copy 0: phi (cx, 2 planes), psi (cx, 2), A_x,A_y,A_z, B_x,B_y,B_z
//   [10,20)  field copy 1: same order (the drift writes the other copy)
//   [20,30)  momenta:      Pi (cx, 2), Psi (cx, 2), E_x,E_y,E_z, H_x,H_y,H_z
// Complex fields are interleaved (re, im); everything is structure of
// arrays with x fastest, site = x + nx (y + ny z).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mts {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
struct Fields {           // one copy of the fields, by sector (0 = p, 1 = q)
    cx<T> *phi[2];
    T *A[2][3];
};

template <typename T>
struct Moms {             // momenta at half steps, by sector
    cx<T> *pi[2];
    T *E[2][3];
};

struct Geom {
    int32_t nx, ny, nz;
    uint32_t nxy;         // nx * ny
};

// Per-step coefficients, computed in double on the host and cast to T once.
template <typename T>
struct StepCoef {
    T h, inv_h, inv_h2, inv_h3, k;
    T cpi, kpi;           // (1 - delta)/(1 + delta), k/(1 + delta)
    T cE, kE;             // (1 - omega)/(1 + omega), k/(1 + omega)
    T lamh[2];            // a^{2s} lambda_0 / 2
    T kap;                // a^{2s} kappa_0
    T sig2[2];            // sigma^2
    T cur[2];             // 2 e_0^2 a^{2s} / h
    // integer-time diagnostics
    T a2s, am2s;          // a^{2s}, a^{-2s}
    T inv_2e2[2];         // 1 / (2 e_0^2)
    T inv_e2h4[2];        // 1 / (e_0^2 h^4)
    T lam4[2];            // lambda_0 / 4
    T kap0;               // kappa_0
    T gsig[2];            // Gauss-law coupling 2 e_0^2 a^{2s} (1 + delta)/(1 + omega)
};

// Reduction slots of one diagnostic record (FP64 partials per block).
enum Slot {
    SL_EPS = 0, SL_LAG, SL_KL, SL_GL, SL_KV, SL_GV,
    SL_GAUSS_ABS_P, SL_GAUSS_ABS_Q, SL_GAUSS_SCALE_P, SL_GAUSS_SCALE_Q,
    SL_WIND_P, SL_WIND_Q, SL_OV_P, SL_OV_Q,
    SL_FIX_P, SL_FIX_Q,   // sum |W| of the sites the fused path left to the fix-up kernel
    NSLOT = 16
};

// Packed |W| byte of a site: |W_x|, |W_y|, |W_z| in two bits each; the fused
// diagnostic step sets WABS_FIX where the fix-up kernel must evaluate the
// site's windings.
constexpr uint8_t WABS_FIX = 0x40;

// Where the partials of one diagnostic step go.
struct Partials {
    double *base;         // [NSLOT][maxblk]
    uint32_t maxblk;
};

// ---- launch wrappers (all enqueue on `st`, return the launch error) ----

// One leapfrog step: reads `in` (fields at n) and `mom` (momenta at n-1/2),
// writes momenta n+1/2 in place and fields n+1 into `out`.  With diag,
// also the integer-time energy / Lagrangian / velocity sums.
template <typename T>
hipError_t launch_step(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, const StepCoef<T> &c,
                       bool diag, Partials part, hipStream_t st);

// One forward-Euler step of the diffusive cooling flow: out = in + k force,
// momenta untouched (c built with kappa = 0, a = 1, k = the cooling step).
template <typename T>
hipError_t launch_cool(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, const StepCoef<T> &c, hipStream_t st);

// The same step with the z-marching LDS-tiled kernel: a workgroup owns a
// 64 x ty column of sites over tz planes; ty in {4, 8, 12}.
struct TileShape {
    int32_t ty, tz;
};
bool tile_supported(TileShape ts, bool fp64);
bool batch_tile_supported(TileShape ts, bool fp64);
uint32_t tile_blocks(const Geom &g, TileShape ts);
// With diag it also writes the phase arg(phi^n) of every site into
// alpha[2][plane] (NaN where phi = 0), the winding kernel's input.
// Bandwidth probes on a state buffer: a copy of the first `bytes_per_copy`
// bytes onto the next ones, and the update's access pattern (no stencil).
hipError_t launch_probe_copy(void *state, uint64_t bytes_per_copy, hipStream_t st);
template <typename T>
hipError_t launch_probe_pattern(T *state, uint64_t plane, uint32_t S, int in, bool nt, hipStream_t st);

// One forward-Euler step of the cooling flow with the tiled kernel: fields
// `in` -> `out`, momenta untouched.
template <typename T>
hipError_t launch_cool_tile(const Geom &g, Fields<T> in, Fields<T> out, const StepCoef<T> &c, TileShape ts,
                            hipStream_t st);

// nt selects streaming (non-temporal) stores for the outputs; pf loads the
// fields of plain steps one plane further ahead (FP32 diagnostic steps always do).
// Momenta are read from `mom` and written to `mom_out` (the same copy: in
// place).  xcd deals the tiles to the XCDs in contiguous runs (block b of
// XCD b mod 8 takes that XCD's next tile in x, y, z order); without it block
// b takes tile b, the hardware's round-robin order.  Results do not depend
// on it.
// With diag and a non-null wabs (FP32, rows 4, 5 or 8, mom_out a different
// copy from mom) the windings of the input fields (packed |W| into wabs) and
// the Gauss residual are computed in the same pass, into partial slots
// SL_EPS .. SL_WIND_Q; alpha is then unused.
template <typename T>
hipError_t launch_step_tile(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> mom, Moms<T> mom_out,
                            const StepCoef<T> &c, bool diag, Partials part, TileShape ts, T *alpha, uint8_t *wabs,
                            uint32_t plane, bool nt, bool pf, bool xcd, hipStream_t st);

// Two steps in one sweep (temporal blocking, FP32): reads fields n from
// `in` and momenta n - 1/2 from `min_`, writes fields n + 2 to `out` and
// momenta n + 3/2 to `mout` (all four distinct); c1, c2 are the
// coefficients of steps n and n + 1.  A workgroup owns 64 x ts.ty sites
// (ty in {3, 7}) over ts.tz planes.  FP64 returns hipErrorNotSupported.
bool pair_tile_supported(TileShape ts);
template <typename T>
hipError_t launch_step_pair(const Geom &g, Fields<T> in, Fields<T> out, Moms<T> min_, Moms<T> mout,
                            const StepCoef<T> &c1, const StepCoef<T> &c2, TileShape ts, bool nt, hipStream_t st);

// One box of an ensemble advanced by a single launch.
template <typename T>
struct BatchBox {
    Geom g;
    Fields<T> f[2];       // field copies 0 and 1
    Moms<T> mom[2];       // momentum copies 0 and 1 (both the state buffer's without a second copy)
    Partials part;        // this box's partials (box-local block index)
    T *alpha;             // this box's phase scratch [2][plane]
    uint8_t *wabs;        // this box's packed |W| bytes (fused diagnostic steps)
    uint32_t plane;
    int32_t ntx, nty, ntz, tz;
    uint32_t blk0;        // first block of this box in the launch
};
// Fields from copy `parity` to the other; momenta from copy `mpin` to copy
// `mpout` (equal: in place).  With diag and fused (FP32, ty 8, mpout != mpin)
// the windings and the Gauss residual are computed in the same pass, as
// launch_step_tile does with wabs.
template <typename T>
hipError_t launch_step_tile_batch(const BatchBox<T> *boxes_dev, int nbox, uint32_t nblk, int parity, int mpin,
                                  int mpout, const StepCoef<T> *coef_dev, bool diag, int ty, bool nt, bool xcd,
                                  bool fused, hipStream_t st);

// One box of an ensemble in the batched post-step launches of a fused
// diagnostic step: the fix-up of the windings, the cells, the overlap and the
// reduction each run as one launch over all boxes.
template <typename T>
struct BatchPost {
    Geom g;
    Fields<T> f[2];       // field copies 0 and 1 (the step's input copy is `parity`)
    Partials part;
    uint8_t *wabs, *cells;
    uint32_t *fixlist;    // the box's list of marked sites (fix-up)
    uint64_t *bits;       // occupancy words (nx % 64 == 0); null: the byte overlap
    uint32_t plane, nwords;
    int32_t radius;
    T h;
    const uint32_t *nblk; // the box's partial counts per slot (fused path)
    double *ring;         // the box's record ring [RING_CAP][NSLOT]
    uint32_t blk_fix, blk_cells, blk_ov;   // the box's first block in each batched launch
};
uint32_t cells_blocks(const Geom &g);
// Records go to ring + ring_idx * NSLOT of every box.
template <typename T>
hipError_t launch_post_batch(const BatchPost<T> *boxes_dev, int nbox, uint32_t nfix, uint32_t ncells, uint32_t nov,
                             int parity, uint32_t ring_idx, hipStream_t st);

// ---- persistent ensemble kernel: a run of plain steps of every box in one launch
//
// Device state of the grid barrier.  count and err are cleared by
// launch_persist_reset before each launch (a kernel, so that a captured graph
// holds no memset node); gen only ever grows.
struct GridSync {
    uint32_t count;              // workgroups arrived at the current barrier
    uint32_t gen;                // barriers completed
    int32_t err;                 // 1: a barrier wait ran out (the grid was not co-resident)
    uint32_t pad;
    unsigned long long next;     // tiles claimed so far in this launch (step j's are j ntiles ...)
};

template <typename T>
struct PersistArgs {
    const BatchBox<T> *boxes;    // the plain-step tile table (rows ty)
    int32_t nbox;
    uint32_t ntiles;             // tiles of all boxes per step
    const StepCoef<T> *coef;     // [nsteps][nbox]
    int32_t nsteps;
    int32_t parity0, mcur0;      // field copy and momentum copy read by the first step
    int32_t mpp;                 // momenta to the other copy every step (else in place)
    GridSync *sync;
    uint64_t limit_ticks;        // longest barrier wait, in wall-clock ticks
};

// Largest co-resident grid of the persistent kernel of this shape on the
// current device (occupancy query times the compute units); 0 for a shape
// it does not support.
hipError_t persist_max_blocks(bool fp64, int ty, bool nt, int *blocks);
hipError_t launch_persist_reset(GridSync *sync, hipStream_t st);
template <typename T>
hipError_t launch_persist(const PersistArgs<T> &a, int ty, bool nt, uint32_t grid, hipStream_t st);

// Phase alpha = arg(phi) of every site and sector into alpha[2][plane]
// (NaN where phi = 0), input of the winding kernel.
template <typename T>
hipError_t launch_phase(const Geom &g, Fields<T> f, T *alpha, uint32_t plane, hipStream_t st);

// Windings of `f` (packed |W| per sector into wabs[2][plane] bytes, sum |W|
// into partials) and the Gauss residual of (f, mom) with g_sigma.
// If `signed_out` is non-null the signed windings go there as int8[6][plane]
// and nothing else is written.
template <typename T>
hipError_t launch_wind_gauss(const Geom &g, Fields<T> f, Moms<T> mom, const T *alpha, T h, T inv_h,
                             const double gcoef[2], uint8_t *wabs, uint32_t plane, int8_t *signed_out, Partials part,
                             hipStream_t st);
uint32_t wind_blocks(const Geom &g);

// Sites the fused diagnostic step marked WABS_FIX: their windings evaluated
// with the guarded link phases of the post-step kernel, bytes rewritten,
// sum |W| into slots SL_FIX_P / SL_FIX_Q (wind_fix_blocks partials).
// The fix-up of the fused windings: a scan that lists the marked sites,
// then a pass that evaluates the list (FIX_PROC_BLOCKS blocks per box).
// list: FIX_LIST_WORDS words per box (a count per scan block, then each
// block's segment of entries).  wind_fix_blocks: the partials of the SL_FIX
// slots (scan blocks, then the evaluation blocks); wind_fix_scan_blocks: the
// scan's.
constexpr uint32_t FIX_LIST_WORDS = 1024u + 1024u * 1024u;
constexpr uint32_t FIX_PROC_BLOCKS = 128;
uint32_t wind_fix_blocks(const Geom &g);
uint32_t wind_fix_scan_blocks(const Geom &g);

// FP64 diagnostic steps: windings (wrap counts, flagged sites marked for the
// fix-up) and the Gauss residual in one z-marching pass of 64 x 8 tiles;
// partials SL_GAUSS_ABS_P .. SL_WIND_Q per block (wind_tile_blocks).
uint32_t wind_tile_blocks(const Geom &g);
template <typename T>
hipError_t launch_wind_gauss_tile(const Geom &g, Fields<T> f, Moms<T> mom, T h, T inv_h, const double gcoef[2],
                                  uint8_t *wabs, uint32_t plane, Partials part, hipStream_t st);
template <typename T>
hipError_t launch_wind_fix(const Geom &g, Fields<T> f, T h, uint8_t *wabs, uint32_t plane, Partials part, uint32_t *list,
                           hipStream_t st);

// Cell values from packed |W| (cells[2][plane] bytes) and, when nx is a
// multiple of 64, the 64-cell occupancy words bits[2][overlap_words]; then
// the overlap counts.
bool overlap_uses_bits(const Geom &g);
uint32_t overlap_words(const Geom &g);
uint32_t overlap_blocks(const Geom &g);
hipError_t launch_cells(const Geom &g, const uint8_t *wabs, uint8_t *cells, uint64_t *bits, uint32_t plane,
                        hipStream_t st);
hipError_t launch_overlap(const Geom &g, const uint8_t *cells, const uint64_t *bits, uint32_t plane, int radius,
                          Partials part, hipStream_t st);

// Robust-method regions of the fast-method pq cells (union-find): region
// sizes into sizes[0 .. min(*n_out, cap)), *n_out = number of regions.
// parent and count are scratch of one uint32 per site.
hipError_t launch_segments(const Geom &g, const uint8_t *cells, uint32_t plane, int radius, uint32_t *parent,
                           uint32_t *count, uint32_t *sizes, uint32_t *n_out, uint32_t cap, hipStream_t st);

// Fixed-order FP64 sum of every slot's partials into rec[NSLOT].
hipError_t launch_reduce(Partials part, const uint32_t *nblk_per_slot_dev, double *rec, hipStream_t st);

// Random-phase initial conditions into field copy `f` and momenta `mom`.
template <typename T>
hipError_t launch_init(const Geom &g, Fields<T> f, Moms<T> mom, uint64_t seed, double sig_p, double sig_q,
                       hipStream_t st);

// Gather the 20 components (host exchange order) of n sites into out[n][20].
template <typename T>
hipError_t launch_gather(Fields<T> f, Moms<T> mom, const uint64_t *sites, int n, double *out, hipStream_t st);

// Number of blocks the per-site kernels use for geometry g (partials needed).
uint32_t site_blocks(const Geom &g);

}  // namespace mts
