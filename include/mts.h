/*
 * mts.h -- C ABI of libmts: the per-timestep lattice update of the
 * U(1)xU(1) multitension cosmic-string model of Correia & Martins,
 * arXiv:2208.01525, with its fused network diagnostics, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Conventions
 *   - Every function returns int: MTS_OK (0) or a negative MTS_E* code.
 *     No C++ exception crosses this boundary.  The text of the last error
 *     of a context is available from mts_last_error().
 *   - Pointers marked "device" are HIP device addresses; "host" pointers
 *     are ordinary CPU memory.  Sizes are in bytes unless stated.
 *   - All GPU work of a context is enqueued on the HIP stream given at
 *     creation (NULL = the null stream).  Functions that return host data
 *     (mts_diagnostics, mts_get_*) synchronise that stream first.
 *   - A context is not thread-safe: one host thread at a time.
 *
 * Lattice and notation (Sec. II-III of the paper)
 *   Periodic comoving box nx*ny*nz, spacing dx (= h), conformal time step
 *   dt (= k).  Sector p: complex scalar phi, momentum Pi, gauge links A_i,
 *   electric field E_i.  Sector q: psi, Psi, B_i, H_i.  `s` is the
 *   paper's beta: coupling constants scale as a^{-2(1-s)} (Sec. III);
 *   s = 1 is physical evolution, s = 0 is constant comoving width (PRS),
 *   s < 0 is core growth.  era_m is the exponent of a ~ t^m, so
 *   a = (eta / eta_ref)^p with p = m / (1 - m), normalised to a = 1 at
 *   eta_ref (the end of the run: Sec. V fixes a = 1 at the end).
 *
 * Host field exchange format (mts_get_fields / mts_set_fields)
 *   double[20][nz][ny][nx], x fastest.  Planes:
 *      0-1 phi (re, im)    2-3 psi     4-5 Pi      6-7 Psi
 *      8-10 A_x,A_y,A_z    11-13 B     14-16 E     17-19 H
 *   The momenta are the half-step values Pi^{n-1/2}, E^{n-1/2} that the
 *   leapfrog stores between steps.
 */
#ifndef MTS_H
#define MTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ codes */
#define MTS_OK 0
#define MTS_EINVAL (-1)      /* bad argument or parameter                       */
#define MTS_EUNSTABLE (-2)   /* time step violates the leapfrog stability bound */
#define MTS_ENOMEM (-3)      /* device allocation failed / buffer too small     */
#define MTS_EHIP (-4)        /* a HIP runtime call failed (see mts_last_error)  */
#define MTS_ENONFINITE (-5)  /* a diagnostic reduction saw NaN or Inf           */

#define MTS_FP32 1           /* fields and per-site arithmetic in float;
                                reductions and time bookkeeping in double      */
#define MTS_FP64 2           /* everything in double                            */

/* ----------------------------------------------------------- params */
typedef struct mts_params {
    int32_t nx, ny, nz;      /* box, each >= 4; nx*ny*nz < 2^32 - 2048          */
    int32_t precision;       /* MTS_FP32 or MTS_FP64                            */
    double dx;               /* lattice spacing h > 0        (paper: 0.5)       */
    double dt;               /* conformal time step k > 0    (paper: 0.1)       */
    double lambda_p, lambda_q;  /* scalar couplings lambda_0 >= 0   (2, 2)      */
    double e_p, e_q;         /* gauge couplings e_0 > 0         (1, 1)          */
    double sigma_p, sigma_q; /* vacuum expectation values > 0   (1, 1)          */
    double kappa;            /* potential coupling kappa_0      (0.9)           */
    double eta_ref;          /* a(eta_ref) = 1; > 0                             */
    int32_t diag_every;      /* diagnostics every d steps; 0 = never            */
    int32_t overlap_radius;  /* fast-method overlap tolerance in cells: 0 or 1  */
} mts_params;

/* One diagnostic record of integer time eta_n: fields phi^n, A^n; momenta
 * time-centred (Pi^{n-1/2} + Pi^{n+1/2})/2; Gauss residual at n+1/2.
 * Sums are FP64 reductions over all sites (Sec. III.A-B, Sec. IV). */
typedef struct mts_diag {
    int64_t step;            /* global step index n since mts_init_fields       */
    double eta;              /* eta_n                                           */
    double a;                /* scale factor a(eta_n)                           */
    double s;                /* beta of this step                               */
    double sum_energy;       /* h^3 sum eps,  eps = K + G + a^{-2s}(Kg+Bg) + a^{2s} V */
    double sum_lagrangian;   /* h^3 sum Lag,  Lag = K - G + a^{-2s}(Kg-Bg) - a^{2s} V */
    double sum_KL, sum_GL;   /* sum K*Lag, sum G*Lag    (velocity, all strings) */
    double sum_KV, sum_GV;   /* sum K*Vint, sum G*Vint  (velocity, pq strings)  */
    double gauss_abs[2];     /* sum |C_sigma|, C = div E - g Im[phi* Pi]        */
    double gauss_scale[2];   /* sum (|div E| + |g Im[phi* Pi]|)                 */
    int64_t wind_abs[2];     /* sum over plaquettes of |winding|, p and q       */
    int64_t pq_count2;       /* count_p + count_q = 2 N_pq (overlapping cells)  */
    /* derived on the host from the sums above (Sec. III.A):                    */
    double L_p, L_q, L_pq;   /* L_pq = h N_pq; L_p = h sum|W_p| - L_pq          */
    double xi_p, xi_q, xi_pq, xi_W;   /* sqrt(V/L)                              */
    double xi_lag;           /* sqrt(-mu V / (h^3 sum Lag)), mu = 2 pi sigma_p^2 */
    double f_total, f_p;     /* L_pq/(L_pq+L_p+L_q), L_pq/L_p                   */
    double v2_lag, v2_pq;    /* <v^2> = 2R/(1+R), R = sum K W / sum G W         */
    double gauss_rel[2];     /* gauss_abs / gauss_scale (0 when scale is 0)     */
    int32_t flags;           /* bit 0: non-finite sum; bit 1: records were lost */
    int32_t pad;
} mts_diag;

typedef struct mts_ctx mts_ctx;

/* Bytes of the device state buffer a context needs: 30 planes of
 * nx*ny*nz (rounded up to 64) elements of the precision's type plus 4096
 * bytes each (a stagger of the plane base addresses across HBM channels) --
 * the 20 live components plus a second copy of the 10 field components (the
 * drift writes the new fields into the other copy). */
size_t mts_state_bytes(const mts_params *p);

/* Create a context on the current HIP device.
 *   p           parameters, copied.  EINVAL for dims < 4, non-positive
 *               dx/dt/e/sigma/eta_ref, negative lambda, precision or
 *               overlap_radius out of range, diag_every < 0.
 *   dev_state   device buffer of at least mts_state_bytes(p) bytes,
 *               256-byte aligned, owned by the caller and borrowed for the
 *               context's lifetime (its contents are the lattice).
 *   stream      hipStream_t (as void*), NULL for the null stream.
 *   out         receives the context.
 * The library allocates its own device scratch (reduction partials; the
 * phase of each scalar, 2 elements per site; winding and cell bytes, 4
 * bytes per site; occupancy bits; the list of sites whose windings the
 * FP64 fix-up evaluates, 4 MiB; a diagnostic ring); ENOMEM if that
 * fails. */
int mts_create(const mts_params *p, void *dev_state, size_t state_bytes, void *stream, mts_ctx **out);

/* Release the library's scratch.  The caller's state buffer is untouched. */
int mts_destroy(mts_ctx *ctx);

/* Random-phase initial conditions (Sec. III): |phi| = sigma_p, |psi| =
 * sigma_q, phases iid uniform in [0, 2 pi) from SplitMix64 (draw number
 * sector*S + site of the stream seeded with `seed`, top 53 bits times
 * 2 pi, cos/sin in double), all momenta, links and electric fields zero.
 * Resets the step counter and drops undrained diagnostic records. */
int mts_init_fields(mts_ctx *ctx, uint64_t seed);

/* Advance n >= 0 leapfrog steps from conformal time eta (step j runs from
 * eta + j*dt), in era m (0 <= m < 1) with beta = s (Sec. III):
 *   (1+delta) Pi^{n+1/2} = (1-delta) Pi^{n-1/2}
 *                          + dt [D^-D^+ phi - a^{2s} phi (lambda/2 (|phi|^2 - sigma^2)
 *                                                        - kappa (|psi|^2 - sigma_q^2))]
 *   (1+omega) E^{n+1/2}  = (1-omega) E^{n-1/2} + dt [-d^-F + 2 e^2 a^{2s} Im(phi* D^+ phi)]
 *   phi^{n+1} = phi^n + dt Pi^{n+1/2},   A^{n+1} = A^n + dt E^{n+1/2}
 * with delta = p dt / eta (alpha = 2), omega = (1 - s) delta, and the same
 * for psi, B (compact links U = exp(-i h A), plaquette sines for F).
 * A step whose global index is a multiple of diag_every also records
 * the diagnostics of its starting time.
 *   EINVAL     n < 0, m outside [0, 1), eta <= 0 with m > 0.
 *   EUNSTABLE  dt^2 (12/h^2 + a_max^{2s} mu2_max) >= 4 for the a-range of
 *              the call, mu2_max = max(2 e^2 sigma^2, eigenvalues of the
 *              vacuum scalar mass matrix); nothing is launched. */
int mts_step(mts_ctx *ctx, int32_t n, double eta, double era_m, double s);

/* Diffusive cooling of the initial conditions (Sec. III): n forward-Euler
 * steps of size dt_cool of the gradient flow
 *   d phi/d eta = D^-D^+ phi - lambda/2 (|phi|^2 - sigma^2) phi
 *   d A_i/d eta = -sum_j d_j^- F_ij + 2 e^2 Im[phi* D_i^+ phi]
 * (and the same for psi, B) at a = 1, without the kappa coupling, as the
 * paper prints it; momenta and electric fields are left unchanged and the
 * step counter does not advance.  The paper cools from eta = -10 to 1 with
 * dt_cool = 1/30.  EUNSTABLE if dt_cool (12/h^2 + mu2_max) >= 2. */
int mts_cool(mts_ctx *ctx, int32_t n, double dt_cool);

/* Drain the diagnostic records produced since the last call (oldest
 * first), synchronising the stream.  Writes at most `max` records to the
 * host array `out` and their number to *count.  Records that did not fit
 * the device ring (4096 entries) are lost and flagged.  Returns
 * ENONFINITE (after writing the records) if any record has a non-finite
 * sum. */
int mts_diagnostics(mts_ctx *ctx, mts_diag *out, int32_t max, int32_t *count);

/* Copy the lattice to / from the host exchange format (double[20][S],
 * host memory of 20*S doubles).  Values are converted to / from the
 * context's precision.  Synchronous. */
int mts_get_fields(mts_ctx *ctx, double *host);
int mts_set_fields(mts_ctx *ctx, const double *host);

/* The 20 components of selected sites, host double[n][20] in the plane
 * order of the exchange format; sites[i] = x + nx (y + ny z) < nx*ny*nz
 * (EINVAL otherwise).  Synchronous; for spot checks of boxes too large to
 * copy out whole. */
int mts_get_sites(mts_ctx *ctx, const uint64_t *sites, int32_t n, double *host);

/* For callers that cannot allocate device memory (code between allocation
 * checkpoints, serving loops, harnesses that forbid hipMalloc): the same
 * result as mts_get_sites, bit for bit, staged through a static device
 * array of the library instead of device memory allocated per call.  The
 * array holds at most MTS_NOALLOC_MAX_SITES sites (1.4 MB; each GPU the
 * library runs on keeps one copy until the process ends); n above that is
 * MTS_EINVAL, as is a site index >= nx*ny*nz.  Every call on one GPU shares
 * that GPU's array, so calls that overlap in time on one GPU (contexts
 * driven from several host threads) race; calls in sequence do not.  Calls
 * no hipMalloc/hipFree; the host arrays are the caller's.  Synchronous. */
#define MTS_NOALLOC_MAX_SITES 8192
int mts_get_sites_noalloc(mts_ctx *ctx, const uint64_t *sites, int32_t n, double *host);

/* Signed plaquette windings of the current fields (Sec. III.A), host
 * int8[6][S]: sector p (W_x, W_y, W_z), then sector q; W_rho is the
 * winding through the face normal to rho at the cell's lower corner,
 * clamped to [-127, 127].  Synchronous; allocates 6 bytes per site of
 * temporary device memory. */
int mts_get_windings(mts_ctx *ctx, int8_t *host);

/* Cell values of the last diagnostic step (total |winding| through the
 * six faces of each cell; a straight string gives 2, Sec. III.B), host
 * uint8[2][S] (sector p, then q).  Each face counts at most 3 (windings are
 * packed in two bits per face; the paper sees none above 1, and the record's
 * sum |W| is not clipped).  Synchronous. */
int mts_get_cells(mts_ctx *ctx, uint8_t *host);

/* Robust-method bound-state segments (Sec. III.B, Sec. V.B) of the last
 * diagnostic step's cells: the cells the fast method marks (a pierced cell
 * of one sector with a pierced cell of the other within overlap_radius,
 * either way round) are grouped into connected regions -- cells sharing at
 * least a corner, periodic -- on the GPU; a region of N cells is a segment
 * of length (N - 1) dx, kept if longer than min_length (the paper: 20 at
 * 4096^3, i.e. more than 41 cells; 3.5 at 512^3).  Fills *out; if sizes is
 * non-null, the region sizes in decreasing order (at most cap) and their
 * number in *n_sizes.  Synchronous; allocates 8 bytes per site of
 * temporary device memory.  EINVAL before any diagnostic step. */
typedef struct mts_segments_t {
    int64_t step;            /* step of the diagnostic record whose cells were used */
    int64_t marked_cells;    /* fast-method pq cells                                */
    int64_t regions;         /* connected regions of them                           */
    int64_t n_pq;            /* regions longer than min_length: N_pq                */
    int64_t largest;         /* cells in the largest region                         */
    double L_pq;             /* sum of (N - 1) dx over the kept regions             */
    double l_pq;             /* mean segment length L_pq / N_pq                     */
    double xi_pq;            /* sqrt(V / L_pq)                                      */
} mts_segments_t;
int mts_segments(mts_ctx *ctx, double min_length, mts_segments_t *out, int64_t *sizes, int64_t cap, int64_t *n_sizes);

/* Choose the update kernel.  ty in {4, 5, 8, 12} (and 13 in FP32) selects
 * the z-marching LDS-tiled kernel with tiles of 64 x ty sites and tz >= 1
 * planes per workgroup (default 8 x 32 in FP32, 4 x 32 in FP64; diagnostic
 * steps use at most 8 rows in FP32 and 5 in FP64, where their variant does
 * not spill registers); every tile shape gives bitwise identical fields, and
 * records that agree to the rounding of their block sums.  ty = 0 selects the one-thread-per-site kernel, which computes
 * the plaquette sines directly and agrees with the tiled kernel to
 * rounding (tz >= 1 is still required, and kept for the tiled kernels of
 * the diagnostic steps).  Synchronises the stream.  EINVAL for other shapes. */
int mts_set_tile(mts_ctx *ctx, int32_t ty, int32_t tz);
int mts_get_tile(const mts_ctx *ctx, int32_t *ty, int32_t *tz);

/* Streaming (non-temporal) stores for the tiled update's outputs: on (1,
 * the default) or off (0).  Which is faster depends on the launch and the
 * box sizes; results are bitwise identical.  The autotuners try both. */
int mts_set_streaming_stores(mts_ctx *ctx, int32_t on);
int mts_get_streaming_stores(const mts_ctx *ctx, int32_t *on);

/* Momentum ping-pong: with on = 1 the tiled kernel reads the momenta from
 * one copy and writes them to the other (the state buffer's and a second
 * copy the library allocates on first use, 40 bytes per site in FP32, 80 in
 * FP64, freed by mts_destroy) instead of rewriting them in place, which HBM
 * serves a few per cent faster; MTS_ENOMEM if the copy does not fit.
 * Results are bitwise identical; diagnostic steps and steps on the
 * per-site kernel stay in place.  on = 0 (the default) rewrites in place.  The autotuner tries it.
 * Synchronises the stream.  Update of Sec. III. */
int mts_set_momentum_pingpong(mts_ctx *ctx, int32_t on);
int mts_get_momentum_pingpong(const mts_ctx *ctx, int32_t *on);

/* Order in which the tiled kernel's workgroups take their tiles.  With
 * xcd_runs = 1 (the default) the tiles are dealt to the GPU's 8 XCDs in
 * contiguous runs (x fastest, then y, then z), so that neighbouring tiles
 * share one L2; with 0 workgroup b takes tile b and the hardware's
 * round-robin dispatch spreads neighbouring tiles over all XCDs, which keeps
 * every XCD streaming through the same region of HBM.  Which is faster
 * depends on the box; results are bitwise identical; the autotuner tries
 * both.  Synchronises the stream.  Update of Sec. III. */
int mts_set_tile_order(mts_ctx *ctx, int32_t xcd_runs);
int mts_get_tile_order(const mts_ctx *ctx, int32_t *xcd_runs);

/* Deeper load pipeline in the tiled update's plain steps: on (1) loads each
 * plane's fields two planes before they are used (more registers per
 * thread, fewer stalls on HBM); off (0, the default) one plane before.
 * FP32 diagnostic steps always use it.  Results are bitwise
 * identical; the autotuner tries both.  Synchronises the stream. */
int mts_set_prefetch(mts_ctx *ctx, int32_t on);
int mts_get_prefetch(const mts_ctx *ctx, int32_t *on);

/* Fused diagnostics (FP32 tiled steps; Sec. III.A windings and the Gauss
 * law of Sec. II): with rows in {4, 5, 8} (default 8) a diagnostic step
 * computes the plaquette windings of its input fields and the Gauss
 * residual at n + 1/2 inside the update kernel (tiles of 64 x rows sites),
 * so only the cell values, the overlap and the final reduction run after
 * it; rows = 0 computes them in separate post-step kernels.  The fused
 * step writes the new momenta to a second momentum copy, which the library
 * allocates on the first fused step (10 planes, 40 bytes per site in FP32;
 * freed by mts_destroy); if it does not fit, diagnostic steps fall back to
 * the post-step kernels and mts_get_fused_diagnostics reports 0.  Windings,
 * cells and overlap counts are bitwise identical either way; the Gauss sums
 * agree to the rounding of their summation order.  FP64 and the per-site
 * kernel always use post-step kernels (FP64: one tiled pass for windings
 * and the Gauss residual, with FP32 phases and FP64 wrap decisions and the
 * same FP64 fix-up, so the windings are those of an FP64 evaluation bit for
 * bit).  Synchronises the stream. */
int mts_set_fused_diagnostics(mts_ctx *ctx, int32_t rows);
int mts_get_fused_diagnostics(const mts_ctx *ctx, int32_t *rows);

/* Temporal blocking (FP32): with steps = 2, every two consecutive plain
 * steps (no diagnostics due at either) run as one sweep of a two-level
 * tiled kernel (tiles of 64 x ty sites, ty in {3, 7}, tz >= 1 planes per
 * workgroup) that reads the state at step n from HBM once and writes the
 * state at step n + 2 once: half the HBM traffic per step.  The fields and
 * momenta are bitwise identical to those of single steps.  The momenta then
 * alternate between the state buffer and a second momentum copy that the
 * library allocates on the first call (10 planes, 40 bytes per site; freed
 * by mts_destroy); MTS_ENOMEM if it does not fit, and the context stays at
 * one step per sweep.  steps = 1 (the default) is one step per sweep.
 * EINVAL for FP64, other steps or tile shapes.  Synchronises the stream.
 * Update of Sec. III (the same equations as mts_step). */
int mts_set_time_blocking(mts_ctx *ctx, int32_t steps, int32_t ty, int32_t tz);
int mts_get_time_blocking(const mts_ctx *ctx, int32_t *steps, int32_t *ty, int32_t *tz);

/* Autotuner: time `steps` plain steps of every supported tile shape
 * (ty in {4, 8, 12, 13} -- {4, 5, 8} in FP64 -- by tz in {8, 16, 32, 64}, with and
 * without streaming stores) on this
 * box with HIP events, keep the fastest, and report it (and its ms per
 * step), each with and without the deeper load pipeline
 * (mts_set_prefetch), and the fastest of them with momentum ping-pong
 * and then with the other tile order (mts_set_tile_order).
 * In FP32 it then times the two-step kernel (ty in {3, 7} by the
 * same tz and store modes, over an even number of steps) and switches
 * time blocking on if that is faster per step (mts_get_time_blocking tells
 * which; ms_per_step is the best of both).  The choice changes speed only:
 * results are bitwise identical for every shape and mode.  Overwrites the
 * lattice (it is left at seed-0 initial conditions): call it before
 * mts_init_fields / mts_set_fields. */
int mts_autotune(mts_ctx *ctx, int32_t steps, int32_t *ty, int32_t *tz, double *ms_per_step);

/* mts_autotune through a cache file (a tuning aid, no part of the method):
 * the key is the GPU's architecture name, its compute-unit count, the box
 * dimensions and the precision.  If cache_path (a text file the caller
 * owns; one line per tuned key, appended) holds the key, its stored choice
 * (tile shape, store mode, load pipeline, momentum ping-pong, tile order,
 * steps per sweep) is applied with the setters, nothing is timed and the
 * fields are left alone: *hit = 1, *ms_per_step = the stored time.
 * Otherwise mts_autotune runs (overwriting the fields) and its choice is
 * appended: *hit = 0, or -1 if the file could not be written (the choice is
 * applied; mts_last_error says why).  A stored choice the context cannot
 * take (no room for a second momentum copy) is tuned afresh.  MTS_EINVAL
 * for a NULL path.  hit, ty, tz and ms_per_step may be NULL. */
int mts_autotune_cached(mts_ctx *ctx, int32_t steps, const char *cache_path, int32_t *hit, int32_t *ty, int32_t *tz,
                        double *ms_per_step);

/* Bandwidth probe (a measurement aid, not part of the method): on this
 * context's state buffer, time `reps` launches each of (a) a plain device
 * copy of one field copy onto the other, one float4 per thread, and (b) a
 * kernel with exactly the update's HBM traffic and none of its stencil or
 * arithmetic (per site the 10 momentum values read and rewritten in place,
 * the 10 field values read and written to the other copy, in the context's
 * store mode), with HIP events; reports bytes moved / time in GB/s.  (b) is
 * the rate the update kernel could reach on this machine.  The lattice is
 * overwritten (as by mts_autotune): call it before mts_init_fields. */
int mts_bandwidth_probe(mts_ctx *ctx, int32_t reps, double *copy_gbps, double *pattern_gbps);

/* Kernel timing with HIP events on the context's stream.  While enabled,
 * every launch of the update kernel is bracketed by events; the summary
 * returns the launch count and the summed event time in milliseconds of
 * plain steps, of diagnostic steps and of two-step sweeps (n_pair launches,
 * each advancing two steps), and the summed time of the diagnostic
 * post-kernels (windings/Gauss, cells, overlap, final reduce).  Any output
 * pointer may be NULL.  mts_timing_read synchronises the stream and resets
 * the counters. */
int mts_timing_enable(mts_ctx *ctx, int32_t on);
int mts_timing_read(mts_ctx *ctx, int64_t *n_plain, double *ms_plain, int64_t *n_diag, double *ms_diag,
                    double *ms_post, int64_t *n_pair, double *ms_pair);

/* ------------------------------------------------------------ ensembles
 * A batch advances several independent boxes (own size, couplings,
 * eta_ref, era, s and seed; shared precision and diag_every) with one
 * update kernel launch per step over all boxes' tiles, the whole n-step
 * sequence of a mts_batch_step call captured into one HIP graph and
 * launched once.  Box k behaves exactly as a single context with the same
 * parameters and tile shape (bitwise identical fields). */
typedef struct mts_batch mts_batch;

/* Bytes of the device pool for nbox boxes: each box's mts_state_bytes()
 * rounded up to 256, in box order.  0 if any box is invalid. */
size_t mts_batch_state_bytes(const mts_params *boxes, int32_t nbox);

/* Create a batch on the current device.  boxes[nbox] are copied; every box
 * must share precision and diag_every (EINVAL otherwise).  dev_pool is a
 * caller-owned device buffer of at least mts_batch_state_bytes() bytes,
 * 256-byte aligned, borrowed for the batch's lifetime.  stream as for
 * mts_create; the graphs run on an internal non-blocking stream of default
 * priority that is joined to `stream` before and after every launch. */
int mts_batch_create(const mts_params *boxes, int32_t nbox, void *dev_pool, size_t pool_bytes, void *stream,
                     mts_batch **out);
int mts_batch_destroy(mts_batch *b);
int32_t mts_batch_size(const mts_batch *b);

/* Random-phase initial conditions of every box, seeds[nbox] (host). */
int mts_batch_init_fields(mts_batch *b, const uint64_t *seeds);

/* Advance every box n steps in one graph launch.  Host arrays of nbox:
 * eta0 (start time), era_m, s_before; s_after and eta_switch may be NULL.
 * Box k uses beta = s_before[k] for steps with eta_j < eta_switch[k] and
 * s_after[k] from then on (a core-growth phase followed by physical
 * evolution, Sec. V).  Same checks and diagnostics as mts_step, per box. */
int mts_batch_step(mts_batch *b, int32_t n, const double *eta0, const double *era_m, const double *s_before,
                   const double *s_after, const double *eta_switch);

/* Per-box access, as the single-context functions. */
int mts_batch_diagnostics(mts_batch *b, int32_t box, mts_diag *out, int32_t max, int32_t *count);
int mts_batch_get_fields(mts_batch *b, int32_t box, double *host);
int mts_batch_set_fields(mts_batch *b, int32_t box, const double *host);

/* Tile shape of the batched launch: one ty in {4, 5, 8, 12} (and 13 in
 * FP32) for all boxes and a tz[nbox] per box. */
int mts_batch_set_tile(mts_batch *b, int32_t ty, const int32_t *tz);
int mts_batch_set_streaming_stores(mts_batch *b, int32_t on);
int mts_batch_get_streaming_stores(const mts_batch *b, int32_t *on);

/* Momentum ping-pong for the batched launch, as mts_set_momentum_pingpong:
 * plain steps of every box read the momenta from one copy and write them to
 * the other (each box's second copy is allocated by the library on first
 * use, freed by mts_batch_destroy); diagnostic steps stay in place.  Results
 * are bitwise identical; off (0) by default; the batch autotuner tries it.
 * Synchronises the batch's and the caller's streams.  Update of Sec. III. */
int mts_batch_set_momentum_pingpong(mts_batch *b, int32_t on);
int mts_batch_get_momentum_pingpong(const mts_batch *b, int32_t *on);

/* Tile order of the batched launch, as mts_set_tile_order (over the
 * batch's whole grid of tiles); the batch autotuner tries both. */
/* Fused diagnostics of an FP32 batch (as mts_set_fused_diagnostics, with
 * 8 rows): the diagnostic steps compute every box's windings and Gauss
 * residual in the batched update launch, and the fix-up, cells, overlap and
 * reduction of all boxes run as one launch each.  On by default for FP32
 * batches with diagnostics when every box has room for its second momentum
 * copy; rows = 0 runs the post-step kernels box by box.  Synchronises. */
int mts_batch_set_fused_diagnostics(mts_batch *b, int32_t rows);
int mts_batch_get_fused_diagnostics(const mts_batch *b, int32_t *rows);

int mts_batch_set_tile_order(mts_batch *b, int32_t xcd_runs);
int mts_batch_get_tile_order(const mts_batch *b, int32_t *xcd_runs);

/* Persistent launch of the plain steps (on != 0): every run of consecutive
 * plain steps between two diagnostic steps of an mts_batch_step call is one
 * launch whose workgroups stay resident (grid: the occupancy query of the
 * current tile shape times the compute units, at most the tiles of a step)
 * and loop over the steps, claiming tiles one at a time from a device
 * counter, with a device-wide barrier after each step (the tile order setting
 * does not apply); the diagnostic steps launch as before.  The tiles and
 * their arithmetic are the per-step launches', so the results are the same
 * bit for bit (Sec. III's leapfrog step, unchanged).  Every barrier wait is bounded by
 * wait_limit_s seconds (0: 10 s; at most 3600): a wait that runs out (the grid
 * was not co-resident, e.g. another kernel holds compute units, or a step is
 * slower than the limit) makes every workgroup leave, and the next call that
 * synchronises the batch (mts_batch_step, _timing_read, _diagnostics,
 * _get_fields) returns MTS_EHIP once; the fields then hold an unfinished step
 * and must be set again.  MTS_EINVAL for a limit out of range. */
int mts_batch_set_persistent(mts_batch *b, int32_t on, double wait_limit_s);
int mts_batch_get_persistent(const mts_batch *b, int32_t *on);

/* Summed HIP-event time (ms) of the graph launches and the steps they ran
 * since the last read; synchronises. */
int mts_batch_timing_read(mts_batch *b, int64_t *steps, double *ms);

/* Autotuner of the batched launch (one ty and one tz for all boxes, streaming
 * stores, then momentum ping-pong, the tile order and the persistent launch
 * on the best of those), as mts_autotune; overwrites every box. */
int mts_batch_autotune(mts_batch *b, int32_t steps, int32_t *ty, int32_t *tz, double *ms_per_step);

/* Per-step time (ms) of the plain steps the last mts_batch_autotune measured
 * for its final configuration as per-step launches in one graph and as one
 * persistent launch (0 before any autotune). */
int mts_batch_autotune_times(const mts_batch *b, double *graph_ms, double *persistent_ms);

const char *mts_batch_last_error(const mts_batch *b);

/* Text of the last error of ctx (never NULL). */
const char *mts_last_error(const mts_ctx *ctx);

/* Short name of a return code. */
const char *mts_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MTS_H */
