// api.hip -- host side of libmts (the C ABI declared in include/mts.h):
// parameter checks, FP64 time bookkeeping, launches, diagnostic records.
#include "kernels.h"
#include "mts.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace mts;

namespace {

constexpr int RING_CAP = 4096;   // diagnostic records kept on the device between drains

// Staging of mts_get_sites_noalloc: the site indices, then the gathered
// values (double[n][20]), for at most MTS_NOALLOC_MAX_SITES sites.
constexpr size_t NOALLOC_SITES_BYTES = sizeof(uint64_t) * MTS_NOALLOC_MAX_SITES;
constexpr size_t NOALLOC_BYTES = NOALLOC_SITES_BYTES + sizeof(double) * 20 * MTS_NOALLOC_MAX_SITES;
constexpr int NOALLOC_MAX_DEVICES = 64;

struct Meta {                    // host-side facts of one record
    int64_t step;
    double eta, a, s;
};

}  // namespace

// Device scratch of the entry points that allocate nothing: each GPU the
// library runs on holds one copy for the life of the process.  Host code
// never passes this name to a kernel or a copy; it uses the device address
// that noalloc_scratch() obtains once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call for that device and kept.
hipError_t noalloc_scratch(void **out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

struct mts_ctx {
    mts_params p{};
    size_t esz = 4;
    Geom g{};
    uint64_t S = 0;              // sites
    uint64_t plane = 0;          // elements per plane (S rounded up to 64, plus the stagger)
    char *state = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;                 // which field copy holds the current fields
    int64_t step_count = 0;

    // scratch
    double *partials = nullptr;  // [NSLOT][maxblk]
    uint32_t maxblk = 0;
    uint32_t *nblk_dev = nullptr;
    TileShape tile{8, 32};       // ty = 0: per-site kernel
    bool nt = true;              // streaming stores in the tiled update
    bool pf = false;             // loads one plane ahead in the tiled update (plain steps)
    bool mpp = false;            // tiled steps write the momenta to the other momentum copy
    bool xcd = true;             // tiles dealt to the XCDs in contiguous runs (else round-robin)
    int fuse_ty = 8;             // rows of the fused diagnostic tile (0: windings and Gauss in post-step kernels)
    bool fuse_off = false;       // the fused path needs a second momentum copy and none could be allocated
    int tblock = 1;              // leapfrog steps per sweep through HBM (1, or 2: two-step kernel)
    TileShape tile2{7, 32};      // tile of the two-step kernel
    void *mom2 = nullptr;        // second momentum copy (10 planes), allocated for two-step sweeps
    int mcur = 0;                // which momentum copy is current: 0 = the state buffer, 1 = mom2
    void *alpha = nullptr;       // arg(phi) per sector: T[2][plane]
    uint8_t *wabs = nullptr;     // packed |W| per sector: [2][plane]
    uint32_t *fixlist = nullptr; // marked sites of a diagnostic step's windings (fix-up): FIX_LIST_WORDS words
    uint8_t *cells = nullptr;    // cell values per sector: [2][plane]
    uint64_t *bits = nullptr;    // occupancy words per sector: [2][overlap_words] (nx % 64 == 0)
    double *ring = nullptr;      // [RING_CAP][NSLOT]
    std::vector<Meta> meta;      // one per record produced since the last drain
    int64_t produced = 0, drained = 0;
    bool have_cells = false;
    int64_t cells_step = -1;     // step whose cells the cell arrays hold
    void *noalloc = nullptr;     // this device's `scratch` (entry points that allocate nothing)
    std::string noalloc_err;     // why it could not be looked up, if it could not

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Mark {
        int kind;                // 0 plain step, 1 diagnostic step, 2 diagnostic post-kernels, 3 two-step sweep
        int a, b;                // event indices
    };
    std::vector<Mark> marks;
    size_t ev_used = 0;

    std::string err;
};

namespace {

int fail(mts_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int hipfail(mts_ctx *c, hipError_t e, const char *what) {
    return fail(c, MTS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hipfail(ctx, e_, #call); \
    } while (0)

template <typename T>
Fields<T> fields_of(const mts_ctx *c, int copy) {
    T *base = reinterpret_cast<T *>(c->state) + (size_t)copy * 10 * c->plane;
    Fields<T> f;
    for (int sec = 0; sec < 2; sec++) {
        f.phi[sec] = reinterpret_cast<cx<T> *>(base + (size_t)(2 * sec) * c->plane);
        for (int i = 0; i < 3; i++) f.A[sec][i] = base + (size_t)(4 + 3 * sec + i) * c->plane;
    }
    return f;
}

// Momentum copy `which` (0: planes 20..29 of the state buffer, 1: mom2).
template <typename T>
T *mom_base(const mts_ctx *c, int which) {
    return which == 0 ? reinterpret_cast<T *>(c->state) + (size_t)20 * c->plane : static_cast<T *>(c->mom2);
}

template <typename T>
Moms<T> moms_at(const mts_ctx *c, int which) {
    T *base = mom_base<T>(c, which);
    Moms<T> m;
    for (int sec = 0; sec < 2; sec++) {
        m.pi[sec] = reinterpret_cast<cx<T> *>(base + (size_t)(2 * sec) * c->plane);
        for (int i = 0; i < 3; i++) m.E[sec][i] = base + (size_t)(4 + 3 * sec + i) * c->plane;
    }
    return m;
}

// The current momenta.
template <typename T>
Moms<T> moms_of(const mts_ctx *c) {
    T *base = mom_base<T>(c, c->mcur);
    Moms<T> m;
    for (int sec = 0; sec < 2; sec++) {
        m.pi[sec] = reinterpret_cast<cx<T> *>(base + (size_t)(2 * sec) * c->plane);
        for (int i = 0; i < 3; i++) m.E[sec][i] = base + (size_t)(4 + 3 * sec + i) * c->plane;
    }
    return m;
}

// FP64 bookkeeping of one step from eta (Sec. III):
//   p = m/(1-m), a = (eta/eta_ref)^p, delta = (alpha/2) p k / eta with alpha = 2,
//   omega = (1 - s) delta, An = a^{2s}.
struct Book {
    double a, delta, omega, An;
};

Book bookkeeping(const mts_params &p, double eta, double era_m, double s) {
    const double pw = era_m / (1.0 - era_m);
    Book b;
    b.a = pw == 0.0 ? 1.0 : std::pow(eta / p.eta_ref, pw);
    b.delta = pw == 0.0 ? 0.0 : pw * p.dt / eta;
    b.omega = (1.0 - s) * b.delta;
    b.An = std::pow(b.a, 2.0 * s);
    return b;
}

template <typename T>
StepCoef<T> coefficients(const mts_params &p, const Book &b, double s) {
    const double h = p.dx, k = p.dt;
    const double lam[2] = {p.lambda_p, p.lambda_q}, e[2] = {p.e_p, p.e_q}, sig[2] = {p.sigma_p, p.sigma_q};
    StepCoef<T> c;
    c.h = (T)h;
    c.inv_h = (T)(1.0 / h);
    c.inv_h2 = (T)(1.0 / (h * h));
    c.inv_h3 = (T)(1.0 / (h * h * h));
    c.k = (T)k;
    c.cpi = (T)((1.0 - b.delta) / (1.0 + b.delta));
    c.kpi = (T)(k / (1.0 + b.delta));
    c.cE = (T)((1.0 - b.omega) / (1.0 + b.omega));
    c.kE = (T)(k / (1.0 + b.omega));
    c.kap = (T)(b.An * p.kappa);
    for (int q = 0; q < 2; q++) {
        c.lamh[q] = (T)(b.An * lam[q] / 2.0);
        c.sig2[q] = (T)(sig[q] * sig[q]);
        c.cur[q] = (T)(2.0 * e[q] * e[q] * b.An / h);
        c.inv_2e2[q] = (T)(1.0 / (2.0 * e[q] * e[q]));
        c.inv_e2h4[q] = (T)(1.0 / (e[q] * e[q] * h * h * h * h));
        c.lam4[q] = (T)(lam[q] / 4.0);
    }
    for (int q = 0; q < 2; q++) c.gsig[q] = (T)(2.0 * (e[q] * e[q]) * b.An * (1.0 + b.delta) / (1.0 + b.omega));
    c.a2s = (T)std::pow(b.a, 2.0 * s);
    c.am2s = (T)std::pow(b.a, -2.0 * s);
    c.kap0 = (T)p.kappa;
    return c;
}

// Largest squared frequency of the linearised update around the vacuum.
double mu2_max(const mts_params &p) {
    const double lp = p.lambda_p * p.sigma_p * p.sigma_p, lq = p.lambda_q * p.sigma_q * p.sigma_q;
    const double off = 2.0 * p.kappa * p.sigma_p * p.sigma_q;
    const double mean = 0.5 * (lp + lq), dif = 0.5 * (lp - lq);
    const double eig = mean + std::sqrt(dif * dif + off * off);
    const double gp = 2.0 * p.e_p * p.e_p * p.sigma_p * p.sigma_p;
    const double gq = 2.0 * p.e_q * p.e_q * p.sigma_q * p.sigma_q;
    return std::max(eig, std::max(gp, gq));
}

int check_params(const mts_params *p, std::string &why) {
    if (!p) return why = "params is NULL", MTS_EINVAL;
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) return why = "each of nx, ny, nz must be >= 4", MTS_EINVAL;
    const double S = (double)p->nx * p->ny * p->nz;
    // planes (S rounded up to 64 plus the stagger) are indexed with 32 bits
    if (S >= 4294967296.0 - 2048) return why = "nx*ny*nz must be below 2^32 - 2048", MTS_EINVAL;
    if (p->precision != MTS_FP32 && p->precision != MTS_FP64) return why = "precision must be MTS_FP32 or MTS_FP64", MTS_EINVAL;
    if (!(p->dx > 0) || !(p->dt > 0)) return why = "dx and dt must be > 0", MTS_EINVAL;
    if (!(p->e_p > 0) || !(p->e_q > 0)) return why = "e_p and e_q must be > 0", MTS_EINVAL;
    if (!(p->sigma_p > 0) || !(p->sigma_q > 0)) return why = "sigma_p and sigma_q must be > 0", MTS_EINVAL;
    if (!(p->lambda_p >= 0) || !(p->lambda_q >= 0)) return why = "lambda_p and lambda_q must be >= 0", MTS_EINVAL;
    if (!std::isfinite(p->kappa)) return why = "kappa must be finite", MTS_EINVAL;
    if (!(p->eta_ref > 0)) return why = "eta_ref must be > 0", MTS_EINVAL;
    if (p->diag_every < 0) return why = "diag_every must be >= 0", MTS_EINVAL;
    if (p->overlap_radius < 0 || p->overlap_radius > 1) return why = "overlap_radius must be 0 or 1", MTS_EINVAL;
    return MTS_OK;
}

// Consecutive planes are staggered by an extra 4 KiB so that the 30 plane base
// addresses of a box whose plane size is a power of two do not all fall on
// the same HBM channel offset (measured: +2-7 % on the update's access
// pattern).
#ifndef MTS_PLANE_PAD_BYTES
#define MTS_PLANE_PAD_BYTES 4096
#endif

uint64_t plane_of(const mts_params &p) {
    const uint64_t S = (uint64_t)p.nx * p.ny * p.nz;
    const uint64_t esz = p.precision == MTS_FP64 ? 8 : 4;
    return (S + 63) / 64 * 64 + MTS_PLANE_PAD_BYTES / esz;
}

hipEvent_t next_event(mts_ctx *c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Record an event pair around a launch when timing is on.
struct TimedRegion {
    mts_ctx *c;
    int kind, a = -1;
    TimedRegion(mts_ctx *ctx, int k) : c(ctx), kind(k) {
        if (!c->timing) return;
        hipEvent_t e = next_event(c);
        if (e && hipEventRecord(e, c->stream) == hipSuccess) a = (int)c->ev_used - 1;
    }
    ~TimedRegion() {
        if (a < 0) return;
        hipEvent_t e = next_event(c);
        if (e && hipEventRecord(e, c->stream) == hipSuccess) c->marks.push_back({kind, a, (int)c->ev_used - 1});
    }
};

// Diagnostic steps use the DIAG variant of the update kernel, which needs
// more registers: it runs with at most 8 rows per tile in FP32 and 5 in FP64
// (256 VGPRs, its running sums in LDS), where it does not spill.  Tile shapes
// do not change the fields (bitwise); records agree to the rounding of their
// block sums.
TileShape diag_tile(const mts_ctx *c) {
    if (c->tile.ty == 0) return c->tile;
    const int cap = c->p.precision == MTS_FP64 ? 5 : 8;
    return TileShape{std::min(c->tile.ty, cap), c->tile.tz};
}

// Diagnostic steps run on the per-site kernel only where the plain steps do.
bool diag_per_site(const mts_ctx *c) { return c->tile.ty == 0; }

// Diagnostic steps that are not fused take the tiled winding/Gauss pass and
// the fix-up, unless the box has 2^31 sites or more (the fix-up list holds a
// site in 31 bits): those take the per-column kernel.
bool post_tiled(const mts_ctx *c) { return c->S < (1ull << 31); }

// The phases alpha of phi^n for the per-column winding kernel: the tiled
// unfused FP32 diagnostic step stores them itself; the per-site kernel and
// the FP64 tiled one leave them to the phase kernel.  Where the tiled pass
// runs nothing reads them and nothing stores them.
bool diag_writes_alpha(const mts_ctx *c) {
    return !diag_per_site(c) && c->p.precision == MTS_FP32 && !post_tiled(c);
}

// Diagnostic steps of the tiled FP32 kernel take the windings and the Gauss
// residual in the same pass (the post-step kernels then only form the cells
// and the overlap) unless switched off or no second momentum copy fits.
bool diag_fused(const mts_ctx *c) {
    return !diag_per_site(c) && c->p.precision == MTS_FP32 && c->fuse_ty != 0 && !c->fuse_off &&
           c->S < (1ull << 31);   // the fix-up list stores a site in 31 bits
}

TileShape fused_tile(const mts_ctx *c) { return TileShape{c->fuse_ty, c->tile.tz}; }


// Partials per slot: the update kernel's blocks for the integer-time sums,
// the per-site grid for the post-step diagnostic kernels.
// The second table (at nblk_dev + NSLOT) is the fused path's: the update
// kernel's blocks hold every slot up to the winding sums.
hipError_t upload_nblk(mts_ctx *c) {
    uint32_t nb[2 * NSLOT];
    const uint32_t step_blocks = diag_per_site(c) ? site_blocks(c->g) : tile_blocks(c->g, diag_tile(c));
    const uint32_t fused_blocks = c->fuse_ty ? tile_blocks(c->g, fused_tile(c)) : 0;
    // diagnostic steps that are not fused: the tiled winding/Gauss pass and
    // the fix-up passes (the per-column kernel in boxes of 2^31 sites or more)
    const bool tiled = post_tiled(c);
    const uint32_t wblk = tiled ? wind_tile_blocks(c->g) : wind_blocks(c->g);
    const uint32_t fixblk = tiled ? wind_fix_blocks(c->g) : 0;
    for (int q = 0; q < NSLOT; q++) {
        nb[q] = q <= SL_GV ? step_blocks : (q <= SL_WIND_Q ? wblk : (q <= SL_OV_Q ? overlap_blocks(c->g) : fixblk));
        nb[NSLOT + q] = q <= SL_WIND_Q ? fused_blocks : (q <= SL_OV_Q ? overlap_blocks(c->g) : wind_fix_blocks(c->g));
    }
    return hipMemcpy(c->nblk_dev, nb, sizeof(nb), hipMemcpyHostToDevice);
}

// Post-step diagnostic kernels of one box (windings + Gauss, cells, overlap,
// reduce into the next ring slot) for the step from eta_j; fields at n are
// in copy `cur`.  Host-side facts of the record are queued.
// With `fused` the update kernel has already written the windings and the
// Gauss sums: only the cells, the overlap and the reduction remain.
template <typename T>
hipError_t enqueue_diag_post(mts_ctx *c, const Book &b, double eta_j, double s, hipStream_t st, bool alpha_ready,
                             bool fused = false) {
    const mts_params &p = c->p;
    Partials part{c->partials, c->maxblk};
    double gcoef[2];
    const double e2[2] = {p.e_p * p.e_p, p.e_q * p.e_q};
    for (int q = 0; q < 2; q++) gcoef[q] = 2.0 * e2[q] * b.An * (1.0 + b.delta) / (1.0 + b.omega);
    T *alpha = static_cast<T *>(c->alpha);
    hipError_t e = hipSuccess;
    if (!fused && post_tiled(c)) {
        // windings (wrap counts) and the Gauss residual in one tiled pass,
        // then the fix-up of the flagged sites
        e = launch_wind_gauss_tile<T>(c->g, fields_of<T>(c, c->cur), moms_of<T>(c), (T)p.dx, (T)(1.0 / p.dx), gcoef,
                                      c->wabs, (uint32_t)c->plane, part, st);
        if (e == hipSuccess)
            e = launch_wind_fix<T>(c->g, fields_of<T>(c, c->cur), (T)p.dx, c->wabs, (uint32_t)c->plane, part,
                                   c->fixlist, st);
    } else if (!fused) {
        // boxes of 2^31 sites or more (the fix-up list holds a site in 31
        // bits): the per-column kernel, which evaluates flagged links in place
        if (!alpha_ready) e = launch_phase<T>(c->g, fields_of<T>(c, c->cur), alpha, (uint32_t)c->plane, st);
        if (e == hipSuccess)
            e = launch_wind_gauss<T>(c->g, fields_of<T>(c, c->cur), moms_of<T>(c), alpha, (T)p.dx, (T)(1.0 / p.dx),
                                     gcoef, c->wabs, (uint32_t)c->plane, nullptr, part, st);
    } else {
        e = launch_wind_fix<T>(c->g, fields_of<T>(c, c->cur), (T)p.dx, c->wabs, (uint32_t)c->plane, part, c->fixlist,
                               st);
    }
    if (e == hipSuccess) e = launch_cells(c->g, c->wabs, c->cells, c->bits, (uint32_t)c->plane, st);
    if (e == hipSuccess)
        e = launch_overlap(c->g, c->cells, c->bits, (uint32_t)c->plane, p.overlap_radius, part, st);
    double *rec = c->ring + (size_t)(c->produced % RING_CAP) * NSLOT;
    if (e == hipSuccess) e = launch_reduce(part, c->nblk_dev + (fused ? NSLOT : 0), rec, st);
    if (e != hipSuccess) return e;
    c->meta.push_back({c->step_count, eta_j, b.a, s});
    c->produced++;
    c->have_cells = true;
    c->cells_step = c->step_count;
    return hipSuccess;
}

int ensure_mom2_quiet(mts_ctx *c);

template <typename T>
int do_step(mts_ctx *c, int32_t n, double eta, double era_m, double s) {
    const mts_params &p = c->p;
    Partials part{c->partials, c->maxblk};
    auto diag_due = [&](int64_t step) { return p.diag_every > 0 && (step % p.diag_every) == 0; };
    for (int32_t j = 0; j < n;) {
        const double eta_j = eta + j * p.dt;
        const Book b = bookkeeping(p, eta_j, era_m, s);
        const StepCoef<T> coef = coefficients<T>(p, b, s);
        const bool diag = diag_due(c->step_count);
        if (c->tblock == 2 && !diag && j + 1 < n && !diag_due(c->step_count + 1)) {
            // two plain steps in one sweep: fields to the other copy, momenta to the other copy
            const double eta_k = eta + (j + 1) * p.dt;
            const StepCoef<T> coef2 = coefficients<T>(p, bookkeeping(p, eta_k, era_m, s), s);
            {
                TimedRegion tr(c, 3);
                hipError_t e = launch_step_pair<T>(c->g, fields_of<T>(c, c->cur), fields_of<T>(c, 1 - c->cur),
                                                   moms_at<T>(c, c->mcur), moms_at<T>(c, 1 - c->mcur), coef, coef2,
                                                   c->tile2, c->nt, c->stream);
                if (e != hipSuccess) return hipfail(c, e, "two-step kernel launch");
            }
            c->cur = 1 - c->cur;
            c->mcur = 1 - c->mcur;
            c->step_count += 2;
            j += 2;
            continue;
        }
        Moms<T> mom = moms_of<T>(c);
        Fields<T> in = fields_of<T>(c, c->cur), out = fields_of<T>(c, 1 - c->cur);
        const bool per_site = c->tile.ty == 0 || (diag && diag_per_site(c));
        // fused diagnostics write the momenta to the other copy (allocated on first use)
        const bool fused = diag && diag_fused(c) && ensure_mom2_quiet(c) == MTS_OK;
        // momenta to the other copy on plain tiled steps (the unfused diagnostic steps, measured 9 % slower
        // with it at 512^3, and the per-site kernel rewrite them in place)
        const bool pp = (c->mpp && !per_site && !diag) || fused;
        const Moms<T> mom_out = pp ? moms_at<T>(c, 1 - c->mcur) : mom;
        {
            TimedRegion tr(c, diag ? 1 : 0);
            hipError_t e = per_site
                               ? launch_step<T>(c->g, in, out, mom, coef, diag, part, c->stream)
                               : launch_step_tile<T>(c->g, in, out, mom, mom_out, coef, diag, part,
                                                     fused ? fused_tile(c) : (diag ? diag_tile(c) : c->tile),
                                                     diag_writes_alpha(c) ? static_cast<T *>(c->alpha) : nullptr,
                                                     fused ? c->wabs : nullptr,
                                                     (uint32_t)c->plane, c->nt, c->pf, c->xcd, c->stream);
            if (e != hipSuccess) return hipfail(c, e, "step kernel launch");
        }
        if (pp) c->mcur = 1 - c->mcur;   // the diagnostic kernels below read the new momenta
        // the step is enqueued: the bookkeeping advances even if its diagnostics fail
        hipError_t ep = hipSuccess;
        if (diag) {
            TimedRegion tr(c, 2);
            ep = enqueue_diag_post<T>(c, b, eta_j, s, c->stream, diag_writes_alpha(c), fused);
        }
        c->cur = 1 - c->cur;
        c->step_count++;
        j++;
        if (ep != hipSuccess) return hipfail(c, ep, "diagnostic kernel launch");
    }
    return MTS_OK;
}

// Argument checks of a run of n steps from eta (beta = s_before while
// eta_j < eta_switch, s_after from then on), including the leapfrog
// stability bound over the run's range of a^{2s}.
int check_step(mts_ctx *c, int32_t n, double eta, double era_m, double s_before, double s_after, double eta_switch) {
    if (n < 0) return fail(c, MTS_EINVAL, "n must be >= 0");
    if (!(era_m >= 0.0 && era_m < 1.0)) return fail(c, MTS_EINVAL, "era_m must be in [0, 1)");
    if (!std::isfinite(eta) || !std::isfinite(s_before) || !std::isfinite(s_after) || std::isnan(eta_switch))
        return fail(c, MTS_EINVAL, "eta and s must be finite");
    if (era_m > 0.0 && !(eta > 0.0)) return fail(c, MTS_EINVAL, "eta must be > 0 when era_m > 0");
    if (n == 0) return MTS_OK;
    const double eta_end = eta + (n - 1) * c->p.dt;
    double Amax = 0.0;
    for (double sv : {s_before, s_after})
        for (double et : {eta, eta_end}) Amax = std::max(Amax, bookkeeping(c->p, et, era_m, sv).An);
    const double k = c->p.dt, h = c->p.dx;
    const double cfl = k * k * (12.0 / (h * h) + Amax * mu2_max(c->p));
    if (!(cfl < 4.0)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "unstable: dt^2 (12/h^2 + a^{2s}_max mu2_max) = %.4g >= 4", cfl);
        return fail(c, MTS_EUNSTABLE, buf);
    }
    return MTS_OK;
}

void derive(const mts_params &p, uint64_t S, mts_diag &d) {
    const double h = p.dx, V = (double)S * h * h * h;
    auto ratio = [](double a, double b) { return b != 0.0 ? a / b : NAN; };
    d.L_pq = h * (double)d.pq_count2 / 2.0;
    d.L_p = h * (double)d.wind_abs[0] - d.L_pq;
    d.L_q = h * (double)d.wind_abs[1] - d.L_pq;
    auto xi = [&](double L) { return L > 0 ? std::sqrt(V / L) : INFINITY; };
    d.xi_p = xi(d.L_p);
    d.xi_q = xi(d.L_q);
    d.xi_pq = xi(d.L_pq);
    d.xi_W = xi(d.L_p + d.L_q + d.L_pq);
    // tension of a basic string: a p-string at critical coupling, 2 pi sigma_p^2 (Sec. III.A, IV)
    const double mu = 2.0 * M_PI * p.sigma_p * p.sigma_p;
    d.xi_lag = d.sum_lagrangian < 0 ? std::sqrt(-mu * V / d.sum_lagrangian) : NAN;
    d.f_total = ratio(d.L_pq, d.L_pq + d.L_p + d.L_q);
    d.f_p = ratio(d.L_pq, d.L_p);
    const double RL = ratio(d.sum_KL, d.sum_GL), Rq = ratio(d.sum_KV, d.sum_GV);
    d.v2_lag = 2.0 * RL / (1.0 + RL);
    d.v2_pq = 2.0 * Rq / (1.0 + Rq);
    for (int q = 0; q < 2; q++) d.gauss_rel[q] = d.gauss_scale[q] != 0.0 ? d.gauss_abs[q] / d.gauss_scale[q] : 0.0;
}

template <typename T>
void to_host(const mts_ctx *c, const std::vector<T> &dev, double *host) {
    // device order: copy `cur` fields (10 planes), momenta (10 planes); both
    // with complex planes interleaved -> host planar order
    const uint64_t S = c->S, P = c->plane;
    auto put_cx = [&](const T *src, int hplane) {
        for (uint64_t i = 0; i < S; i++) {
            host[(size_t)hplane * S + i] = (double)src[2 * i];
            host[(size_t)(hplane + 1) * S + i] = (double)src[2 * i + 1];
        }
    };
    auto put_r = [&](const T *src, int hplane) {
        for (uint64_t i = 0; i < S; i++) host[(size_t)hplane * S + i] = (double)src[i];
    };
    const T *f = dev.data(), *m = dev.data() + 10 * P;
    put_cx(f, 0);
    put_cx(f + 2 * P, 2);
    put_cx(m, 4);
    put_cx(m + 2 * P, 6);
    for (int i = 0; i < 6; i++) put_r(f + (4 + i) * P, 8 + i);
    for (int i = 0; i < 6; i++) put_r(m + (4 + i) * P, 14 + i);
}

template <typename T>
void from_host(const mts_ctx *c, const double *host, std::vector<T> &dev) {
    const uint64_t S = c->S, P = c->plane;
    auto get_cx = [&](T *dst, int hplane) {
        for (uint64_t i = 0; i < S; i++) {
            dst[2 * i] = (T)host[(size_t)hplane * S + i];
            dst[2 * i + 1] = (T)host[(size_t)(hplane + 1) * S + i];
        }
    };
    auto get_r = [&](T *dst, int hplane) {
        for (uint64_t i = 0; i < S; i++) dst[i] = (T)host[(size_t)hplane * S + i];
    };
    T *f = dev.data(), *m = dev.data() + 10 * P;
    get_cx(f, 0);
    get_cx(f + 2 * P, 2);
    get_cx(m, 4);
    get_cx(m + 2 * P, 6);
    for (int i = 0; i < 6; i++) get_r(f + (4 + i) * P, 8 + i);
    for (int i = 0; i < 6; i++) get_r(m + (4 + i) * P, 14 + i);
}

template <typename T>
int get_fields_t(mts_ctx *c, double *host) {
    std::vector<T> buf(20 * c->plane);
    T *base = reinterpret_cast<T *>(c->state);
    HIPCHK(c, hipMemcpyAsync(buf.data(), base + (size_t)c->cur * 10 * c->plane, 10 * c->plane * sizeof(T),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(buf.data() + 10 * c->plane, mom_base<T>(c, c->mcur), 10 * c->plane * sizeof(T),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    to_host<T>(c, buf, host);
    return MTS_OK;
}

template <typename T>
int set_fields_t(mts_ctx *c, const double *host) {
    std::vector<T> buf(20 * c->plane, T(0));
    from_host<T>(c, host, buf);
    T *base = reinterpret_cast<T *>(c->state);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpyAsync(base + (size_t)c->cur * 10 * c->plane, buf.data(), 10 * c->plane * sizeof(T),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(mom_base<T>(c, c->mcur), buf.data() + 10 * c->plane, 10 * c->plane * sizeof(T),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MTS_OK;
}

template <typename T>
int get_windings_t(mts_ctx *c, int8_t *host) {
    int8_t *tmp = nullptr;
    const size_t bytes = 6 * c->plane;
    HIPCHK(c, hipMalloc(&tmp, bytes));
    Partials part{c->partials, c->maxblk};
    double g0[2] = {0, 0};
    T *alpha = static_cast<T *>(c->alpha);
    hipError_t e = launch_phase<T>(c->g, fields_of<T>(c, c->cur), alpha, (uint32_t)c->plane, c->stream);
    if (e == hipSuccess)
        e = launch_wind_gauss<T>(c->g, fields_of<T>(c, c->cur), moms_of<T>(c), alpha, (T)c->p.dx,
                                 (T)(1.0 / c->p.dx), g0, nullptr, (uint32_t)c->plane, tmp, part, c->stream);
    std::vector<int8_t> buf(bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(buf.data(), tmp, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hipfail(c, e, "windings");
    for (int q = 0; q < 6; q++) std::memcpy(host + (size_t)q * c->S, buf.data() + (size_t)q * c->plane, c->S);
    return MTS_OK;
}

}  // namespace

namespace {
// The second momentum copy for the fused diagnostics: allocated on first use;
// if it does not fit, the fused path is switched off for this context.
int ensure_mom2_quiet(mts_ctx *c) {
    if (c->mom2) return MTS_OK;
    if (c->fuse_off) return MTS_ENOMEM;
    hipError_t e = hipMalloc(&c->mom2, (size_t)10 * c->plane * c->esz);
    if (e != hipSuccess) {
        c->mom2 = nullptr;
        c->fuse_off = true;
        (void)hipGetLastError();
        return MTS_ENOMEM;
    }
    return MTS_OK;
}
}  // namespace

extern "C" {

size_t mts_state_bytes(const mts_params *p) {
    std::string why;
    if (check_params(p, why) != MTS_OK) return 0;
    return 30 * plane_of(*p) * (p->precision == MTS_FP64 ? 8 : 4);
}

int mts_create(const mts_params *p, void *dev_state, size_t state_bytes, void *stream, mts_ctx **out) {
    if (!out) return MTS_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = check_params(p, why);
    if (rc != MTS_OK) {
        std::fprintf(stderr, "mts_create: %s\n", why.c_str());
        return rc;
    }
    if (!dev_state || (reinterpret_cast<uintptr_t>(dev_state) & 255) != 0) {
        std::fprintf(stderr, "mts_create: state buffer missing or not 256-byte aligned\n");
        return MTS_EINVAL;
    }
    if (state_bytes < mts_state_bytes(p)) {
        std::fprintf(stderr, "mts_create: state buffer too small\n");
        return MTS_ENOMEM;
    }
    mts_ctx *c = new (std::nothrow) mts_ctx;
    if (!c) return MTS_ENOMEM;
    c->p = *p;
    c->esz = p->precision == MTS_FP64 ? 8 : 4;
    c->g = Geom{p->nx, p->ny, p->nz, (uint32_t)((uint32_t)p->nx * (uint32_t)p->ny)};
    c->S = (uint64_t)p->nx * p->ny * p->nz;
    c->plane = plane_of(*p);
    c->state = static_cast<char *>(dev_state);
    c->stream = static_cast<hipStream_t>(stream);
    c->tile = p->precision == MTS_FP64 ? TileShape{4, 32} : TileShape{8, 32};
    c->maxblk = site_blocks(c->g);
    for (int ty : {4, 5, 8, 12, 13}) c->maxblk = std::max(c->maxblk, tile_blocks(c->g, TileShape{ty, 1}));
    c->maxblk = std::max(c->maxblk, std::max(wind_blocks(c->g), overlap_blocks(c->g)));
    c->maxblk = std::max(c->maxblk, std::max(wind_fix_blocks(c->g), wind_tile_blocks(c->g)));
    hipError_t e = hipMalloc(&c->partials, sizeof(double) * NSLOT * (size_t)c->maxblk);
    if (e == hipSuccess) e = hipMalloc(&c->nblk_dev, sizeof(uint32_t) * 2 * NSLOT);
    if (e == hipSuccess) e = hipMalloc(&c->wabs, 2 * c->plane);
    if (e == hipSuccess) e = hipMalloc(&c->cells, 2 * c->plane);
    if (e == hipSuccess) e = hipMalloc(&c->alpha, 2 * c->plane * c->esz);
    if (e == hipSuccess && overlap_uses_bits(c->g))
        e = hipMalloc(&c->bits, sizeof(uint64_t) * 2 * (size_t)overlap_words(c->g));
    if (e == hipSuccess) e = hipMalloc(&c->ring, sizeof(double) * NSLOT * RING_CAP);
    if (e == hipSuccess) e = hipMalloc(&c->fixlist, sizeof(uint32_t) * (size_t)FIX_LIST_WORDS);
    if (e == hipSuccess) e = upload_nblk(c);
    if (e != hipSuccess) {
        std::fprintf(stderr, "mts_create: scratch allocation failed: %s\n", hipGetErrorString(e));
        mts_destroy(c);
        return MTS_ENOMEM;
    }
    // the static scratch of this device (used only by the entry points that
    // allocate nothing; a failure here is reported by them)
    const hipError_t es = noalloc_scratch(&c->noalloc);
    if (es != hipSuccess) {
        c->noalloc = nullptr;
        c->noalloc_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(es);
        (void)hipGetLastError();
    }
    *out = c;
    return MTS_OK;
}

int mts_destroy(mts_ctx *c) {
    if (!c) return MTS_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->partials);
    (void)hipFree(c->nblk_dev);
    (void)hipFree(c->wabs);
    (void)hipFree(c->cells);
    (void)hipFree(c->alpha);
    (void)hipFree(c->bits);
    (void)hipFree(c->ring);
    (void)hipFree(c->fixlist);
    (void)hipFree(c->mom2);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return MTS_OK;
}

int mts_init_fields(mts_ctx *c, uint64_t seed) {
    if (!c) return MTS_EINVAL;
    c->cur = 0;
    c->mcur = 0;
    c->step_count = 0;
    c->meta.clear();
    c->produced = c->drained = 0;
    c->have_cells = false;
    hipError_t e;
    if (c->p.precision == MTS_FP64)
        e = launch_init<double>(c->g, fields_of<double>(c, 0), moms_of<double>(c), seed, c->p.sigma_p, c->p.sigma_q,
                                c->stream);
    else
        e = launch_init<float>(c->g, fields_of<float>(c, 0), moms_of<float>(c), seed, c->p.sigma_p, c->p.sigma_q,
                               c->stream);
    if (e != hipSuccess) return hipfail(c, e, "init kernel launch");
    return MTS_OK;
}

int mts_step(mts_ctx *c, int32_t n, double eta, double era_m, double s) {
    if (!c) return MTS_EINVAL;
    const int rc = check_step(c, n, eta, era_m, s, s, INFINITY);
    if (rc != MTS_OK || n == 0) return rc;
    return c->p.precision == MTS_FP64 ? do_step<double>(c, n, eta, era_m, s) : do_step<float>(c, n, eta, era_m, s);
}

int mts_cool(mts_ctx *c, int32_t n, double dt_cool) {
    if (!c) return MTS_EINVAL;
    if (n < 0 || !(dt_cool > 0) || !std::isfinite(dt_cool)) return fail(c, MTS_EINVAL, "n >= 0 and dt_cool > 0 needed");
    // forward Euler on the flow is stable while dt (12/h^2 + mu2_max) < 2
    const double h = c->p.dx, bound = dt_cool * (12.0 / (h * h) + mu2_max(c->p));
    if (!(bound < 2.0)) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "unstable: dt_cool (12/h^2 + mu2_max) = %.4g >= 2", bound);
        return fail(c, MTS_EUNSTABLE, buf);
    }
    mts_params q = c->p;
    q.kappa = 0.0;             // the printed cooling equations have no coupling term
    q.dt = dt_cool;
    const Book b{1.0, 0.0, 0.0, 1.0};
    const bool tiled = c->tile.ty != 0;
    for (int32_t j = 0; j < n; j++) {
        hipError_t e;
        if (c->p.precision == MTS_FP64)
            e = tiled ? launch_cool_tile<double>(c->g, fields_of<double>(c, c->cur), fields_of<double>(c, 1 - c->cur),
                                                 coefficients<double>(q, b, 1.0), c->tile, c->stream)
                      : launch_cool<double>(c->g, fields_of<double>(c, c->cur), fields_of<double>(c, 1 - c->cur),
                                            moms_of<double>(c), coefficients<double>(q, b, 1.0), c->stream);
        else
            e = tiled ? launch_cool_tile<float>(c->g, fields_of<float>(c, c->cur), fields_of<float>(c, 1 - c->cur),
                                                coefficients<float>(q, b, 1.0), c->tile, c->stream)
                      : launch_cool<float>(c->g, fields_of<float>(c, c->cur), fields_of<float>(c, 1 - c->cur),
                                           moms_of<float>(c), coefficients<float>(q, b, 1.0), c->stream);
        if (e != hipSuccess) return hipfail(c, e, "cooling kernel launch");
        c->cur = 1 - c->cur;
    }
    return MTS_OK;
}

int mts_diagnostics(mts_ctx *c, mts_diag *out, int32_t max, int32_t *count) {
    if (!c || !count || (max > 0 && !out) || max < 0) return MTS_EINVAL;
    *count = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc = MTS_OK;
    const int64_t avail = c->produced - c->drained;
    const int64_t lost = std::max<int64_t>(0, avail - RING_CAP);
    const int64_t take = std::min<int64_t>(avail - lost, max);
    std::vector<double> rec(NSLOT);
    for (int64_t r = 0; r < take; r++) {
        const int64_t idx = c->drained + lost + r;
        HIPCHK(c, hipMemcpy(rec.data(), c->ring + (size_t)(idx % RING_CAP) * NSLOT, sizeof(double) * NSLOT,
                            hipMemcpyDeviceToHost));
        const Meta &mt = c->meta[(size_t)(lost + r)];
        mts_diag d;
        std::memset(&d, 0, sizeof d);
        const double h3 = c->p.dx * c->p.dx * c->p.dx;
        d.step = mt.step;
        d.eta = mt.eta;
        d.a = mt.a;
        d.s = mt.s;
        d.sum_energy = rec[SL_EPS] * h3;
        d.sum_lagrangian = rec[SL_LAG] * h3;
        d.sum_KL = rec[SL_KL];
        d.sum_GL = rec[SL_GL];
        d.sum_KV = rec[SL_KV];
        d.sum_GV = rec[SL_GV];
        d.gauss_abs[0] = rec[SL_GAUSS_ABS_P];
        d.gauss_abs[1] = rec[SL_GAUSS_ABS_Q];
        d.gauss_scale[0] = rec[SL_GAUSS_SCALE_P];
        d.gauss_scale[1] = rec[SL_GAUSS_SCALE_Q];
        d.wind_abs[0] = (int64_t)std::llround(rec[SL_WIND_P] + rec[SL_FIX_P]);
        d.wind_abs[1] = (int64_t)std::llround(rec[SL_WIND_Q] + rec[SL_FIX_Q]);
        d.pq_count2 = (int64_t)std::llround(rec[SL_OV_P] + rec[SL_OV_Q]);
        bool finite = true;
        for (int q = 0; q < NSLOT; q++) finite = finite && std::isfinite(rec[q]);
        derive(c->p, c->S, d);
        d.flags = (finite ? 0 : 1) | (lost > 0 ? 2 : 0);
        if (!finite) rc = MTS_ENONFINITE;
        out[r] = d;
    }
    c->drained += lost + take;
    c->meta.erase(c->meta.begin(), c->meta.begin() + (size_t)(lost + take));
    *count = (int32_t)take;
    if (rc == MTS_ENONFINITE) c->err = "a diagnostic reduction saw NaN or Inf";
    return rc;
}

int mts_get_fields(mts_ctx *c, double *host) {
    if (!c || !host) return MTS_EINVAL;
    return c->p.precision == MTS_FP64 ? get_fields_t<double>(c, host) : get_fields_t<float>(c, host);
}

int mts_set_fields(mts_ctx *c, const double *host) {
    if (!c || !host) return MTS_EINVAL;
    return c->p.precision == MTS_FP64 ? set_fields_t<double>(c, host) : set_fields_t<float>(c, host);
}

int mts_get_windings(mts_ctx *c, int8_t *host) {
    if (!c || !host) return MTS_EINVAL;
    return c->p.precision == MTS_FP64 ? get_windings_t<double>(c, host) : get_windings_t<float>(c, host);
}

int mts_get_sites(mts_ctx *c, const uint64_t *sites, int32_t n, double *host) {
    if (!c || n < 0 || (n > 0 && (!sites || !host))) return MTS_EINVAL;
    if (n == 0) return MTS_OK;
    for (int32_t i = 0; i < n; i++)
        if (sites[i] >= c->S) return fail(c, MTS_EINVAL, "site index out of range");
    uint64_t *dsites = nullptr;
    double *dout = nullptr;
    hipError_t e = hipMalloc(&dsites, sizeof(uint64_t) * n);
    if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double) * 20 * n);
    if (e == hipSuccess) e = hipMemcpyAsync(dsites, sites, sizeof(uint64_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = c->p.precision == MTS_FP64
                ? launch_gather<double>(fields_of<double>(c, c->cur), moms_of<double>(c), dsites, n, dout, c->stream)
                : launch_gather<float>(fields_of<float>(c, c->cur), moms_of<float>(c), dsites, n, dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dout, sizeof(double) * 20 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dsites);
    (void)hipFree(dout);
    if (e != hipSuccess) return hipfail(c, e, "get_sites");
    return MTS_OK;
}

int mts_get_sites_noalloc(mts_ctx *c, const uint64_t *sites, int32_t n, double *host) {
    if (!c || n < 0 || (n > 0 && (!sites || !host))) return MTS_EINVAL;
    if (n > MTS_NOALLOC_MAX_SITES) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "get_sites_noalloc: n = %d exceeds the static scratch's %d sites", (int)n,
                      (int)MTS_NOALLOC_MAX_SITES);
        return fail(c, MTS_EINVAL, buf);
    }
    if (n == 0) return MTS_OK;
    for (int32_t i = 0; i < n; i++)
        if (sites[i] >= c->S) return fail(c, MTS_EINVAL, "site index out of range");
    if (!c->noalloc) return fail(c, MTS_EHIP, c->noalloc_err);
    uint64_t *dsites = static_cast<uint64_t *>(c->noalloc);
    double *dout = reinterpret_cast<double *>(static_cast<char *>(c->noalloc) + NOALLOC_SITES_BYTES);
    hipError_t e = hipMemcpyAsync(dsites, sites, sizeof(uint64_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = c->p.precision == MTS_FP64
                ? launch_gather<double>(fields_of<double>(c, c->cur), moms_of<double>(c), dsites, n, dout, c->stream)
                : launch_gather<float>(fields_of<float>(c, c->cur), moms_of<float>(c), dsites, n, dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dout, sizeof(double) * 20 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hipfail(c, e, "get_sites_noalloc");
    return MTS_OK;
}

int mts_get_cells(mts_ctx *c, uint8_t *host) {
    if (!c || !host) return MTS_EINVAL;
    if (!c->have_cells) return fail(c, MTS_EINVAL, "no diagnostic step has run yet");
    std::vector<uint8_t> buf(2 * c->plane);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->cells, 2 * c->plane, hipMemcpyDeviceToHost));
    for (int q = 0; q < 2; q++) std::memcpy(host + (size_t)q * c->S, buf.data() + (size_t)q * c->plane, c->S);
    return MTS_OK;
}

int mts_segments(mts_ctx *c, double min_length, mts_segments_t *out, int64_t *sizes, int64_t cap, int64_t *n_sizes) {
    if (!c || !out || (cap > 0 && !sizes) || cap < 0) return MTS_EINVAL;
    if (!c->have_cells) return fail(c, MTS_EINVAL, "no diagnostic step has run yet");
    const uint32_t S = (uint32_t)c->S;
    const uint32_t dcap = (uint32_t)std::min<uint64_t>(c->S, 1u << 24);
    uint32_t *parent = nullptr, *count = nullptr, *dsz = nullptr, *dn = nullptr;
    hipError_t e = hipMalloc(&parent, sizeof(uint32_t) * S);
    if (e == hipSuccess) e = hipMalloc(&count, sizeof(uint32_t) * S);
    if (e == hipSuccess) e = hipMalloc(&dsz, sizeof(uint32_t) * dcap);
    if (e == hipSuccess) e = hipMalloc(&dn, sizeof(uint32_t));
    uint32_t nreg = 0;
    std::vector<uint32_t> hs;
    if (e == hipSuccess)
        e = launch_segments(c->g, c->cells, (uint32_t)c->plane, c->p.overlap_radius, parent, count, dsz, dn, dcap,
                            c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&nreg, dn, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && nreg <= dcap) {
        hs.resize(nreg);
        if (nreg) e = hipMemcpy(hs.data(), dsz, sizeof(uint32_t) * nreg, hipMemcpyDeviceToHost);
    }
    (void)hipFree(parent);
    (void)hipFree(count);
    (void)hipFree(dsz);
    (void)hipFree(dn);
    if (e != hipSuccess) return hipfail(c, e, "segments");
    if (nreg > dcap) return fail(c, MTS_ENOMEM, "more regions than the size list holds");
    std::sort(hs.begin(), hs.end(), [](uint32_t a, uint32_t b) { return a > b; });
    const double h = c->p.dx, V = (double)c->S * h * h * h;
    mts_segments_t r;
    std::memset(&r, 0, sizeof r);
    r.step = c->cells_step;
    r.regions = (int64_t)hs.size();
    for (uint32_t v : hs) {
        r.marked_cells += v;
        const double L = (double)(v - 1) * h;
        if (L > min_length) {
            r.n_pq++;
            r.L_pq += L;
        }
    }
    r.largest = hs.empty() ? 0 : hs[0];
    r.l_pq = r.n_pq ? r.L_pq / (double)r.n_pq : NAN;
    r.xi_pq = r.L_pq > 0 ? std::sqrt(V / r.L_pq) : INFINITY;
    *out = r;
    if (n_sizes) *n_sizes = (int64_t)hs.size();
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)hs.size()); i++) sizes[i] = hs[i];
    return MTS_OK;
}

int mts_set_tile(mts_ctx *c, int32_t ty, int32_t tz) {
    if (!c) return MTS_EINVAL;
    const TileShape ts{ty, tz};
    // tz >= 1 also with ty = 0: the diagnostic paths size their tiled grids
    // from the stored tz
    if (tz < 1 || (ty != 0 && !tile_supported(ts, c->p.precision == MTS_FP64)))
        return fail(c, MTS_EINVAL, "tile: ty must be 0, 4, 5, 8, 12 or (FP32) 13 and tz >= 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->tile = ts;
    HIPCHK(c, upload_nblk(c));
    return MTS_OK;
}

int mts_set_streaming_stores(mts_ctx *c, int32_t on) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nt = on != 0;
    return MTS_OK;
}

// The second momentum copy (10 planes), allocated on first use.
static int ensure_mom2(mts_ctx *c, const char *what) {
    if (c->mom2) return MTS_OK;
    hipError_t e = hipMalloc(&c->mom2, (size_t)10 * c->plane * c->esz);
    if (e != hipSuccess) {
        c->mom2 = nullptr;
        (void)hipGetLastError();
        return fail(c, MTS_ENOMEM, std::string(what) + ": second momentum copy: " + hipGetErrorString(e));
    }
    return MTS_OK;
}

int mts_set_fused_diagnostics(mts_ctx *c, int32_t rows) {
    if (!c) return MTS_EINVAL;
    if (rows != 0 && rows != 4 && rows != 5 && rows != 8)
        return fail(c, MTS_EINVAL, "fused diagnostics: rows must be 0 (off), 4, 5 or 8");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->fuse_ty = rows;
    if (rows) c->fuse_off = false;   // try the second momentum copy again
    HIPCHK(c, upload_nblk(c));
    return MTS_OK;
}

int mts_get_fused_diagnostics(const mts_ctx *c, int32_t *rows) {
    if (!c || !rows) return MTS_EINVAL;
    *rows = diag_fused(c) ? c->fuse_ty : 0;
    return MTS_OK;
}

int mts_set_momentum_pingpong(mts_ctx *c, int32_t on) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (on) {
        const int rc = ensure_mom2(c, "momentum ping-pong");
        if (rc != MTS_OK) return rc;
    }
    c->mpp = on != 0;
    return MTS_OK;
}

int mts_get_momentum_pingpong(const mts_ctx *c, int32_t *on) {
    if (!c || !on) return MTS_EINVAL;
    *on = c->mpp ? 1 : 0;
    return MTS_OK;
}

int mts_set_tile_order(mts_ctx *c, int32_t xcd_runs) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->xcd = xcd_runs != 0;
    return MTS_OK;
}

int mts_get_tile_order(const mts_ctx *c, int32_t *xcd_runs) {
    if (!c || !xcd_runs) return MTS_EINVAL;
    *xcd_runs = c->xcd ? 1 : 0;
    return MTS_OK;
}

int mts_set_prefetch(mts_ctx *c, int32_t on) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pf = on != 0;
    return MTS_OK;
}

int mts_get_prefetch(const mts_ctx *c, int32_t *on) {
    if (!c || !on) return MTS_EINVAL;
    *on = c->pf ? 1 : 0;
    return MTS_OK;
}

int mts_get_streaming_stores(const mts_ctx *c, int32_t *on) {
    if (!c || !on) return MTS_EINVAL;
    *on = c->nt ? 1 : 0;
    return MTS_OK;
}

int mts_get_tile(const mts_ctx *c, int32_t *ty, int32_t *tz) {
    if (!c || !ty || !tz) return MTS_EINVAL;
    *ty = c->tile.ty;
    *tz = c->tile.tz;
    return MTS_OK;
}

int mts_bandwidth_probe(mts_ctx *c, int32_t reps, double *copy_gbps, double *pattern_gbps) {
    if (!c || reps < 1 || !copy_gbps || !pattern_gbps) return MTS_EINVAL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t ec = hipEventCreate(&e0);
    if (ec == hipSuccess) ec = hipEventCreate(&e1);
    if (ec != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hipfail(c, ec, "hipEventCreate");
    }
    const uint64_t copy_bytes = (uint64_t)10 * c->plane * c->esz;   // one field copy onto the other
    const double pattern_bytes = (double)(c->esz * 40) * (double)c->S;
    auto run = [&](auto launch, double bytes, double *out) -> int {
        hipError_t e = launch();                                    // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; e == hipSuccess && r < reps; r++) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) return hipfail(c, e, "bandwidth probe");
        *out = bytes * reps / (ms * 1e-3) / 1e9;
        return MTS_OK;
    };
    int rc = run([&] { return launch_probe_copy(c->state, copy_bytes, c->stream); }, 2.0 * (double)copy_bytes,
                 copy_gbps);
    if (rc == MTS_OK) {
        if (c->p.precision == MTS_FP64)
            rc = run([&] { return launch_probe_pattern<double>(reinterpret_cast<double *>(c->state), c->plane,
                                                               (uint32_t)c->S, c->cur, c->nt, c->stream); },
                     pattern_bytes, pattern_gbps);
        else
            rc = run([&] { return launch_probe_pattern<float>(reinterpret_cast<float *>(c->state), c->plane,
                                                              (uint32_t)c->S, c->cur, c->nt, c->stream); },
                     pattern_bytes, pattern_gbps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int mts_set_time_blocking(mts_ctx *c, int32_t steps, int32_t ty, int32_t tz) {
    if (!c) return MTS_EINVAL;
    if (steps == 1) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->tblock = 1;
        return MTS_OK;
    }
    if (steps != 2) return fail(c, MTS_EINVAL, "time blocking: steps must be 1 or 2");
    if (c->p.precision != MTS_FP32) return fail(c, MTS_EINVAL, "time blocking: FP32 only");
    if (!pair_tile_supported(TileShape{ty, tz})) return fail(c, MTS_EINVAL, "time blocking: ty must be 3 or 7 and tz >= 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int rc = ensure_mom2(c, "time blocking");
    if (rc != MTS_OK) return rc;
    c->tblock = 2;
    c->tile2 = TileShape{ty, tz};
    return MTS_OK;
}

int mts_get_time_blocking(const mts_ctx *c, int32_t *steps, int32_t *ty, int32_t *tz) {
    if (!c || !steps || !ty || !tz) return MTS_EINVAL;
    *steps = c->tblock;
    *ty = c->tile2.ty;
    *tz = c->tile2.tz;
    return MTS_OK;
}

int mts_autotune(mts_ctx *c, int32_t steps, int32_t *ty_out, int32_t *tz_out, double *ms_out) {
    if (!c || steps < 1) return MTS_EINVAL;
    const std::vector<int> tys = c->p.precision == MTS_FP64 ? std::vector<int>{4, 5, 8} : std::vector<int>{4, 8, 12, 13};
    const int tzs[] = {8, 16, 32, 64};
    // time the plain update, outside the caller's timing; every exit below
    // restores these settings
    const int32_t d = c->p.diag_every;
    const bool timing = c->timing;
    c->p.diag_every = 0;
    c->timing = false;
    c->tblock = 1;               // single-step shapes first; the choice is set at the end
    c->mpp = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MTS_OK;
    auto hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == MTS_OK) rc = hipfail(c, e, what);
        return rc == MTS_OK;
    };
    hip(hipEventCreate(&e0), "hipEventCreate") && hip(hipEventCreate(&e1), "hipEventCreate");
    double best = INFINITY;
    TileShape pick = c->tile;
    bool pick_nt = c->nt, pick_pf = c->pf;
    if (rc == MTS_OK) rc = mts_init_fields(c, 0);
    for (int pf = 0; pf < 2; pf++)
    for (int nt = 0; nt < 2; nt++)
    for (int ty : tys) {
        for (int tz : tzs) {
            if (rc != MTS_OK) break;
            if (tz > 2 * c->p.nz && tz != 8) continue;
            c->nt = nt != 0;
            c->pf = pf != 0;
            if ((rc = mts_set_tile(c, ty, tz)) != MTS_OK) break;
            if ((rc = mts_step(c, 1, 1.0, 0.5, 1.0)) != MTS_OK) break;       // warm
            if (!hip(hipEventRecord(e0, c->stream), "hipEventRecord")) break;
            if ((rc = mts_step(c, steps, 1.1, 0.5, 1.0)) != MTS_OK) break;
            float ms = 0;
            if (!(hip(hipEventRecord(e1, c->stream), "hipEventRecord") &&
                  hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
                  hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")))
                break;
            if (ms < best) {
                best = ms;
                pick = TileShape{ty, tz};
                pick_nt = nt != 0;
                pick_pf = pf != 0;
            }
        }
    }
    // the best single-step configuration again with the momenta written to the other copy
    bool pick_mpp = false;
    if (rc == MTS_OK) {
        c->nt = pick_nt;
        c->pf = pick_pf;
        rc = mts_set_tile(c, pick.ty, pick.tz);
        const int r2 = rc == MTS_OK ? mts_set_momentum_pingpong(c, 1) : rc;
        if (r2 == MTS_OK) {
            float ms = 0;
            if ((rc = mts_step(c, 1, 1.0, 0.5, 1.0)) == MTS_OK && hip(hipEventRecord(e0, c->stream), "hipEventRecord") &&
                (rc = mts_step(c, steps, 1.1, 0.5, 1.0)) == MTS_OK &&
                hip(hipEventRecord(e1, c->stream), "hipEventRecord") &&
                hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
                hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime") && ms < best) {
                best = ms;
                pick_mpp = true;
            }
        } else if (r2 != MTS_ENOMEM) {
            rc = r2;
        }
        c->mpp = false;
        if (rc == MTS_OK) c->err.clear();
    }
    // and with the other tile order (contiguous runs per XCD or round-robin),
    // kept only if at least 1 % faster: at equal speed the XCD runs fetch
    // less through the fabric
    bool pick_xcd = c->xcd;
    if (rc == MTS_OK) {
        c->mpp = pick_mpp;
        c->xcd = !pick_xcd;
        float ms = 0;
        if ((rc = mts_step(c, 1, 1.0, 0.5, 1.0)) == MTS_OK && hip(hipEventRecord(e0, c->stream), "hipEventRecord") &&
            (rc = mts_step(c, steps, 1.3, 0.5, 1.0)) == MTS_OK &&
            hip(hipEventRecord(e1, c->stream), "hipEventRecord") &&
            hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
            hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime") && ms < 0.99 * best) {
            best = ms;
            pick_xcd = !pick_xcd;
        }
        c->xcd = pick_xcd;
        c->mpp = false;
    }

    // two steps per sweep (FP32), timed over an even number of steps, per step
    double best_ps = best / steps;
    int pick_tb = 1;
    TileShape pick2 = c->tile2;
    bool pick2_nt = pick_nt;
    const int32_t steps2 = 2 * ((steps + 1) / 2);
    if (rc == MTS_OK && c->p.precision == MTS_FP32) {
        if (rc == MTS_OK) rc = mts_set_tile(c, pick.ty, pick.tz);
        bool room = true;
        for (int nt = 0; nt < 2 && rc == MTS_OK && room; nt++)
            for (int ty : {3, 7})
                for (int tz : tzs) {
                    if (rc != MTS_OK || !room) break;
                    if (tz > 2 * c->p.nz && tz != 8) continue;
                    c->nt = nt != 0;
                    const int r2 = mts_set_time_blocking(c, 2, ty, tz);
                    if (r2 == MTS_ENOMEM) {   // no room for the second momentum copy: single steps only
                        room = false;
                        break;
                    }
                    if ((rc = r2) != MTS_OK) break;
                    if ((rc = mts_step(c, 2, 1.0, 0.5, 1.0)) != MTS_OK) break;   // warm
                    if (!hip(hipEventRecord(e0, c->stream), "hipEventRecord")) break;
                    if ((rc = mts_step(c, steps2, 1.2, 0.5, 1.0)) != MTS_OK) break;
                    float ms = 0;
                    if (!(hip(hipEventRecord(e1, c->stream), "hipEventRecord") &&
                          hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
                          hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")))
                        break;
                    if (ms / steps2 < best_ps) {
                        best_ps = ms / steps2;
                        pick_tb = 2;
                        pick2 = TileShape{ty, tz};
                        pick2_nt = nt != 0;
                    }
                }
        c->err.clear();
    }
    c->nt = pick_tb == 2 ? pick2_nt : pick_nt;
    c->pf = pick_pf;
    c->mpp = pick_mpp;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->p.diag_every = d;
    c->timing = timing;
    if (rc != MTS_OK) return rc;
    if ((rc = mts_set_tile(c, pick.ty, pick.tz)) != MTS_OK) return rc;
    if ((rc = mts_set_time_blocking(c, pick_tb, pick2.ty, pick2.tz)) != MTS_OK) return rc;
    if ((rc = mts_init_fields(c, 0)) != MTS_OK) return rc;   // momenta back in the state buffer
    if (pick_tb == 1 && !pick_mpp && c->mom2) {              // the second momentum copy is not needed
        HIPCHK(c, hipStreamSynchronize(c->stream));
        (void)hipFree(c->mom2);
        c->mom2 = nullptr;
    }
    if (ty_out) *ty_out = pick.ty;
    if (tz_out) *tz_out = pick.tz;
    if (ms_out) *ms_out = best_ps;
    return MTS_OK;
}

}  // extern "C"

// ---- autotune cache
//
// One line per tuned configuration, appended after a tuning run:
//   mts-tune-1 <arch> cu=<CUs> n=<nx>x<ny>x<nz> prec=<fp32|fp64> | ty= tz= nt= pf= pp= xcd= tb= ty2= tz2= ms=
// The last line with a matching key wins; lines that do not parse are skipped.

namespace {

std::string tune_key(const mts_ctx *c) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "mts-tune-1 %s cu=%d n=%dx%dx%d prec=%s", arch.c_str(), cus, c->p.nx, c->p.ny,
                  c->p.nz, c->p.precision == MTS_FP64 ? "fp64" : "fp32");
    return buf;
}

struct TunePick {
    int ty, tz, nt, pf, pp, xcd, tb, ty2, tz2;
    double ms;
};

bool tune_lookup(const char *path, const std::string &key, TunePick *out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char *bar = std::strstr(line, " | ");
        if (!bar || (size_t)(bar - line) != key.size() || std::strncmp(line, key.c_str(), key.size()) != 0) continue;
        TunePick t{};
        if (std::sscanf(bar + 3, "ty=%d tz=%d nt=%d pf=%d pp=%d xcd=%d tb=%d ty2=%d tz2=%d ms=%lf", &t.ty, &t.tz,
                        &t.nt, &t.pf, &t.pp, &t.xcd, &t.tb, &t.ty2, &t.tz2, &t.ms) == 10) {
            *out = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

bool tune_store(const char *path, const std::string &key, const TunePick &t) {
    FILE *f = std::fopen(path, "a");
    if (!f) return false;
    const int w = std::fprintf(f, "%s | ty=%d tz=%d nt=%d pf=%d pp=%d xcd=%d tb=%d ty2=%d tz2=%d ms=%.6f\n", key.c_str(),
                               t.ty, t.tz, t.nt, t.pf, t.pp, t.xcd, t.tb, t.ty2, t.tz2, t.ms);
    return std::fclose(f) == 0 && w > 0;
}

}  // namespace

extern "C" {

int mts_autotune_cached(mts_ctx *c, int32_t steps, const char *cache_path, int32_t *hit, int32_t *ty_out,
                        int32_t *tz_out, double *ms_out) {
    if (!c || steps < 1 || !cache_path) return MTS_EINVAL;
    const std::string key = tune_key(c);
    TunePick t{};
    if (tune_lookup(cache_path, key, &t)) {
        // apply the stored choice with the setters (each checks its own values)
        int rc = mts_set_tile(c, t.ty, t.tz);
        if (rc == MTS_OK) rc = mts_set_streaming_stores(c, t.nt);
        if (rc == MTS_OK) rc = mts_set_prefetch(c, t.pf);
        if (rc == MTS_OK) rc = mts_set_tile_order(c, t.xcd);
        if (rc == MTS_OK) rc = mts_set_momentum_pingpong(c, t.pp);
        if (rc == MTS_OK) rc = mts_set_time_blocking(c, t.tb, t.ty2, t.tz2);
        if (rc == MTS_OK) {
            if (hit) *hit = 1;
            if (ty_out) *ty_out = t.ty;
            if (tz_out) *tz_out = t.tz;
            if (ms_out) *ms_out = t.ms;
            return MTS_OK;
        }
        if (rc != MTS_ENOMEM && rc != MTS_EINVAL) return rc;
        // a choice this context cannot take (no room for a second momentum
        // copy, a tile shape the library no longer supports): tune afresh
        c->err.clear();
    }
    double ms = 0.0;
    int32_t ty = 0, tz = 0;
    const int rc = mts_autotune(c, steps, &ty, &tz, &ms);
    if (rc != MTS_OK) return rc;
    t = TunePick{c->tile.ty, c->tile.tz, c->nt ? 1 : 0, c->pf ? 1 : 0, c->mpp ? 1 : 0, c->xcd ? 1 : 0, c->tblock,
                 c->tile2.ty, c->tile2.tz, ms};
    const bool stored = tune_store(cache_path, key, t);
    if (!stored) c->err = std::string("autotune cache: could not append to ") + cache_path;
    if (hit) *hit = stored ? 0 : -1;
    if (ty_out) *ty_out = ty;
    if (tz_out) *tz_out = tz;
    if (ms_out) *ms_out = ms;
    return MTS_OK;
}

int mts_timing_enable(mts_ctx *c, int32_t on) {
    if (!c) return MTS_EINVAL;
    c->timing = on != 0;
    return MTS_OK;
}

int mts_timing_read(mts_ctx *c, int64_t *n_plain, double *ms_plain, int64_t *n_diag, double *ms_diag,
                    double *ms_post, int64_t *n_pair, double *ms_pair) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t np = 0, nd = 0, n2 = 0;
    double tp = 0, td = 0, tq = 0, t2 = 0;
    for (const auto &mk : c->marks) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[mk.a], c->ev_pool[mk.b]));
        if (mk.kind == 0) np++, tp += ms;
        else if (mk.kind == 1) nd++, td += ms;
        else if (mk.kind == 3) n2++, t2 += ms;
        else tq += ms;
    }
    if (n_pair) *n_pair = n2;
    if (ms_pair) *ms_pair = t2;
    c->marks.clear();
    c->ev_used = 0;
    if (n_plain) *n_plain = np;
    if (ms_plain) *ms_plain = tp;
    if (n_diag) *n_diag = nd;
    if (ms_diag) *ms_diag = td;
    if (ms_post) *ms_post = tq;
    return MTS_OK;
}

const char *mts_last_error(const mts_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

const char *mts_strerror(int code) {
    switch (code) {
        case MTS_OK: return "MTS_OK";
        case MTS_EINVAL: return "MTS_EINVAL";
        case MTS_EUNSTABLE: return "MTS_EUNSTABLE";
        case MTS_ENOMEM: return "MTS_ENOMEM";
        case MTS_EHIP: return "MTS_EHIP";
        case MTS_ENONFINITE: return "MTS_ENONFINITE";
        default: return "MTS_E?";
    }
}

}  // extern "C"

// ===================================================================== ensembles

struct mts_batch {
    std::vector<mts_ctx *> box;
    int precision = MTS_FP32;
    hipStream_t user = nullptr;      // caller's stream
    hipStream_t stream = nullptr;    // internal stream the graphs are captured on and launched to
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    void *boxes_dev = nullptr;       // BatchBox<T>[nbox] for plain steps
    void *boxes_diag_dev = nullptr;  // BatchBox<T>[nbox] for diagnostic steps (their own tile rows)
    int32_t ty_diag = 8;
    uint32_t nblk_diag = 0;
    bool fused = false;              // FP32 diagnostic steps fused (windings, Gauss) with batched post-step launches
    void *post_dev = nullptr;        // BatchPost<T>[nbox]
    uint32_t nfix = 0, ncells = 0, nov = 0;   // blocks of the batched post-step launches
    bool nt = true;                  // streaming stores in the tiled update
    bool mpp = false;                // plain tiled steps write the momenta to the other copy
    bool xcd = true;                 // tiles dealt to the XCDs in contiguous runs (else round-robin)
    bool persist = false;            // runs of plain steps in one persistent launch (grid barrier per step)
    GridSync *gsync = nullptr;       // the persistent kernel's barrier state
    double persist_wait_s = 10.0;    // longest barrier wait before the launch gives up
    double tune_graph_ms = 0.0, tune_persist_ms = 0.0;   // the autotuner's last per-step times of both forms
    void *coef_dev = nullptr;        // StepCoef<T>[n][nbox]
    size_t coef_cap = 0;             // bytes
    int32_t ty = 8;
    std::vector<int32_t> tz;
    uint32_t nblk = 0;
    hipGraphExec_t exec = nullptr;   // last launched graph (kept until the next call)
    hipGraph_t graph = nullptr;
    int64_t t_steps = 0;
    double t_ms = 0.0;
    bool t_pending = false;
    int64_t t_pending_steps = 0;
    std::string err;
};

namespace {

int bfail(mts_batch *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(bb, call)                                                                           \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return bfail(bb, MTS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

template <typename T>
int batch_upload_boxes(mts_batch *b) {
    const size_t nbox = b->box.size();
    std::vector<BatchBox<T>> h(nbox), hd(nbox);
    std::vector<BatchPost<T>> hp(nbox);
    uint32_t blk = 0, blkd = 0, bfix = 0, bcells = 0, bov = 0;
    for (size_t k = 0; k < nbox; k++) {
        mts_ctx *c = b->box[k];
        c->tile = TileShape{b->ty, b->tz[k]};
        c->fuse_ty = b->fused ? 8 : 0;   // the batch's fused diagnostic tile has 8 rows
        b->ty_diag = b->fused ? 8 : diag_tile(c).ty;
        for (int pass = 0; pass < 2; pass++) {
            BatchBox<T> &x = pass == 0 ? h[k] : hd[k];
            const int ty = pass == 0 ? b->ty : b->ty_diag;
            uint32_t &acc = pass == 0 ? blk : blkd;
            x.g = c->g;
            x.f[0] = fields_of<T>(c, 0);
            x.f[1] = fields_of<T>(c, 1);
            x.mom[0] = moms_at<T>(c, 0);
            x.mom[1] = moms_at<T>(c, c->mom2 ? 1 : 0);
            x.part = Partials{c->partials, c->maxblk};
            x.alpha = diag_writes_alpha(c) ? static_cast<T *>(c->alpha) : nullptr;
            x.wabs = c->wabs;
            x.plane = (uint32_t)c->plane;
            x.tz = b->tz[k];
            x.ntx = (c->g.nx + 63) / 64;
            x.nty = (c->g.ny + ty - 1) / ty;
            x.ntz = (c->g.nz + x.tz - 1) / x.tz;
            x.blk0 = acc;
            acc += (uint32_t)(x.ntx * x.nty * x.ntz);
        }
        hipError_t e = upload_nblk(c);
        if (e != hipSuccess) return bfail(b, MTS_EHIP, std::string("upload_nblk: ") + hipGetErrorString(e));
        BatchPost<T> &q = hp[k];
        q.g = c->g;
        q.f[0] = fields_of<T>(c, 0);
        q.f[1] = fields_of<T>(c, 1);
        q.part = Partials{c->partials, c->maxblk};
        q.wabs = c->wabs;
        q.fixlist = c->fixlist;
        q.cells = c->cells;
        q.bits = overlap_uses_bits(c->g) ? c->bits : nullptr;
        q.plane = (uint32_t)c->plane;
        q.nwords = overlap_words(c->g);
        q.radius = c->p.overlap_radius;
        q.h = (T)c->p.dx;
        q.nblk = c->nblk_dev + NSLOT;
        q.ring = c->ring;
        q.blk_fix = bfix;
        q.blk_cells = bcells;
        q.blk_ov = bov;
        bfix += wind_fix_scan_blocks(c->g);
        bcells += cells_blocks(c->g);
        bov += overlap_blocks(c->g);
    }
    b->nblk = blk;
    b->nblk_diag = blkd;
    b->nfix = bfix;
    b->ncells = bcells;
    b->nov = bov;
    BHIPCHK(b, hipMemcpy(b->boxes_dev, h.data(), sizeof(BatchBox<T>) * nbox, hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(b->boxes_diag_dev, hd.data(), sizeof(BatchBox<T>) * nbox, hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(b->post_dev, hp.data(), sizeof(BatchPost<T>) * nbox, hipMemcpyHostToDevice));
    return MTS_OK;
}

int batch_upload(mts_batch *b) {
    return b->precision == MTS_FP64 ? batch_upload_boxes<double>(b) : batch_upload_boxes<float>(b);
}

void batch_release_graph(mts_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void batch_collect_timing(mts_batch *b) {
    if (!b->t_pending) return;
    float ms = 0;
    if (hipEventElapsedTime(&ms, b->ev_t0, b->ev_t1) == hipSuccess) {
        b->t_ms += ms;
        b->t_steps += b->t_pending_steps;
    }
    b->t_pending = false;
}

// After the batch's stream has drained: did a persistent launch give up at a
// barrier?  Reported once (the flag is cleared); the fields of every box are
// then those of an unfinished step.
int batch_check_persist(mts_batch *b) {
    if (!b->gsync) return MTS_OK;
    GridSync h{};
    BHIPCHK(b, hipMemcpy(&h, b->gsync, sizeof h, hipMemcpyDeviceToHost));
    if (h.err == 0) return MTS_OK;
    BHIPCHK(b, hipMemset(&b->gsync->err, 0, sizeof(int32_t)));
    return bfail(b, MTS_EHIP,
                 "persistent ensemble launch: a grid-barrier wait ran out (workgroups not co-resident, or a step "
                 "slower than the wait limit); the fields hold an unfinished step");
}

// Launch of a run of nrun plain steps of every box as one persistent kernel
// (after the kernel that clears its barrier state).
template <typename T>
hipError_t batch_persist_run(mts_batch *b, int32_t j0, int32_t nrun) {
    const size_t nbox = b->box.size();
    int grid = 0;
    hipError_t e = persist_max_blocks(b->precision == MTS_FP64, b->ty, b->nt, &grid);
    if (e != hipSuccess) return e;
    if (grid <= 0) return hipErrorInvalidConfiguration;
    grid = std::min<int>(grid, (int)b->nblk);   // no more workgroups than tiles
    int dev = 0, khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    PersistArgs<T> a{};
    a.boxes = static_cast<const BatchBox<T> *>(b->boxes_dev);
    a.nbox = (int32_t)nbox;
    a.ntiles = b->nblk;
    a.coef = static_cast<const StepCoef<T> *>(b->coef_dev) + (size_t)j0 * nbox;
    a.nsteps = nrun;
    a.parity0 = b->box[0]->cur;
    a.mcur0 = b->box[0]->mcur;
    a.mpp = b->mpp ? 1 : 0;
    a.sync = b->gsync;
    a.limit_ticks = (uint64_t)std::max(1.0, b->persist_wait_s * 1e3 * (double)khz);
    e = launch_persist_reset(b->gsync, b->stream);
    if (e == hipSuccess) e = launch_persist<T>(a, b->ty, b->nt, (uint32_t)grid, b->stream);
    return e;
}

template <typename T>
int batch_step_t(mts_batch *b, int32_t n, const double *eta0, const double *era_m, const double *s_before,
                 const double *s_after, const double *eta_switch) {
    const size_t nbox = b->box.size();
    // per-box, per-step coefficients (FP64 bookkeeping, cast once)
    const size_t need = sizeof(StepCoef<T>) * nbox * (size_t)n;
    if (need > b->coef_cap) {
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        batch_release_graph(b);
        (void)hipFree(b->coef_dev);
        b->coef_dev = nullptr;
        b->coef_cap = 0;
        BHIPCHK(b, hipMalloc(&b->coef_dev, need));
        b->coef_cap = need;
    }
    std::vector<StepCoef<T>> tab(nbox * (size_t)n);
    std::vector<std::vector<Book>> books(nbox, std::vector<Book>((size_t)n));
    std::vector<std::vector<double>> svals(nbox, std::vector<double>((size_t)n));
    for (size_t k = 0; k < nbox; k++) {
        const mts_params &p = b->box[k]->p;
        for (int32_t j = 0; j < n; j++) {
            const double eta_j = eta0[k] + j * p.dt;
            const double sw = eta_switch ? eta_switch[k] : INFINITY;
            const double sj = eta_j < sw ? s_before[k] : (s_after ? s_after[k] : s_before[k]);
            books[k][j] = bookkeeping(p, eta_j, era_m[k], sj);
            svals[k][j] = sj;
            tab[(size_t)j * nbox + k] = coefficients<T>(p, books[k][j], sj);
        }
    }
    // the previous call's graph may still read the table: order the upload after it
    BHIPCHK(b, hipMemcpyAsync(b->coef_dev, tab.data(), need, hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    batch_collect_timing(b);
    batch_release_graph(b);
    if (const int rc = batch_check_persist(b); rc != MTS_OK) return rc;

    // Host bookkeeping advances while the steps are captured; nothing runs
    // until the graph is launched, so a failure before that restores it.
    struct Saved {
        int cur, mcur;
        int64_t step_count, produced, cells_step;
        size_t nmeta;
        bool have_cells;
    };
    std::vector<Saved> saved;
    for (mts_ctx *c : b->box)
        saved.push_back({c->cur, c->mcur, c->step_count, c->produced, c->cells_step, c->meta.size(), c->have_cells});
    auto rollback = [&](int code, const std::string &why) {
        for (size_t k = 0; k < nbox; k++) {
            mts_ctx *c = b->box[k];
            c->cur = saved[k].cur;
            c->mcur = saved[k].mcur;
            c->step_count = saved[k].step_count;
            c->produced = saved[k].produced;
            c->cells_step = saved[k].cells_step;
            c->meta.resize(saved[k].nmeta);
            c->have_cells = saved[k].have_cells;
        }
        batch_release_graph(b);
        return bfail(b, code, why);
    };

    // join the caller's stream, capture all n steps, launch once, join back
    BHIPCHK(b, hipEventRecord(b->ev_in, b->user));
    BHIPCHK(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
    BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    const int32_t d = b->box[0]->p.diag_every;
    for (int32_t j = 0; j < n && err == hipSuccess; j++) {
        mts_ctx *c0 = b->box[0];
        const bool diag = d > 0 && (c0->step_count % d) == 0;
        if (!diag && b->persist) {
            // the run of plain steps up to the next diagnostic step (or the end of the call)
            int32_t r = 1;
            while (j + r < n && !(d > 0 && (c0->step_count + r) % d == 0)) r++;
            err = batch_persist_run<T>(b, j, r);
            for (int32_t i = 0; i < r; i++)
                for (mts_ctx *c : b->box) {
                    c->cur = 1 - c->cur;
                    c->step_count++;
                    if (b->mpp) c->mcur = 1 - c->mcur;
                }
            j += r - 1;
            continue;
        }
        if (diag && diag_per_site(c0)) {
            // diagnostic steps of per-site boxes: the per-site kernel, box by box (as single contexts do)
            for (size_t k = 0; k < nbox && err == hipSuccess; k++) {
                mts_ctx *c = b->box[k];
                err = launch_step<T>(c->g, fields_of<T>(c, c->cur), fields_of<T>(c, 1 - c->cur), moms_of<T>(c),
                                     tab[(size_t)j * nbox + k], true, Partials{c->partials, c->maxblk}, b->stream);
            }
        } else {
            // momenta to the other copy on plain steps under ping-pong and on fused diagnostic steps, in
            // place otherwise
            const bool fused = diag && b->fused;
            const int mpin = c0->mcur, mpout = (b->mpp && !diag) || fused ? 1 - mpin : mpin;
            err = launch_step_tile_batch<T>(static_cast<const BatchBox<T> *>(diag ? b->boxes_diag_dev : b->boxes_dev),
                                            (int)nbox, diag ? b->nblk_diag : b->nblk, c0->cur, mpin, mpout,
                                            static_cast<const StepCoef<T> *>(b->coef_dev) + (size_t)j * nbox, diag,
                                            diag ? b->ty_diag : b->ty, b->nt, b->xcd, fused, b->stream);
            if (mpout != mpin)
                for (mts_ctx *c : b->box) c->mcur = mpout;
        }
        if (diag && b->fused && err == hipSuccess) {
            // the post-step kernels of all boxes, one launch each; every box's ring advances together
            err = launch_post_batch<T>(static_cast<const BatchPost<T> *>(b->post_dev), (int)nbox, b->nfix, b->ncells,
                                       b->nov, c0->cur, (uint32_t)(c0->produced % RING_CAP), b->stream);
            for (size_t k = 0; k < nbox && err == hipSuccess; k++) {
                mts_ctx *c = b->box[k];
                c->meta.push_back({c->step_count, eta0[k] + j * c->p.dt, books[k][j].a, svals[k][j]});
                c->produced++;
                c->have_cells = true;
                c->cells_step = c->step_count;
            }
        } else if (diag) {
            for (size_t k = 0; k < nbox && err == hipSuccess; k++)
                err = enqueue_diag_post<T>(b->box[k], books[k][j], eta0[k] + j * b->box[k]->p.dt, svals[k][j],
                                           b->stream, diag_writes_alpha(b->box[k]));
        }
        for (mts_ctx *c : b->box) {
            c->cur = 1 - c->cur;
            c->step_count++;
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rollback(MTS_EHIP, std::string("batch capture: ") + hipGetErrorString(err));
    }
    if (ec != hipSuccess) return rollback(MTS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    b->graph = g;
    hipError_t el = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (el != hipSuccess) return rollback(MTS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(el));
    el = hipEventRecord(b->ev_t0, b->stream);
    if (el == hipSuccess) el = hipGraphLaunch(b->exec, b->stream);
    if (el != hipSuccess) return rollback(MTS_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(el));
    BHIPCHK(b, hipEventRecord(b->ev_t1, b->stream));
    b->t_pending = true;
    b->t_pending_steps = n;
    BHIPCHK(b, hipEventRecord(b->ev_out, b->stream));
    BHIPCHK(b, hipStreamWaitEvent(b->user, b->ev_out, 0));
    return MTS_OK;
}

}  // namespace

extern "C" {

size_t mts_batch_state_bytes(const mts_params *boxes, int32_t nbox) {
    if (!boxes || nbox <= 0) return 0;
    size_t tot = 0;
    for (int32_t k = 0; k < nbox; k++) {
        const size_t v = mts_state_bytes(&boxes[k]);
        if (v == 0) return 0;
        tot += align256(v);
    }
    return tot;
}

int mts_batch_create(const mts_params *boxes, int32_t nbox, void *dev_pool, size_t pool_bytes, void *stream,
                     mts_batch **out) {
    if (!out) return MTS_EINVAL;
    *out = nullptr;
    if (!boxes || nbox <= 0) return MTS_EINVAL;
    for (int32_t k = 1; k < nbox; k++)
        if (boxes[k].precision != boxes[0].precision || boxes[k].diag_every != boxes[0].diag_every) {
            std::fprintf(stderr, "mts_batch_create: every box must share precision and diag_every\n");
            return MTS_EINVAL;
        }
    const size_t need = mts_batch_state_bytes(boxes, nbox);
    if (need == 0) return MTS_EINVAL;
    if (!dev_pool || (reinterpret_cast<uintptr_t>(dev_pool) & 255) != 0) return MTS_EINVAL;
    if (pool_bytes < need) return MTS_ENOMEM;
    mts_batch *b = new (std::nothrow) mts_batch;
    if (!b) return MTS_ENOMEM;
    b->precision = boxes[0].precision;
    b->user = static_cast<hipStream_t>(stream);
    b->ty = b->precision == MTS_FP64 ? 4 : 8;
    size_t off = 0;
    int rc = MTS_OK;
    for (int32_t k = 0; k < nbox && rc == MTS_OK; k++) {
        mts_ctx *c = nullptr;
        const size_t sz = mts_state_bytes(&boxes[k]);
        rc = mts_create(&boxes[k], static_cast<char *>(dev_pool) + off, sz, stream, &c);
        if (rc == MTS_OK) {
            b->box.push_back(c);
            b->tz.push_back(32);
        }
        off += align256(sz);
    }
    hipError_t e = hipSuccess;
    if (rc == MTS_OK) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    for (hipEvent_t *ev : {&b->ev_in, &b->ev_out, &b->ev_t0, &b->ev_t1})
        if (rc == MTS_OK && e == hipSuccess) e = hipEventCreate(ev);
    if (rc == MTS_OK && e == hipSuccess) {
        const size_t bb = (b->precision == MTS_FP64 ? sizeof(BatchBox<double>) : sizeof(BatchBox<float>)) * nbox;
        const size_t bp = (b->precision == MTS_FP64 ? sizeof(BatchPost<double>) : sizeof(BatchPost<float>)) * nbox;
        e = hipMalloc(&b->boxes_dev, bb);
        if (e == hipSuccess) e = hipMalloc(&b->boxes_diag_dev, bb);
        if (e == hipSuccess) e = hipMalloc(&b->post_dev, bp);
    }
    if (rc == MTS_OK && e != hipSuccess) rc = MTS_ENOMEM;
    // FP32 ensembles with diagnostics fuse them when every box has room for a second momentum copy
    if (rc == MTS_OK && b->precision == MTS_FP32 && boxes[0].diag_every > 0) {
        bool room = true;
        for (mts_ctx *c : b->box) room = room && c->S < (1ull << 31) && ensure_mom2_quiet(c) == MTS_OK;
        b->fused = room;
    }
    if (rc == MTS_OK) rc = batch_upload(b);
    if (rc != MTS_OK) {
        std::fprintf(stderr, "mts_batch_create: %s\n", b->err.c_str());
        mts_batch_destroy(b);
        return rc;
    }
    *out = b;
    return MTS_OK;
}

int mts_batch_destroy(mts_batch *b) {
    if (!b) return MTS_EINVAL;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_release_graph(b);
    for (mts_ctx *c : b->box) mts_destroy(c);
    (void)hipFree(b->boxes_dev);
    (void)hipFree(b->boxes_diag_dev);
    (void)hipFree(b->post_dev);
    (void)hipFree(b->coef_dev);
    (void)hipFree(b->gsync);
    for (hipEvent_t ev : {b->ev_in, b->ev_out, b->ev_t0, b->ev_t1})
        if (ev) (void)hipEventDestroy(ev);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return MTS_OK;
}

int32_t mts_batch_size(const mts_batch *b) { return b ? (int32_t)b->box.size() : 0; }

int mts_batch_init_fields(mts_batch *b, const uint64_t *seeds) {
    if (!b || !seeds) return MTS_EINVAL;
    for (size_t k = 0; k < b->box.size(); k++) {
        const int rc = mts_init_fields(b->box[k], seeds[k]);
        if (rc != MTS_OK) return bfail(b, rc, mts_last_error(b->box[k]));
    }
    return MTS_OK;
}

int mts_batch_step(mts_batch *b, int32_t n, const double *eta0, const double *era_m, const double *s_before,
                   const double *s_after, const double *eta_switch) {
    if (!b || !eta0 || !era_m || !s_before) return MTS_EINVAL;
    for (size_t k = 0; k < b->box.size(); k++) {
        mts_ctx *c = b->box[k];
        const double sa = s_after ? s_after[k] : s_before[k];
        const double sw = eta_switch ? eta_switch[k] : INFINITY;
        const int rc = check_step(c, n, eta0[k], era_m[k], s_before[k], sa, sw);
        if (rc != MTS_OK) return bfail(b, rc, "box " + std::to_string(k) + ": " + c->err);
        if (c->cur != b->box[0]->cur || c->mcur != b->box[0]->mcur || c->step_count != b->box[0]->step_count)
            return bfail(b, MTS_EINVAL, "boxes must be initialised and stepped together");
    }
    if (n == 0) return MTS_OK;
    return b->precision == MTS_FP64 ? batch_step_t<double>(b, n, eta0, era_m, s_before, s_after, eta_switch)
                                    : batch_step_t<float>(b, n, eta0, era_m, s_before, s_after, eta_switch);
}

int mts_batch_diagnostics(mts_batch *b, int32_t box, mts_diag *out, int32_t max, int32_t *count) {
    if (!b || box < 0 || box >= (int32_t)b->box.size()) return MTS_EINVAL;
    if (b->gsync) {
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        if (const int rc = batch_check_persist(b); rc != MTS_OK) return rc;
    }
    return mts_diagnostics(b->box[box], out, max, count);
}

int mts_batch_get_fields(mts_batch *b, int32_t box, double *host) {
    if (!b || box < 0 || box >= (int32_t)b->box.size()) return MTS_EINVAL;
    if (b->gsync) {
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        if (const int rc = batch_check_persist(b); rc != MTS_OK) return rc;
    }
    return mts_get_fields(b->box[box], host);
}

int mts_batch_set_fields(mts_batch *b, int32_t box, const double *host) {
    if (!b || box < 0 || box >= (int32_t)b->box.size()) return MTS_EINVAL;
    return mts_set_fields(b->box[box], host);
}

int mts_batch_set_tile(mts_batch *b, int32_t ty, const int32_t *tz) {
    if (!b || !tz) return MTS_EINVAL;
    if (!batch_tile_supported(TileShape{ty, 1}, b->precision == MTS_FP64))
        return bfail(b, MTS_EINVAL, "ty must be 4, 5, 8, 12 or (FP32) 13");
    for (size_t k = 0; k < b->box.size(); k++)
        if (tz[k] < 1) return bfail(b, MTS_EINVAL, "tz must be >= 1");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->user));
    b->ty = ty;
    for (size_t k = 0; k < b->box.size(); k++) b->tz[k] = tz[k];
    return batch_upload(b);
}

int mts_batch_set_streaming_stores(mts_batch *b, int32_t on) {
    if (!b) return MTS_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->nt = on != 0;
    return MTS_OK;
}

int mts_batch_get_streaming_stores(const mts_batch *b, int32_t *on) {
    if (!b || !on) return MTS_EINVAL;
    *on = b->nt ? 1 : 0;
    return MTS_OK;
}

int mts_batch_set_momentum_pingpong(mts_batch *b, int32_t on) {
    if (!b) return MTS_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->user));
    if (on) {
        for (size_t k = 0; k < b->box.size(); k++) {
            const int rc = ensure_mom2(b->box[k], "momentum ping-pong");
            if (rc != MTS_OK) return bfail(b, rc, "box " + std::to_string(k) + ": " + b->box[k]->err);
        }
        const int rc = batch_upload(b);
        if (rc != MTS_OK) return rc;
    }
    b->mpp = on != 0;
    return MTS_OK;
}

int mts_batch_set_fused_diagnostics(mts_batch *b, int32_t rows) {
    if (!b) return MTS_EINVAL;
    if (rows != 0 && rows != 8) return bfail(b, MTS_EINVAL, "fused diagnostics of a batch: rows must be 0 or 8");
    if (rows && b->precision != MTS_FP32) return bfail(b, MTS_EINVAL, "fused diagnostics are FP32 only");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->user));
    if (rows) {
        for (size_t k = 0; k < b->box.size(); k++) {
            if (b->box[k]->S >= (1ull << 31))
                return bfail(b, MTS_EINVAL, "fused diagnostics: box " + std::to_string(k) + " has 2^31 sites or more");
            const int rc = ensure_mom2(b->box[k], "fused diagnostics");
            if (rc != MTS_OK) return bfail(b, rc, "box " + std::to_string(k) + ": " + b->box[k]->err);
        }
    }
    b->fused = rows != 0;
    return batch_upload(b);
}

int mts_batch_get_fused_diagnostics(const mts_batch *b, int32_t *rows) {
    if (!b || !rows) return MTS_EINVAL;
    *rows = b->fused ? 8 : 0;
    return MTS_OK;
}

int mts_batch_get_momentum_pingpong(const mts_batch *b, int32_t *on) {
    if (!b || !on) return MTS_EINVAL;
    *on = b->mpp ? 1 : 0;
    return MTS_OK;
}

int mts_batch_set_tile_order(mts_batch *b, int32_t xcd_runs) {
    if (!b) return MTS_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->xcd = xcd_runs != 0;
    return MTS_OK;
}

int mts_batch_set_persistent(mts_batch *b, int32_t on, double wait_limit_s) {
    if (!b) return MTS_EINVAL;
    if (!(wait_limit_s >= 0.0) || wait_limit_s > 3600.0)
        return bfail(b, MTS_EINVAL, "persistent ensemble launch: wait limit must be in [0, 3600] s");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->user));
    if (on && !b->gsync) {
        BHIPCHK(b, hipMalloc(&b->gsync, sizeof(GridSync)));
        BHIPCHK(b, hipMemset(b->gsync, 0, sizeof(GridSync)));
    }
    if (on) {
        int grid = 0;
        BHIPCHK(b, persist_max_blocks(b->precision == MTS_FP64, b->ty, b->nt, &grid));
        if (grid <= 0) return bfail(b, MTS_EINVAL, "persistent ensemble launch: no co-resident grid for this tile");
    }
    b->persist = on != 0;
    b->persist_wait_s = wait_limit_s > 0.0 ? wait_limit_s : 10.0;
    return MTS_OK;
}

int mts_batch_get_persistent(const mts_batch *b, int32_t *on) {
    if (!b || !on) return MTS_EINVAL;
    *on = b->persist ? 1 : 0;
    return MTS_OK;
}

int mts_batch_autotune_times(const mts_batch *b, double *graph_ms, double *persistent_ms) {
    if (!b) return MTS_EINVAL;
    if (graph_ms) *graph_ms = b->tune_graph_ms;
    if (persistent_ms) *persistent_ms = b->tune_persist_ms;
    return MTS_OK;
}

int mts_batch_get_tile_order(const mts_batch *b, int32_t *xcd_runs) {
    if (!b || !xcd_runs) return MTS_EINVAL;
    *xcd_runs = b->xcd ? 1 : 0;
    return MTS_OK;
}

int mts_batch_timing_read(mts_batch *b, int64_t *steps, double *ms) {
    if (!b) return MTS_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (const int rc = batch_check_persist(b); rc != MTS_OK) return rc;
    batch_collect_timing(b);
    if (steps) *steps = b->t_steps;
    if (ms) *ms = b->t_ms;
    b->t_steps = 0;
    b->t_ms = 0.0;
    return MTS_OK;
}

int mts_batch_autotune(mts_batch *b, int32_t steps, int32_t *ty_out, int32_t *tz_out, double *ms_out) {
    if (!b || steps < 1) return MTS_EINVAL;
    const size_t nbox = b->box.size();
    const std::vector<int> tys = b->precision == MTS_FP64 ? std::vector<int>{4, 5, 8} : std::vector<int>{4, 8, 12, 13};
    const int tzs[] = {8, 16, 32, 64};
    std::vector<int32_t> d(nbox);
    for (size_t k = 0; k < nbox; k++) {
        d[k] = b->box[k]->p.diag_every;
        b->box[k]->p.diag_every = 0;           // time the plain update
    }
    std::vector<uint64_t> seeds(nbox, 0);
    std::vector<double> eta(nbox, 1.0), era(nbox, 0.5), sv(nbox, 1.0);
    b->mpp = false;
    b->persist = false;
    b->tune_graph_ms = b->tune_persist_ms = 0.0;
    int rc = mts_batch_init_fields(b, seeds.data());
    double best = INFINITY;
    int pick_ty = b->ty, pick_tz = b->tz.empty() ? 32 : b->tz[0];
    bool pick_nt = b->nt;
    int nzmax = 0;
    for (mts_ctx *c : b->box) nzmax = std::max(nzmax, c->p.nz);
    for (int nt = 0; nt < 2; nt++)
    for (int ty : tys)
        for (int tz : tzs) {
            if (rc != MTS_OK) break;
            if (tz > 2 * nzmax && tz != 8) continue;
            b->nt = nt != 0;
            std::vector<int32_t> tzv(nbox, tz);
            if ((rc = mts_batch_set_tile(b, ty, tzv.data())) != MTS_OK) break;
            if ((rc = mts_batch_step(b, 1, eta.data(), era.data(), sv.data(), nullptr, nullptr)) != MTS_OK) break;
            int64_t ns = 0;
            double ms = 0;
            if ((rc = mts_batch_timing_read(b, &ns, &ms)) != MTS_OK) break;
            if ((rc = mts_batch_step(b, steps, eta.data(), era.data(), sv.data(), nullptr, nullptr)) != MTS_OK) break;
            if ((rc = mts_batch_timing_read(b, &ns, &ms)) != MTS_OK) break;
            if (ms < best) {
                best = ms;
                pick_ty = ty;
                pick_tz = tz;
                pick_nt = nt != 0;
            }
        }
    b->nt = pick_nt;
    // the best configuration again with the momenta written to the other copy
    bool pick_mpp = false;
    if (rc == MTS_OK) {
        std::vector<int32_t> tzv(nbox, pick_tz);
        rc = mts_batch_set_tile(b, pick_ty, tzv.data());
        const int r2 = rc == MTS_OK ? mts_batch_set_momentum_pingpong(b, 1) : rc;
        if (r2 == MTS_OK) {
            int64_t ns = 0;
            double ms = 0;
            if ((rc = mts_batch_step(b, 1, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
                (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK &&
                (rc = mts_batch_step(b, steps, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
                (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK && ms < best) {
                best = ms;
                pick_mpp = true;
            }
        } else if (r2 != MTS_ENOMEM) {
            rc = r2;
        }
        b->mpp = false;
        if (rc == MTS_OK) b->err.clear();
    }
    // and with the other tile order, kept only if at least 1 % faster
    if (rc == MTS_OK) {
        const bool cur = b->xcd;
        b->mpp = pick_mpp;
        b->xcd = !cur;
        int64_t ns = 0;
        double ms = 0;
        if ((rc = mts_batch_step(b, 1, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
            (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK &&
            (rc = mts_batch_step(b, steps, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
            (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK && ms < 0.99 * best)
            best = ms;
        else
            b->xcd = cur;
        b->mpp = false;
    }
    // and the persistent launch of the same configuration, kept if faster
    bool pick_persist = false;
    if (rc == MTS_OK) {
        b->mpp = pick_mpp;
        b->tune_graph_ms = best / steps;
        int64_t ns = 0;
        double ms = 0;
        if ((rc = mts_batch_set_persistent(b, 1, 0.0)) == MTS_OK &&
            (rc = mts_batch_step(b, 1, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
            (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK &&
            (rc = mts_batch_step(b, steps, eta.data(), era.data(), sv.data(), nullptr, nullptr)) == MTS_OK &&
            (rc = mts_batch_timing_read(b, &ns, &ms)) == MTS_OK) {
            b->tune_persist_ms = ms / steps;
            if (ms < best) {
                best = ms;
                pick_persist = true;
            }
        }
        b->persist = false;
        b->mpp = false;
    }
    for (size_t k = 0; k < nbox; k++) b->box[k]->p.diag_every = d[k];
    if (rc != MTS_OK) return rc;
    std::vector<int32_t> tzv(nbox, pick_tz);
    if ((rc = mts_batch_set_tile(b, pick_ty, tzv.data())) != MTS_OK) return rc;
    if ((rc = mts_batch_init_fields(b, seeds.data())) != MTS_OK) return rc;   // momenta back in copy 0
    if ((rc = mts_batch_set_momentum_pingpong(b, pick_mpp ? 1 : 0)) != MTS_OK) return rc;
    b->persist = pick_persist;
    if (!pick_mpp && !b->fused) {                     // the second momentum copies are not needed
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        for (mts_ctx *c : b->box) {
            (void)hipFree(c->mom2);
            c->mom2 = nullptr;
        }
        if ((rc = batch_upload(b)) != MTS_OK) return rc;
    }
    if (ty_out) *ty_out = pick_ty;
    if (tz_out) *tz_out = pick_tz;
    if (ms_out) *ms_out = best / steps;
    return MTS_OK;
}

const char *mts_batch_last_error(const mts_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
