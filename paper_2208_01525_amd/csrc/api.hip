// api.hip -- host side of libmts (the C ABI declared in include/mts.h):
// parameter checks, FP64 time bookkeeping, launches, diagnostic records.
#include "kernels.h"
#include "mts.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace mts;

namespace {

constexpr int RING_CAP = 4096;   // diagnostic records kept on the device between drains

struct Meta {                    // host-side facts of one record
    int64_t step;
    double eta, a, s;
};

}  // namespace

struct mts_ctx {
    mts_params p{};
    size_t esz = 4;
    Geom g{};
    uint64_t S = 0;              // sites
    uint64_t plane = 0;          // elements per plane (S rounded up to 64)
    char *state = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;                 // which field copy holds the current fields
    int64_t step_count = 0;

    // scratch
    double *partials = nullptr;  // [NSLOT][maxblk]
    uint32_t maxblk = 0;
    uint32_t *nblk_dev = nullptr;
    uint8_t *wabs = nullptr;     // packed |W| per sector: [2][plane]
    uint8_t *cells = nullptr;    // cell values per sector: [2][plane]
    double *ring = nullptr;      // [RING_CAP][NSLOT]
    std::vector<Meta> meta;      // one per record produced since the last drain
    int64_t produced = 0, drained = 0;
    bool have_cells = false;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Mark {
        int kind;                // 0 plain step, 1 diagnostic step, 2 diagnostic post-kernels
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

template <typename T>
Moms<T> moms_of(const mts_ctx *c) {
    T *base = reinterpret_cast<T *>(c->state) + (size_t)20 * c->plane;
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
    if (S >= 4294967296.0 - 64) return why = "nx*ny*nz must be below 2^32", MTS_EINVAL;
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

uint64_t plane_of(const mts_params &p) {
    const uint64_t S = (uint64_t)p.nx * p.ny * p.nz;
    return (S + 63) / 64 * 64;
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

template <typename T>
int do_step(mts_ctx *c, int32_t n, double eta, double era_m, double s) {
    const mts_params &p = c->p;
    Moms<T> mom = moms_of<T>(c);
    Partials part{c->partials, c->maxblk};
    for (int32_t j = 0; j < n; j++) {
        const double eta_j = eta + j * p.dt;
        const Book b = bookkeeping(p, eta_j, era_m, s);
        const StepCoef<T> coef = coefficients<T>(p, b, s);
        const bool diag = p.diag_every > 0 && (c->step_count % p.diag_every) == 0;
        Fields<T> in = fields_of<T>(c, c->cur), out = fields_of<T>(c, 1 - c->cur);
        {
            TimedRegion tr(c, diag ? 1 : 0);
            hipError_t e = launch_step<T>(c->g, in, out, mom, coef, diag, part, c->stream);
            if (e != hipSuccess) return hipfail(c, e, "step kernel launch");
        }
        if (diag) {
            TimedRegion tr(c, 2);
            double gcoef[2];
            const double e2[2] = {p.e_p * p.e_p, p.e_q * p.e_q};
            for (int q = 0; q < 2; q++) gcoef[q] = 2.0 * e2[q] * b.An * (1.0 + b.delta) / (1.0 + b.omega);
            hipError_t e = launch_wind_gauss<T>(c->g, in, mom, (T)p.dx, gcoef, c->wabs, (uint32_t)c->plane, nullptr,
                                                part, c->stream);
            if (e == hipSuccess) e = launch_cells(c->g, c->wabs, c->cells, (uint32_t)c->plane, c->stream);
            if (e == hipSuccess) e = launch_overlap(c->g, c->cells, (uint32_t)c->plane, p.overlap_radius, part, c->stream);
            double *rec = c->ring + (size_t)(c->produced % RING_CAP) * NSLOT;
            if (e == hipSuccess) e = launch_reduce(part, c->nblk_dev, rec, c->stream);
            if (e != hipSuccess) return hipfail(c, e, "diagnostic kernel launch");
            c->meta.push_back({c->step_count, eta_j, b.a, s});
            c->produced++;
            c->have_cells = true;
        }
        c->cur = 1 - c->cur;
        c->step_count++;
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
    const double mu = 2.0 * M_PI;   // tension of a basic string at criticality, sigma = 1 (Sec. IV)
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
    HIPCHK(c, hipMemcpyAsync(buf.data() + 10 * c->plane, base + 20 * c->plane, 10 * c->plane * sizeof(T),
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
    HIPCHK(c, hipMemcpyAsync(base + 20 * c->plane, buf.data() + 10 * c->plane, 10 * c->plane * sizeof(T),
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
    hipError_t e = launch_wind_gauss<T>(c->g, fields_of<T>(c, c->cur), moms_of<T>(c), (T)c->p.dx, g0, nullptr,
                                        (uint32_t)c->plane, tmp, part, c->stream);
    std::vector<int8_t> buf(bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(buf.data(), tmp, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hipfail(c, e, "windings");
    for (int q = 0; q < 6; q++) std::memcpy(host + (size_t)q * c->S, buf.data() + (size_t)q * c->plane, c->S);
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
    c->maxblk = site_blocks(c->g);
    hipError_t e = hipMalloc(&c->partials, sizeof(double) * NSLOT * (size_t)c->maxblk);
    if (e == hipSuccess) e = hipMalloc(&c->nblk_dev, sizeof(uint32_t) * NSLOT);
    if (e == hipSuccess) e = hipMalloc(&c->wabs, 2 * c->plane);
    if (e == hipSuccess) e = hipMalloc(&c->cells, 2 * c->plane);
    if (e == hipSuccess) e = hipMalloc(&c->ring, sizeof(double) * NSLOT * RING_CAP);
    if (e == hipSuccess) {
        uint32_t nb[NSLOT];
        for (int q = 0; q < NSLOT; q++) nb[q] = q < SL_OV_Q + 1 ? c->maxblk : 0;
        e = hipMemcpy(c->nblk_dev, nb, sizeof(nb), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        std::fprintf(stderr, "mts_create: scratch allocation failed: %s\n", hipGetErrorString(e));
        mts_destroy(c);
        return MTS_ENOMEM;
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
    (void)hipFree(c->ring);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return MTS_OK;
}

int mts_init_fields(mts_ctx *c, uint64_t seed) {
    if (!c) return MTS_EINVAL;
    c->cur = 0;
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
    if (n < 0) return fail(c, MTS_EINVAL, "n must be >= 0");
    if (!(era_m >= 0.0 && era_m < 1.0)) return fail(c, MTS_EINVAL, "era_m must be in [0, 1)");
    if (!std::isfinite(eta) || !std::isfinite(s)) return fail(c, MTS_EINVAL, "eta and s must be finite");
    if (era_m > 0.0 && !(eta > 0.0)) return fail(c, MTS_EINVAL, "eta must be > 0 when era_m > 0");
    if (n == 0) return MTS_OK;
    // leapfrog stability over the call's a-range (a^{2s} is monotone in eta)
    const Book b0 = bookkeeping(c->p, eta, era_m, s), b1 = bookkeeping(c->p, eta + (n - 1) * c->p.dt, era_m, s);
    const double Amax = std::max(b0.An, b1.An), k = c->p.dt, h = c->p.dx;
    const double cfl = k * k * (12.0 / (h * h) + Amax * mu2_max(c->p));
    if (!(cfl < 4.0)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "unstable: dt^2 (12/h^2 + a^{2s}_max mu2_max) = %.4g >= 4", cfl);
        return fail(c, MTS_EUNSTABLE, buf);
    }
    return c->p.precision == MTS_FP64 ? do_step<double>(c, n, eta, era_m, s) : do_step<float>(c, n, eta, era_m, s);
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
        d.wind_abs[0] = (int64_t)std::llround(rec[SL_WIND_P]);
        d.wind_abs[1] = (int64_t)std::llround(rec[SL_WIND_Q]);
        d.pq_count2 = (int64_t)std::llround(rec[SL_OV_P] + rec[SL_OV_Q]);
        bool finite = true;
        for (int q = 0; q <= SL_OV_Q; q++) finite = finite && std::isfinite(rec[q]);
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

int mts_get_cells(mts_ctx *c, uint8_t *host) {
    if (!c || !host) return MTS_EINVAL;
    if (!c->have_cells) return fail(c, MTS_EINVAL, "no diagnostic step has run yet");
    std::vector<uint8_t> buf(2 * c->plane);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->cells, 2 * c->plane, hipMemcpyDeviceToHost));
    for (int q = 0; q < 2; q++) std::memcpy(host + (size_t)q * c->S, buf.data() + (size_t)q * c->plane, c->S);
    return MTS_OK;
}

int mts_timing_enable(mts_ctx *c, int32_t on) {
    if (!c) return MTS_EINVAL;
    c->timing = on != 0;
    return MTS_OK;
}

int mts_timing_read(mts_ctx *c, int64_t *n_plain, double *ms_plain, int64_t *n_diag, double *ms_diag,
                    double *ms_post) {
    if (!c) return MTS_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t np = 0, nd = 0;
    double tp = 0, td = 0, tq = 0;
    for (const auto &mk : c->marks) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[mk.a], c->ev_pool[mk.b]));
        if (mk.kind == 0) np++, tp += ms;
        else if (mk.kind == 1) nd++, td += ms;
        else tq += ms;
    }
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
