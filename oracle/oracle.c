/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the U(1)xU(1) multitension
 * string lattice update of Correia & Martins, arXiv:2208.01525.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP implementation; the two agree
 * only on the host field exchange format (20 planar FP64 components per
 * site, x fastest) and on the published SplitMix64 definition used for the
 * random-phase initial conditions.
 *
 * What is computed, and where it comes from in the paper:
 *   - Model: two complex scalars phi (sector p) and psi (sector q), two U(1)
 *     gauge fields A, B; potential with the kappa coupling (Sec. II, the
 *     Lagrangian and potential).
 *   - Update: the damped leapfrog of Sec. III (scalar momentum kick with the
 *     Hubble damping delta, gauge momentum kick with omega = delta(1-beta),
 *     then the drift of all fields), with the couplings scaled by a^{2 beta}
 *     (Sec. III, PRS / core-growth prescription).  beta is called `s` here.
 *   - Diagnostics: the winding-based lengths and the bound-state overlap
 *     ("fast method", Sec. III.A-B), the Lagrangian length estimator and
 *     the weighted scalar velocity estimator (Sec. III.A), and the two
 *     Gauss laws (Sec. II, checked in Sec. IV).
 * The paper names the lattice operators D^-D^+, d^-F and Im[phi* D^+ phi]
 * but does not spell them out; the compact-link reading used here is:
 *   U_i(x)     = exp(-i h A_i(x))          (A carries the gauge coupling)
 *   D_i^+phi   = (U_i(x) phi(x+i) - phi(x)) / h
 *   theta_ij   = h [A_i(x) + A_j(x+i) - A_i(x+j) - A_j(x)]   (= h^2 F_ij)
 * With a = 1 the update is exactly Hamilton's equations of the lattice
 * energy in orc_hamiltonian() (pinned by finite differences in the tests).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fcx-limited-range -shared -fPIC
 * (-fcx-limited-range makes complex products the textbook formula).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Model and lattice.  Sector 0 = p (phi, Pi, A, E); sector 1 = q (psi, Psi, B, H). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t overlap_radius; /* 0: same cell only; 1: one cell in any direction */
    double h;               /* lattice spacing, Delta x */
    double k;               /* conformal time step, Delta eta */
    double lam[2];          /* lambda_p0, lambda_q0 */
    double e[2];            /* e_p0, e_q0 */
    double sig[2];          /* sigma_p, sigma_q */
    double kappa;           /* kappa_0 */
    double eta_ref;         /* a(eta_ref) = 1 */
} orc_model;

/* One record of the integer-time diagnostics (fields at eta_n, momenta
 * averaged over n-1/2 and n+1/2; Gauss residual at n+1/2). */
typedef struct {
    double eta, a;
    double sum_eps;        /* h^3 sum of the energy density */
    double sum_lag;        /* h^3 sum of the Lagrangian density */
    double sum_KL, sum_GL; /* sum K*Lag, sum G*Lag   (velocity, all strings) */
    double sum_KV, sum_GV; /* sum K*Vint, sum G*Vint (velocity, bound states) */
    double gauss_abs[2];   /* sum |C_sigma| */
    double gauss_scale[2]; /* sum (|div E| + |g rho|) */
    int64_t wind_abs[2];   /* sum |W| over all plaquettes, per sector */
    int64_t pq_count2;     /* count_p + count_q = 2 N_pq */
} orc_diag;

/* ---------------------------------------------------------------- layout */

static int64_t nsites(const orc_model *m) { return (int64_t)m->nx * m->ny * m->nz; }

static int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

/* site index of (x,y,z) + d, periodic; x fastest */
static int64_t site(const orc_model *m, const int c[3], const int d[3]) {
    int x = wrap(c[0] + d[0], m->nx), y = wrap(c[1] + d[1], m->ny), z = wrap(c[2] + d[2], m->nz);
    return x + (int64_t)m->nx * (y + (int64_t)m->ny * z);
}

/* site displaced by a*i_hat + b*j_hat */
static int64_t shifted(const orc_model *m, const int c[3], int i, int a, int j, int b) {
    int d[3] = {0, 0, 0};
    d[i] += a;
    d[j] += b;
    return site(m, c, d);
}

/* component planes of the 20-real state */
static int c_scal(int sec) { return 2 * sec; }          /* phi, psi      : 0-1, 2-3   */
static int c_mom(int sec) { return 4 + 2 * sec; }       /* Pi, Psi       : 4-5, 6-7   */
static int c_link(int sec, int i) { return 8 + 3 * sec + i; }   /* A, B : 8-10, 11-13 */
static int c_elec(int sec, int i) { return 14 + 3 * sec + i; }  /* E, H : 14-16, 17-19 */

static cplx get_c(const orc_model *m, const double *st, int comp, int64_t s) {
    int64_t S = nsites(m);
    return st[comp * S + s] + I * st[(comp + 1) * S + s];
}
static double get_r(const orc_model *m, const double *st, int comp, int64_t s) {
    return st[comp * nsites(m) + s];
}

/* ---------------------------------------------------- lattice operators */

/* link phasor U_i(x) = exp(-i h A_i(x)) */
static cplx link_U(const orc_model *m, const double *st, int sec, int i, int64_t s) {
    return cexp(-I * m->h * get_r(m, st, c_link(sec, i), s));
}

/* plaquette angle theta_ij(x) = h [A_i(x) + A_j(x+i) - A_i(x+j) - A_j(x)] */
static double plaquette(const orc_model *m, const double *st, int sec, int i, int j, const int c[3]) {
    int64_t x = shifted(m, c, i, 0, j, 0);
    int64_t xi = shifted(m, c, i, 1, j, 0);
    int64_t xj = shifted(m, c, i, 0, j, 1);
    return m->h * (get_r(m, st, c_link(sec, i), x) + get_r(m, st, c_link(sec, j), xi)
                   - get_r(m, st, c_link(sec, i), xj) - get_r(m, st, c_link(sec, j), x));
}

/* ------------------------------------------------------------- forces */

/*
 * Right-hand sides of the momentum kicks at time n (Sec. III, the Pi/Psi and
 * E/H update equations), with the a^{2 beta} factor passed in as An:
 *   F_phi = D^-D^+ phi - An phi [lam/2 (|phi|^2 - sig^2) - kappa (|psi|^2 - sig_q^2)]
 *   F_A_i = -sum_{j != i} d_j^- F_ij + 2 e^2 An Im[phi* D_i^+ phi]
 * Lattice forms:
 *   D^-D^+ phi = h^-2 sum_i [U_i(x) phi(x+i) - 2 phi(x) + conj(U_i(x-i)) phi(x-i)]
 *   d_j^- F_ij -> h^-3 [sin theta_ij(x) - sin theta_ij(x-j)]      (compact)
 *   Im[phi* D_i^+ phi] = h^-1 Im[conj(phi(x)) U_i(x) phi(x+i)]
 * F has 10 planes: F_phi (re, im), F_psi (re, im), F_A (x,y,z), F_B (x,y,z).
 */
void orc_forces(const orc_model *m, const double *st, double An, double *F) {
    const int64_t S = nsites(m);
    const double h = m->h;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < m->nz; z++)
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                const int zero[3] = {0, 0, 0};
                const int64_t s0 = site(m, c, zero);
                for (int sec = 0; sec < 2; sec++) {
                    const int oth = 1 - sec;
                    cplx phi = get_c(m, st, c_scal(sec), s0);
                    cplx lap = 0.0;
                    for (int i = 0; i < 3; i++) {
                        int64_t sp = shifted(m, c, i, 1, i, 0);
                        int64_t sm = shifted(m, c, i, -1, i, 0);
                        lap += link_U(m, st, sec, i, s0) * get_c(m, st, c_scal(sec), sp)
                             - 2.0 * phi
                             + conj(link_U(m, st, sec, i, sm)) * get_c(m, st, c_scal(sec), sm);
                    }
                    lap /= h * h;
                    cplx chi = get_c(m, st, c_scal(oth), s0);
                    double mod2 = creal(phi) * creal(phi) + cimag(phi) * cimag(phi);
                    double oth2 = creal(chi) * creal(chi) + cimag(chi) * cimag(chi);
                    double bracket = m->lam[sec] / 2.0 * (mod2 - m->sig[sec] * m->sig[sec])
                                   - m->kappa * (oth2 - m->sig[oth] * m->sig[oth]);
                    cplx fphi = lap - An * phi * bracket;
                    F[(2 * sec) * S + s0] = creal(fphi);
                    F[(2 * sec + 1) * S + s0] = cimag(fphi);

                    for (int i = 0; i < 3; i++) {
                        double curl = 0.0;
                        for (int j = 0; j < 3; j++) {
                            if (j == i) continue;
                            int dm[3] = {0, 0, 0};
                            dm[j] = -1;
                            int cm[3] = {c[0] + dm[0], c[1] + dm[1], c[2] + dm[2]};
                            curl += sin(plaquette(m, st, sec, i, j, c)) - sin(plaquette(m, st, sec, i, j, cm));
                        }
                        double mag = -curl / (h * h * h);
                        int64_t sp = shifted(m, c, i, 1, i, 0);
                        cplx hop = conj(phi) * link_U(m, st, sec, i, s0) * get_c(m, st, c_scal(sec), sp);
                        double cur = 2.0 * m->e[sec] * m->e[sec] * An * cimag(hop) / h;
                        F[(4 + 3 * sec + i) * S + s0] = mag + cur;
                    }
                }
            }
}

/* ------------------------------------------------ energy and Lagrangian */

/* Per-site pieces of the energy/Lagrangian at one site, given momenta
 * (pi, E) to use for the kinetic parts:
 *   K   = |Pi|^2 + |Psi|^2
 *   G   = sum_i |D_i^+ phi|^2 + |D_i^+ psi|^2
 *   Kg  = sum_sigma 1/(2 e^2) sum_i E_i^2
 *   Bg  = sum_sigma 1/(e^2 h^4) sum_{i<j} (1 - cos theta_ij)
 *   V   = lam_p/4 (|phi|^2-sig_p^2)^2 + lam_q/4 (|psi|^2-sig_q^2)^2
 *         - kappa (|phi|^2-sig_p^2)(|psi|^2-sig_q^2)          (Sec. II)
 *   Vint= kappa (|phi|^2-sig_p^2)(|psi|^2-sig_q^2)             (Sec. III.B, Fig. 2)
 * `fld` supplies phi, psi, A, B; `mom` supplies Pi, Psi, E, H (same layout). */
typedef struct { double K, G, Kg, Bg, V, Vint; } site_terms;

static site_terms terms_at(const orc_model *m, const double *fld, const double *mom, const int c[3]) {
    const int zero[3] = {0, 0, 0};
    const int64_t s0 = site(m, c, zero);
    const double h = m->h;
    site_terms t = {0, 0, 0, 0, 0, 0};
    double dev[2];
    for (int sec = 0; sec < 2; sec++) {
        cplx pi = get_c(m, mom, c_mom(sec), s0);
        t.K += creal(pi) * creal(pi) + cimag(pi) * cimag(pi);
        cplx phi = get_c(m, fld, c_scal(sec), s0);
        for (int i = 0; i < 3; i++) {
            int64_t sp = shifted(m, c, i, 1, i, 0);
            cplx d = (link_U(m, fld, sec, i, s0) * get_c(m, fld, c_scal(sec), sp) - phi) / h;
            t.G += creal(d) * creal(d) + cimag(d) * cimag(d);
            double ei = get_r(m, mom, c_elec(sec, i), s0);
            t.Kg += ei * ei / (2.0 * m->e[sec] * m->e[sec]);
        }
        for (int i = 0; i < 3; i++)
            for (int j = i + 1; j < 3; j++)
                t.Bg += (1.0 - cos(plaquette(m, fld, sec, i, j, c))) / (m->e[sec] * m->e[sec] * h * h * h * h);
        dev[sec] = creal(phi) * creal(phi) + cimag(phi) * cimag(phi) - m->sig[sec] * m->sig[sec];
    }
    t.Vint = m->kappa * dev[0] * dev[1];
    t.V = m->lam[0] / 4.0 * dev[0] * dev[0] + m->lam[1] / 4.0 * dev[1] * dev[1] - t.Vint;
    return t;
}

/* Lattice Hamiltonian at a = 1 using the momenta stored in the state:
 *   H = h^3 sum_x [K + G + Kg + Bg + V]
 * The update at a = 1 is Hamilton's equations of this H:
 *   dPi/deta = -(1/(2 h^3)) (dH/dRe phi + i dH/dIm phi),  dE_i/deta = -(e^2/h^3) dH/dA_i. */
double orc_hamiltonian(const orc_model *m, const double *st) {
    double *plane = (double *)calloc((size_t)m->nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < m->nz; z++) {
        double acc = 0.0;
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                site_terms t = terms_at(m, st, st, c);
                acc += t.K + t.G + t.Kg + t.Bg + t.V;
            }
        plane[z] = acc;
    }
    double H = 0.0;
    for (int z = 0; z < m->nz; z++) H += plane[z];
    free(plane);
    return H * m->h * m->h * m->h;
}

/* ------------------------------------------------------------ windings */

/* covariant phase of the link: chi_mu(x) = arg(conj(phi(x)) U_mu(x) phi(x+mu)) in (-pi, pi];
 * zero when the product vanishes (the sign of a zero does not pick a branch) */
static double link_phase(const orc_model *m, const double *st, int sec, int mu, const int c[3]) {
    const int zero[3] = {0, 0, 0};
    int64_t s0 = site(m, c, zero);
    int64_t sp = shifted(m, c, mu, 1, mu, 0);
    cplx z = conj(get_c(m, st, c_scal(sec), s0)) * link_U(m, st, sec, mu, s0) * get_c(m, st, c_scal(sec), sp);
    if (creal(z) == 0.0 && cimag(z) == 0.0) return 0.0; /* no phase where phi vanishes */
    double a = carg(z);
    return a <= -M_PI ? M_PI : a;
}

/*
 * Gauge-invariant plaquette winding through the face normal to rho, with
 * (mu, nu, rho) cyclic:
 *   W_rho(x) = [chi_mu(x) + chi_nu(x+mu) - chi_mu(x+nu) - chi_nu(x) + theta_mu,nu(x)] / 2 pi
 * This is an integer (rounded to the nearest one); the windings through the
 * six faces of any cell add up to zero.  These are the "non-zero plaquettes"
 * whose count gives the string length in each sector (Sec. III.A).
 * W has 6 planes: sector p (W_x, W_y, W_z), then sector q.
 */
void orc_windings(const orc_model *m, const double *st, int32_t *W) {
    const int64_t S = nsites(m);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < m->nz; z++)
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                const int zero[3] = {0, 0, 0};
                const int64_t s0 = site(m, c, zero);
                for (int sec = 0; sec < 2; sec++)
                    for (int rho = 0; rho < 3; rho++) {
                        int mu = (rho + 1) % 3, nu = (rho + 2) % 3;
                        int cmu[3] = {c[0], c[1], c[2]};
                        cmu[mu] += 1;
                        int cnu[3] = {c[0], c[1], c[2]};
                        cnu[nu] += 1;
                        double loop = link_phase(m, st, sec, mu, c) + link_phase(m, st, sec, nu, cmu)
                                    - link_phase(m, st, sec, mu, cnu) - link_phase(m, st, sec, nu, c)
                                    + plaquette(m, st, sec, mu, nu, c);
                        W[(3 * sec + rho) * S + s0] = (int32_t)lrint(loop / (2.0 * M_PI));
                    }
            }
}

/* Cell value: total |winding| through the six faces of the cell [x, x+1]^3
 * (Sec. III.B: a straight string pierces two faces, giving 2).
 * n has 2 planes (sector p, sector q). */
void orc_cells(const orc_model *m, const int32_t *W, int32_t *n) {
    const int64_t S = nsites(m);
    for (int z = 0; z < m->nz; z++)
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                const int zero[3] = {0, 0, 0};
                int64_t s0 = site(m, c, zero);
                for (int sec = 0; sec < 2; sec++) {
                    int32_t tot = 0;
                    for (int rho = 0; rho < 3; rho++) {
                        int64_t up = shifted(m, c, rho, 1, rho, 0);
                        tot += abs(W[(3 * sec + rho) * S + s0]) + abs(W[(3 * sec + rho) * S + up]);
                    }
                    n[sec * S + s0] = tot;
                }
            }
}

/*
 * Fast-method bound-state overlap (Sec. III.B): a pierced cell of one sector
 * counts when a pierced cell of the other sector sits in the same cell or,
 * for radius 1, in any of the 26 neighbouring cells.  Both directions are
 * counted; N_pq = (count_p + count_q) / 2.
 */
void orc_overlap(const orc_model *m, const int32_t *n, int radius, int64_t *count_p, int64_t *count_q) {
    const int64_t S = nsites(m);
    int64_t cnt[2] = {0, 0};
    for (int z = 0; z < m->nz; z++)
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                const int zero[3] = {0, 0, 0};
                int64_t s0 = site(m, c, zero);
                for (int sec = 0; sec < 2; sec++) {
                    if (n[sec * S + s0] == 0) continue;
                    int found = 0;
                    for (int dz = -radius; dz <= radius && !found; dz++)
                        for (int dy = -radius; dy <= radius && !found; dy++)
                            for (int dx = -radius; dx <= radius && !found; dx++) {
                                const int d[3] = {dx, dy, dz};
                                if (n[(1 - sec) * S + site(m, c, d)] > 0) found = 1;
                            }
                    cnt[sec] += found;
                }
            }
    *count_p = cnt[0];
    *count_q = cnt[1];
}

/*
 * Robust-method segments (Sec. III.B, Sec. V.B): the cells marked by the
 * fast method (a pierced cell of one sector with a pierced cell of the other
 * in its (2r+1)^3 neighbourhood, either way round) are split into connected
 * regions -- cells sharing at least a corner (26-neighbourhood), periodic --
 * by a breadth-first flood fill.  Writes the size of every region to sizes
 * (capacity cap) and returns their number (or -1 if cap is too small).
 */
int64_t orc_segments(const orc_model *m, const int32_t *n, int radius, int64_t *sizes, int64_t cap) {
    const int64_t S = nsites(m);
    uint8_t *mark = (uint8_t *)calloc((size_t)S, 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
    for (int z = 0; z < m->nz; z++)
        for (int y = 0; y < m->ny; y++)
            for (int x = 0; x < m->nx; x++) {
                const int c[3] = {x, y, z};
                const int zero[3] = {0, 0, 0};
                int64_t s0 = site(m, c, zero);
                for (int sec = 0; sec < 2 && !mark[s0]; sec++) {
                    if (n[sec * S + s0] == 0) continue;
                    for (int dz = -radius; dz <= radius; dz++)
                        for (int dy = -radius; dy <= radius; dy++)
                            for (int dx = -radius; dx <= radius; dx++) {
                                const int d[3] = {dx, dy, dz};
                                if (n[(1 - sec) * S + site(m, c, d)] > 0) mark[s0] = 1;
                            }
                }
            }
    int64_t ncomp = 0;
    for (int64_t start = 0; start < S; start++) {
        if (mark[start] != 1) continue;
        int64_t head = 0, tail = 0, size = 0;
        queue[tail++] = start;
        mark[start] = 2;
        while (head < tail) {
            const int64_t s0 = queue[head++];
            size++;
            const int c[3] = {(int)(s0 % m->nx), (int)((s0 / m->nx) % m->ny), (int)(s0 / ((int64_t)m->nx * m->ny))};
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        const int d[3] = {dx, dy, dz};
                        const int64_t nb = site(m, c, d);
                        if (mark[nb] == 1) {
                            mark[nb] = 2;
                            queue[tail++] = nb;
                        }
                    }
        }
        if (ncomp < cap) sizes[ncomp] = size;
        ncomp++;
    }
    free(mark);
    free(queue);
    return ncomp <= cap ? ncomp : -1;
}

/* -------------------------------------------------------------- initial */

/* SplitMix64 output number `counter` of the stream started at `seed`
 * (Steele, Lea & Flood, OOPSLA 2014; the mixing constants of that
 * publication's reference generator). */
static uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Random-phase initial conditions (Sec. III): |phi| = sig_p, |psi| = sig_q,
 * phases iid uniform in [0, 2 pi) -- draw number sector*S + site of the
 * SplitMix64 stream, top 53 bits as a fraction of 2 pi; momenta, links and
 * electric fields zero. */
void orc_init_random_phase(const orc_model *m, uint64_t seed, double *st) {
    const int64_t S = nsites(m);
    memset(st, 0, sizeof(double) * 20 * (size_t)S);
    for (int sec = 0; sec < 2; sec++)
        for (int64_t s = 0; s < S; s++) {
            uint64_t r = splitmix64(seed, (uint64_t)(sec * S + s));
            double phase = 2.0 * M_PI * ((double)(r >> 11) * 0x1.0p-53);
            st[(2 * sec) * S + s] = m->sig[sec] * cos(phase);
            st[(2 * sec + 1) * S + s] = m->sig[sec] * sin(phase);
        }
}

/* ----------------------------------------------------------------- step */

/* Time bookkeeping of one step from eta (Sec. III):
 *   a      = (eta / eta_ref)^p,  p = m / (1 - m)   (a ~ t^m, so a ~ eta^p)
 *   delta  = (1/2) alpha p Delta eta / eta, alpha = 2
 *   omega  = delta (1 - s)
 *   An     = a^{2 s} */
void orc_coefficients(const orc_model *m, double eta, double era_m, double s, double out[4]) {
    double p = era_m / (1.0 - era_m);
    double a = (p == 0.0) ? 1.0 : pow(eta / m->eta_ref, p);
    double alpha = 2.0;
    double delta = (p == 0.0) ? 0.0 : 0.5 * alpha * p * m->k / eta;
    double omega = delta * (1.0 - s);
    out[0] = a;
    out[1] = delta;
    out[2] = omega;
    out[3] = pow(a, 2.0 * s);
}

/*
 * One leapfrog step from eta_n to eta_n + k, in place (Sec. III):
 *   (1+delta) Pi^{n+1/2} = (1-delta) Pi^{n-1/2} + k F_phi(n)
 *   (1+omega) E^{n+1/2}  = (1-omega) E^{n-1/2}  + k F_A(n)
 *   phi^{n+1} = phi^n + k Pi^{n+1/2},   A^{n+1} = A^n + k E^{n+1/2}
 * If `d` is non-null, the diagnostics of integer time n are filled in.
 */
void orc_step_coeffs(const orc_model *m, double *st, double eta, double a, double delta, double omega,
                     double s, orc_diag *d);

void orc_step(const orc_model *m, double *st, double eta, double era_m, double s, orc_diag *d) {
    double co[4];
    orc_coefficients(m, eta, era_m, s, co);
    orc_step_coeffs(m, st, eta, co[0], co[1], co[2], s, d);
}

/* The same step with the scale factor and damping given explicitly
 * (An = a^{2s}); with delta = omega = 0 and a held fixed it evolves the
 * equations of Sec. III at a frozen instant of the expansion. */
void orc_step_coeffs(const orc_model *m, double *st, double eta, double a, double delta, double omega,
                     double s, orc_diag *d) {
    const int64_t S = nsites(m);
    const double k = m->k;
    const double An = pow(a, 2.0 * s);

    double *F = (double *)malloc(sizeof(double) * 10 * (size_t)S);
    orc_forces(m, st, An, F);

    double *old = NULL;
    if (d) {
        old = (double *)malloc(sizeof(double) * 20 * (size_t)S);
        memcpy(old, st, sizeof(double) * 20 * (size_t)S);
    }

    /* kicks */
    for (int sec = 0; sec < 2; sec++) {
        for (int part = 0; part < 2; part++) {
            double *pi = st + (c_mom(sec) + part) * S;
            const double *f = F + (2 * sec + part) * S;
            for (int64_t s0 = 0; s0 < S; s0++)
                pi[s0] = ((1.0 - delta) * pi[s0] + k * f[s0]) / (1.0 + delta);
        }
        for (int i = 0; i < 3; i++) {
            double *E = st + c_elec(sec, i) * S;
            const double *f = F + (4 + 3 * sec + i) * S;
            for (int64_t s0 = 0; s0 < S; s0++)
                E[s0] = ((1.0 - omega) * E[s0] + k * f[s0]) / (1.0 + omega);
        }
    }

    if (d) {
        /* time-centred momenta at integer time n */
        double *avg = (double *)malloc(sizeof(double) * 20 * (size_t)S);
        memcpy(avg, st, sizeof(double) * 20 * (size_t)S);
        for (int comp = 4; comp < 8; comp++)
            for (int64_t s0 = 0; s0 < S; s0++)
                avg[comp * S + s0] = 0.5 * (old[comp * S + s0] + st[comp * S + s0]);
        for (int comp = 14; comp < 20; comp++)
            for (int64_t s0 = 0; s0 < S; s0++)
                avg[comp * S + s0] = 0.5 * (old[comp * S + s0] + st[comp * S + s0]);

        const double a2s = pow(a, 2.0 * s), am2s = pow(a, -2.0 * s);
        double g[2];
        for (int sec = 0; sec < 2; sec++)
            g[sec] = 2.0 * m->e[sec] * m->e[sec] * An * (1.0 + delta) / (1.0 + omega);

        double *acc = (double *)calloc((size_t)m->nz * 10, sizeof(double));
#pragma omp parallel for schedule(static)
        for (int z = 0; z < m->nz; z++) {
            double *az = acc + 10 * z;
            for (int y = 0; y < m->ny; y++)
                for (int x = 0; x < m->nx; x++) {
                    const int c[3] = {x, y, z};
                    const int zero[3] = {0, 0, 0};
                    const int64_t s0 = site(m, c, zero);
                    /* fields at n come from `old` (not yet drifted, same as st) */
                    site_terms t = terms_at(m, old, avg, c);
                    double eps = t.K + t.G + am2s * (t.Kg + t.Bg) + a2s * t.V;
                    double lag = t.K - t.G + am2s * (t.Kg - t.Bg) - a2s * t.V;
                    az[0] += eps;
                    az[1] += lag;
                    az[2] += t.K * lag;
                    az[3] += t.G * lag;
                    az[4] += t.K * t.Vint;
                    az[5] += t.G * t.Vint;
                    /* Gauss law at n+1/2 (Sec. II; residual of the discrete form) */
                    for (int sec = 0; sec < 2; sec++) {
                        double div = 0.0;
                        for (int i = 0; i < 3; i++) {
                            int64_t sm = shifted(m, c, i, -1, i, 0);
                            div += (get_r(m, st, c_elec(sec, i), s0) - get_r(m, st, c_elec(sec, i), sm)) / m->h;
                        }
                        cplx phi = get_c(m, old, c_scal(sec), s0);
                        cplx pi = get_c(m, st, c_mom(sec), s0);
                        double rho = cimag(conj(phi) * pi);
                        double C = div - g[sec] * rho;
                        az[6 + sec] += fabs(C);
                        az[8 + sec] += fabs(div) + fabs(g[sec] * rho);
                    }
                }
        }
        double tot[10] = {0};
        for (int z = 0; z < m->nz; z++)
            for (int q = 0; q < 10; q++) tot[q] += acc[10 * z + q];
        free(acc);

        const double h3 = m->h * m->h * m->h;
        d->eta = eta;
        d->a = a;
        d->sum_eps = tot[0] * h3;
        d->sum_lag = tot[1] * h3;
        d->sum_KL = tot[2];
        d->sum_GL = tot[3];
        d->sum_KV = tot[4];
        d->sum_GV = tot[5];
        d->gauss_abs[0] = tot[6];
        d->gauss_abs[1] = tot[7];
        d->gauss_scale[0] = tot[8];
        d->gauss_scale[1] = tot[9];

        int32_t *W = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)S);
        int32_t *n = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)S);
        orc_windings(m, old, W);
        for (int sec = 0; sec < 2; sec++) {
            int64_t w = 0;
            for (int64_t q = 0; q < 3 * S; q++) w += abs(W[3 * sec * S + q]);
            d->wind_abs[sec] = w;
        }
        orc_cells(m, W, n);
        int64_t cp, cq;
        orc_overlap(m, n, m->overlap_radius, &cp, &cq);
        d->pq_count2 = cp + cq;
        free(W);
        free(n);
        free(avg);
        free(old);
    }

    /* drift */
    for (int sec = 0; sec < 2; sec++) {
        for (int part = 0; part < 2; part++) {
            double *phi = st + (c_scal(sec) + part) * S;
            const double *pi = st + (c_mom(sec) + part) * S;
            for (int64_t s0 = 0; s0 < S; s0++) phi[s0] = phi[s0] + k * pi[s0];
        }
        for (int i = 0; i < 3; i++) {
            double *A = st + c_link(sec, i) * S;
            const double *E = st + c_elec(sec, i) * S;
            for (int64_t s0 = 0; s0 < S; s0++) A[s0] = A[s0] + k * E[s0];
        }
    }
    free(F);
}

/* Diffusive cooling of the initial conditions (Sec. III): n forward-Euler
 * steps of size dt of the first-order flow
 *   d phi/d eta = D^-D^+ phi - lam/2 (|phi|^2 - sig^2) phi
 *   d A_i/d eta = -sum_j d_j^- F_ij + 2 e^2 Im[phi* D_i^+ phi]
 * for both sectors, at a = 1 and without the kappa coupling (the printed
 * cooling equations have none).  Momenta and electric fields are not
 * touched. */
void orc_cool(const orc_model *m, double *st, int n, double dt) {
    const int64_t S = nsites(m);
    orc_model q = *m;
    q.kappa = 0.0;
    double *F = (double *)malloc(sizeof(double) * 10 * (size_t)S);
    for (int it = 0; it < n; it++) {
        orc_forces(&q, st, 1.0, F);
        for (int sec = 0; sec < 2; sec++) {
            for (int part = 0; part < 2; part++) {
                double *phi = st + (c_scal(sec) + part) * S;
                const double *f = F + (2 * sec + part) * S;
                for (int64_t s0 = 0; s0 < S; s0++) phi[s0] += dt * f[s0];
            }
            for (int i = 0; i < 3; i++) {
                double *A = st + c_link(sec, i) * S;
                const double *f = F + (4 + 3 * sec + i) * S;
                for (int64_t s0 = 0; s0 < S; s0++) A[s0] += dt * f[s0];
            }
        }
    }
    free(F);
}

/* Advance n steps from eta0 (eta_j = eta0 + j k, not accumulated).  If
 * diag_every > 0, records are written for steps j with (j0 + j) % diag_every
 * == 0 into d (capacity max_d); the number written is returned. */
int orc_run(const orc_model *m, double *st, int n, double eta0, double era_m, double s,
            int64_t j0, int diag_every, orc_diag *d, int max_d) {
    int nd = 0;
    for (int j = 0; j < n; j++) {
        double eta = eta0 + j * m->k;
        orc_diag *rec = NULL;
        if (diag_every > 0 && (j0 + j) % diag_every == 0 && nd < max_d) rec = &d[nd++];
        orc_step(m, st, eta, era_m, s, rec);
    }
    return nd;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing aid; results do not depend on it). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
