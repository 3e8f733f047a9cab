/*
 * sanitize_check.c -- drives every entry point of the oracle on small ragged
 * boxes, to be built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers_cpu.py).  TEST INFRASTRUCTURE ONLY: it includes
 * oracle.c itself, so the checked code is the oracle as the tests use it.
 * Exit status 0 and the line "sanitize_check: ok" mean no sanitizer report.
 */
#include <stdio.h>

#include "oracle.c"

static double frand(uint64_t *s) {
    /* a small LCG for input values only (no part of the method) */
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static int run_box(int nx, int ny, int nz, int radius) {
    orc_model m;
    memset(&m, 0, sizeof m);
    m.nx = nx;
    m.ny = ny;
    m.nz = nz;
    m.overlap_radius = radius;
    m.h = 0.5;
    m.k = 0.1;
    m.lam[0] = 2.0;
    m.lam[1] = 1.6;
    m.e[0] = 1.0;
    m.e[1] = 0.9;
    m.sig[0] = 1.0;
    m.sig[1] = 1.1;
    m.kappa = 0.7;
    m.eta_ref = 3.0;
    const int64_t S = (int64_t)nx * ny * nz;
    double *st = calloc((size_t)(20 * S), sizeof(double));
    double *F = calloc((size_t)(10 * S), sizeof(double));
    int32_t *W = calloc((size_t)(6 * S), sizeof(int32_t));
    int32_t *n = calloc((size_t)(2 * S), sizeof(int32_t));
    int64_t *sizes = calloc((size_t)S, sizeof(int64_t));
    orc_diag d[8];
    if (!st || !F || !W || !n || !sizes) return 1;

    orc_init_random_phase(&m, 7, st);
    uint64_t seed = 11;
    for (int64_t i = 8 * S; i < 20 * S; i++) st[i] = 0.6 * (frand(&seed) - 0.5);   /* links, momenta */
    st[0] = st[S] = 0.0;                                                           /* a zero of phi */

    orc_cool(&m, st, 3, 1.0 / 30.0);
    orc_forces(&m, st, 1.3, F);
    volatile double e = orc_hamiltonian(&m, st);
    (void)e;
    double c[4];
    orc_coefficients(&m, 1.5, 0.5, 1.0, c);
    int nd = orc_run(&m, st, 6, 1.0, 0.5, 1.0, 0, 2, d, 8);
    nd += orc_run(&m, st, 3, 1.6, 2.0 / 3.0, -0.26, 6, 3, d, 8);
    orc_windings(&m, st, W);
    orc_cells(&m, W, n);
    int64_t cp = 0, cq = 0;
    orc_overlap(&m, n, radius, &cp, &cq);
    const int64_t k = orc_segments(&m, n, radius, sizes, S);
    free(st);
    free(F);
    free(W);
    free(n);
    free(sizes);
    return (nd == 4 && k >= 0) ? 0 : 1;
}

int main(void) {
    const int boxes[][4] = {{9, 7, 5, 1}, {4, 4, 4, 0}, {13, 5, 6, 1}};
    for (int b = 0; b < 3; b++) {
        for (int t = 1; t <= 3; t += 2) {
            orc_set_num_threads(t);
            if (run_box(boxes[b][0], boxes[b][1], boxes[b][2], boxes[b][3]) != 0) {
                printf("sanitize_check: unexpected result on box %d\n", b);
                return 1;
            }
        }
    }
    printf("sanitize_check: ok\n");
    return 0;
}
