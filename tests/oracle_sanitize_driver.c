/*
 * oracle_sanitize_driver.c -- exercises every entry point of the C oracle on
 * small grids, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py compiles and runs it on the CPU).  Each array
 * is allocated to its exact length, so any read or write past a field, a
 * ghost layer or a side-data array is reported by the sanitizer.  The driver
 * also checks that the solves converge; it prints one line per case and
 * returns non-zero on a failed check.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mg_oracle.h"

static int failures = 0;

static double *field(int n) { return (double *)calloc(og_field_len(n), sizeof(double)); }

static void fill_random(int n, double *a, unsigned *seed, int zero_mean) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            *seed = *seed * 1664525u + 1013904223u;
            const double v = (double)(*seed >> 8) / 16777216.0 - 0.5;
            a[(size_t)(j + 1) * (n + 2) + i + 1] = v;
            s += v;
        }
    if (zero_mean)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) a[(size_t)(j + 1) * (n + 2) + i + 1] -= s / ((double)n * n);
}

static void check(int ok, const char *what, int n, const int bc[4]) {
    printf("%s n=%d bc=%d%d%d%d %s\n", what, n, bc[0], bc[1], bc[2], bc[3], ok ? "ok" : "FAILED");
    if (!ok) ++failures;
}

static og_params params(int n, const int bc[4], double alpha, double beta) {
    og_params p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.h = 1.0 / n;
    p.alpha = alpha;
    p.beta = beta;
    memcpy(p.bc, bc, sizeof(p.bc));
    p.nu1 = p.nu2 = 2;
    p.nu_bottom = 50;
    p.max_cycles = 60;
    p.rtol = 1e-10;
    p.n_bottom = 2;
    return p;
}

int main(void) {
    static const int sides[5][2] = {{OG_PERIODIC, OG_PERIODIC}, {OG_DIRICHLET, OG_DIRICHLET},
                                    {OG_NEUMANN, OG_NEUMANN}, {OG_DIRICHLET, OG_NEUMANN},
                                    {OG_NEUMANN, OG_DIRICHLET}};
    unsigned seed = 12345u;
    const int sizes[] = {2, 4, 16, 32};
    for (int si = 0; si < 4; ++si) {
        const int n = sizes[si];
        for (int ax = 0; ax < 5; ++ax)
            for (int ay = 0; ay < 5; ++ay) {
                const int bc[4] = {sides[ax][0], sides[ax][1], sides[ay][0], sides[ay][1]};
                const int singular = bc[0] != OG_DIRICHLET && bc[1] != OG_DIRICHLET && bc[2] != OG_DIRICHLET &&
                                     bc[3] != OG_DIRICHLET;
                for (int op = 0; op < 2; ++op) {
                    const double alpha = op ? 1.0 : 0.0, beta = op ? 0.37 / ((double)n * n) : -1.0;
                    og_params p = params(n, bc, alpha, beta);
                    double *f = field(n), *phi = field(n), *r = field(n);
                    fill_random(n, f, &seed, singular && op == 0);
                    og_fill(n, bc, f);
                    og_smooth(n, p.h, alpha, beta, bc, phi, f, 2);
                    og_residual(n, p.h, alpha, beta, bc, phi, f, r);
                    if (n >= 4) {
                        double *c = field(n / 2);
                        og_restrict(n, r, c);
                        og_prolong_add(n / 2, bc, c, phi);
                        free(c);
                    }
                    (void)og_norm(n, p.h, r);
                    (void)og_mean(n, r);
                    og_vcycle(&p, phi, f);
                    og_result res;
                    const int st = og_solve(&p, phi, f, 0, &res);
                    check(st == OG_OK && res.rel_resid <= 1e-10, "solve", n, bc);
                    if (n >= 8 && !(singular && op == 0)) {
                        og_params q = p;
                        q.n_bottom = 4;
                        const int s2 = og_solve(&q, phi, f, 0, &res);
                        check(s2 == OG_OK && res.rel_resid <= 1e-10, "solve_exact_bottom", n, bc);
                    }
                    {  /* full multigrid start from 2^2 and from the middle level */
                        double *g = field(n);
                        const int s6 = og_fmg(&p, g, f, 2, 1, 1);
                        check(s6 == OG_OK, "fmg", n, bc);
                        const int s7 = og_fmg(&p, g, f, n > 4 ? n / 4 : n, 2, 2);
                        check(s7 == OG_OK, "fmg_top", n, bc);
                        free(g);
                    }
                    if (n <= 16) {
                        double *g = field(n);
                        og_params q = p;
                        q.max_cycles = 200000;
                        const int s3 = og_smooth_solve(&q, g, f, 200000, &res);
                        check(s3 == OG_OK || s3 == OG_NOT_CONVERGED, "smooth_solve", n, bc);
                        free(g);
                    }
                    if (op == 1) {  /* Crank-Nicolson step: alpha = 1 */
                        double *w = field(n);
                        fill_random(n, phi, &seed, 0);
                        og_cn_rhs(n, p.h, beta, bc, phi, w);
                        const int s4 = og_cn_step(&p, phi, w, &res);
                        check(s4 == OG_OK, "cn_step", n, bc);
                        free(w);
                    }
                    /* side data on every non-periodic side: arrays of exactly n values */
                    double *b[4] = {NULL, NULL, NULL, NULL};
                    for (int sd = 0; sd < 4; ++sd)
                        if (bc[sd] != OG_PERIODIC) {
                            b[sd] = (double *)malloc(sizeof(double) * n);
                            for (int k = 0; k < n; ++k) b[sd][k] = 0.1 * (k + 1) / n;
                        }
                    double *fo = field(n);
                    og_bc_rhs(n, p.h, beta, bc, (const double *const *)b, f, fo);
                    og_fill_bc(n, p.h, bc, (const double *const *)b, phi);
                    if (!(singular && op == 0)) {
                        const int s5 = og_solve_bc(&p, phi, f, (const double *const *)b, 0, &res);
                        check(s5 == OG_OK, "solve_bc", n, bc);
                    }
                    for (int sd = 0; sd < 4; ++sd) free(b[sd]);
                    free(fo);
                    free(f);
                    free(phi);
                    free(r);
                }
            }
        /* projection: doubly periodic Poisson */
        {
            const int bc[4] = {OG_PERIODIC, OG_PERIODIC, OG_PERIODIC, OG_PERIODIC};
            og_params p = params(n, bc, 0.0, -1.0);
            double *u = field(n), *v = field(n), *phi = field(n), *d = field(n);
            fill_random(n, u, &seed, 0);
            fill_random(n, v, &seed, 0);
            og_divergence(n, p.h, u, v, d);
            og_result res;
            const int st = og_project(&p, u, v, phi, &res);
            check(st == OG_OK, "project", n, bc);
            og_subtract_gradient(n, p.h, phi, u, v);
            free(u);
            free(v);
            free(phi);
            free(d);
        }
    }
    printf("failures: %d\n", failures);
    return failures ? 1 : 0;
}
