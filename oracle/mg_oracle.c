/*
 * mg_oracle.c -- plain FP64 CPU multigrid for the cell-centred
 * constant-coefficient Helmholtz problem  (alpha - beta Lap) phi = f.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library's
 * results are checked against.  Only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant
 * with the GPU library and includes nothing from it.
 *
 * What it follows (pyro paper, Sec. 3.3 "Multigrid"):
 *   - the operator of Eq. (helmholtz); Poisson is (alpha, beta) = (0, -1);
 *   - the second difference of Sec. 2 ("Design"), applied along x and y with
 *     the same spacing (square cells);
 *   - red-black Gauss-Seidel relaxation; restriction = mean of the four fine
 *     cells; prolongation = centred slopes in x and y of each coarse cell,
 *     bilinear without the xy cross term;
 *   - homogeneous ghost cells: Dirichlet  phi[lo-1] = -phi[lo],
 *     Neumann phi[lo-1] = +phi[lo] (the two ghost-cell equations of Sec. 3.3);
 *     periodic (not in the paper; needed by the periodic workloads) wraps;
 *   - pure V-cycles down to a 2x2 grid, solved there by relaxation only
 *     (50 sweeps by default);
 *   - stop when ||r||_2 / ||f||_2 falls to the tolerance (Poisson test
 *     problem, Sec. 3.3.1).
 * Where the paper is silent the readings are: red = (i+j) even (0-based),
 * red first; ghosts refreshed before each colour; V(nu1, nu2) with the counts
 * given by the caller; coarse operators re-discretised with h_l = 2^l h and
 * the same alpha, beta; coarse levels use the homogeneous version of the
 * finest BC types; L2 norms are sqrt(h^2 sum v^2) over valid cells; the stop
 * test runs before every cycle and uses "<="; zero initial guess unless one
 * is given.  Singular problems (alpha == 0 and no Dirichlet side): the mean of
 * each restricted coarse right-hand side is removed and the mean of phi is
 * pinned to zero after each cycle.
 *
 * Storage: every field is (n+2) x (n+2) doubles, row-major, x contiguous,
 * one ghost layer; valid cell (i, j) (0 <= i, j < n) lives at
 * a[(j+1)*(n+2) + (i+1)].  Corner ghosts are never read or written.
 *
 * Parallelism: the only OpenMP use is over rows inside one colour of a
 * sweep (cells of one colour are independent) and over rows of pointwise
 * passes.  Sums are formed per row and then added in row order, so every
 * result is independent of the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mg_oracle.h"

#define IDX(n, i, j) ((size_t)((j) + 1) * (size_t)((n) + 2) + (size_t)((i) + 1))

static int is_singular(double alpha, const int bc[4]) {
    if (alpha != 0.0) return 0;
    for (int s = 0; s < 4; ++s)
        if (bc[s] == OG_DIRICHLET) return 0;
    return 1;
}

/* Ghost cells of one side-type: Dirichlet -> minus the adjacent valid cell,
 * Neumann -> plus it, periodic -> the valid cell on the opposite side. */
void og_fill(int n, const int bc[4], double *a) {
    for (int j = 0; j < n; ++j) {
        /* x-lo ghost (i = -1) and x-hi ghost (i = n) */
        double lo = a[IDX(n, 0, j)], hi = a[IDX(n, n - 1, j)];
        a[IDX(n, -1, j)] = bc[OG_XLO] == OG_PERIODIC ? hi : (bc[OG_XLO] == OG_DIRICHLET ? -lo : lo);
        a[IDX(n, n, j)] = bc[OG_XHI] == OG_PERIODIC ? lo : (bc[OG_XHI] == OG_DIRICHLET ? -hi : hi);
    }
    for (int i = 0; i < n; ++i) {
        double lo = a[IDX(n, i, 0)], hi = a[IDX(n, i, n - 1)];
        a[IDX(n, i, -1)] = bc[OG_YLO] == OG_PERIODIC ? hi : (bc[OG_YLO] == OG_DIRICHLET ? -lo : lo);
        a[IDX(n, i, n)] = bc[OG_YHI] == OG_PERIODIC ? lo : (bc[OG_YHI] == OG_DIRICHLET ? -hi : hi);
    }
}

/* One colour of Gauss-Seidel: every cell with (i+j)%2 == colour solves its
 * own row of (alpha - beta Lap) phi = f for phi_ij with the neighbours held:
 *   phi_ij = (f_ij + (beta/h^2)(phiE + phiW + phiN + phiS)) / (alpha + 4 beta/h^2) */
static void relax_colour(int n, double h, double alpha, double beta, const int bc[4],
                         double *phi, const double *f, int colour) {
    og_fill(n, bc, phi);
    const double c = beta / (h * h);
    const double diag = alpha + 4.0 * c;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        for (int i = (j + colour) & 1; i < n; i += 2) {
            double nb = phi[IDX(n, i + 1, j)] + phi[IDX(n, i - 1, j)] + phi[IDX(n, i, j + 1)] +
                        phi[IDX(n, i, j - 1)];
            phi[IDX(n, i, j)] = (f[IDX(n, i, j)] + c * nb) / diag;
        }
    }
}

void og_smooth(int n, double h, double alpha, double beta, const int bc[4], double *phi,
               const double *f, int iters) {
    for (int it = 0; it < iters; ++it) {
        relax_colour(n, h, alpha, beta, bc, phi, f, 0); /* red   */
        relax_colour(n, h, alpha, beta, bc, phi, f, 1); /* black */
    }
}

/* r = f - (alpha phi - beta Lap phi), Lap written as differences from the
 * centre to limit cancellation. */
void og_residual(int n, double h, double alpha, double beta, const int bc[4], double *phi,
                 const double *f, double *r) {
    og_fill(n, bc, phi);
    const double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double p = phi[IDX(n, i, j)];
            double lap = ((phi[IDX(n, i + 1, j)] - p) + (phi[IDX(n, i - 1, j)] - p) +
                          (phi[IDX(n, i, j + 1)] - p) + (phi[IDX(n, i, j - 1)] - p)) * ih2;
            r[IDX(n, i, j)] = f[IDX(n, i, j)] - (alpha * p - beta * lap);
        }
    }
}

/* coarse(I, J) = mean of fine (2I..2I+1, 2J..2J+1); fine has n cells/side. */
void og_restrict(int n, const double *fine, double *coarse) {
    int nc = n / 2;
#pragma omp parallel for schedule(static)
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I)
            coarse[IDX(nc, I, J)] =
                0.25 * (fine[IDX(n, 2 * I, 2 * J)] + fine[IDX(n, 2 * I + 1, 2 * J)] +
                        fine[IDX(n, 2 * I, 2 * J + 1)] + fine[IDX(n, 2 * I + 1, 2 * J + 1)]);
}

/* fine += P coarse.  Centred slopes of each coarse cell (ghosts from the
 * homogeneous BCs), then each of the four fine cells, which sit a quarter
 * coarse width from the coarse centre, gets e + dx*mx + dy*my with
 * dx, dy = -1/4 or +1/4 and mx, my the centred differences per coarse cell. */
void og_prolong_add(int nc, const int bc[4], double *coarse, double *fine) {
    int n = 2 * nc;
    og_fill(nc, bc, coarse);
#pragma omp parallel for schedule(static)
    for (int J = 0; J < nc; ++J) {
        for (int I = 0; I < nc; ++I) {
            double e = coarse[IDX(nc, I, J)];
            double mx = 0.5 * (coarse[IDX(nc, I + 1, J)] - coarse[IDX(nc, I - 1, J)]);
            double my = 0.5 * (coarse[IDX(nc, I, J + 1)] - coarse[IDX(nc, I, J - 1)]);
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    double dx = a ? 0.25 : -0.25, dy = b ? 0.25 : -0.25;
                    fine[IDX(n, 2 * I + a, 2 * J + b)] += e + dx * mx + dy * my;
                }
        }
    }
}

/* Sum over valid cells, formed per row then over rows in order. */
static double valid_sum(int n, const double *a, int squares) {
    double *row = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            double v = a[IDX(n, i, j)];
            s += squares ? v * v : v;
        }
        row[j] = s;
    }
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += row[j];
    free(row);
    return s;
}

double og_norm(int n, double h, const double *a) { return sqrt(h * h * valid_sum(n, a, 1)); }

double og_mean(int n, const double *a) { return valid_sum(n, a, 0) / ((double)n * (double)n); }

static void add_const(int n, double *a, double c) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) a[IDX(n, i, j)] += c;
}

size_t og_field_len(int n) { return (size_t)(n + 2) * (size_t)(n + 2); }

/* Exact solve of one level, an alternative bottom for the V-cycle (Sec. 3.3
 * leaves the coarsest solve open): the level's operator alpha - beta Lap_h,
 * side rules included, written out as a dense matrix over the n*n valid cells
 * (unknown k = j n + i) and solved by Gaussian elimination with partial
 * pivoting.  A singular operator (constants in its null space) gets c 1 1^T
 * added, c = beta / h^2: for a right-hand side of zero sum, 1^T A = 0 makes
 * the modified system's solution the zero-sum solution of the original. */
static void direct_solve(int n, double h, double alpha, double beta, const int bc[4], int singular,
                         double *phi, const double *f) {
    int m = n * n, w = m + 1;
    double c = beta / (h * h);
    double *A = (double *)calloc((size_t)m * (size_t)w, sizeof(double)); /* rows [A | b] */
    static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1}; /* sides x-lo, x-hi, y-lo, y-hi */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int k = j * n + i;
            double *row = A + (size_t)k * w;
            row[k] += alpha + 4.0 * c;
            for (int s = 0; s < 4; ++s) {
                int ii = i + di[s], jj = j + dj[s];
                if (ii >= 0 && ii < n && jj >= 0 && jj < n)
                    row[jj * n + ii] -= c;
                else if (bc[s] == OG_PERIODIC)
                    row[((jj + n) % n) * n + (ii + n) % n] -= c;
                else if (bc[s] == OG_DIRICHLET)
                    row[k] += c; /* ghost = -cell */
                else
                    row[k] -= c; /* ghost = +cell */
            }
            if (singular)
                for (int q = 0; q < m; ++q) row[q] += c;
            row[m] = f[IDX(n, i, j)];
        }
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[(size_t)r * w + col]) > fabs(A[(size_t)piv * w + col])) piv = r;
        if (piv != col)
            for (int q = 0; q < w; ++q) {
                double t = A[(size_t)col * w + q];
                A[(size_t)col * w + q] = A[(size_t)piv * w + q];
                A[(size_t)piv * w + q] = t;
            }
        for (int r = col + 1; r < m; ++r) {
            double g = A[(size_t)r * w + col] / A[(size_t)col * w + col];
            for (int q = col; q < w; ++q) A[(size_t)r * w + q] -= g * A[(size_t)col * w + q];
        }
    }
    for (int k = m - 1; k >= 0; --k) {
        double s = A[(size_t)k * w + m];
        for (int q = k + 1; q < m; ++q) s -= A[(size_t)k * w + q] * A[(size_t)q * w + m];
        A[(size_t)k * w + m] = s / A[(size_t)k * w + k];
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) phi[IDX(n, i, j)] = A[(size_t)(j * n + i) * w + m];
    free(A);
}

/* Recursive V(nu1, nu2) cycle on level `lev` of the hierarchy.  phi[l] and
 * f[l] hold the level-l fields; r is scratch of the finest size. */
static void vcycle(const og_params *p, int lev, double **phi, double **f, double *r, int singular) {
    int n = p->n >> lev;
    double h = p->h * (double)(1 << lev);
    if (n >= 4 && n == p->n_bottom) {
        direct_solve(n, h, p->alpha, p->beta, p->bc, singular, phi[lev], f[lev]);
        return;
    }
    if (n == 2) {
        og_smooth(n, h, p->alpha, p->beta, p->bc, phi[lev], f[lev], p->nu_bottom);
        return;
    }
    og_smooth(n, h, p->alpha, p->beta, p->bc, phi[lev], f[lev], p->nu1);
    og_residual(n, h, p->alpha, p->beta, p->bc, phi[lev], f[lev], r);
    og_restrict(n, r, f[lev + 1]);
    if (singular) add_const(n / 2, f[lev + 1], -og_mean(n / 2, f[lev + 1]));
    memset(phi[lev + 1], 0, sizeof(double) * og_field_len(n / 2));
    vcycle(p, lev + 1, phi, f, r, singular);
    og_prolong_add(n / 2, p->bc, phi[lev + 1], phi[lev]);
    og_smooth(n, h, p->alpha, p->beta, p->bc, phi[lev], f[lev], p->nu2);
}

static int num_levels(int n) {
    int L = 0;
    while ((n >> L) >= 2) ++L;
    return L; /* n, n/2, ..., 2 */
}

static int valid_n(int n) { return n >= 2 && (n & (n - 1)) == 0; }

/* Hierarchy helpers: level 0 aliases the caller's arrays. */
static int alloc_levels(const og_params *p, double *phi0, const double *f0, double ***phi,
                        double ***f, double **r) {
    int L = num_levels(p->n);
    *phi = (double **)calloc((size_t)L, sizeof(double *));
    *f = (double **)calloc((size_t)L, sizeof(double *));
    *r = (double *)calloc(og_field_len(p->n), sizeof(double));
    (*phi)[0] = phi0;
    (*f)[0] = (double *)f0;
    for (int l = 1; l < L; ++l) {
        (*phi)[l] = (double *)calloc(og_field_len(p->n >> l), sizeof(double));
        (*f)[l] = (double *)calloc(og_field_len(p->n >> l), sizeof(double));
    }
    return L;
}

static void free_levels(int L, double **phi, double **f, double *r) {
    for (int l = 1; l < L; ++l) {
        free(phi[l]);
        free(f[l]);
    }
    free(phi);
    free(f);
    free(r);
}

int og_vcycle(const og_params *p, double *phi, const double *f) {
    if (!valid_n(p->n)) return OG_EINVAL;
    double **P, **F, *r;
    int L = alloc_levels(p, phi, f, &P, &F, &r);
    vcycle(p, 0, P, F, r, is_singular(p->alpha, p->bc));
    free_levels(L, P, F, r);
    return OG_OK;
}

int og_solve(const og_params *p, double *phi, const double *f, int use_guess, og_result *out) {
    if (!valid_n(p->n)) return OG_EINVAL;
    int n = p->n;
    int singular = is_singular(p->alpha, p->bc);
    if (!use_guess) memset(phi, 0, sizeof(double) * og_field_len(n));
    memset(out, 0, sizeof(*out));

    double fnorm = og_norm(n, p->h, f);
    if (fnorm == 0.0) {
        memset(phi, 0, sizeof(double) * og_field_len(n));
        out->status = OG_OK;
        return OG_OK;
    }
    if (singular) add_const(n, phi, -og_mean(n, phi));

    double **P, **F, *r;
    int L = alloc_levels(p, phi, f, &P, &F, &r);
    int status = OG_NOT_CONVERGED;
    int cycles = 0;
    for (;;) {
        og_residual(n, p->h, p->alpha, p->beta, p->bc, phi, f, r);
        double rho = og_norm(n, p->h, r) / fnorm;
        if (cycles < OG_HISTORY) out->history[cycles] = rho;
        if (cycles == 0) out->rel_resid0 = rho;
        out->rel_resid = rho;
        if (rho <= p->rtol) {
            status = OG_OK;
            break;
        }
        if (cycles >= p->max_cycles) break;
        vcycle(p, 0, P, F, r, singular);
        if (singular) add_const(n, phi, -og_mean(n, phi));
        ++cycles;
    }
    og_fill(n, p->bc, phi);
    out->cycles = cycles;
    out->status = status;
    free_levels(L, P, F, r);
    return status;
}

/* Full multigrid (FMG): a start for the V-cycles that the paper does not
 * describe (its Sec. 3.3 cycles from a zero guess and leaves the coarse-grid
 * solver open); this is the standard nested iteration of the multigrid
 * literature (Brandt 1977; Briggs, Henson and McCormick, "A Multigrid
 * Tutorial", 2nd ed., Ch. 3), assembled from the operators above.
 *   1. f is restricted (four-cell mean) level by level down to the FMG's
 *      coarsest level, the one of top_n cells per side; on a singular problem
 *      each restricted f has its mean removed.
 *   2. There phi starts at zero and gets ncyc_top V-cycles.
 *   3. On each finer level, phi = P phi_coarse (the prolongation of Sec. 3.3
 *      added to a zero field), then ncyc V-cycles against that level's f.
 *      The V-cycles are those of og_vcycle, rooted at that level; a singular
 *      problem gets the mean of phi removed after each, as og_solve does.
 * The result is the finest phi with its ghosts filled. */
int og_fmg(const og_params *p, double *phi, const double *f, int top_n, int ncyc_top, int ncyc) {
    if (!valid_n(p->n) || !valid_n(top_n) || top_n > p->n || ncyc_top < 0 || ncyc < 0) return OG_EINVAL;
    int singular = is_singular(p->alpha, p->bc);
    double **P, **F, *r;
    int L = alloc_levels(p, phi, f, &P, &F, &r);
    int c = 0;
    while ((p->n >> c) > top_n) ++c;
    for (int l = 1; l <= c; ++l) {
        og_restrict(p->n >> (l - 1), F[l - 1], F[l]);
        if (singular) add_const(p->n >> l, F[l], -og_mean(p->n >> l, F[l]));
    }
    memset(P[c], 0, sizeof(double) * og_field_len(p->n >> c));
    for (int k = 0; k < ncyc_top; ++k) {
        vcycle(p, c, P, F, r, singular);
        if (singular) add_const(p->n >> c, P[c], -og_mean(p->n >> c, P[c]));
    }
    for (int l = c - 1; l >= 0; --l) {
        memset(P[l], 0, sizeof(double) * og_field_len(p->n >> l));
        og_prolong_add(p->n >> (l + 1), p->bc, P[l + 1], P[l]);
        for (int k = 0; k < ncyc; ++k) {
            vcycle(p, l, P, F, r, singular);
            if (singular) add_const(p->n >> l, P[l], -og_mean(p->n >> l, P[l]));
        }
    }
    og_fill(p->n, p->bc, phi);
    free_levels(L, P, F, r);
    return OG_OK;
}

/* Relaxation alone (no coarse grids), the paper's first suggested exercise:
 * whole red-black iterations until the same stopping rule holds. */
int og_smooth_solve(const og_params *p, double *phi, const double *f, int max_iters,
                    og_result *out) {
    if (!valid_n(p->n)) return OG_EINVAL;
    int n = p->n;
    int singular = is_singular(p->alpha, p->bc);
    memset(out, 0, sizeof(*out));
    double *r = (double *)calloc(og_field_len(n), sizeof(double));
    double fnorm = og_norm(n, p->h, f);
    int it = 0, status = OG_NOT_CONVERGED;
    for (;;) {
        og_residual(n, p->h, p->alpha, p->beta, p->bc, phi, f, r);
        double rho = fnorm > 0 ? og_norm(n, p->h, r) / fnorm : 0.0;
        out->rel_resid = rho;
        if (rho <= p->rtol) {
            status = OG_OK;
            break;
        }
        if (it >= max_iters) break;
        og_smooth(n, p->h, p->alpha, p->beta, p->bc, phi, f, 1);
        if (singular) add_const(n, phi, -og_mean(n, phi));
        ++it;
    }
    out->cycles = it;
    out->status = status;
    free(r);
    return status;
}

/* Crank-Nicolson step of the diffusion equation phi_t = k Lap phi (pyro
 * paper, Sec. 3.4 "Implicit diffusion"): the step averages k Lap phi over
 * the old and the new time level, so with beta = k dt / 2 the new phi solves
 * (1 - beta Lap) phi' = phi + beta Lap phi -- the Helmholtz problem of
 * Sec. 3.3 with alpha = 1 and that right-hand side.
 * og_cn_rhs: f = phi + beta Lap phi on valid cells (phi's ghosts filled
 * first; Lap written as differences from the centre, as in og_residual). */
void og_cn_rhs(int n, double h, double beta, const int bc[4], double *phi, double *f) {
    og_fill(n, bc, phi);
    const double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double p = phi[IDX(n, i, j)];
            double lap = ((phi[IDX(n, i + 1, j)] - p) + (phi[IDX(n, i - 1, j)] - p) +
                          (phi[IDX(n, i, j + 1)] - p) + (phi[IDX(n, i, j - 1)] - p)) * ih2;
            f[IDX(n, i, j)] = p + beta * lap;
        }
    }
}

/* One step in place: work <- the right-hand side, then V-cycles from phi
 * (the old level as the initial guess) to the tolerance.  p->alpha must be
 * 1 and p->beta = k dt / 2. */
int og_cn_step(const og_params *p, double *phi, double *work, og_result *out) {
    if (!valid_n(p->n) || p->alpha != 1.0) return OG_EINVAL;
    og_cn_rhs(p->n, p->h, p->beta, p->bc, phi, work);
    return og_solve(p, phi, work, 1, out);
}

/* Inhomogeneous side data (Sec. 3.3: the boundary value itself then enters
 * the ghost cell's expression).  b[s] holds n values along side s (index j
 * for the x sides, i for the y sides; NULL = homogeneous on that side; a
 * periodic side takes none).  Second-order ghosts:
 *   Dirichlet, value v at the face:  ghost = 2 v - phi_adjacent;
 *   Neumann, derivative d = dphi/dx (x sides) or dphi/dy (y sides) at the
 *   face:  lo ghost = phi_adjacent - h d,  hi ghost = phi_adjacent + h d. */
static double side_value(const double *const b[4], int s, int k) { return b && b[s] ? b[s][k] : 0.0; }

void og_fill_bc(int n, double h, const int bc[4], const double *const b[4], double *a) {
    og_fill(n, bc, a);
    for (int j = 0; j < n; ++j) {
        double vl = side_value(b, OG_XLO, j), vh = side_value(b, OG_XHI, j);
        if (bc[OG_XLO] == OG_DIRICHLET) a[IDX(n, -1, j)] += 2.0 * vl;
        if (bc[OG_XLO] == OG_NEUMANN) a[IDX(n, -1, j)] -= h * vl;
        if (bc[OG_XHI] == OG_DIRICHLET) a[IDX(n, n, j)] += 2.0 * vh;
        if (bc[OG_XHI] == OG_NEUMANN) a[IDX(n, n, j)] += h * vh;
    }
    for (int i = 0; i < n; ++i) {
        double vl = side_value(b, OG_YLO, i), vh = side_value(b, OG_YHI, i);
        if (bc[OG_YLO] == OG_DIRICHLET) a[IDX(n, i, -1)] += 2.0 * vl;
        if (bc[OG_YLO] == OG_NEUMANN) a[IDX(n, i, -1)] -= h * vl;
        if (bc[OG_YHI] == OG_DIRICHLET) a[IDX(n, i, n)] += 2.0 * vh;
        if (bc[OG_YHI] == OG_NEUMANN) a[IDX(n, i, n)] += h * vh;
    }
}

/* The problem with side data as a homogeneous one: the data's part of each
 * ghost (ghost with data minus ghost without) multiplies beta / h^2 in the
 * operator, so it moves to the right-hand side:
 *   f_out = f + (beta / h^2) * sum over the cell's out-of-domain neighbours of
 *           (data part of that ghost).
 * The coarse levels then solve the homogeneous correction problem, as the
 * paper's V-cycle does. */
void og_bc_rhs(int n, double h, double beta, const int bc[4], const double *const b[4], const double *f,
               double *f_out) {
    double *g0 = (double *)calloc(og_field_len(n), sizeof(double));
    og_fill_bc(n, h, bc, b, g0); /* the data part of every ghost (phi = 0) */
    const double c = beta / (h * h);
    memcpy(f_out, f, sizeof(double) * og_field_len(n));
    for (int j = 0; j < n; ++j) {
        f_out[IDX(n, 0, j)] += c * (bc[OG_XLO] == OG_PERIODIC ? 0.0 : g0[IDX(n, -1, j)]);
        f_out[IDX(n, n - 1, j)] += c * (bc[OG_XHI] == OG_PERIODIC ? 0.0 : g0[IDX(n, n, j)]);
    }
    for (int i = 0; i < n; ++i) {
        f_out[IDX(n, i, 0)] += c * (bc[OG_YLO] == OG_PERIODIC ? 0.0 : g0[IDX(n, i, -1)]);
        f_out[IDX(n, i, n - 1)] += c * (bc[OG_YHI] == OG_PERIODIC ? 0.0 : g0[IDX(n, i, n)]);
    }
    free(g0);
}

/* Solve with side data: V-cycles on the shifted right-hand side, then the
 * returned field's ghosts filled with the data. */
int og_solve_bc(const og_params *p, double *phi, const double *f, const double *const b[4], int use_guess,
                og_result *out) {
    if (!valid_n(p->n)) return OG_EINVAL;
    double *f2 = (double *)calloc(og_field_len(p->n), sizeof(double));
    og_bc_rhs(p->n, p->h, p->beta, p->bc, b, f, f2);
    int st = og_solve(p, phi, f2, use_guess, out);
    og_fill_bc(p->n, p->h, p->bc, b, phi);
    free(f2);
    return st;
}

/* Cell-centred approximate projection (pyro paper, Sec. 3.5, incompressible
 * flow): a velocity field U* = (u, v) at cell centres is split as U^d + grad
 * phi by solving Lap phi = D U* and setting U = U* - G phi, where D and G are
 * centred differences across two cells and Lap the 5-point operator (so
 * D G != Lap: the projection is approximate).  Doubly periodic domain (the
 * paper's convergence test); the Poisson problem is then singular and its
 * zero-mean solution is taken. */
void og_divergence(int n, double h, const double *u, const double *v, double *f) {
    const int bc[4] = {OG_PERIODIC, OG_PERIODIC, OG_PERIODIC, OG_PERIODIC};
    double *uu = (double *)malloc(sizeof(double) * og_field_len(n));
    double *vv = (double *)malloc(sizeof(double) * og_field_len(n));
    memcpy(uu, u, sizeof(double) * og_field_len(n));
    memcpy(vv, v, sizeof(double) * og_field_len(n));
    og_fill(n, bc, uu);
    og_fill(n, bc, vv);
    const double i2h = 1.0 / (2.0 * h);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            f[IDX(n, i, j)] = (uu[IDX(n, i + 1, j)] - uu[IDX(n, i - 1, j)]) * i2h +
                              (vv[IDX(n, i, j + 1)] - vv[IDX(n, i, j - 1)]) * i2h;
    free(uu);
    free(vv);
}

/* u -= (phi[i+1] - phi[i-1]) / 2h, v -= (phi[j+1] - phi[j-1]) / 2h */
void og_subtract_gradient(int n, double h, double *phi, double *u, double *v) {
    const int bc[4] = {OG_PERIODIC, OG_PERIODIC, OG_PERIODIC, OG_PERIODIC};
    og_fill(n, bc, phi);
    const double i2h = 1.0 / (2.0 * h);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            u[IDX(n, i, j)] -= (phi[IDX(n, i + 1, j)] - phi[IDX(n, i - 1, j)]) * i2h;
            v[IDX(n, i, j)] -= (phi[IDX(n, i, j + 1)] - phi[IDX(n, i, j - 1)]) * i2h;
        }
}

/* In place on u, v; phi receives the zero-mean potential.  p must describe
 * the periodic Poisson problem (alpha 0, beta -1, all sides periodic). */
int og_project(const og_params *p, double *u, double *v, double *phi, og_result *out) {
    if (!valid_n(p->n) || p->alpha != 0.0 || p->beta != -1.0) return OG_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] != OG_PERIODIC) return OG_EINVAL;
    double *f = (double *)calloc(og_field_len(p->n), sizeof(double));
    og_divergence(p->n, p->h, u, v, f);
    int st = og_solve(p, phi, f, 0, out);
    og_subtract_gradient(p->n, p->h, phi, u, v);
    free(f);
    return st;
}
