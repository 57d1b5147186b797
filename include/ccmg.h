/*
 * ccmg.h -- C ABI of the MI355X (gfx950) cell-centred multigrid library.
 *
 * Problem (pyro paper, Sec. 3.3, Eq. (helmholtz)):
 *     (alpha - beta Lap) phi = f     on a square grid of n x n square cells,
 * Poisson is (alpha, beta) = (0, -1).  The method: pure V-cycles of red-black
 * Gauss-Seidel relaxation, restriction by averaging the four fine cells,
 * prolongation by centred slopes per coarse cell (bilinear without the xy
 * term), coarsening down to a 2 x 2 grid that is solved by relaxation alone
 * (50 sweeps by default), stopping when ||r||_2 / ||f||_2 <= rtol
 * (Sec. 3.3 and its Poisson test problem, Sec. 3.3.1).  Ghost cells follow
 * the paper's homogeneous rules: Dirichlet phi[lo-1] = -phi[lo], Neumann
 * phi[lo-1] = +phi[lo]; periodic sides wrap.
 *
 * Conventions for every entry point:
 *   - Device arrays hold one grid level *with* one ghost layer: (n+2) rows of
 *     `pitch` elements (pitch >= n+2, and (n+2) * pitch < 2^31), row-major,
 *     x contiguous; valid cell (i, j) is element (j+1)*pitch + (i+1).
 *     Pitches are in elements; a pitch outside these bounds is CCMG_EINVAL.
 *   - Arrays are owned by the caller; the library never allocates device
 *     memory.  Plans work inside a caller-provided workspace.
 *   - All GPU work is enqueued on the plan's stream (a hipStream_t passed as
 *     void*; NULL = the default stream).
 *   - Functions return a ccmg status; none aborts or throws.  Arguments are
 *     validated before any device work is enqueued.
 *   - A plan is not re-entrant: one call at a time per plan.  Distinct plans
 *     (with distinct workspaces) may run on distinct streams concurrently.
 */
#ifndef CCMG_H
#define CCMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Side types (Sec. 3.3; periodic is an addition for doubly periodic work). */
enum { CCMG_BC_DIRICHLET = 0, CCMG_BC_NEUMANN = 1, CCMG_BC_PERIODIC = 2 };
/* Side order inside ccmg_problem.bc */
enum { CCMG_XLO = 0, CCMG_XHI = 1, CCMG_YLO = 2, CCMG_YHI = 3 };
/* Precision forms.
 *   CCMG_FP64 : every level relaxed, restricted and prolonged in FP64.
 *   CCMG_MIXED: iterative refinement -- the FP64 residual of the FP64 iterate
 *               is rounded to FP32, FP32 V-cycles solve for the correction
 *               (2x2 bottom solve in FP64), the correction is added in FP64,
 *               and the stop test always uses the FP64 residual.  With
 *               nu1 = nu2 = 2 a refinement step runs several FP32 V-cycles
 *               from a zero correction: the first step 2, later steps as
 *               many as the contraction measured so far says the tolerance
 *               needs, at most 3 (option CCMG_OPT_MIXED_INNER, 1..8; one
 *               more when that is expected to end the solve); the finest
 *               level's post-smoothing of one inner cycle and pre-smoothing
 *               of the next share one launch. */
enum { CCMG_FP64 = 0, CCMG_MIXED = 1 };

/* Status codes */
enum {
    CCMG_OK = 0,
    CCMG_NOT_CONVERGED = 1, /* max_cycles reached; last iterate and history kept */
    CCMG_EINVAL = -1,       /* NULL pointer, bad count, bad pitch, bad level     */
    CCMG_ESIZE = -2,        /* n not a power of two in [2, 16384]                */
    CCMG_EBC = -3,          /* unknown side type, or periodic not paired         */
    CCMG_EINCOMPAT = -4,    /* singular problem with |sum f| > 1e-12 sum |f|     */
    CCMG_ENONFINITE = -5,   /* NaN / Inf in f, or a residual norm went NaN / Inf */
    CCMG_EHIP = -6,         /* a HIP runtime call failed                         */
    CCMG_EWORKSPACE = -7    /* workspace NULL, too small or misaligned (256 B)   */
};

#define CCMG_HISTORY 128

typedef struct {
    int n;                 /* cells per side: power of two, 2 <= n <= 16384     */
    int ng;                /* ghost layers: must be 1                           */
    double xmin, xmax;     /* domain; cells must be square:                     */
    double ymin, ymax;     /*   xmax - xmin == ymax - ymin > 0                  */
    int bc[4];             /* side types, order CCMG_XLO, XHI, YLO, YHI         */
    double alpha, beta;    /* (alpha - beta Lap) phi = f                        */
    int nu1, nu2;          /* relaxations before / after the coarse correction, 0..8 */
    int nu_bottom;         /* relaxations on the 2 x 2 grid (paper: 50)         */
    int max_cycles;        /* >= 0, at most CCMG_HISTORY - 1                    */
    double rtol;           /* stop when ||r|| / ||f|| <= rtol                   */
    int prec;              /* CCMG_FP64 or CCMG_MIXED                           */
} ccmg_problem;

typedef struct {
    int status;            /* same value the call returned                      */
    int cycles;            /* V-cycles (MIXED: refinement steps) performed      */
    double rel_resid0;     /* ||f - A phi0|| / ||f|| of the starting iterate    */
    double rel_resid;      /* ... of the returned iterate                       */
    double history[CCMG_HISTORY]; /* history[k] after k cycles, k <= cycles     */
    float ms;              /* device time of the call (HIP events)              */
    int inner_cycles;      /* MIXED: FP32 V-cycles performed in total           */
} ccmg_result;

typedef struct ccmg_plan ccmg_plan;

/* Text for a status code (static storage). */
const char *ccmg_status_str(int status);

/* Fill *p with the defaults: unit square, all sides Dirichlet, Poisson
 * (Eq. helmholtz with alpha = 0, beta = -1), V(2,2), 50 bottom relaxations
 * (Sec. 3.3, "by default"), 100 cycles, rtol 1e-10, FP64. */
int ccmg_problem_init(ccmg_problem *p, int n);

/* Validate a problem without touching the GPU: n a power of two (the
 * hierarchy n, n/2, ..., 2 of Sec. 3.3), square cells, known side types with
 * periodic sides paired, counts in range. */
int ccmg_problem_check(const ccmg_problem *p);

/* Bytes of device workspace ccmg_plan_create needs for *p (0 if invalid): the
 * coarse levels of the hierarchy (Sec. 3.3) and the solve's scalars. */
size_t ccmg_workspace_bytes(const ccmg_problem *p);

/* Create a plan (the grid hierarchy of Sec. 3.3 laid out in a caller-owned
 * device workspace of >= ccmg_workspace_bytes bytes, 256-byte aligned).  The workspace must outlive the plan and must not
 * be shared with another live plan.  `stream` is a hipStream_t (or NULL). */
int ccmg_plan_create(const ccmg_problem *p, void *d_ws, size_t ws_bytes, void *stream,
                     ccmg_plan **out);
int ccmg_plan_destroy(ccmg_plan *plan);

/* Solve (alpha - beta Lap) phi = f by V-cycles to the plan's tolerance
 * (Sec. 3.3; stop test as in Sec. 3.3.1).  d_f, d_phi: device arrays of the
 * finest level, same pitch.  f's ghosts are ignored.  On entry d_phi holds the
 * starting iterate if use_guess != 0 (else it is ignored and zero is used);
 * on return it holds the last iterate with its ghost cells filled.  Blocks
 * until the result is known (the stop test needs it).  Singular problems
 * (alpha == 0, no Dirichlet side) are checked for compatibility and return
 * the zero-mean solution.  ||f|| == 0 gives phi = 0 and CCMG_OK.
 * `out` may be NULL.  FP64 plans with nu1 = nu2 = 2 and more than 32 cells
 * per side run the finest level's post-smoothing of one cycle and
 * pre-smoothing of the next in one launch (the same iterates; see
 * CCMG_OPT_FUSED); from a zero start they also take f's statistics (for the
 * checks above and ||f||) in the first cycle's first launch and check them
 * after that cycle.  On an error status (CCMG_EINCOMPAT, CCMG_ENONFINITE,
 * ...) d_phi's contents are unspecified. */
int ccmg_solve(ccmg_plan *plan, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess,
               ccmg_result *out);

/* Full multigrid (FMG) into d_phi: a start for the V-cycles that the paper
 * does not describe (Sec. 3.3 cycles from zero and leaves the coarse solve
 * open); it is the nested iteration of the multigrid literature (Brandt
 * 1977; Briggs, Henson and McCormick, A Multigrid Tutorial, ch. 3) built from
 * the operators of Sec. 3.3.  f is restricted (four-cell means) down to the
 * top level of the plan's coarse tail (32 x 32 cells, or the finest level if
 * smaller); there phi starts at zero and gets ncyc_top V-cycles; on each
 * finer level phi = P (coarser phi), the Sec. 3.3 prolongation added to a
 * zero field, then ncyc V-cycles of that level (on the finest level too).
 * FP64 plans only; 1 <= ncyc_top <= 16, 0 <= ncyc <= 16; d_f and d_phi as
 * for ccmg_solve (d_phi's contents on entry are not read; its ghosts are
 * filled on return).  Uses the plan's workspace; enqueues device work on the
 * plan's stream and returns without waiting.  For singular problems the
 * result is defined up to an additive constant. */
int ccmg_fmg(ccmg_plan *plan, const double *d_f, double *d_phi, ptrdiff_t pitch, int ncyc_top, int ncyc);

/* Plan options (all optional; read at every solve).
 *   CCMG_OPT_FUSED       0 or 1 (default 1): the fused finest launch of FP64
 *                        V(2,2) solves (0: one launch per half cycle, the
 *                        same iterates).
 *   CCMG_OPT_FUSED_KEEP  >= 0 (default 1): a fused launch also writes the
 *                        iterate after its post-smoothing (the solve's result
 *                        if that cycle meets the tolerance) while the residual
 *                        extrapolated from the last two cycles is within this
 *                        factor of the tolerance (at least 100 until three
 *                        cycles' residuals are known); 0 never (the solve then
 *                        returns the next cycle's pre-smoothed iterate, checked
 *                        by its own residual).
 *   CCMG_OPT_MIXED_INNER 1..8 (default 3): most FP32 V-cycles per refinement
 *                        step of MIXED plans with V(2,2).
 *   CCMG_OPT_FMG         0..4 (default 0, off): FP64 solves without a guess
 *                        start from a full multigrid pass (ccmg_fmg with this
 *                        many V-cycles on every level but the finest) instead
 *                        of zero; the V-cycles on the finest level are then
 *                        the solve's own, counted in `cycles` as usual.  With
 *                        the fused finest launch the finest level's
 *                        prolongation runs inside the first pre-smoothing and
 *                        the start's residual is not formed: rel_resid0 and
 *                        history[0] are NaN.
 *   CCMG_OPT_VISIT       0, 1 or 2 (default 1): in V(2,2) cycles a level below
 *                        the finest and above the one-workgroup tail, whose
 *                        correction starts from zero, may run as a visit:
 *                        its restricting launch on the way down (two
 *                        red-black iterations from zero, residual,
 *                        restriction; Sec. 3.3) stores no iterate, and one
 *                        launch on the way up recomputes those two
 *                        iterations, adds the prolongated correction and
 *                        runs the two post-smoothing iterations.  Each cell
 *                        of the level is written and read once less; the
 *                        iterates are bitwise those of the two-launch form.
 *                        The same holds for the finest level of FP64 solves
 *                        from zero with the fused launch (at least 2 cycles
 *                        allowed): the first pre-smoothing stores no iterate
 *                        and the first fused launch recomputes it from f.
 *                        0: never; 1: where ccmg_plan_autotune found it
 *                        faster (nowhere on an untuned plan); 2: wherever it
 *                        applies.
 * ccmg_plan_set_option returns CCMG_EINVAL for an unknown option or a value
 * outside its range; ccmg_plan_get_option writes the current value. */
enum { CCMG_OPT_FUSED = 1, CCMG_OPT_FUSED_KEEP = 2, CCMG_OPT_MIXED_INNER = 3, CCMG_OPT_FMG = 4, CCMG_OPT_VISIT = 5 };
int ccmg_plan_set_option(ccmg_plan *plan, int option, double value);
int ccmg_plan_get_option(ccmg_plan *plan, int option, double *value);

/* Bottom of the V-cycle (Sec. 3.3 leaves the coarsest solve open).
 * n_bottom = 2 (the default): nu_bottom red-black relaxations on the 2 x 2
 * grid.  n_bottom = 4 or 8: the cycle ends on the level of n_bottom x
 * n_bottom cells with an exact solve, phi = A^-1 f (A: the level's operator
 * alpha - beta Lap_h with the plan's side rules; for a singular plan
 * A + c 1 1^T, c = beta / h^2, whose solution of a zero-mean f is the
 * zero-mean solution), and the levels below it are not visited; nu_bottom is
 * then unused.  A^-1 is computed here on the device (Gauss-Jordan in FP64,
 * n_bottom^4 doubles in the plan's workspace) and applied in FP64 from LDS by
 * the one-workgroup tail, also in the FP32 cycles of mixed plans.  Applies to
 * every later ccmg_solve, ccmg_vcycle, ccmg_solve_bc, ccmg_cn_step and
 * ccmg_project of the plan.  Returns CCMG_EINVAL for another size, a size
 * above min(n, 32), or an indefinite operator (alpha beta < 0 or beta == 0);
 * blocks until the inverse is written. */
int ccmg_plan_set_bottom(ccmg_plan *plan, int n_bottom);

/* ---- Inhomogeneous side data (Sec. 3.3: the V-cycle's levels use the
 * homogeneous rules; with data the boundary value enters the ghost cell's
 * expression).  d_b is a host array of four device arrays, one per side in
 * the order CCMG_XLO, CCMG_XHI, CCMG_YLO, CCMG_YHI, each of n values along the
 * side (index j on the x sides, i on the y sides), or NULL for a homogeneous
 * side (d_b itself may be NULL: all homogeneous).  A periodic side takes
 * NULL (else CCMG_EINVAL).  Dirichlet: the value v at the face, ghost =
 * 2 v - phi.  Neumann: the derivative d along +x (x sides) or +y (y sides) at
 * the face, ghost = phi - h d on a lo side and phi + h d on a hi side.  The
 * arrays are only read. */
/* d_f_out = d_f plus (beta / h^2) times the data part of each ghost next to
 * a cell: the right-hand side of the equivalent homogeneous problem.  Out of
 * place, same pitch, asynchronous. */
int ccmg_bc_rhs(ccmg_plan *plan, const double *d_f, double *d_f_out, ptrdiff_t pitch, const double *const d_b[4]);
/* Ghost cells of d_phi (finest level) from its valid cells with the data. */
int ccmg_fill_ghosts_bc(ccmg_plan *plan, double *d_phi, ptrdiff_t pitch, const double *const d_b[4]);
/* ccmg_solve of the problem with side data: d_work <- ccmg_bc_rhs(d_f), the
 * solve on d_work (its stop test uses ||r|| / ||d_work||, which stays
 * meaningful when f = 0 and only the data drive the solution), then the
 * returned field's ghosts filled with the data.  d_work: caller-owned
 * scratch of the same layout, distinct from d_f and d_phi.  Singular
 * problems need compatible data (the shifted right-hand side sums to 0). */
int ccmg_solve_bc(ccmg_plan *plan, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess,
                  const double *const d_b[4], double *d_work, ccmg_result *out);

/* ---- Cell-centred approximate projection (Sec. 3.5, incompressible flow).
 * In place on a cell-centred velocity (d_u, d_v) of the doubly periodic
 * square: d_work <- D U (centred differences across two cells), then
 * ccmg_solve(plan, d_work, d_phi) for Lap phi = D U (zero-mean phi, ghosts
 * filled), then U -= G phi (the same centred differences).  D G differs from
 * the 5-point Lap, so D U is small afterwards, not zero.  The plan must be the
 * periodic Poisson problem (alpha 0, beta -1, all sides periodic), else
 * CCMG_EINVAL, as are NULL or coinciding arrays.  Ghost cells of d_u, d_v are
 * not read or written; all four arrays share one pitch.  Blocks like
 * ccmg_solve. */
int ccmg_project(ccmg_plan *plan, double *d_u, double *d_v, ptrdiff_t pitch, double *d_phi, double *d_work,
                 ccmg_result *out);

/* ---- Crank-Nicolson implicit diffusion (Sec. 3.4).
 * A step of phi_t = k Lap phi averages k Lap phi over the old and new time
 * levels; with beta = k dt / 2 the new level solves the Helmholtz problem
 * (1 - beta Lap) phi' = phi + beta Lap phi.  Both calls use a plan made for
 * alpha = 1, beta = k dt / 2 (the plan's sides, spacing and precision). */
/* d_f = d_phi + beta Lap d_phi on the finest level's valid cells, with the
 * plan's side rules applied where a neighbour is read (d_phi's ghost cells
 * are not read; d_f's are not written).  Out of place, same pitch.
 * Asynchronous on the plan's stream.  CCMG_EINVAL for NULL or equal pointers
 * or a bad pitch. */
int ccmg_cn_rhs(ccmg_plan *plan, const double *d_phi, double *d_f, ptrdiff_t pitch);
/* One step in place: d_work <- the right-hand side of d_phi, then
 * ccmg_solve(plan, d_work, d_phi, pitch, use_guess = 1, out) -- the old level
 * is the initial guess.  d_work: caller-owned scratch of the same layout.
 * CCMG_EINVAL also when the plan's alpha is not 1.  Blocks like ccmg_solve. */
int ccmg_cn_step(ccmg_plan *plan, double *d_phi, double *d_work, ptrdiff_t pitch, ccmg_result *out);

/* Exactly one V-cycle (Sec. 3.3: nu1 relaxations, restriction of the
 * residual, the coarse correction from zero, prolongation, nu2 relaxations)
 * of FP64 plans, or one refinement step of MIXED plans, on the finest level,
 * in place on d_phi, without a stop test.  Asynchronous. */
int ccmg_vcycle(ccmg_plan *plan, const double *d_f, double *d_phi, ptrdiff_t pitch);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): ccmg_vcycle of the FP64
 * problem *p without a plan or workspace.  Exactly one V-cycle in place on
 * d_phi (same kernels, launch shapes and iterates as ccmg_vcycle on an
 * untuned plan of *p), enqueued on `stream` (a hipStream_t, NULL = default)
 * and asynchronous.  The levels below the finest live in a static device
 * array of ccmg_noalloc_scratch_bytes() bytes (32 MiB), one per device, which
 * every call on that device shares and which keeps the last call's contents;
 * a V-cycle writes every part of it before reading it.  Nothing is allocated,
 * on the device or the host.  Returns CCMG_EWORKSPACE when the problem's
 * coarse levels need more than the scratch (FP64 grids of more than
 * 1024 x 1024 cells), CCMG_EINVAL for a MIXED problem, NULL arrays, a bad
 * pitch or a device index of 16 or more, and ccmg_problem_check's status for
 * an invalid problem.  Calls that overlap on one device race on the scratch:
 * order them on one stream (calls on distinct devices are independent). */
int ccmg_vcycle_noalloc(const ccmg_problem *p, const double *d_f, double *d_phi, ptrdiff_t pitch, void *stream);
size_t ccmg_noalloc_scratch_bytes(void);

/* ---- single steps at one level, for checking each kernel (asynchronous).
 * `level` l has n >> l cells per side and spacing h * 2^l; every level uses
 * the homogeneous version of the plan's side types and the plan's
 * alpha, beta.  Out-of-place: input and output arrays must not overlap. */

/* Fill the ghost cells of d_a (level l) from its valid cells with the
 * homogeneous side rules (Sec. 3.3 ghost equations; periodic sides wrap). */
int ccmg_fill_ghosts(ccmg_plan *plan, int level, double *d_a, ptrdiff_t pitch);
/* phi_out = `iters` (1 or 2) red-black Gauss-Seidel iterations applied to
 * phi_in (Sec. 3.3 smoother; the relaxation of Eq. helmholtz solved for the
 * centre cell, red cells (i + j even) first, ghosts refreshed per colour). */
int ccmg_smooth(ccmg_plan *plan, int level, int iters, const double *d_f, const double *d_phi_in,
                double *d_phi_out, ptrdiff_t pitch);
/* r = f - (alpha phi - beta Lap phi) on valid cells of level l (the residual
 * of Eq. helmholtz with the 5-point Laplacian, Sec. 2 / Sec. 3.3). */
int ccmg_residual(ccmg_plan *plan, int level, const double *d_f, const double *d_phi, double *d_r,
                  ptrdiff_t pitch);
/* d_fc (level l+1) = four-cell average of r = f - A phi (level l): the
 * residual restricted as a V-cycle does it (Sec. 3.3). */
int ccmg_restrict_residual(ccmg_plan *plan, int level, const double *d_f, const double *d_phi,
                           ptrdiff_t pitch, double *d_fc, ptrdiff_t pitch_c);
/* d_coarse (level l+1) = the average of the four cells of d_fine (level l)
 * that cover each coarse cell (Sec. 3.3, restriction), valid cells only; the
 * two arrays must not overlap. */
int ccmg_restrict(ccmg_plan *plan, int level, const double *d_fine, ptrdiff_t pitch, double *d_coarse,
                  ptrdiff_t pitch_c);
/* phi_out = phi_in + P e  with e on level l+1 (its ghosts are not read):
 * the prolongation of Sec. 3.3, centred slopes per coarse cell with the
 * homogeneous side rules, bilinear without the xy term. */
int ccmg_prolong_add(ccmg_plan *plan, int level, const double *d_ec, ptrdiff_t pitch_c,
                     const double *d_phi_in, double *d_phi_out, ptrdiff_t pitch);

/* ---- batched solves.
 * m independent problems of any sizes and side types advanced together (the
 * same refinement as CCMG_MIXED: FP32 V(2,2) cycles for the correction, FP64
 * update and FP64 stop test, whatever each problem's `prec` says).  Each batch
 * step is one fixed sequence of launches (per level size class, one
 * persistent launch over the tiles of every problem that has a level of that
 * size; one launch for all problems' levels of <= 32 cells; one launch for
 * all problems' stop tests) captured in a hipGraph and replayed; converged
 * problems are skipped.  Every problem needs nu1 == nu2 == 2.
 * Pointer arrays (d_f, d_phi, pitch) are host arrays of m entries; f[i] and
 * phi[i] are device arrays of problem i as for ccmg_solve.  The batch works
 * on an internal stream ordered after, and before, the caller's `stream`. */
typedef struct ccmg_batch ccmg_batch;
typedef struct {
    int steps;             /* batch steps replayed                              */
    int converged;         /* problems that reached their rtol                  */
    float ms;              /* device time of the solve (HIP events)             */
} ccmg_batch_info;

size_t ccmg_batch_workspace_bytes(int m, const ccmg_problem *probs);
int ccmg_batch_create(int m, const ccmg_problem *probs, void *d_ws, size_t ws_bytes, void *stream,
                      ccmg_batch **out);
int ccmg_batch_destroy(ccmg_batch *batch);
/* Solve all problems (each as ccmg_solve would, Sec. 3.3 V-cycles with the
 * refinement of CCMG_MIXED); out (m entries, may be NULL) receives each problem's
 * result, info (may be NULL) the batch summary.  Returns CCMG_OK if every
 * problem converged, else the first error status, else CCMG_NOT_CONVERGED. */
int ccmg_batch_solve(ccmg_batch *batch, const double *const *d_f, double *const *d_phi, const ptrdiff_t *pitch,
                     int use_guess, ccmg_result *out, ccmg_batch_info *info);
/* Batch options.  CCMG_BATCH_OPT_EAGER 0 or 1 (default 0): issue each batch
 * step's launches directly instead of replaying the captured graphs (the same
 * launches; for checking the replays).  CCMG_EINVAL for anything else. */
enum { CCMG_BATCH_OPT_EAGER = 1 };
int ccmg_batch_set_option(ccmg_batch *batch, int option, double value);
/* Time the candidate rows-per-band of each level size class and the number of
 * persistent wavefronts over whole batch steps on the given arrays and keep the
 * fastest.  d_phi is used as scratch (overwritten). */
int ccmg_batch_autotune(ccmg_batch *batch, const double *const *d_f, double *const *d_phi,
                        const ptrdiff_t *pitch);
/* Level size classes (descending), their rows per band, and the wavefront count. */
int ccmg_batch_shapes(ccmg_batch *batch, int *sizes, int *ty, int max, int *count, int *waves);

/* ---- learned initial guess.
 * A linear network of six 3x3 convolutions with circular padding and
 * dilations 1, 2, 4, 8, 16, 32 on a 128 x 128 grid (channels 1 -> 32 -> ... ->
 * 32 -> 1, no biases; the 32 -> 32 layers on the matrix cores with weights
 * and activations as BF16 hi + lo pairs and FP32 accumulation, the first and
 * last layers with FP32 weights)
 * maps a right-hand side, averaged onto that grid and divided by its RMS, to
 * the solution averaged the same way.  The guess for an n x n problem
 * (n >= 256, power of two) is that output times the RMS, prolonged back to
 * n x n by multigrid prolongations; the solver then continues from it
 * (ccmg_solve with use_guess = 1) to the same tolerance.  Parameters: FP32,
 * ccmg_net_param_count() of them, in layer order ([32][9], four x
 * [32][9][32] (out, tap, in), [9][32]); tap = 3 (dy + 1) + (dx + 1) reads the
 * input at (y + dy d, x + dx d).  Network inputs / targets: nb x 128 x 128
 * FP32 device arrays.  All work on the net's stream. */
typedef struct ccmg_net ccmg_net;
int ccmg_net_param_count(void);
/* Workspace for training batches of up to `batch` samples and guesses for
 * problems of up to n_max cells per side (0 if invalid). */
size_t ccmg_net_workspace_bytes(int batch, int n_max);
int ccmg_net_create(int batch, int n_max, void *d_ws, size_t ws_bytes, void *stream, ccmg_net **out);
int ccmg_net_destroy(ccmg_net *net);
/* Load parameters (device FP32); resets the optimiser state. */
int ccmg_net_set_params(ccmg_net *net, const float *d_params);
int ccmg_net_get_params(ccmg_net *net, float *d_params);
/* Training state, for checkpoints: ccmg_net_state_count() FP32 values -- the
 * parameters, then Adam's first and second moments, each in parameter order
 * (3 x ccmg_net_param_count()) -- and Adam's step counter (its bias
 * corrections depend on it).  get copies the state to the device array
 * d_state (asynchronous on the net's stream) and *step (host); set restores
 * both, so that the next ccmg_net_train_step continues exactly where the
 * saved net stopped. */
int ccmg_net_state_count(void);
int ccmg_net_get_state(ccmg_net *net, float *d_state, int *step);
int ccmg_net_set_state(ccmg_net *net, const float *d_state, int step);
/* y = net(x) for nb samples (the network is not in the paper: it only
 * supplies the starting iterate of a Sec. 3.3 solve). */
int ccmg_net_forward(ccmg_net *net, const float *d_x, float *d_y, int nb);
/* Mean squared error of net(x) against t and its gradient with respect to
 * every parameter (device FP32, may be NULL); *loss (host, may be NULL). */
int ccmg_net_loss_grad(ccmg_net *net, const float *d_x, const float *d_t, int nb, float *d_grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss with rate lr. */
int ccmg_net_train_step(ccmg_net *net, const float *d_x, const float *d_t, int nb, float lr, float *loss);
/* Encoder: block means of `a` (n x n, ghosted FP64) on the 128 x 128 grid
 * divided by the RMS of `scale_src` (the sample's right-hand side). */
int ccmg_net_encode(ccmg_net *net, const double *d_a, ptrdiff_t pitch, int n, const double *d_scale_src,
                    ptrdiff_t scale_pitch, float *d_x);
/* The guess for f (n x n, ghosted FP64, 256 <= n <= n_max) on a square of
 * side `length`: encode, network, `coarse_iters` (0..64) red-black
 * Gauss-Seidel iterations of the periodic Poisson problem on the network's
 * grid (they remove the grid-scale noise of the network output), then
 * multigrid prolongations to n x n.  Writes the valid cells of d_phi. */
int ccmg_net_guess(ccmg_net *net, const double *d_f, ptrdiff_t pitch, int n, double length, int coarse_iters,
                   double *d_phi, ptrdiff_t phi_pitch);
/* Learned solve for the problem the network is trained on (alpha = 0,
 * beta = -1, square domain, all four sides periodic): ccmg_net_guess, then ccmg_solve from
 * that guess to the plan's tolerance.  A guess whose relative residual is not
 * finite or above 1e6 is discarded and the solve starts from zero instead
 * (*guess_used = 0, may be NULL).  out->ms covers guess and solve,
 * out->rel_resid0 is the guess's relative residual.  The plan and the net
 * must share one stream; the plan's n must lie in [256, n_max].  Returns
 * ccmg_solve's status (CCMG_EINVAL for a problem the network does not fit). */
int ccmg_solve_learned(ccmg_plan *plan, ccmg_net *net, const double *d_f, double *d_phi, ptrdiff_t pitch,
                       int coarse_iters, ccmg_result *out, int *guess_used);

/* ---- launch-shape autotuning.
 * Times every candidate tile shape (rows per wavefront band x wavefronts per
 * workgroup, or the 2-D tile kernel below the finest level) of the two
 * launches of each level, of the same level run as a visit (see
 * CCMG_OPT_VISIT; the visit is kept where its pair is faster), and of the
 * fused finest launch, on the given data and keeps the fastest for this plan.
 * d_f and d_phi are only read (finest level, same layout as ccmg_solve);
 * blocks until done.  Optional: untuned plans use a fixed size-based choice. */
int ccmg_plan_autotune(ccmg_plan *plan, const double *d_f, double *d_phi, ptrdiff_t pitch);
/* Set one launch shape by hand: kind 0 = the nu1 (restricting) launch of
 * `level`, 1 = the nu2 (prolongating) launch; ty even, >= 8 unless it covers
 * the level; 1 <= wpb <= 4.  ty = 0 selects the 2-D LDS tile kernel instead
 * of the row march (levels below the finest with at least 64 cells per side
 * that are not in the one-workgroup tail).  kind 2 = the fused finest launch
 * of FP64 solves, 3 = its FP32 form in mixed-precision steps (level 0 only,
 * ty even and >= 8, no tile kernel).  Levels below the finest that are not
 * in the tail, run as a visit (CCMG_OPT_VISIT): kind 4 = the restricting
 * launch without the stored iterate (as kind 0), kind 5 = the visit launch
 * (row march only, ty even and >= 16 unless it covers the level; ty = 0 sets
 * the level to run its two launches instead, and with CCMG_OPT_VISIT = 1
 * any other ty sets it to run as a visit).  kind 6 (level 0, FP64): the
 * first fused launch of a solve from zero that recomputes the first
 * pre-smoothing (ty as for kind 5; 0: the pre-smoothing is stored and the
 * ordinary fused launch reads it).  Results do not depend on the shape. */
int ccmg_plan_set_shape(ccmg_plan *plan, int level, int kind, int ty, int wpb);
/* One launch shape, kinds as for ccmg_plan_set_shape (kinds 5 and 6 give
 * ty = 0, wpb = 1 where the recomputing form is not chosen for
 * CCMG_OPT_VISIT = 1). */
int ccmg_plan_shape(ccmg_plan *plan, int level, int kind, int *ty, int *wpb);
/* The fused finest launch's shape: kind 2 (FP64) or 3 (FP32), as for
 * ccmg_plan_set_shape. */
int ccmg_plan_fused_shape(ccmg_plan *plan, int kind, int *ty, int *wpb);
/* The plan's launch shapes per level (arrays of max_levels entries). */
int ccmg_plan_shapes(ccmg_plan *plan, int *ty_pre, int *wpb_pre, int *ty_post, int *wpb_post,
                     int max_levels);

/* ---- kernel timing (diagnostics).
 * While profiling is on, the plan brackets each launch of the two
 * finest-level row-march kernels of a V-cycle with HIP events on its stream:
 *   "finest_pre":  nu1 relaxations + residual + four-cell restriction,
 *   "finest_post": prolongation + nu2 relaxations (+ residual norm);
 * MIXED plans: "mixed_finest_pre" (the same in FP32) and "mixed_finest_post_ir"
 * (FP32 prolongation + relaxations, then the FP64 update of the iterate and
 * its FP64 residual, rounded to FP32 for the next step); FP64 solves with
 * fused launches: "finest_fused" (prolongation + 2 relaxations + residual
 * norm [+ that iterate kept], then 2 relaxations + residual + restriction);
 * "finest_fused_first" (the first such launch of a solve from zero: the
 * first cycle's two pre-smoothing relaxations, not stored by its first
 * launch, recomputed from f, then what "finest_fused" does);
 * MIXED steps with several inner cycles: "mixed_finest_fused" (the same in
 * FP32 between two inner cycles, without norm or kept iterate); the
 * Crank-Nicolson right-hand side "cn_rhs"; the projection's "divergence" and
 * "subtract_gradient" passes.
 * `bytes` is the algorithmic traffic of one launch: each valid cell of each
 * array the launch reads or writes, counted once (ghost cells and halo
 * re-reads excluded).  Launches of a cycle queued after the one that met the
 * tolerance (they exit as soon as they start) are not counted. */
typedef struct {
    char name[32];
    int launches;          /* launches timed since profiling was (re)enabled */
    double ms;             /* their summed device time                       */
    double bytes;          /* their summed algorithmic bytes                 */
} ccmg_kernel_stat;

/* Enable (1) or disable (0) kernel timing; either way the counters restart. */
int ccmg_plan_profile(ccmg_plan *plan, int enable);
/* Copy up to `max` kernel records into out; *count receives how many exist.
 * Call after the timed work has completed (e.g. after ccmg_solve returned). */
int ccmg_plan_kernel_stats(ccmg_plan *plan, ccmg_kernel_stat *out, int max, int *count);

/* Streaming probe (diagnostics): d_c = d_a + d_b over `count` doubles, each
 * array read or written once -- the access pattern of a launch that reads two
 * arrays and writes one -- in several launch shapes (2, 4, 8, 32 and 128
 * workgroups of 256 threads per compute unit, 16-byte accesses, ordinary and
 * nontemporal), each timed with HIP events on `stream` over `reps` launches
 * after one untimed launch.  *ms receives the fastest mean time per launch,
 * *config (may be NULL) its shape: workgroups per compute unit, plus 1000 if
 * nontemporal.  It states what the device's memory system delivers for that
 * pattern, beside the nameplate bandwidth.  count even, arrays 16-byte aligned
 * and not overlapping, else CCMG_EINVAL.  Blocks until done. */
int ccmg_probe_stream(const double *d_a, const double *d_b, double *d_c, size_t count, int reps, void *stream,
                      float *ms, int *config);

#ifdef __cplusplus
}
#endif
#endif
