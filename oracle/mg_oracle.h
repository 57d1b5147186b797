/*
 * mg_oracle.h -- interface of the FP64 CPU multigrid oracle (test
 * infrastructure only; see mg_oracle.c).  Independent of the GPU library's
 * header: none of these names or values are shared with it.
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OG_DIRICHLET = 0, OG_NEUMANN = 1, OG_PERIODIC = 2 };
enum { OG_XLO = 0, OG_XHI = 1, OG_YLO = 2, OG_YHI = 3 };
enum { OG_OK = 0, OG_NOT_CONVERGED = 1, OG_EINVAL = -1 };
#define OG_HISTORY 256

typedef struct {
    int n;          /* cells per side, a power of two >= 2          */
    double h;       /* cell width (square cells)                    */
    double alpha;   /* (alpha - beta Lap) phi = f                   */
    double beta;
    int bc[4];      /* x-lo, x-hi, y-lo, y-hi side types            */
    int nu1, nu2;   /* pre / post relaxations per level             */
    int nu_bottom;  /* relaxations on the 2x2 grid                  */
    int max_cycles;
    double rtol;    /* stop when ||r|| / ||f|| <= rtol              */
    int n_bottom;   /* 4, 8, ...: exact solve on the level of that  */
                    /* size, nothing below it; else the 2x2 grid's  */
                    /* nu_bottom relaxations                        */
} og_params;

typedef struct {
    int status;
    int cycles;
    double rel_resid0;
    double rel_resid;
    double history[OG_HISTORY];
} og_result;

size_t og_field_len(int n);
void og_fill(int n, const int bc[4], double *a);
void og_smooth(int n, double h, double alpha, double beta, const int bc[4], double *phi,
               const double *f, int iters);
void og_residual(int n, double h, double alpha, double beta, const int bc[4], double *phi,
                 const double *f, double *r);
void og_restrict(int n, const double *fine, double *coarse);
void og_prolong_add(int nc, const int bc[4], double *coarse, double *fine);
double og_norm(int n, double h, const double *a);
double og_mean(int n, const double *a);
int og_vcycle(const og_params *p, double *phi, const double *f);
int og_solve(const og_params *p, double *phi, const double *f, int use_guess, og_result *out);
int og_fmg(const og_params *p, double *phi, const double *f, int top_n, int ncyc_top, int ncyc);
int og_smooth_solve(const og_params *p, double *phi, const double *f, int max_iters,
                    og_result *out);
void og_cn_rhs(int n, double h, double beta, const int bc[4], double *phi, double *f);
int og_cn_step(const og_params *p, double *phi, double *work, og_result *out);
void og_fill_bc(int n, double h, const int bc[4], const double *const b[4], double *a);
void og_bc_rhs(int n, double h, double beta, const int bc[4], const double *const b[4], const double *f,
               double *f_out);
int og_solve_bc(const og_params *p, double *phi, const double *f, const double *const b[4], int use_guess,
                og_result *out);
void og_divergence(int n, double h, const double *u, const double *v, double *f);
void og_subtract_gradient(int n, double h, double *phi, double *u, double *v);
int og_project(const og_params *p, double *u, double *v, double *phi, og_result *out);

#ifdef __cplusplus
}
#endif
#endif
