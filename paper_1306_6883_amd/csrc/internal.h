// internal.h -- shared declarations of the ccmg HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccmg.h"

namespace ccmg {

// Device scalars of a solve (workspace): statistics of f, mean of phi.
enum { S_FSUM = 0, S_FABS = 1, S_F2 = 2, S_FBAD = 3, S_PHIMEAN = 4, S_RHO0 = 5, kScal = 16 };

enum Post {
    POST_NONE = 0,
    POST_RESTRICT = 1,  // residual -> four-cell restriction into aux (+ partial sums)
    POST_NORM = 2,      // residual -> sum r^2, sum phi per tile
    POST_RESID = 3,     // residual -> aux
    POST_IR = 4,        // (float launches) relaxed e -> phi64_out = phi64_in + e, FP64 residual
                        // of phi64_out -> r32 (+ sum r^2, sum phi64, sum r32 per tile)
    POST_R32 = 5,       // (double launches) residual -> r32 (+ the same three sums)
    POST_FUSED = 6,     // (finest level, NU = 4) the post-smoothing of one cycle and the
                        // pre-smoothing of the next in one launch: after the first two iterations
                        // the residual norm (sum r^2, sum phi per tile -> partial_norm, if set) and the
                        // iterate (-> phi_mid, if set); after all four, RESTRICT as above
    POST_VISIT = 7,     // (levels below the finest, NU = 4, from zero, with prolongation) a
                        // level's whole visit in one launch: the two pre-smoothing iterations
                        // from zero (recomputed: the restricting launch of the way down then
                        // stores no iterate), the prolongation of the coarse correction, the
                        // two post-smoothing iterations; stores the result
    POST_FUSED0 = 8,    // (finest level, NU = 6, from zero) the first fused launch of a solve
                        // from zero: the first cycle's two pre-smoothing iterations recomputed
                        // from zero as in POST_VISIT, then everything POST_FUSED does
    POST_CNPRE = 9      // (finest level, FP64, NU = 2, from a loaded iterate) POST_RESTRICT
                        // whose right-hand side is the Crank-Nicolson one of the loaded
                        // iterate, f = phi + cn_beta Lap phi, formed here and written to cn_f
                        // (not loaded)
};

// Arguments of one row-march launch over one grid level (see march.hip).
template <typename T>
struct MarchArgs {
    const T *f;          // right-hand side, ghosted, pitch pf
    int pf;
    const T *phi_in;     // starting iterate (ignored when the launch assumes zero)
    int pin;
    T *phi_out;          // relaxed iterate (valid cells only)
    int pout;
    const T *ec;         // coarse correction e (level l+1) for the prolongation
    int pc;
    T *aux;              // POST_RESTRICT: coarse rhs (level l+1); POST_RESID: r
    int paux;
    double *partial;     // per-tile sums: RESTRICT -> sum of coarse rhs; NORM -> sum r^2, sum phi
    const double *fmean_part;  // partial sums whose total / (n*n) is subtracted from f (or null)
    int fmean_count;
    const int *fmean_count_ptr;  // if set, the number of partial sums is read from here
    const double *phi_shift;   // device scalar subtracted from loaded phi (or null)
    const int *skip;     // device flag: when set (solve converged) the launch does nothing
    int n;               // cells per side of this level
    int bc[4];
    T cc, invd;          // relaxation: phi = (f + cc * sum of neighbours) * invd
    T alpha, beta, ih2;  // residual: r = f - (alpha phi - beta ih2 * lap)
    int strips, chunks, ty, outw, ntiles, groups_per_xcd;
    // Edge strips (x sides Dirichlet or Neumann): the first and last strip run
    // bands of ety rows (echunks of them, after the (strips - 2) * chunks
    // interior tiles); echunks = 0: every strip runs bands of ty rows.
    int ety, echunks;
    // mixed precision (POST_IR / POST_R32)
    const double *q_in;  // FP64 iterate, read (POST_IR)
    int pq_in;
    double *q_out;       // FP64 iterate + e, written (POST_IR)
    int pq_out;
    const double *g;     // FP64 right-hand side (POST_IR)
    int pg;
    float *r_out;        // FP32 copy of the FP64 residual
    int pr;
    double *partial3;    // per tile: sum of the FP32 residual (mean removal of singular problems)
    double alpha64, beta64, ih2_64;
    int q_zero;          // POST_IR: the FP64 iterate is zero (q_in is not used)
    int *count_out;      // if set, receives ntiles (producers of per-tile sums)
    // POST_FUSED: the iterate after the post-smoothing and its per-tile norm sums
    T *phi_mid;
    int pmid;
    double *partial_norm;
    // POST_RESTRICT: if set, per tile (4 * tile + q) the statistics of f over
    // the tile's output cells: sum f, sum |f|, sum f^2 over finite values and
    // the count of non-finite ones (f as loaded, before any mean shift)
    double *fstat_part;
    // POST_RESTRICT with LOADPHI: if set, per tile (2 * tile + q) the sums
    // (r^2, phi) of the residual of the loaded iterate, before any relaxation
    // (the residual norm of a solve's starting guess); no mean shift may apply
    double *in_norm_part;
    // POST_CNPRE: the right-hand side formed from the loaded iterate goes here
    T *cn_f;
    int pcnf;
    T cn_beta;
};

// One unit of work of a batched launch: tile `tile` of level descriptor `desc`.
struct WorkItem {
    int desc;
    int tile;
};

// Columns of a row-march tile: a wavefront loads 128 (two per lane) and
// outputs the middle ones; each side gives up one column per stage (2 nu
// relaxations, the residual when there is a post stage) and one lane for the
// prolongation's slope, rounded up to whole lanes.
constexpr int march_halo_x(int nu, bool prolong, bool post) {
    return (2 * nu + (post ? 1 : 0) + (prolong ? 2 : 0) + 1) & ~1;
}
constexpr int march_outw(int nu, bool prolong, bool post) { return 128 - 2 * march_halo_x(nu, prolong, post); }

// A tile on a Dirichlet or Neumann x side applies the ghost rule in every
// stage (about a quarter more instructions per row), so with one wave per band
// it would finish last: bands of at least kEdgeSplitMinTy rows are halved in
// the two edge strips.
constexpr int kEdgeSplitMinTy = 64;
constexpr int edge_band_rows(int ty) { return ((ty / 2) + 1) & ~1; }

// Launch description chosen by the host for one level.
struct MarchShape {
    int ty;       // rows per tile (even); 0: the 2-D LDS tile kernel (tile.hip)
    int wpb;      // waves per workgroup
};

// The 2-D LDS tile kernel (levels below the finest, n >= kTileMinN): the same
// launches as the row march for POST_NONE / POST_RESTRICT without a phi shift.
constexpr int kTileMinN = 64;
template <typename T>
hipError_t launch_tile(const MarchArgs<T> &a, int nu, bool load_phi, bool prolong, int post, hipStream_t s,
                       int *ntiles_out);

// Host launchers (march.hip).  nu in {0,1,2}; load_phi=false means phi starts at 0.
// *ntiles_out receives the number of tiles (= partial-sum slots) of the launch.
template <typename T>
hipError_t launch_march(const MarchArgs<T> &a, int nu, bool load_phi, bool prolong, int post,
                        MarchShape shape, hipStream_t s, int *ntiles_out);
// The fused finest-level launch (POST_FUSED; march_f64_fused.hip).
hipError_t dispatch_fused(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt);
hipError_t dispatch_fused(const MarchArgs<float> &a, MarchShape sh, hipStream_t s, int *nt);
// The first fused launch of a solve from zero (POST_FUSED0; march_f64_fused.hip).
hipError_t dispatch_fused0(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt);
// The first pre-smoothing of a Crank-Nicolson step (POST_CNPRE; march_f64_cn.hip).
hipError_t dispatch_cnpre(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt);
// A coarse level's whole visit (POST_VISIT; march_visit.hip).
hipError_t dispatch_visit(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt);
hipError_t dispatch_visit(const MarchArgs<float> &a, MarchShape sh, hipStream_t s, int *nt);
// One march variant family with NU fused iterations; defined in march_impl.h and
// instantiated per (T, NU) in the march_*.hip files.
template <typename T, int NU>
hipError_t dispatch_nu(const MarchArgs<T> &a, bool load_phi, bool prolong, int post, MarchShape sh,
                       hipStream_t s, int *nt);

// Coarse tail: a whole V-cycle from level `n_top` (<= kCoarseMax) down to 2x2 and
// back, one workgroup, all levels resident in LDS (coarse.hip).
constexpr int kCoarseMax = 32;
template <typename T>
struct CoarseArgs {
    const T *f;          // rhs at the top level, ghosted
    long pf;
    const T *phi_in;     // starting iterate at the top level (if load_phi)
    long pin;
    T *phi_out;          // result at the top level (valid cells)
    long pout;
    const double *phi_shift;  // subtracted from loaded phi (or null)
    const int *skip;          // device flag: when set the launch does nothing
    int n_top;
    int bc[4];
    double alpha, beta, h_top;
    // per level l below the top (n_top >> l cells): relaxation phi = (f + cc*sum) * invd,
    // residual r = f - (alpha phi - beta ih2 lap); filled by launch_coarse
    double cc[8], invd[8], ih2[8];
    int nu1, nu2, nu_bottom;
    int load_phi;        // 1: top level starts from phi_in; 0: from zero
    int sub_top_mean;    // 1: remove the mean of the top-level rhs (singular, not finest)
    int singular;        // remove the mean of every restricted rhs below the top
    // exact bottom: n_bottom in {4, 8} (<= n_top) ends the cycle on that level
    // with phi = ainv f (ainv: the level's inverse operator, FP64, column-major
    // m x m, m = n_bottom^2); otherwise (0 or 2) the 2 x 2 relaxations.
    int n_bottom;
    const double *ainv;
};
// Largest exact-bottom level (cells per side): its inverse is held in LDS.
constexpr int kDirectMax = 8;
// Inverse of (alpha - beta Lap_h) on an nb x nb level with the side rules bc
// (plus c 1 1^T, c = beta / h^2, when singular), column-major into out
// (nb^4 doubles).  The operator must be definite (alpha beta >= 0, beta != 0).
hipError_t launch_bottom_inverse(int nb, const int bc[4], double alpha, double beta, double h, int singular,
                                 double *out, hipStream_t s);
template <typename T>
hipError_t launch_coarse(const CoarseArgs<T> &a, hipStream_t s);
// One workgroup per entry of a device array of tail descriptors (batches).
// The descriptors must hold the per-level constants (see coarse_fill_consts).
template <typename T>
hipError_t launch_coarse_list(const CoarseArgs<T> *list, int count, hipStream_t s);
template <typename T>
void coarse_fill_consts(CoarseArgs<T> &a);

// util.hip
hipError_t launch_fill_ghosts_f64(double *a, long pitch, int n, const int bc[4], const double *shift,
                                  hipStream_t s);
// End of a cycle: sum the (sum r^2, sum phi) tile pairs in a fixed order, then
//   *rho_out = sqrt(sum r^2) / sqrt(*f2),  *phi_mean = sum phi / n^2 (singular) or 0,
//   *done = 1 if rho <= rtol or rho is not finite.
// Does nothing if *done is already set.  One workgroup.
// host_rho (optional): host-mapped address that also receives rho.
// Side data (bcdata.hip): per side its type and a device array of n values
// (nullptr: homogeneous).
struct BcData {
    const double *b[4];
    int type[4];
};
hipError_t launch_bc_rhs(const double *f, double *f_out, long pitch, int n, const BcData &d, double beta, double h,
                         hipStream_t s);
hipError_t launch_add_ghost_data(double *a, long pitch, int n, const BcData &d, double h, hipStream_t s);

// Approximate projection (proj.hip), doubly periodic: f = D U; U -= G phi.
hipError_t launch_divergence(const double *u, const double *v, double *f, long pitch, int n, double h,
                             hipStream_t s);
hipError_t launch_subtract_gradient(const double *phi, double *u, double *v, long pitch, int n, double h,
                                    hipStream_t s);

// Crank-Nicolson right-hand side f = phi + beta Lap phi on valid cells (cn.hip).
hipError_t launch_cn_rhs(const double *phi, long pp, double *f, long pf, int n, const int bc[4], double beta,
                         double h, hipStream_t s);
hipError_t launch_cycle_end(const double *partial, int count, int n, int singular, const double *f2,
                            double rtol, double *rho_out, double *phi_mean, int *done, double *host_rho,
                            hipStream_t s);
// Statistics of f (sum, sum |f|, sum f^2, non-finite count) -> out4; `blocks` partials.
hipError_t launch_fstats(const double *f, long pitch, int n, double *partial, int blocks, double *out4,
                         hipStream_t s);
// The same, and coarse (n/2 cells, pitch pc) = the four-cell restriction of f.
hipError_t launch_fstats_restrict(const double *f, long pitch, int n, double *partial, int blocks, double *out4,
                                  double *coarse, long pc, hipStream_t s);
hipError_t launch_set(double *p, int count, double v, hipStream_t s);
// out4[q] = sum over i < count of partial[4 i + q], in a fixed order (one workgroup).
hipError_t launch_reduce4(const double *partial, int count, double *out4, hipStream_t s);
hipError_t launch_set_int(int *p, int count, int v, hipStream_t s);
// coarse = four-cell average of fine (valid cells; nc cells per side of the coarse level).
hipError_t launch_restrict(const double *fine, long pf, double *coarse, long pc, int nc, hipStream_t s);
// c = a + b over `count` doubles (even count, 16-byte aligned): a streaming probe.
hipError_t launch_probe_stream(const double *a, const double *b, double *c, long count, int blocks, hipStream_t s);

// The library's static device scratch (noalloc.hip): its address on device
// `dev` (looked up once per device, with that device current) and its size.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
hipError_t static_scratch(int dev, void **ptr, size_t *bytes);

// The stream and finest size of a plan (for entry points outside plan.cpp).
hipStream_t plan_stream(const ccmg_plan *P);
int plan_n(const ccmg_plan *P);
const ccmg_problem *plan_problem(const ccmg_plan *P);
// ccmg_solve with a bound on the guess's relative residual (see plan.cpp).
constexpr int kGuessRejected = 100;
int solve_impl(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess, ccmg_result *out,
               double guess_reject, double *cn_f = nullptr);

}  // namespace ccmg
