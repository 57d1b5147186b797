// cn.hip -- right-hand side of a Crank-Nicolson diffusion step (Sec. 3.4).
//
// The step averages k Lap phi over the old and new time levels; with
// beta = k dt / 2 the new level solves (1 - beta Lap) phi' = f with
// f = phi + beta Lap phi.  This kernel forms f in one pass: each thread owns
// one column and walks a band of rows, keeping the rows above and below in
// registers; east / west neighbours are loaded directly (they are the
// neighbouring lanes' values, so they come from cache).  Side rules are
// applied where a neighbour is read: a Dirichlet ghost is minus the cell, a
// Neumann ghost the cell itself, a periodic side wraps.  Lap is written as
// differences from the centre, the same order as the residual.
#include "internal.h"

namespace ccmg {

namespace {

constexpr int kCnThreads = 256;
constexpr int kCnRows = 32;  // rows per band

__global__ __launch_bounds__(kCnThreads) void k_cn_rhs(const double *__restrict__ phi, long pp,
                                                       double *__restrict__ f, long pf, int n, int bxl,
                                                       int bxh, int byl, int byh, double beta, double ih2) {
    const int x = blockIdx.x * kCnThreads + threadIdx.x;
    const int y0 = blockIdx.y * kCnRows;
    if (x >= n) return;
    const int nm = n - 1;
    const bool px = bxl == CCMG_BC_PERIODIC, py = byl == CCMG_BC_PERIODIC;
    const double sxl = bxl == CCMG_BC_DIRICHLET ? -1.0 : 1.0, sxh = bxh == CCMG_BC_DIRICHLET ? -1.0 : 1.0;
    const double syl = byl == CCMG_BC_DIRICHLET ? -1.0 : 1.0, syh = byh == CCMG_BC_DIRICHLET ? -1.0 : 1.0;
    // columns of the west / east neighbours (the cell's own column at a
    // non-periodic side: the ghost rule then scales it)
    const int xw = x > 0 ? x - 1 : (px ? nm : 0), xe = x < nm ? x + 1 : (px ? 0 : nm);
    const double gw = (x == 0 && !px) ? sxl : 1.0, ge = (x == nm && !px) ? sxh : 1.0;
    auto row = [&](int y) { return phi + (long)(y + 1) * pp + 1; };
    const int y1 = min(y0 + kCnRows, n);
    // the row below the band
    double cur = row(y0)[x];
    double below;
    if (y0 > 0) below = row(y0 - 1)[x];
    else below = py ? row(nm)[x] : syl * cur;
    for (int y = y0; y < y1; ++y) {
        double above;
        if (y < nm) above = row(y + 1)[x];
        else above = py ? row(0)[x] : syh * cur;
        const double *r = row(y);
        const double w = gw * r[xw], e = ge * r[xe];
        const double lap = (((e - cur) + (w - cur)) + (above - cur) + (below - cur)) * ih2;
        f[(long)(y + 1) * pf + 1 + x] = cur + beta * lap;
        below = cur;
        cur = above;
    }
}

}  // namespace

hipError_t launch_cn_rhs(const double *phi, long pp, double *f, long pf, int n, const int bc[4], double beta,
                         double h, hipStream_t s) {
    if (n < 2 || !phi || !f) return hipErrorInvalidValue;
    const dim3 grid((n + kCnThreads - 1) / kCnThreads, (n + kCnRows - 1) / kCnRows);
    hipLaunchKernelGGL(k_cn_rhs, grid, dim3(kCnThreads), 0, s, phi, pp, f, pf, n, bc[CCMG_XLO], bc[CCMG_XHI],
                       bc[CCMG_YLO], bc[CCMG_YHI], beta, 1.0 / (h * h));
    return hipGetLastError();
}

}  // namespace ccmg
