// bcdata.hip -- inhomogeneous side data (Sec. 3.3).
//
// The V-cycle's levels use the homogeneous side rules.  With data on a side
// (a Dirichlet value v at the face, or a Neumann derivative d across it) the
// second-order ghost becomes the homogeneous one plus a data part:
// Dirichlet 2v, Neumann -h d on a lo side and +h d on a hi side.  That part
// multiplies beta / h^2 in the operator, so it moves to the right-hand side:
// the problem with data is the homogeneous problem with
//     f' = f + (beta / h^2) * (data part of each out-of-domain neighbour),
// which the existing solve handles; the returned field's ghosts then get the
// data part added to the homogeneous ghosts.
#include "internal.h"

namespace ccmg {

namespace {

constexpr int kBcThreads = 256;
constexpr int kBcRows = 32;

// data part of the ghost beyond side s at position k (0 without data)
__device__ __forceinline__ double data_part(const BcData &d, int s, int k, double h) {
    const double *v = d.b[s];
    if (!v) return 0.0;
    if (d.type[s] == CCMG_BC_DIRICHLET) return 2.0 * v[k];
    if (d.type[s] == CCMG_BC_NEUMANN) return (s == CCMG_XLO || s == CCMG_YLO) ? -(h * v[k]) : h * v[k];
    return 0.0;  // periodic sides carry no data
}

// f_out = f plus the data terms on the cells next to a side: one thread per
// column walking a band of rows (x sides before y sides, lo before hi)
__global__ __launch_bounds__(kBcThreads) void k_bc_rhs(const double *__restrict__ f, double *__restrict__ fo,
                                                       long pitch, int n, BcData d, double c, double h) {
    const int x = blockIdx.x * kBcThreads + threadIdx.x;
    if (x >= n) return;
    const int y0 = blockIdx.y * kBcRows, y1 = min(y0 + kBcRows, n);
    for (int y = y0; y < y1; ++y) {
        const long o = (long)(y + 1) * pitch + 1 + x;
        double v = f[o];
        if (x == 0) v += c * data_part(d, CCMG_XLO, y, h);
        if (x == n - 1) v += c * data_part(d, CCMG_XHI, y, h);
        if (y == 0) v += c * data_part(d, CCMG_YLO, x, h);
        if (y == n - 1) v += c * data_part(d, CCMG_YHI, x, h);
        fo[o] = v;
    }
}

// add the data parts to ghosts that already hold the homogeneous values
__global__ __launch_bounds__(kBcThreads) void k_add_ghost_data(double *__restrict__ a, long pitch, int n, BcData d,
                                                               double h) {
    const int k = blockIdx.x * kBcThreads + threadIdx.x;
    if (k >= n) return;
    a[(long)(k + 1) * pitch + 0] += data_part(d, CCMG_XLO, k, h);
    a[(long)(k + 1) * pitch + n + 1] += data_part(d, CCMG_XHI, k, h);
    a[1 + k] += data_part(d, CCMG_YLO, k, h);
    a[(long)(n + 1) * pitch + 1 + k] += data_part(d, CCMG_YHI, k, h);
}

}  // namespace

hipError_t launch_bc_rhs(const double *f, double *f_out, long pitch, int n, const BcData &d, double beta, double h,
                         hipStream_t s) {
    const dim3 grid((n + kBcThreads - 1) / kBcThreads, (n + kBcRows - 1) / kBcRows);
    hipLaunchKernelGGL(k_bc_rhs, grid, dim3(kBcThreads), 0, s, f, f_out, pitch, n, d, beta / (h * h), h);
    return hipGetLastError();
}

hipError_t launch_add_ghost_data(double *a, long pitch, int n, const BcData &d, double h, hipStream_t s) {
    hipLaunchKernelGGL(k_add_ghost_data, dim3((n + kBcThreads - 1) / kBcThreads), dim3(kBcThreads), 0, s, a,
                       pitch, n, d, h);
    return hipGetLastError();
}

}  // namespace ccmg
