// proj.hip -- the cell-centred approximate projection (Sec. 3.5).
//
// A cell-centred velocity U* = (u, v) on the doubly periodic square is split
// as U^d + grad phi: Lap phi = D U*, then U = U* - G phi.  D and G are
// centred differences across two cells, Lap the solver's 5-point operator
// (D G != Lap: the projection is approximate).  Both passes here are one
// thread per column walking a band of rows; neighbours wrap.
#include "internal.h"

namespace ccmg {

namespace {

constexpr int kPjThreads = 256;
constexpr int kPjRows = 32;

__global__ __launch_bounds__(kPjThreads) void k_divergence(const double *__restrict__ u, const double *__restrict__ v,
                                                           double *__restrict__ f, long pitch, int n, double i2h) {
    const int x = blockIdx.x * kPjThreads + threadIdx.x;
    if (x >= n) return;
    const int nm = n - 1;
    const int xw = x > 0 ? x - 1 : nm, xe = x < nm ? x + 1 : 0;
    const int y0 = blockIdx.y * kPjRows, y1 = min(y0 + kPjRows, n);
    for (int y = y0; y < y1; ++y) {
        const int yS = y > 0 ? y - 1 : nm, yN = y < nm ? y + 1 : 0;
        const double *ur = u + (long)(y + 1) * pitch + 1;
        const double dux = (ur[xe] - ur[xw]) * i2h;
        const double dvy = (v[(long)(yN + 1) * pitch + 1 + x] - v[(long)(yS + 1) * pitch + 1 + x]) * i2h;
        f[(long)(y + 1) * pitch + 1 + x] = dux + dvy;
    }
}

__global__ __launch_bounds__(kPjThreads) void k_subtract_gradient(const double *__restrict__ phi,
                                                                  double *__restrict__ u, double *__restrict__ v,
                                                                  long pitch, int n, double i2h) {
    const int x = blockIdx.x * kPjThreads + threadIdx.x;
    if (x >= n) return;
    const int nm = n - 1;
    const int xw = x > 0 ? x - 1 : nm, xe = x < nm ? x + 1 : 0;
    const int y0 = blockIdx.y * kPjRows, y1 = min(y0 + kPjRows, n);
    for (int y = y0; y < y1; ++y) {
        const int yS = y > 0 ? y - 1 : nm, yN = y < nm ? y + 1 : 0;
        const long o = (long)(y + 1) * pitch + 1 + x;
        const double *pr = phi + (long)(y + 1) * pitch + 1;
        u[o] -= (pr[xe] - pr[xw]) * i2h;
        v[o] -= (phi[(long)(yN + 1) * pitch + 1 + x] - phi[(long)(yS + 1) * pitch + 1 + x]) * i2h;
    }
}

}  // namespace

hipError_t launch_divergence(const double *u, const double *v, double *f, long pitch, int n, double h,
                             hipStream_t s) {
    const dim3 grid((n + kPjThreads - 1) / kPjThreads, (n + kPjRows - 1) / kPjRows);
    hipLaunchKernelGGL(k_divergence, grid, dim3(kPjThreads), 0, s, u, v, f, pitch, n, 1.0 / (2.0 * h));
    return hipGetLastError();
}

hipError_t launch_subtract_gradient(const double *phi, double *u, double *v, long pitch, int n, double h,
                                    hipStream_t s) {
    const dim3 grid((n + kPjThreads - 1) / kPjThreads, (n + kPjRows - 1) / kPjRows);
    hipLaunchKernelGGL(k_subtract_gradient, grid, dim3(kPjThreads), 0, s, phi, u, v, pitch, n, 1.0 / (2.0 * h));
    return hipGetLastError();
}

}  // namespace ccmg
