// coarse.hip -- the bottom of the V-cycle in one workgroup.
//
// Levels with at most kCoarseMax cells per side are too small to fill the
// GPU, so one workgroup runs the whole rest of the V-cycle for them: from the
// top level (n_top cells per side) down to the 2 x 2 grid and back up, every
// level held in LDS (phi and f, no ghost layer: side rules are applied where a
// neighbour is read).  The steps are those of the paper's V-cycle (Sec. 3.3):
// nu1 red-black Gauss-Seidel iterations, residual and four-cell restriction,
// recursion, centred-slope prolongation without the xy term, nu2 iterations;
// on the 2 x 2 grid nu_bottom relaxations, done in FP64 whatever T is.
#include "internal.h"

namespace ccmg {

namespace {

constexpr int kThreads = 256;

// Neighbour values of cell (x, y) of an n x n level stored row-major in A.
template <typename T>
__device__ __forceinline__ void neighbours(const T *A, int n, int x, int y, const int *bc, T self,
                                           T &e, T &w, T &nn, T &s) {
    const int nm = n - 1;
    auto sgn = [](int b) { return b == CCMG_BC_DIRICHLET ? T(-1) : T(1); };
    e = x < nm ? A[y * n + x + 1] : (bc[CCMG_XHI] == CCMG_BC_PERIODIC ? A[y * n] : sgn(bc[CCMG_XHI]) * self);
    w = x > 0 ? A[y * n + x - 1] : (bc[CCMG_XLO] == CCMG_BC_PERIODIC ? A[y * n + nm] : sgn(bc[CCMG_XLO]) * self);
    nn = y < nm ? A[(y + 1) * n + x] : (bc[CCMG_YHI] == CCMG_BC_PERIODIC ? A[x] : sgn(bc[CCMG_YHI]) * self);
    s = y > 0 ? A[(y - 1) * n + x] : (bc[CCMG_YLO] == CCMG_BC_PERIODIC ? A[nm * n + x] : sgn(bc[CCMG_YLO]) * self);
}

// Block-wide sum in a fixed order (per-thread strided sums, per-wave butterfly,
// then the four wave totals in order).  All threads get the result.
__device__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

template <typename T>
__device__ void relax(T *P, const T *F, int n, const int *bc, T cc, T invd, int iters) {
    const int half = (n * n) >> 1, hn = n >> 1;
    for (int it = 0; it < iters; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int i = threadIdx.x; i < half; i += kThreads) {
                const int y = i / hn;
                const int x = 2 * (i - y * hn) + ((y + colour) & 1);
                const T self = P[y * n + x];
                T e, w, nn, s;
                neighbours(P, n, x, y, bc, self, e, w, nn, s);
                P[y * n + x] = (F[y * n + x] + cc * (((e + w) + nn) + s)) * invd;
            }
            __syncthreads();
        }
    }
}

// Fc = four-cell average of r = F - A P (fine level of n cells per side).
template <typename T>
__device__ void restrict_residual(const T *P, const T *F, T *Fc, int n, const int *bc, T alpha, T beta,
                                  T ih2) {
    const int nc = n >> 1;
    for (int i = threadIdx.x; i < nc * nc; i += kThreads) {
        const int J = i / nc, I = i - J * nc;
        T r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = 2 * I + (q & 1), y = 2 * J + (q >> 1);
            const T p = P[y * n + x];
            T e, w, nn, s;
            neighbours(P, n, x, y, bc, p, e, w, nn, s);
            const T lap = ((((e - p) + (w - p)) + (nn - p)) + (s - p)) * ih2;
            r[q] = F[y * n + x] - (alpha * p - beta * lap);
        }
        Fc[i] = T(0.25) * (((r[0] + r[1]) + r[2]) + r[3]);
    }
    __syncthreads();
}

template <typename T>
__device__ void remove_mean(T *A, int n, double *red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n * n; i += kThreads) s += (double)A[i];
    const T m = T(block_sum(s, red) / ((double)n * (double)n));
    for (int i = threadIdx.x; i < n * n; i += kThreads) A[i] -= m;
    __syncthreads();
}

// P (fine, n per side) += prolongation of E (coarse, n/2 per side).
template <typename T>
__device__ void prolong_add(const T *E, T *P, int n, const int *bc) {
    const int nc = n >> 1;
    for (int i = threadIdx.x; i < n * n; i += kThreads) {
        const int y = i / n, x = i - y * n;
        const int I = x >> 1, J = y >> 1;
        const T e = E[J * nc + I];
        T ee, ew, en, es;
        neighbours(E, nc, I, J, bc, e, ee, ew, en, es);
        const T mx = T(0.5) * (ee - ew), my = T(0.5) * (en - es);
        const T dx = (x & 1) ? T(0.25) : T(-0.25), dy = (y & 1) ? T(0.25) : T(-0.25);
        P[i] = P[i] + ((e + dx * mx) + dy * my);
    }
    __syncthreads();
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kThreads) void k_coarse(const CoarseArgs<T> a) {
    __shared__ T sP[kCoarseMax * kCoarseMax * 4 / 3 + 8];
    __shared__ T sF[kCoarseMax * kCoarseMax * 4 / 3 + 8];
    __shared__ double red[kThreads / 64];
    __shared__ int bc[4];
    if (a.skip && *a.skip) return;  // uniform over the workgroup
    if (threadIdx.x < 4) bc[threadIdx.x] = a.bc[threadIdx.x];
    __syncthreads();

    const int n0 = a.n_top;
    int L = 0;
    while ((n0 >> L) >= 2) ++L;  // levels n0, n0/2, ..., 2
    int off[16];
    off[0] = 0;
    for (int l = 1; l < L; ++l) off[l] = off[l - 1] + (n0 >> (l - 1)) * (n0 >> (l - 1));

    // top level in
    const T shift = (a.load_phi && a.phi_shift) ? T(*a.phi_shift) : T(0);
    for (int i = threadIdx.x; i < n0 * n0; i += kThreads) {
        const int y = i / n0, x = i - y * n0;
        sF[i] = a.f[(long)(y + 1) * a.pf + 1 + x];
        sP[i] = a.load_phi ? a.phi_in[(long)(y + 1) * a.pin + 1 + x] - shift : T(0);
    }
    __syncthreads();
    if (a.sub_top_mean) remove_mean(sF, n0, red);

    auto consts = [&](int l, T &cc, T &invd, T &ih2) {
        const double h = a.h_top * (double)(1 << l);
        const double c = a.beta / (h * h);
        cc = T(c);
        invd = T(1.0 / (a.alpha + 4.0 * c));
        ih2 = T(1.0 / (h * h));
    };

    // down
    for (int l = 0; l + 1 < L; ++l) {
        const int n = n0 >> l;
        T cc, invd, ih2;
        consts(l, cc, invd, ih2);
        relax(sP + off[l], sF + off[l], n, bc, cc, invd, a.nu1);
        restrict_residual(sP + off[l], sF + off[l], sF + off[l + 1], n, bc, T(a.alpha), T(a.beta), ih2);
        if (a.singular) remove_mean(sF + off[l + 1], n >> 1, red);
        for (int i = threadIdx.x; i < (n >> 1) * (n >> 1); i += kThreads) sP[off[l + 1] + i] = T(0);
        __syncthreads();
    }
    // bottom: 2 x 2 grid, relaxation only, in FP64 registers of one thread
    if (threadIdx.x == 0) {
        const int l = L - 1;
        const double h = a.h_top * (double)(1 << l);
        const double c = a.beta / (h * h), invd = 1.0 / (a.alpha + 4.0 * c);
        double p[4], f[4];
        for (int q = 0; q < 4; ++q) {
            p[q] = (double)sP[off[l] + q];
            f[q] = (double)sF[off[l] + q];
        }
        auto sgn = [](int b) { return b == CCMG_BC_DIRICHLET ? -1.0 : 1.0; };
        // cell q = y*2 + x; its x-neighbour is q^1, its y-neighbour q^2.  On a
        // 2 x 2 grid the periodic image of that neighbour is the same cell, and a
        // D / N ghost is -/+ the cell itself.
        for (int it = 0; it < a.nu_bottom; ++it) {
            for (int colour = 0; colour < 2; ++colour) {
                for (int q = 0; q < 4; ++q) {
                    const int x = q & 1, y = q >> 1;
                    if (((x + y) & 1) != colour) continue;
                    const double self = p[q];
                    const double ex = p[q ^ 1], ey = p[q ^ 2];
                    const double e = x == 0 ? ex : (bc[CCMG_XHI] == CCMG_BC_PERIODIC ? ex : sgn(bc[CCMG_XHI]) * self);
                    const double w = x == 1 ? ex : (bc[CCMG_XLO] == CCMG_BC_PERIODIC ? ex : sgn(bc[CCMG_XLO]) * self);
                    const double nn = y == 0 ? ey : (bc[CCMG_YHI] == CCMG_BC_PERIODIC ? ey : sgn(bc[CCMG_YHI]) * self);
                    const double s = y == 1 ? ey : (bc[CCMG_YLO] == CCMG_BC_PERIODIC ? ey : sgn(bc[CCMG_YLO]) * self);
                    p[q] = (f[q] + c * (((e + w) + nn) + s)) * invd;
                }
            }
        }
        for (int q = 0; q < 4; ++q) sP[off[l] + q] = T(p[q]);
    }
    __syncthreads();
    // up
    for (int l = L - 2; l >= 0; --l) {
        const int n = n0 >> l;
        T cc, invd, ih2;
        consts(l, cc, invd, ih2);
        prolong_add(sP + off[l + 1], sP + off[l], n, bc);
        relax(sP + off[l], sF + off[l], n, bc, cc, invd, a.nu2);
    }
    // top level out
    for (int i = threadIdx.x; i < n0 * n0; i += kThreads) {
        const int y = i / n0, x = i - y * n0;
        a.phi_out[(long)(y + 1) * a.pout + 1 + x] = sP[i];
    }
}

template <typename T>
hipError_t launch_coarse(const CoarseArgs<T> &a, hipStream_t s) {
    if (a.n_top < 2 || a.n_top > kCoarseMax || (a.n_top & (a.n_top - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_coarse<double>(const CoarseArgs<double> &, hipStream_t);
template hipError_t launch_coarse<float>(const CoarseArgs<float> &, hipStream_t);

}  // namespace ccmg
