// coarse.hip -- the bottom of the V-cycle in one workgroup.
//
// Levels with at most kCoarseMax cells per side are too small to fill the
// GPU, so one workgroup runs the whole rest of the V-cycle for them: from the
// top level (n_top cells per side) down to the 2 x 2 grid and back up, every
// level held in LDS (phi and f, no ghost layer: side rules are applied where a
// neighbour is read).  The steps are those of the paper's V-cycle (Sec. 3.3):
// nu1 red-black Gauss-Seidel iterations, residual and four-cell restriction,
// recursion, centred-slope prolongation without the xy term, nu2 iterations;
// on the 2 x 2 grid nu_bottom relaxations, done in FP64 whatever T is.  Or an
// exact bottom on a 4 x 4 or 8 x 8 level: its inverse operator (computed once
// per plan by k_bottom_inverse) is held in LDS and applied in FP64.
#include <cstdlib>

#include "internal.h"

namespace ccmg {

namespace {

// Workgroup size NT (a template parameter): 512 gives one thread per cell of a
// colour on the 32 x 32 level (64, 128 and 256 measured slower).  With NT = 64
// (one wavefront) no workgroup barrier would be needed -- a wave's LDS
// operations complete in issue order, so ordering the compiler's code is
// enough between phases.
constexpr int kCoarseThreads = 512;

template <int NT>
__device__ __forceinline__ void sync() {
    if constexpr (NT == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Side rules, held in scalar registers for the whole kernel.
struct Sides {
    bool px, py;          // periodic in x / y
    float sxl, sxh, syl, syh;  // ghost sign of a Dirichlet (-1) / Neumann (+1) side
};

// Neighbour values of cell (x, y) of an n x n level (n = 1 << lg) stored
// row-major in A.  Branch-free: every neighbour is one LDS read at a wrapped
// (periodic) or clamped (own cell) index, times the ghost sign (-1 Dirichlet,
// +1 Neumann) where the neighbour is a ghost; times 1 (exact) elsewhere.
template <typename T>
__device__ __forceinline__ void neighbours(const T *A, int lg, int x, int y, const Sides &sd, T self,
                                           T &e, T &w, T &nn, T &s) {
    (void)self;
    const int nm = (1 << lg) - 1;
    const bool xh = x == nm, xl = x == 0, yh = y == nm, yl = y == 0;
    const int xe = xh ? (sd.px ? 0 : x) : x + 1;
    const int xw = xl ? (sd.px ? nm : x) : x - 1;
    const int yn = yh ? (sd.py ? 0 : y) : y + 1;
    const int yS = yl ? (sd.py ? nm : y) : y - 1;
    const T ge = (xh && !sd.px) ? T(sd.sxh) : T(1);
    const T gw = (xl && !sd.px) ? T(sd.sxl) : T(1);
    const T gn = (yh && !sd.py) ? T(sd.syh) : T(1);
    const T gs = (yl && !sd.py) ? T(sd.syl) : T(1);
    const int row = y << lg;
    e = ge * A[row + xe];
    w = gw * A[row + xw];
    nn = gn * A[(yn << lg) + x];
    s = gs * A[(yS << lg) + x];
}

// Block-wide sum in a fixed order (per-thread strided sums, per-wave butterfly,
// then the wave totals in order).  All threads get the result.
template <int NT>
__device__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if constexpr (NT == 64) {
        return v;
    } else {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = v;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t += red[i];
        __syncthreads();
        return t;
    }
}

template <int NT, typename T>
__device__ void relax(T *P, const T *F, int lg, const Sides &sd, T cc, T invd, int iters) {
    const int n = 1 << lg, half = (n * n) >> 1, lgh = lg - 1;
    for (int it = 0; it < iters; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int i = threadIdx.x; i < half; i += NT) {
                const int y = i >> lgh;
                const int x = 2 * (i - (y << lgh)) + ((y + colour) & 1);
                const T self = P[(y << lg) + x];
                T e, w, nn, s;
                neighbours(P, lg, x, y, sd, self, e, w, nn, s);
                P[(y << lg) + x] = (F[(y << lg) + x] + cc * (((e + w) + nn) + s)) * invd;
            }
            sync<NT>();
        }
    }
}

// Fc = four-cell average of r = F - A P (fine level of n = 1 << lg cells per side).
template <int NT, typename T>
__device__ void restrict_residual(const T *P, const T *F, T *Fc, int lg, const Sides &sd, T alpha, T beta,
                                  T ih2) {
    const int lgc = lg - 1, nc = 1 << lgc;
    for (int i = threadIdx.x; i < nc * nc; i += NT) {
        const int J = i >> lgc, I = i - (J << lgc);
        T r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = 2 * I + (q & 1), y = 2 * J + (q >> 1);
            const T p = P[(y << lg) + x];
            T e, w, nn, s;
            neighbours(P, lg, x, y, sd, p, e, w, nn, s);
            const T lap = ((((e - p) + (w - p)) + (nn - p)) + (s - p)) * ih2;
            r[q] = F[(y << lg) + x] - (alpha * p - beta * lap);
        }
        Fc[i] = T(0.25) * (((r[0] + r[1]) + r[2]) + r[3]);
    }
    sync<NT>();
}

template <int NT, typename T>
__device__ void remove_mean(T *A, int lg, double *red) {
    const int nn = 1 << (2 * lg);
    double s = 0.0;
    for (int i = threadIdx.x; i < nn; i += NT) s += (double)A[i];
    const T m = T(block_sum<NT>(s, red) / (double)nn);
    for (int i = threadIdx.x; i < nn; i += NT) A[i] -= m;
    sync<NT>();
}

// P (fine, n = 1 << lg per side) += prolongation of E (coarse, n/2 per side).
template <int NT, typename T>
__device__ void prolong_add(const T *E, T *P, int lg, const Sides &sd) {
    const int n = 1 << lg, lgc = lg - 1;
    for (int i = threadIdx.x; i < n * n; i += NT) {
        const int y = i >> lg, x = i - (y << lg);
        const int I = x >> 1, J = y >> 1;
        const T e = E[(J << lgc) + I];
        T ee, ew, en, es;
        neighbours(E, lgc, I, J, sd, e, ee, ew, en, es);
        const T mx = T(0.5) * (ee - ew), my = T(0.5) * (en - es);
        const T dx = (x & 1) ? T(0.25) : T(-0.25), dy = (y & 1) ? T(0.25) : T(-0.25);
        P[i] = P[i] + ((e + dx * mx) + dy * my);
    }
    sync<NT>();
}

}  // namespace

// Levels with at most 2^kWaveLg cells per side run on one wave (see coarse_body).
constexpr int kWaveLg = 3;

// One level on the way down: nu1 relaxations, residual restricted to the
// next level (its mean removed for singular problems), next level's
// correction zeroed.  NTW threads (the workgroup, or the first wave) take part.
template <int NTW, typename T>
__device__ void down_level(const CoarseArgs<T> &a, const Sides &sd, T *sP, T *sF, const int *off, int lg0, int l,
                           double *red) {
    const int lg = lg0 - l;
    relax<NTW>(sP + off[l], sF + off[l], lg, sd, T(a.cc[l]), T(a.invd[l]), a.nu1);
    restrict_residual<NTW>(sP + off[l], sF + off[l], sF + off[l + 1], lg, sd, T(a.alpha), T(a.beta),
                           T(a.ih2[l]));
    if (a.singular) remove_mean<NTW>(sF + off[l + 1], lg - 1, red);
    for (int i = threadIdx.x; i < (1 << (2 * (lg - 1))); i += NTW) sP[off[l + 1] + i] = T(0);
    sync<NTW>();
}

// One level on the way up: prolongation of the next level's correction, nu2
// relaxations.
template <int NTW, typename T>
__device__ void up_level(const CoarseArgs<T> &a, const Sides &sd, T *sP, const T *sF, const int *off, int lg0,
                         int l) {
    const int lg = lg0 - l;
    prolong_add<NTW>(sP + off[l + 1], sP + off[l], lg, sd);
    relax<NTW>(sP + off[l], sF + off[l], lg, sd, T(a.cc[l]), T(a.invd[l]), a.nu2);
}

// Bottom: 2 x 2 grid, relaxation only, in FP64 registers of thread 0.
// Cell q = 2y + x; its x-neighbour is q^1 and its y-neighbour q^2.  On a
// 2 x 2 grid the periodic image of that neighbour is the same cell, and a
// Dirichlet / Neumann ghost is -/+ the cell itself.
template <typename T>
__device__ void bottom(const CoarseArgs<T> &a, const Sides &sd, T *sP, const T *sF, const int *off, int L) {
    if (threadIdx.x != 0) return;
    const int l = L - 1;
    const double c = a.cc[l], invd = a.invd[l];
    double p0 = sP[off[l] + 0], p1 = sP[off[l] + 1], p2 = sP[off[l] + 2], p3 = sP[off[l] + 3];
    const double f0 = sF[off[l] + 0], f1 = sF[off[l] + 1], f2 = sF[off[l] + 2], f3 = sF[off[l] + 3];
    const double xl = sd.px ? 1.0 : (double)sd.sxl, xh = sd.px ? 1.0 : (double)sd.sxh;
    const double yl = sd.py ? 1.0 : (double)sd.syl, yh = sd.py ? 1.0 : (double)sd.syh;
    // x-ghost of a cell at x = 0 is its west side (x-lo), at x = 1 its east side (x-hi)
    auto upd = [&](double self, double ex, double ey, double f, bool x0, bool y0) {
        const double e = x0 ? ex : (sd.px ? ex : xh * self);
        const double w = x0 ? (sd.px ? ex : xl * self) : ex;
        const double nn = y0 ? ey : (sd.py ? ey : yh * self);
        const double s = y0 ? (sd.py ? ey : yl * self) : ey;
        return (f + c * (((e + w) + nn) + s)) * invd;
    };
    for (int it = 0; it < a.nu_bottom; ++it) {
        const double q0 = upd(p0, p1, p2, f0, true, true);    // red (0,0)
        const double q3 = upd(p3, p2, p1, f3, false, false);  // red (1,1)
        const double q1 = upd(p1, q0, q3, f1, false, true);   // black (1,0)
        const double q2 = upd(p2, q3, q0, f2, true, false);   // black (0,1)
        // an iteration that changes nothing is a fixed point: the remaining
        // iterations would return exactly these values
        const bool same = q0 == p0 && q1 == p1 && q2 == p2 && q3 == p3;
        p0 = q0, p1 = q1, p2 = q2, p3 = q3;
        if (same) break;
    }
    sP[off[l] + 0] = T(p0);
    sP[off[l] + 1] = T(p1);
    sP[off[l] + 2] = T(p2);
    sP[off[l] + 3] = T(p3);
}

// Exact bottom on level l (n = 1 << lg cells per side, m = n^2 unknowns), on
// the first wave: lane i computes P[i] = sum_j ainv[i][j] F[j] in FP64 in
// column order.  ainv is column-major in LDS, so a lane reads consecutive
// doubles and F[j] is one broadcast.
template <typename T>
__device__ void direct_bottom(const double *sInv, T *P, const T *F, int lg) {
    const int m = 1 << (2 * lg);
    const int i = threadIdx.x;
    if (i < m) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += sInv[j * m + i] * (double)F[j];
        P[i] = T(s);
    }
}

template <int NT, typename T, bool DIRECT>
__device__ void coarse_body(const CoarseArgs<T> &a) {
    __shared__ T sP[kCoarseMax * kCoarseMax * 4 / 3 + 8];
    __shared__ T sF[kCoarseMax * kCoarseMax * 4 / 3 + 8];
    __shared__ double red[NT / 64];
    __shared__ double sInv[DIRECT ? kDirectMax * kDirectMax * kDirectMax * kDirectMax : 1];
    if (a.skip && *a.skip) return;  // uniform over the workgroup

    Sides sd;
    sd.px = a.bc[CCMG_XLO] == CCMG_BC_PERIODIC;
    sd.py = a.bc[CCMG_YLO] == CCMG_BC_PERIODIC;
    sd.sxl = a.bc[CCMG_XLO] == CCMG_BC_DIRICHLET ? -1.f : 1.f;
    sd.sxh = a.bc[CCMG_XHI] == CCMG_BC_DIRICHLET ? -1.f : 1.f;
    sd.syl = a.bc[CCMG_YLO] == CCMG_BC_DIRICHLET ? -1.f : 1.f;
    sd.syh = a.bc[CCMG_YHI] == CCMG_BC_DIRICHLET ? -1.f : 1.f;

    const int n0 = a.n_top;
    const int lg0 = 31 - __clz(n0);
    // levels n0, n0/2, ..., n_bottom (2 unless the bottom is exact)
    const int lgb = DIRECT ? 31 - __clz(a.n_bottom) : 1;
    const int L = lg0 - lgb + 1;
    if (DIRECT) {  // the inverse into LDS; its loads overlap the top level's
        const int mm = 1 << (4 * lgb);
        for (int i = threadIdx.x; i < mm; i += NT) sInv[i] = a.ainv[i];
    }
    int off[8];
    off[0] = 0;
    for (int l = 1; l < L; ++l) off[l] = off[l - 1] + (1 << (2 * (lg0 - l + 1)));

    // top level in
    const T shift = (a.load_phi && a.phi_shift) ? T(*a.phi_shift) : T(0);
    for (int i = threadIdx.x; i < n0 * n0; i += NT) {
        const int y = i >> lg0, x = i - (y << lg0);
        sF[i] = a.f[(long)(y + 1) * a.pf + 1 + x];
        sP[i] = a.load_phi ? a.phi_in[(long)(y + 1) * a.pin + 1 + x] - shift : T(0);
    }
    sync<NT>();
    if (a.sub_top_mean) remove_mean<NT>(sF, lg0, red);

    // Levels of at most 8 x 8 cells (and the bottom) run on the first wave
    // alone: 64 lanes cover such a level's colour in one pass, and a wave
    // needs no workgroup barrier between phases.  lw = first such level.
    int lw = 0;
    while (lw < L && lg0 - lw > kWaveLg) ++lw;
    // down, whole workgroup
    for (int l = 0; l < lw && l + 1 < L; ++l) down_level<NT>(a, sd, sP, sF, off, lg0, l, red);
    if (NT == 64 || threadIdx.x < 64) {
        for (int l = lw; l + 1 < L; ++l) down_level<64>(a, sd, sP, sF, off, lg0, l, red);
        if (DIRECT)
            direct_bottom(sInv, sP + off[L - 1], sF + off[L - 1], lgb);
        else
            bottom(a, sd, sP, sF, off, L);
        sync<64>();
        for (int l = L - 2; l >= lw; --l) up_level<64>(a, sd, sP, sF, off, lg0, l);
    }
    sync<NT>();
    // up, whole workgroup
    for (int l = (lw < L - 1 ? lw : L - 1) - 1; l >= 0; --l) up_level<NT>(a, sd, sP, sF, off, lg0, l);
    // top level out
    for (int i = threadIdx.x; i < n0 * n0; i += NT) {
        const int y = i >> lg0, x = i - (y << lg0);
        a.phi_out[(long)(y + 1) * a.pout + 1 + x] = sP[i];
    }
}

template <int NT, typename T, bool DIRECT>
__global__ __launch_bounds__(NT) void k_coarse(const CoarseArgs<T> a) {
    coarse_body<NT, T, DIRECT>(a);
}

// Batches: one workgroup per problem (relaxation bottom).
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_coarse_list(const CoarseArgs<T> *__restrict__ list) {
    coarse_body<NT, T, false>(list[blockIdx.x]);
}

// Inverse of a small level's operator by Gauss-Jordan elimination on [A | I]
// in LDS, one workgroup.  No pivoting: the operator is definite (symmetric,
// all eigenvalues of one sign; a singular one is made definite by c 1 1^T with
// c of the operator's sign), so every pivot is a nonzero Schur complement
// entry.  Four threads per row, each a quarter of the 2m columns.
constexpr int kInvThreads = 256;
__global__ __launch_bounds__(kInvThreads) void k_bottom_inverse(int lgb, int bc0, int bc1, int bc2, int bc3,
                                                                double alpha, double beta, double h, int singular,
                                                                double *__restrict__ out) {
    constexpr int kM = kDirectMax * kDirectMax;
    __shared__ double M[kM][2 * kM];
    const int nb = 1 << lgb, m = nb * nb, w = 2 * m;
    const int bc[4] = {bc0, bc1, bc2, bc3};
    const double c = beta / (h * h);
    for (int k = threadIdx.x; k < m; k += kInvThreads) {
        for (int q = 0; q < m; ++q) M[k][q] = singular ? c : 0.0;  // A (+ c 1 1^T) ...
        for (int q = m; q < w; ++q) M[k][q] = (q == k + m) ? 1.0 : 0.0;  // ... | I
        const int i = k % nb, j = k / nb;
        M[k][k] += alpha + 4.0 * c;
        const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
        for (int s = 0; s < 4; ++s) {
            const bool inside = ni[s] >= 0 && ni[s] < nb && nj[s] >= 0 && nj[s] < nb;
            if (inside || bc[s] == CCMG_BC_PERIODIC)
                M[k][((nj[s] + nb) % nb) * nb + (ni[s] + nb) % nb] -= c;
            else  // ghost = -cell (Dirichlet) or +cell (Neumann)
                M[k][k] -= (bc[s] == CCMG_BC_DIRICHLET ? -c : c);
        }
    }
    const int r = threadIdx.x >> 2, part = threadIdx.x & 3;
    const int q0 = part * (w / 4), q1 = q0 + w / 4;
    for (int col = 0; col < m; ++col) {
        __syncthreads();
        const double piv = M[col][col];
        const double g = (r < m && r != col) ? M[r][col] / piv : 0.0;
        __syncthreads();
        if (r < m && r != col)
            for (int q = q0; q < q1; ++q) M[r][q] -= g * M[col][q];
        __syncthreads();
        if (r == col)
            for (int q = q0; q < q1; ++q) M[col][q] /= piv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += kInvThreads) {
        const int k = t % m, q = t / m;  // out[q * m + k] = inverse[k][q]
        out[t] = M[k][m + q];
    }
}

hipError_t launch_bottom_inverse(int nb, const int bc[4], double alpha, double beta, double h, int singular,
                                 double *out, hipStream_t s) {
    if (nb < 4 || nb > kDirectMax || (nb & (nb - 1)) || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bottom_inverse, dim3(1), dim3(kInvThreads), 0, s, 31 - __builtin_clz(nb), bc[0], bc[1],
                       bc[2], bc[3], alpha, beta, h, singular, out);
    return hipGetLastError();
}

template <typename T>
void coarse_fill_consts(CoarseArgs<T> &a) {
    for (int l = 0; (a.n_top >> l) >= 2 && l < 8; ++l) {
        const double h = a.h_top * (double)(1 << l);
        const double c = a.beta / (h * h);
        a.cc[l] = c;
        a.invd[l] = 1.0 / (a.alpha + 4.0 * c);
        a.ih2[l] = 1.0 / (h * h);
    }
}

template <typename T>
hipError_t launch_coarse(const CoarseArgs<T> &a0, hipStream_t s) {
    if (a0.n_top < 2 || a0.n_top > kCoarseMax || (a0.n_top & (a0.n_top - 1))) return hipErrorInvalidValue;
    CoarseArgs<T> a = a0;
    coarse_fill_consts(a);
    const bool direct = a.n_bottom >= 4;
    if (direct && (a.n_bottom > kDirectMax || a.n_bottom > a.n_top || (a.n_bottom & (a.n_bottom - 1)) || !a.ainv))
        return hipErrorInvalidValue;
    constexpr int NT = kCoarseThreads;
    if (direct) hipLaunchKernelGGL((k_coarse<NT, T, true>), dim3(1), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((k_coarse<NT, T, false>), dim3(1), dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_list(const CoarseArgs<T> *list, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_coarse_list<kCoarseThreads, T>), dim3(count), dim3(kCoarseThreads), 0, s, list);
    return hipGetLastError();
}

template hipError_t launch_coarse<double>(const CoarseArgs<double> &, hipStream_t);
template hipError_t launch_coarse<float>(const CoarseArgs<float> &, hipStream_t);
template hipError_t launch_coarse_list<float>(const CoarseArgs<float> *, int, hipStream_t);
template hipError_t launch_coarse_list<double>(const CoarseArgs<double> *, int, hipStream_t);
template void coarse_fill_consts<float>(CoarseArgs<float> &);
template void coarse_fill_consts<double>(CoarseArgs<double> &);

}  // namespace ccmg
