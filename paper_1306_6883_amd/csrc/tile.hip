// tile.hip -- the half-V-cycle launches of the smaller levels as 2-D LDS tiles.
//
// A level below the finest does little work per launch, so the row march's
// serial walk down its band dominates there.  Here one workgroup owns a
// 32 x 32 block of output cells: it loads the block with a halo of
// 2 nu (+1 when it restricts) cells into LDS in one round trip, runs the nu
// red-black Gauss-Seidel iterations there (the valid region shrinks by one cell
// per colour sweep; halo cells are recomputed by the neighbouring blocks), and
// writes the block -- plus, for the restricting launch, the residual's
// four-cell averages and their per-block sum.  The arithmetic of every cell
// (relaxation, residual, restriction, prolongation, ghost rule) is written in
// the same order as in the row march, so both give the same bits.
#include "internal.h"

// Products fused into additions only within one expression, as in the row
// march: both kernels give the same bits for any operator.
#pragma clang fp contract(on)

namespace ccmg {

namespace {

constexpr int TS = 32;        // output block side
constexpr int kTileThreads = 256;

__device__ __forceinline__ double block_sum_256(double v, double *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T, int NU, bool LOADPHI, bool PROLONG, bool RESTRICT>
__global__ __launch_bounds__(kTileThreads) void k_tile(const MarchArgs<T> a) {
    constexpr int H = 2 * NU + (RESTRICT ? 1 : 0);  // halo cells per side
    constexpr int R = TS + 2 * H;                    // LDS block side
    constexpr int RC = R / 2 + 3;                    // coarse block side (prolongation)
    __shared__ T u[R][R + 1];
    __shared__ T fv[R][R + 1];
    __shared__ T ec[PROLONG ? RC : 1][PROLONG ? RC + 1 : 1];
    __shared__ double red[4];
    if (a.skip && *a.skip) return;  // uniform over the workgroup

    const int n = a.n, nm = n - 1, tid = threadIdx.x;
    const int tpr = n / TS, nb = tpr * tpr;
    // neighbouring blocks (which share halo cells) stay on one XCD's L2:
    // workgroups are dealt to the 8 XCDs round robin
    int b = blockIdx.x;
    if (nb >= 8 && (nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int X0 = (b % tpr) * TS, Y0 = (b / tpr) * TS;
    const bool px = a.bc[CCMG_XLO] == CCMG_BC_PERIODIC, py = a.bc[CCMG_YLO] == CCMG_BC_PERIODIC;
    const T sxl = a.bc[CCMG_XLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T sxh = a.bc[CCMG_XHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syl = a.bc[CCMG_YLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syh = a.bc[CCMG_YHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    // global coordinate of local index l (axis origin o); -1 when outside a
    // non-periodic domain
    auto gco = [&](int o, int l, bool per) -> int {
        const int g = o - H + l;
        if (per) return g & nm;
        return (g < 0 || g > nm) ? -1 : g;
    };

    // 1. every global load of the block is issued before the first is used
    // (one memory round trip): f and phi (or zero) with the halo, the coarse
    // correction, then the partial sums of f's mean
    constexpr int NL = (R * R + kTileThreads - 1) / kTileThreads;
    constexpr int NC = PROLONG ? (RC * RC + kTileThreads - 1) / kTileThreads : 1;
    T fr[NL], pr[NL], cr[NC];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int k = tid + q * kTileThreads;
        fr[q] = pr[q] = T(0);
        if (k < R * R) {
            const int lj = k / R, li = k - lj * R;
            const int gx = gco(X0, li, px), gy = gco(Y0, lj, py);
            if (gx >= 0 && gy >= 0) {
                fr[q] = a.f[(long)(gy + 1) * a.pf + 1 + gx];
                if constexpr (LOADPHI) pr[q] = a.phi_in[(long)(gy + 1) * a.pin + 1 + gx];
            }
        }
    }
    // coarse cells covering the block and its halo, one more for the slopes
    const int CX0 = ((X0 - H) >> 1) - 1, CY0 = ((Y0 - H) >> 1) - 1;
    if constexpr (PROLONG) {
        const int ncm = (n >> 1) - 1;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int k = tid + q * kTileThreads;
            cr[q] = T(0);
            if (k < RC * RC) {
                const int cj = k / RC, ci = k - cj * RC;
                int I = CX0 + ci, J = CY0 + cj;
                if (px) I &= ncm;
                if (py) J &= ncm;
                if (I >= 0 && I <= ncm && J >= 0 && J <= ncm) cr[q] = a.ec[(long)(J + 1) * a.pc + 1 + I];
            }
        }
    }
    T fsub = T(0);
    if (a.fmean_part) {
        const int cnt = a.fmean_count_ptr ? *a.fmean_count_ptr : a.fmean_count;
        // every 64th partial per lane in turn, loaded 16 at a time (predicated)
        double s = 0.0;
        for (int i = tid & 63; i < cnt; i += 16 * 64) {
            double v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = i + 64 * k < cnt ? a.fmean_part[i + 64 * k] : 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (i + 64 * k < cnt) s += v[k];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        fsub = T(s / ((double)n * (double)n));
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int k = tid + q * kTileThreads;
        if (k < R * R) {
            const int lj = k / R, li = k - lj * R;
            T fval = fr[q];
            if (a.fmean_part && gco(X0, li, px) >= 0 && gco(Y0, lj, py) >= 0) fval -= fsub;
            fv[lj][li] = fval;
            u[lj][li] = pr[q];
        }
    }
    if constexpr (PROLONG) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int k = tid + q * kTileThreads;
            if (k < RC * RC) {
                const int cj = k / RC, ci = k - cj * RC;
                ec[cj][ci] = cr[q];
            }
        }
        __syncthreads();
        for (int k = tid; k < R * R; k += kTileThreads) {
            const int lj = k / R, li = k - lj * R;
            const int gx = gco(X0, li, px), gy = gco(Y0, lj, py);
            if (gx < 0 || gy < 0) continue;
            const int gxr = X0 - H + li, gyr = Y0 - H + lj;  // unwrapped: selects the coarse cell
            const int ci = (gxr >> 1) - CX0, cj = (gyr >> 1) - CY0;
            const int I = gx >> 1, J = gy >> 1;
            const T c0 = ec[cj][ci];
            T ew = ec[cj][ci - 1], ee = ec[cj][ci + 1], cm = ec[cj - 1][ci], cp = ec[cj + 1][ci];
            if (!px) {
                if (I == 0) ew = sxl * c0;
                if (I == (n >> 1) - 1) ee = sxh * c0;
            }
            if (!py) {
                if (J == 0) cm = syl * c0;
                if (J == (n >> 1) - 1) cp = syh * c0;
            }
            const T mx = T(0.5) * (ee - ew);
            const T my = T(0.5) * (cp - cm);
            const T dx = (gx & 1) ? T(0.25) : T(-0.25);
            const T dy = (gy & 1) ? T(0.25) : T(-0.25);
            u[lj][li] = u[lj][li] + ((c0 + dx * mx) + dy * my);
        }
    }
    __syncthreads();

    // 2. red-black iterations; colour sweep p updates the cells of its colour in
    // [p + 1, R - p - 1) of both axes.  Block origins are even and 2H is even,
    // so a cell's colour is (li + lj) & 1.
    const T cc = a.cc, invd = a.invd;
#pragma unroll
    for (int p = 0; p < 2 * NU; ++p) {
        const int c = p & 1;  // red (even) first
        const int lo = p + 1, wr = R - 2 * p - 2, half = wr >> 1;
        for (int k = tid; k < wr * half; k += kTileThreads) {
            const int row = k / half, pos = k - row * half;
            const int lj = lo + row;
            const int li = lo + 2 * pos + ((lo + lj + c) & 1);
            const int gx = gco(X0, li, px), gy = gco(Y0, lj, py);
            if (gx < 0 || gy < 0) continue;
            const T self = u[lj][li];
            T e = u[lj][li + 1], w = u[lj][li - 1], nn = u[lj + 1][li], ss = u[lj - 1][li];
            if (!px) {
                if (gx == 0) w = sxl * self;
                if (gx == nm) e = sxh * self;
            }
            if (!py) {
                if (gy == nm) nn = syh * self;
                if (gy == 0) ss = syl * self;
            }
            u[lj][li] = (fv[lj][li] + cc * (((e + w) + nn) + ss)) * invd;
        }
        __syncthreads();
    }

    // 3. the block's cells out (unless the iterate is not wanted: a level run
    // as a visit recomputes it on the way up)
    for (int k = tid; a.phi_out && k < TS * TS; k += kTileThreads) {
        const int j = k / TS, i = k - j * TS;
        const int gx = X0 + i, gy = Y0 + j;
        a.phi_out[(long)(gy + 1) * a.pout + 1 + gx] = u[H + j][H + i];
    }

    // 4. residual -> four-cell averages (one coarse cell per thread) + block sum
    if constexpr (RESTRICT) {
        const T ih2 = a.ih2, alpha = a.alpha, beta = a.beta;
        auto resid = [&](int li, int lj) -> T {
            const int gx = X0 - H + li, gy = Y0 - H + lj;  // inside the domain (block cells)
            const T p = u[lj][li];
            T e = u[lj][li + 1], w = u[lj][li - 1], nn = u[lj + 1][li], ss = u[lj - 1][li];
            if (!px) {
                if (gx == 0) w = sxl * p;
                if (gx == nm) e = sxh * p;
            }
            if (!py) {
                if (gy == nm) nn = syh * p;
                if (gy == 0) ss = syl * p;
            }
            const T lap = ((((e - p) + (w - p)) + (nn - p)) + (ss - p)) * ih2;
            return fv[lj][li] - (alpha * p - beta * lap);
        };
        const int cj = tid >> 4, ci = tid & 15;  // 16 x 16 coarse cells
        const int li = H + 2 * ci, lj = H + 2 * cj;
        const T r00 = resid(li, lj), r01 = resid(li + 1, lj);
        const T r10 = resid(li, lj + 1), r11 = resid(li + 1, lj + 1);
        const T v = T(0.25) * (((r00 + r01) + r10) + r11);
        const int I = (X0 >> 1) + ci, J = (Y0 >> 1) + cj;
        a.aux[(long)(J + 1) * a.paux + 1 + I] = v;
        const double s = block_sum_256((double)v, red);
        if (tid == 0) a.partial[blockIdx.x] = s;
    }
}

template <typename T, int NU>
hipError_t go_nu(const MarchArgs<T> &a, bool load_phi, bool prolong, bool restrict_, int nb, hipStream_t s) {
    const dim3 g(nb), blk(kTileThreads);
    if (!load_phi && !prolong && restrict_) hipLaunchKernelGGL((k_tile<T, NU, false, false, true>), g, blk, 0, s, a);
    else if (load_phi && !prolong && restrict_) hipLaunchKernelGGL((k_tile<T, NU, true, false, true>), g, blk, 0, s, a);
    else if (load_phi && !prolong && !restrict_) hipLaunchKernelGGL((k_tile<T, NU, true, false, false>), g, blk, 0, s, a);
    else if (load_phi && prolong && !restrict_) hipLaunchKernelGGL((k_tile<T, NU, true, true, false>), g, blk, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_tile(const MarchArgs<T> &a, int nu, bool load_phi, bool prolong, int post, hipStream_t s,
                       int *ntiles_out) {
    // levels below the finest only: no phi shift, no norms, at least 2 x 2 blocks
    if (a.n < kTileMinN || a.n < 2 * TS || (a.n & (a.n - 1)) || a.phi_shift || (post != POST_NONE && post != POST_RESTRICT))
        return hipErrorInvalidValue;
    const int tpr = a.n / TS, nb = tpr * tpr;
    if (ntiles_out) *ntiles_out = nb;
    const bool rs = post == POST_RESTRICT;
    switch (nu) {
        case 0: return go_nu<T, 0>(a, load_phi, prolong, rs, nb, s);
        case 1: return go_nu<T, 1>(a, load_phi, prolong, rs, nb, s);
        case 2: return go_nu<T, 2>(a, load_phi, prolong, rs, nb, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_tile<double>(const MarchArgs<double> &, int, bool, bool, int, hipStream_t, int *);
template hipError_t launch_tile<float>(const MarchArgs<float> &, int, bool, bool, int, hipStream_t, int *);

}  // namespace ccmg
