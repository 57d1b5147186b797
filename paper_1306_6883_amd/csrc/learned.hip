// learned.hip -- kernels of the learned initial guess.
//
// The network maps the right-hand side, averaged onto a G x G grid (G = 128),
// to the solution on that grid.  The map it has to learn is linear, so the
// network is linear: six 3x3 convolutions with circular padding and dilations
// 1, 2, 4, 8, 16, 32 (receptive field 127 cells: the whole periodic grid),
// channels 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, no biases.  Activations are
// pixel-major with the 32 channels contiguous ([b][y][x][c]) and carried
// between layers as a pair of BF16 planes (hi + lo, about 16 significant bits:
// a single BF16 activation puts a noise floor of about 1% on the output);
// weights are BF16 copies of FP32 master weights; gradients are single BF16.
//
// The 32 -> 32 layers are implicit GEMMs on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation): M = 32 pixels of one row,
// N = 32 output channels, K = 9 taps x 32 input channels.  The input gradient
// of such a layer is the same product with transposed, tap-flipped weights;
// the weight gradient is a product with K running over pixels.  The 1-channel
// first and last layers are small and run on the vector units.
//
// Operand layouts of v_mfma_f32_32x32x16_bf16 (wave64): lane l holds
//   A (32 x 16): row l % 32, k = 8 (l / 32) + i, i = 0..7;
//   B (16 x 32): column l % 32, k = 8 (l / 32) + i;
//   D (32 x 32, FP32): register j holds row 8 (j / 4) + 4 (l / 32) + j % 4,
//   column l % 32.
#include "learned.h"

namespace ccmg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ int wrapg(int v) { return v & (kNetG - 1); }
// tap t = 3 ky + kx -> offset (ky - 1, kx - 1) * dilation
__device__ __forceinline__ int tap_dy(int t, int d) { return (t / 3 - 1) * d; }
__device__ __forceinline__ int tap_dx(int t, int d) { return (t % 3 - 1) * d; }

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// Workgroups are dealt to the 8 XCDs round robin; when the grid divides by 8,
// give each XCD a contiguous run of workgroup indices instead, so that the
// rows one XCD's waves read for their (dilated) taps stay in its L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

}  // namespace

// out[b][y][x][co] = sum_{tap, ci} w[co][tap][ci] * in[b][y + dy][x + dx][ci]
// One wavefront per 32 pixels of one row.  An activation is carried as a pair
// of BF16 values (hi + lo, about 16 significant bits): with `in_lo` the
// products take two MFMAs (hi and lo against the same BF16 weights), and with
// `out_lo` the FP32 sum is written as such a pair.  Without them (gradients)
// one BF16 value.
// SPLIT = 1: four tiles per workgroup of 256, one per wavefront.  SPLIT = 3
// (small batches, too few tiles to occupy the GPU): one tile per workgroup of
// 192; wavefront s takes taps 3s .. 3s + 2 and the first adds the other two's
// partial sums from LDS, (acc0 + acc1) + acc2.
template <int SPLIT>
__global__ __launch_bounds__(256) void k_conv32(const __bf16 *__restrict__ in, const __bf16 *__restrict__ in_lo,
                                                const __bf16 *__restrict__ w, const __bf16 *__restrict__ w_lo,
                                                __bf16 *__restrict__ out, __bf16 *__restrict__ out_lo, int nb,
                                                int dil) {
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wave = SPLIT == 1 ? xcd_block() * 4 + wib : xcd_block();
    const int tiles_per_row = kNetG / 32;
    if (wave >= nb * kNetG * tiles_per_row) return;  // uniform over the workgroup when SPLIT > 1
    const int b = wave / (kNetG * tiles_per_row);
    const int rem = wave - b * kNetG * tiles_per_row;
    const int y = rem / tiles_per_row;
    const int x0 = (rem - y * tiles_per_row) * 32;
    const int r = lane & 31, hk = lane >> 5;
    const size_t img = (size_t)b * kNetG * kNetG * kNetC;
    f32x16 acc = {};
    const int t0 = SPLIT == 1 ? 0 : 3 * wib;
#pragma unroll
    for (int tt = 0; tt < 9 / SPLIT; ++tt) {
        const int t = t0 + tt;
        const int ys = wrapg(y + tap_dy(t, dil));
        const int xs = wrapg(x0 + r + tap_dx(t, dil));
        const size_t px = img + ((size_t)ys * kNetG + xs) * kNetC;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t wo = ((size_t)r * 9 + t) * kNetC + 16 * h + 8 * hk;
            const bf16x8 bv = load8(w + wo);
            const bf16x8 av = load8(in + px + 16 * h + 8 * hk);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            if (in_lo)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(in_lo + px + 16 * h + 8 * hk), bv, acc, 0, 0, 0);
            if (w_lo)  // the weights' low parts (hi activations; lo x lo is below the FP32 sums' rounding)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, load8(w_lo + wo), acc, 0, 0, 0);
        }
    }
    if constexpr (SPLIT > 1) {
        __shared__ float part[SPLIT - 1][16][64];
        if (wib > 0)
#pragma unroll
            for (int j = 0; j < 16; ++j) part[wib - 1][j][lane] = acc[j];
        __syncthreads();
        if (wib > 0) return;
#pragma unroll
        for (int s = 0; s < SPLIT - 1; ++s)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] += part[s][j][lane];
    }
    const size_t o = (((size_t)b * kNetG + y) * kNetG + x0) * kNetC;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j / 4) + 4 * hk + (j % 4);  // pixel within the tile
        const __bf16 hi = (__bf16)acc[j];
        out[o + (size_t)row * kNetC + r] = hi;
        if (out_lo) out_lo[o + (size_t)row * kNetC + r] = (__bf16)(acc[j] - (float)hi);
    }
}

template __global__ void k_conv32<1>(const __bf16 *, const __bf16 *, const __bf16 *, const __bf16 *, __bf16 *,
                                      __bf16 *, int, int);
template __global__ void k_conv32<3>(const __bf16 *, const __bf16 *, const __bf16 *, const __bf16 *, __bf16 *,
                                      __bf16 *, int, int);

// Weight gradient of a 32 -> 32 layer:
//   dw[co][tap][ci] = sum_{b, y, x} g[b][y][x][co] * in[b][y + dy][x + dx][ci]
// K runs over pixels, which are the strided dimension of the pixel-major
// layout, so each operand tile (16 pixels x 32 channels, 1 KB) is loaded with
// one 16-byte load per lane (pixel l / 4, channels 8 (l % 4) ..), stored
// transposed in the wave's own LDS slot ([channel][pixel]) and read back as one
// 16-byte LDS load per lane (channel l % 32, pixels 8 (l / 32) ..).  Runs of 16
// pixels start at multiples of 16, so a run lies in one row; shifted runs wrap
// pixel by pixel.  Three wavefronts share a chunk of `chunk` pixels (a
// multiple of 16), one per row of three taps, and write the chunk's
// 9 x 32 x 32 partial sums; the next run's tiles load during this run's
// products.
namespace {
// Order this wave's LDS writes before its later LDS reads of other lanes'
// data (a wave's LDS operations complete in issue order; this keeps the
// compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ void store_transposed(__bf16 (*tile)[16], int px, int cg, bf16x8 v) {
#pragma unroll
    for (int j = 0; j < 8; ++j) tile[cg + j][px] = v[j];
}
}  // namespace

__global__ __launch_bounds__(256) void k_conv32_wgrad(const __bf16 *__restrict__ g, const __bf16 *__restrict__ in,
                                                      float *__restrict__ part, int npix, int chunk, int dil) {
    __shared__ __attribute__((aligned(16))) __bf16 lds[4][4][kNetC][16];
    const int lane = threadIdx.x & 63;
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wave = xcd_block() * 4 + wl;
    const int nchunks = (npix + chunk - 1) / chunk;
    if (wave >= 3 * nchunks) return;
    const int ck = wave / 3, trow = wave - 3 * ck;  // pixel chunk, tap row (taps 3 trow .. 3 trow + 2)
    __bf16(*tl)[kNetC][16] = lds[wl];              // tile 0: g, tiles 1..3: shifted inputs
    const int r = lane & 31, hk = lane >> 5;        // operand lane roles
    const int px = lane >> 2, cg = 8 * (lane & 3);  // loader lane roles
    f32x16 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = f32x16{};
    const int p0 = ck * chunk;
    const int p1 = min(p0 + chunk, npix);
    bf16x8 v[4];
    auto load_run = [&](int p) {
        const int bb = p / (kNetG * kNetG);
        const int rem = p - bb * kNetG * kNetG;
        const int y = rem / kNetG, x0 = rem % kNetG;
        const __bf16 *img = in + (size_t)bb * kNetG * kNetG * kNetC;
        v[0] = load8(g + (size_t)(p + px) * kNetC + cg);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int t = 3 * trow + k;
            const int ys = wrapg(y + tap_dy(t, dil));
            const int xs = wrapg(x0 + px + tap_dx(t, dil));
            v[1 + k] = load8(img + ((size_t)ys * kNetG + xs) * kNetC + cg);
        }
    };
    load_run(p0);
    for (int p = p0; p < p1; p += 16) {
        wave_lds_sync();  // the previous run's operand reads are done before the tiles are rewritten
#pragma unroll
        for (int k = 0; k < 4; ++k) store_transposed(tl[k], px, cg, v[k]);
        if (p + 16 < p1) load_run(p + 16);  // next run's tiles in flight during this run's products
        wave_lds_sync();
        const bf16x8 av = load8(&tl[0][r][8 * hk]);  // A (32 co x 16 px)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const bf16x8 bv = load8(&tl[1 + k][r][8 * hk]);  // B (16 px x 32 ci)
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[k], 0, 0, 0);
        }
    }
    float *o = part + (size_t)ck * 9 * kNetC * kNetC;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int co = 8 * (j / 4) + 4 * hk + (j % 4);
            o[((size_t)co * 9 + 3 * trow + k) * kNetC + r] = acc[k][j];
        }
}

// out[i] = sum over `count` partial vectors of length len, in a fixed order.
__global__ void k_sum_partials(const float *__restrict__ part, int count, int len, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int k = 0; k < count; ++k) s += part[(size_t)k * len + i];
    out[i] = s;
}

// Partial sums, first stage: out[grp][i] = sum of partials k = grp, grp + groups, ...
// (grid: x over i, y over groups); the second stage is k_sum_partials over the groups.
__global__ void k_sum_partials_grouped(const float *__restrict__ part, int count, int len, int groups,
                                       float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = blockIdx.y;
    if (i >= len) return;
    float s = 0.f;
    for (int k = grp; k < count; k += groups) s += part[(size_t)k * len + i];
    out[(size_t)grp * len + i] = s;
}

// wt[ci][tap][co] = w[co][8 - tap][ci]: the input gradient of a layer is the
// same convolution with these weights applied to the output gradient.
__global__ void k_transpose_flip(const __bf16 *__restrict__ w, __bf16 *__restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNetC * 9 * kNetC) return;
    const int ci = i / (9 * kNetC), t = (i / kNetC) % 9, co = i % kNetC;
    wt[i] = w[((size_t)co * 9 + (8 - t)) * kNetC + ci];
}

// First layer (1 -> 32): one thread per pixel; FP32 input and weights, the
// output as a BF16 (hi, lo) pair.
__global__ void k_conv_in(const float *__restrict__ x, const float *__restrict__ w1, __bf16 *__restrict__ out,
                          __bf16 *__restrict__ out_lo, int nb, int dil) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb * kNetG * kNetG) return;
    const int b = q / (kNetG * kNetG), rem = q - b * kNetG * kNetG, y = rem / kNetG, xx = rem % kNetG;
    float v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        v[t] = x[((size_t)b * kNetG + wrapg(y + tap_dy(t, dil))) * kNetG + wrapg(xx + tap_dx(t, dil))];
    // the pixel's 32 channels (64 B each for hi and lo) as 16-byte stores
#pragma unroll
    for (int c8 = 0; c8 < kNetC; c8 += 8) {
        bf16x8 h8, l8;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int co = c8 + k;
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) s += w1[co * 9 + t] * v[t];
            const __bf16 hi = (__bf16)s;
            h8[k] = hi;
            l8[k] = (__bf16)(s - (float)hi);
        }
        *reinterpret_cast<bf16x8 *>(out + (size_t)q * kNetC + c8) = h8;
        *reinterpret_cast<bf16x8 *>(out_lo + (size_t)q * kNetC + c8) = l8;
    }
}

// Last layer (32 -> 1): one thread per pixel, (hi + lo) activations, FP32
// weights and output.
__global__ void k_conv_out(const __bf16 *__restrict__ in, const __bf16 *__restrict__ in_lo,
                           const float *__restrict__ w6, float *__restrict__ y, int nb, int dil) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb * kNetG * kNetG) return;
    const int b = q / (kNetG * kNetG), rem = q - b * kNetG * kNetG, yy = rem / kNetG, xx = rem % kNetG;
    float s = 0.f;
#pragma unroll 3
    for (int t = 0; t < 9; ++t) {
        const size_t px =
            (((size_t)b * kNetG + wrapg(yy + tap_dy(t, dil))) * kNetG + wrapg(xx + tap_dx(t, dil))) * kNetC;
        // the neighbour's 32 channels as four 16-byte loads of hi and of lo;
        // the sum runs over ci in order as before
        bf16x8 h8[4], l8[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h8[c] = load8(in + px + 8 * c);
            l8[c] = load8(in_lo + px + 8 * c);
        }
#pragma unroll
        for (int ci = 0; ci < kNetC; ++ci)
            s += w6[t * kNetC + ci] * ((float)h8[ci >> 3][ci & 7] + (float)l8[ci >> 3][ci & 7]);
    }
    y[q] = s;
}

// Input gradient of the last layer: g[b][p][ci] = sum_tap w6[tap][ci] * dy[b][p - off(tap)].
__global__ void k_conv_out_bwd(const float *__restrict__ dy, const float *__restrict__ w6, __bf16 *__restrict__ g,
                               int nb, int dil) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb * kNetG * kNetG) return;
    const int b = q / (kNetG * kNetG), rem = q - b * kNetG * kNetG, yy = rem / kNetG, xx = rem % kNetG;
    float d[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        d[t] = (float)(__bf16)dy[((size_t)b * kNetG + wrapg(yy - tap_dy(t, dil))) * kNetG + wrapg(xx - tap_dx(t, dil))];
#pragma unroll
    for (int c8 = 0; c8 < kNetC; c8 += 8) {  // 16-byte stores of 8 channels
        bf16x8 g8;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) s += (float)(__bf16)w6[t * kNetC + c8 + k] * d[t];
            g8[k] = (__bf16)s;
        }
        *reinterpret_cast<bf16x8 *>(g + (size_t)q * kNetC + c8) = g8;
    }
}

// Weight gradients of the 1-channel layers, per-block partials:
//   mode 0 (first layer): part[blk][co][tap] = sum_p g[p][co] * x[p + off(tap)]
//   mode 1 (last layer):  part[blk][tap][ci] = sum_p dy[p] * in[p + off(tap)][ci]
// (in = act + act_lo, the activation pair).
// 256 threads: channel c = thread % 32, pixel group = thread / 32 (8 groups).
__global__ __launch_bounds__(256) void k_wgrad_small(int mode, const __bf16 *__restrict__ act,
                                                     const __bf16 *__restrict__ act_lo,
                                                     const float *__restrict__ vec, float *__restrict__ part,
                                                     int npix, int chunk, int dil) {
    __shared__ float red[8][9 * kNetC];
    const int c = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, npix);
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.f;
    for (int q = p0 + grp; q < p1; q += 8) {
        const int b = q / (kNetG * kNetG), rem = q - b * kNetG * kNetG, yy = rem / kNetG, xx = rem % kNetG;
        if (mode == 0) {
            const float gv = (float)act[(size_t)q * kNetC + c];
#pragma unroll
            for (int t = 0; t < 9; ++t)
                acc[t] += gv * vec[((size_t)b * kNetG + wrapg(yy + tap_dy(t, dil))) * kNetG +
                                   wrapg(xx + tap_dx(t, dil))];
        } else {
            const float dv = (float)(__bf16)vec[q];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const size_t a = (((size_t)b * kNetG + wrapg(yy + tap_dy(t, dil))) * kNetG +
                                  wrapg(xx + tap_dx(t, dil))) * kNetC + c;
                acc[t] += dv * ((float)act[a] + (float)act_lo[a]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) red[grp][t * kNetC + c] = acc[t];
    __syncthreads();
    for (int i = threadIdx.x; i < 9 * kNetC; i += 256) {
        float s = 0.f;
        for (int k = 0; k < 8; ++k) s += red[k][i];
        const int t = i / kNetC, ch = i % kNetC;
        // mode 0 stores [co][tap], mode 1 [tap][ci]
        part[(size_t)blockIdx.x * 9 * kNetC + (mode == 0 ? ch * 9 + t : t * kNetC + ch)] = s;
    }
}

// Mean squared error: dy = 2 (y - t) / count, and per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                             float *__restrict__ dy, double *__restrict__ part, int count) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const float e = y[i] - t[i];
        dy[i] = 2.f * e / (float)count;
        s += (double)e * (double)e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_finish(const double *__restrict__ part, int blocks, int count, float *__restrict__ loss) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < blocks; ++i) s += part[i];
        *loss = (float)(s / count);
    }
}

// Adam on FP32 master weights; refreshes the BF16 copy of the 32 -> 32 layers.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, __bf16 *__restrict__ w16, int count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    w16[i] = (__bf16)wi;
}

// BF16 copy of the weights as a (hi, lo) pair: hi = bf16(a), lo = bf16(a - hi).
__global__ void k_to_bf16(const float *__restrict__ a, __bf16 *__restrict__ b, __bf16 *__restrict__ lo, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const __bf16 h = (__bf16)a[i];
        b[i] = h;
        if (lo) lo[i] = (__bf16)(a[i] - (float)h);
    }
}

// Scale of a right-hand side: its RMS over the valid cells, sqrt(sum f^2 / n^2);
// 1 when no statistics are given.
__device__ __forceinline__ double rms_scale(const double *sumsq, int n) {
    if (!sumsq) return 1.0;
    const double s = sqrt(*sumsq / ((double)n * (double)n));
    return s > 0.0 ? s : 1.0;
}

// Encoder: out[y][x] = mean of the r x r block of f (FP64, ghosted, pitch) / scale,
// with r = n / G (a mean of four-cell means is this block mean).  A workgroup
// covers 64 blocks of one block row; its four waves take every fourth fine
// row, each lane summing its block's r columns (a wave reads 64 r contiguous
// values per row), and the four row sums meet in LDS.
__global__ __launch_bounds__(256) void k_encode(const double *__restrict__ f, long pitch, int n,
                                                const double *__restrict__ sumsq, float *__restrict__ out) {
    __shared__ double red[4][64];
    const int xi = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + xi, y = blockIdx.y;
    const int r = n / kNetG;
    double s = 0.0;
    for (int j = ph; j < r; j += 4) {
        const double *row = f + (long)(y * r + j + 1) * pitch + 1 + (long)x * r;
        for (int i = 0; i < r; ++i) s += row[i];
    }
    red[ph][xi] = s;
    __syncthreads();
    if (ph == 0) {
        const double t = (red[0][xi] + red[1][xi]) + (red[2][xi] + red[3][xi]);
        out[y * kNetG + x] = (float)(t / ((double)r * r) / rms_scale(sumsq, n));
    }
}

// Decoder, first step: the network output on the G x G grid in physical units
// (times the RMS of f when given, and the square of the domain side), then
// `iters` red-black Gauss-Seidel iterations of the periodic Poisson problem
// Lap u = f on that grid against the encoded right-hand side (x times the
// RMS), red ((row + column) even) first, which remove the grid-scale noise of
// the network output.  FP32 (it is only a guess).  One workgroup of 1024
// threads, each keeping a 4 x 4 block in registers and exchanging only block
// edges through LDS.  Output: G x G FP64 (no ghosts).
// LDS layout of the G x G grid: one pad word after every 4 columns and rows of
// kRelaxRow words, so that the 64 lanes of a wave (32 blocks across, 2 block
// rows down) reading or writing one edge cell each hit 64 different banks
// (a plain 128-word row put them on far fewer).
constexpr int kRelaxB = 4;
constexpr int kRelaxRow = 168;
__device__ __forceinline__ int relax_at(int r, int c) { return r * kRelaxRow + c + (c >> 2); }

__global__ __launch_bounds__(kRelaxThreads) void k_coarse_relax(const float *__restrict__ y,
                                                                const float *__restrict__ x,
                                                                const double *__restrict__ sumsq, int nfine,
                                                                double length, int iters,
                                                                double *__restrict__ out) {
    constexpr int B = kRelaxB, NB = kNetG / B, m = kNetG - 1;  // 32 x 32 blocks of 4 x 4 cells
    static_assert(NB * NB <= kRelaxThreads, "one block per thread");
    __shared__ float u[kNetG * kRelaxRow];
    const int t = threadIdx.x;
    const double rms = rms_scale(sumsq, nfine);
    const float su = (float)(rms * length * length);
    const float h2 = (float)(length * length / ((double)kNetG * kNetG));
    for (int q = t; q < kNetG * kNetG; q += kRelaxThreads) u[relax_at(q / kNetG, q % kNetG)] = y[q] * su;
    __syncthreads();
    if (t < NB * NB) {
        const int R0 = B * (t / NB), C0 = B * (t % NB);  // block origin (even: block parity = global parity)
        float v[B][B], hf[B][B];
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int j = 0; j < B; ++j) {
                v[i][j] = u[relax_at(R0 + i, C0 + j)];
                hf[i][j] = -h2 * (float)(x[(R0 + i) * kNetG + C0 + j] * rms);
            }
        const int up = (R0 - 1) & m, dn = (R0 + B) & m, lf = (C0 - 1) & m, rt = (C0 + B) & m;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // updates of colour c: neighbours inside the block from registers,
                // outside from the edges the neighbouring blocks published
#pragma unroll
                for (int i = 0; i < B; ++i)
#pragma unroll
                    for (int j = 0; j < B; ++j) {
                        if (((i + j) & 1) != c) continue;
                        const float w = j > 0 ? v[i][j - 1] : u[relax_at(R0 + i, lf)];
                        const float e = j < B - 1 ? v[i][j + 1] : u[relax_at(R0 + i, rt)];
                        const float nn = i > 0 ? v[i - 1][j] : u[relax_at(up, C0 + j)];
                        const float ss = i < B - 1 ? v[i + 1][j] : u[relax_at(dn, C0 + j)];
                        v[i][j] = 0.25f * (hf[i][j] + ((e + w) + (ss + nn)));  // u = (sum - h^2 f) / 4
                    }
                // publish the updated edge cells
#pragma unroll
                for (int i = 0; i < B; ++i)
#pragma unroll
                    for (int j = 0; j < B; ++j) {
                        if (((i + j) & 1) != c) continue;
                        if (i == 0 || i == B - 1 || j == 0 || j == B - 1) u[relax_at(R0 + i, C0 + j)] = v[i][j];
                    }
                __syncthreads();
            }
        }
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int j = 0; j < B; ++j) u[relax_at(R0 + i, C0 + j)] = v[i][j];
    } else {
        for (int it = 0; it < 2 * iters; ++it) __syncthreads();  // keep the barrier count of the relaxing threads
    }
    __syncthreads();
    for (int q = t; q < kNetG * kNetG; q += kRelaxThreads) out[q] = (double)u[relax_at(q / kNetG, q % kNetG)];
}

// Decoder step: one multigrid prolongation (centred slopes, no xy term,
// periodic) from an nc x nc FP64 grid (no ghosts) to 2nc x 2nc, written plain
// (out_pitch = 2nc) or into the valid cells of a ghosted field.
__global__ void k_decode_step(const double *__restrict__ c, int nc, double *__restrict__ fine, long out_pitch,
                              int ghosted) {
    const int n = 2 * nc;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * n) return;
    const int y = q / n, x = q % n, I = x >> 1, J = y >> 1, m = nc - 1;
    auto at = [&](int jj, int ii) -> double { return c[(jj & m) * nc + (ii & m)]; };
    const double e = at(J, I);
    const double mx = 0.5 * (at(J, I + 1) - at(J, I - 1)), my = 0.5 * (at(J + 1, I) - at(J - 1, I));
    const double dx = (x & 1) ? 0.25 : -0.25, dy = (y & 1) ? 0.25 : -0.25;
    const double v = (e + dx * mx) + dy * my;
    if (ghosted) fine[(long)(y + 1) * out_pitch + x + 1] = v;
    else fine[q] = v;
}


}  // namespace ccmg
