// learned.h -- shapes and kernels of the learned initial guess (learned.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ccmg {

constexpr int kNetG = 128;     // grid of the network
constexpr int kNetC = 32;      // channels of the hidden layers
constexpr int kNetLayers = 6;  // dilations 1, 2, 4, 8, 16, 32
// parameter blocks (FP32 master copy, contiguous):
//   layer 0: [32 co][9 tap]            layers 1..4: [32 co][9 tap][32 ci]
//   layer 5: [9 tap][32 ci]
constexpr int kW0 = kNetC * 9;
constexpr int kWmid = kNetC * 9 * kNetC;
constexpr int kW5 = 9 * kNetC;
constexpr int kNetParams = kW0 + 4 * kWmid + kW5;  // 37440
inline int net_param_offset(int layer) { return layer == 0 ? 0 : kW0 + (layer - 1) * kWmid; }
inline int net_dilation(int layer) { return 1 << layer; }

template <int SPLIT>
__global__ void k_conv32(const __bf16 *in, const __bf16 *in_lo, const __bf16 *w, const __bf16 *w_lo, __bf16 *out,
                         __bf16 *out_lo, int nb, int dil);
// batches of at most this many images run k_conv32<3> in the forward pass
constexpr int kConvSplitMaxBatch = 2;
__global__ void k_conv32_wgrad(const __bf16 *g, const __bf16 *in, float *part, int npix, int chunk, int dil);
__global__ void k_sum_partials(const float *part, int count, int len, float *out);
__global__ void k_sum_partials_grouped(const float *part, int count, int len, int groups, float *out);
__global__ void k_transpose_flip(const __bf16 *w, __bf16 *wt);
__global__ void k_conv_in(const float *x, const float *w1, __bf16 *out, __bf16 *out_lo, int nb, int dil);
__global__ void k_conv_out(const __bf16 *in, const __bf16 *in_lo, const float *w6, float *y, int nb, int dil);
__global__ void k_conv_out_bwd(const float *dy, const float *w6, __bf16 *g, int nb, int dil);
__global__ void k_wgrad_small(int mode, const __bf16 *act, const __bf16 *act_lo, const float *vec, float *part,
                              int npix, int chunk, int dil);
__global__ void k_mse(const float *y, const float *t, float *dy, double *part, int count);
__global__ void k_loss_finish(const double *part, int blocks, int count, float *loss);
__global__ void k_adam(float *w, const float *g, float *m, float *v, __bf16 *w16, int count, float lr, float b1,
                       float b2, float eps, float c1, float c2);
__global__ void k_to_bf16(const float *a, __bf16 *b, __bf16 *lo, int count);
__global__ void k_encode(const double *f, long pitch, int n, const double *sumsq, float *out);
constexpr int kRelaxThreads = 1024;
__global__ void k_coarse_relax(const float *y, const float *x, const double *sumsq, int nfine, double length,
                               int iters, double *out);
__global__ void k_decode_step(const double *c, int nc, double *fine, long out_pitch, int ghosted);

}  // namespace ccmg
