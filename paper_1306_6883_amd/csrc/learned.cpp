// learned.cpp -- host side of the learned initial guess: the network object,
// its training step (forward, mean squared error, backward through every layer,
// Adam) and the guess for a fine right-hand side (encode, network, decode).
// Kernels in learned.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "learned.h"

using namespace ccmg;

namespace {

constexpr int kPix = kNetG * kNetG;
constexpr int kWgChunk = 1024;    // pixels per wavefront of the MFMA weight gradient
constexpr int kSmallChunk = 512;  // pixels per workgroup of the 1-channel weight gradients
constexpr int kSumGroups = 32;    // first-stage groups of the partial-sum reduction
constexpr int kLossBlocks = 256;
// A guess whose relative residual exceeds this is discarded (zero guess instead).
constexpr double kGuessReject = 1e6;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct NetLayout {
    size_t w, m, v, grad, w16, w16lo, wt16, act, g0, g1, y, dy, part, part2, lpart, loss, x1, y1, dec0, dec1, stats, fpart;
    size_t total;
};

NetLayout net_layout(int batch, int nmax) {
    NetLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = al(off + b);
        return o;
    };
    const size_t npix = (size_t)batch * kPix;
    L.w = take(sizeof(float) * kNetParams);
    L.m = take(sizeof(float) * kNetParams);
    L.v = take(sizeof(float) * kNetParams);
    L.grad = take(sizeof(float) * kNetParams);
    L.w16 = take(2 * (size_t)kNetParams);
    L.w16lo = take(2 * (size_t)kNetParams);
    L.wt16 = take(2 * (size_t)4 * kWmid);
    L.act = take(2 * npix * kNetC * 10);  // a1 .. a5 (hi), then a1 .. a5 (lo)
    L.g0 = take(2 * npix * kNetC);
    L.g1 = take(2 * npix * kNetC);
    L.y = take(sizeof(float) * npix);
    L.dy = take(sizeof(float) * npix);
    const size_t wg_waves = (npix + kWgChunk - 1) / kWgChunk;
    const size_t sm_blocks = (npix + kSmallChunk - 1) / kSmallChunk;
    L.part = take(sizeof(float) * std::max(wg_waves * kWmid, sm_blocks * kW0));
    L.part2 = take(sizeof(float) * kSumGroups * kWmid);
    L.lpart = take(sizeof(double) * kLossBlocks);
    L.loss = take(sizeof(float) * 4);
    L.x1 = take(sizeof(float) * kPix);
    L.y1 = take(sizeof(float) * kPix);
    const size_t nm = (size_t)std::max(nmax, kNetG);
    L.dec0 = take(sizeof(double) * nm * nm);
    L.dec1 = take(sizeof(double) * nm * nm);
    L.stats = take(sizeof(double) * 8);
    L.fpart = take(sizeof(double) * 4 * 512);
    L.total = off;
    return L;
}

}  // namespace

struct ccmg_net {
    int batch = 0, nmax = 0;
    NetLayout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timing of the learned solve
    int step = 0;

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    float *w() const { return at<float>(L.w); }
    __bf16 *w16() const { return at<__bf16>(L.w16); }
    __bf16 *act(int i) const { return at<__bf16>(L.act) + (size_t)i * batch * kPix * kNetC; }  // a1 = act(0)
    __bf16 *act_lo(int i) const { return act(5 + i); }
};

namespace {

int hs(hipError_t e) { return e == hipSuccess ? CCMG_OK : CCMG_EHIP; }

hipError_t refresh_bf16(ccmg_net *N) {
    hipLaunchKernelGGL(k_to_bf16, dim3((kNetParams + 255) / 256), dim3(256), 0, N->stream, N->w(), N->w16(),
                       N->at<__bf16>(N->L.w16lo), kNetParams);
    for (int l = 1; l <= 4; ++l)
        hipLaunchKernelGGL(k_transpose_flip, dim3((kWmid + 255) / 256), dim3(256), 0, N->stream,
                           N->w16() + net_param_offset(l), N->at<__bf16>(N->L.wt16) + (size_t)(l - 1) * kWmid);
    return hipGetLastError();
}

// Forward through the six layers: x (nb x G x G, FP32) -> y (FP32); keeps the
// activation pairs a1..a5.
hipError_t forward(ccmg_net *N, const float *x, float *y, int nb) {
    hipStream_t s = N->stream;
    const int npix = nb * kPix;
    hipLaunchKernelGGL(k_conv_in, dim3((npix + 255) / 256), dim3(256), 0, s, x, N->w() + net_param_offset(0),
                       N->act(0), N->act_lo(0), nb, net_dilation(0));
    const int waves = nb * kNetG * (kNetG / 32);
    for (int l = 1; l <= 4; ++l) {
        const __bf16 *wl = N->w16() + net_param_offset(l), *wlo = N->at<__bf16>(N->L.w16lo) + net_param_offset(l);
        if (nb <= kConvSplitMaxBatch)  // too few tiles for the GPU: three wavefronts per tile
            hipLaunchKernelGGL(k_conv32<3>, dim3(waves), dim3(192), 0, s, N->act(l - 1), N->act_lo(l - 1), wl, wlo,
                               N->act(l), N->act_lo(l), nb, net_dilation(l));
        else
            hipLaunchKernelGGL(k_conv32<1>, dim3((waves + 3) / 4), dim3(256), 0, s, N->act(l - 1),
                               N->act_lo(l - 1), wl, wlo, N->act(l), N->act_lo(l), nb, net_dilation(l));
    }
    hipLaunchKernelGGL(k_conv_out, dim3((npix + 255) / 256), dim3(256), 0, s, N->act(4), N->act_lo(4),
                       N->w() + net_param_offset(5), y, nb, net_dilation(5));
    return hipGetLastError();
}

// out[len] = sum of `count` partial vectors, in a fixed order (two stages).
void sum_partials(ccmg_net *N, const float *part, int count, int len, float *out) {
    const int groups = std::min(count, kSumGroups);
    float *p2 = N->at<float>(N->L.part2);
    hipLaunchKernelGGL(k_sum_partials_grouped, dim3((len + 255) / 256, groups), dim3(256), 0, N->stream, part, count,
                       len, groups, p2);
    hipLaunchKernelGGL(k_sum_partials, dim3((len + 255) / 256), dim3(256), 0, N->stream, p2, groups, len, out);
}

// Loss and gradients of all parameters into N->grad (after forward() on x).
hipError_t backward(ccmg_net *N, const float *x, const float *t, int nb) {
    hipStream_t s = N->stream;
    const int npix = nb * kPix;
    float *grad = N->at<float>(N->L.grad);
    float *part = N->at<float>(N->L.part);
    float *y = N->at<float>(N->L.y), *dy = N->at<float>(N->L.dy);
    hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(256), 0, s, y, t, dy, N->at<double>(N->L.lpart), npix);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(64), 0, s, N->at<double>(N->L.lpart), kLossBlocks, npix,
                       N->at<float>(N->L.loss));
    const int sm_blocks = (npix + kSmallChunk - 1) / kSmallChunk;
    // last layer: weights, then the gradient of a5
    hipLaunchKernelGGL(k_wgrad_small, dim3(sm_blocks), dim3(256), 0, s, 1, N->act(4), N->act_lo(4), dy, part, npix,
                       kSmallChunk, net_dilation(5));
    sum_partials(N, part, sm_blocks, kW5, grad + net_param_offset(5));
    __bf16 *gcur = N->at<__bf16>(N->L.g0), *gnext = N->at<__bf16>(N->L.g1);
    hipLaunchKernelGGL(k_conv_out_bwd, dim3((npix + 255) / 256), dim3(256), 0, s, dy, N->w() + net_param_offset(5),
                       gcur, nb, net_dilation(5));
    // layers 4 .. 1 (32 -> 32): weight gradient from (g, input activation), then g of the input
    const int wg_waves = (npix + kWgChunk - 1) / kWgChunk;
    const int cv_waves = nb * kNetG * (kNetG / 32);
    for (int l = 4; l >= 1; --l) {
        hipLaunchKernelGGL(k_conv32_wgrad, dim3((3 * wg_waves + 3) / 4), dim3(256), 0, s, gcur, N->act(l - 1), part, npix,
                           kWgChunk, net_dilation(l));
        sum_partials(N, part, wg_waves, kWmid, grad + net_param_offset(l));
        hipLaunchKernelGGL(k_conv32<1>, dim3((cv_waves + 3) / 4), dim3(256), 0, s, gcur, (const __bf16 *)nullptr,
                           N->at<__bf16>(N->L.wt16) + (size_t)(l - 1) * kWmid, (const __bf16 *)nullptr, gnext, (__bf16 *)nullptr, nb,
                           net_dilation(l));
        std::swap(gcur, gnext);
    }
    // first layer: weights only (its input is data)
    hipLaunchKernelGGL(k_wgrad_small, dim3(sm_blocks), dim3(256), 0, s, 0, gcur, (const __bf16 *)nullptr, x, part,
                       npix, kSmallChunk, net_dilation(0));
    sum_partials(N, part, sm_blocks, kW0, grad + net_param_offset(0));
    return hipGetLastError();
}

}  // namespace

extern "C" {

int ccmg_net_param_count(void) { return kNetParams; }

size_t ccmg_net_workspace_bytes(int batch, int n_max) {
    if (batch < 1 || batch > 1024 || n_max < kNetG || n_max > 16384 || (n_max & (n_max - 1))) return 0;
    return net_layout(batch, n_max).total;
}

int ccmg_net_create(int batch, int n_max, void *d_ws, size_t ws_bytes, void *stream, ccmg_net **out) {
    if (!out) return CCMG_EINVAL;
    *out = nullptr;
    const size_t need = ccmg_net_workspace_bytes(batch, n_max);
    if (need == 0) return CCMG_EINVAL;
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return CCMG_EWORKSPACE;
    ccmg_net *N = new (std::nothrow) ccmg_net();
    if (!N) return CCMG_EINVAL;
    N->batch = batch;
    N->nmax = n_max;
    N->L = net_layout(batch, n_max);
    N->ws = static_cast<char *>(d_ws);
    N->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemsetAsync(N->ws, 0, N->L.total, N->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    if (e == hipSuccess) e = hipEventCreate(&N->ev0);
    if (e == hipSuccess) e = hipEventCreate(&N->ev1);
    if (e != hipSuccess) {
        ccmg_net_destroy(N);
        return CCMG_EHIP;
    }
    *out = N;
    return CCMG_OK;
}

int ccmg_net_destroy(ccmg_net *N) {
    if (!N) return CCMG_EINVAL;
    if (N->ev0) hipEventDestroy(N->ev0);
    if (N->ev1) hipEventDestroy(N->ev1);
    delete N;
    return CCMG_OK;
}

int ccmg_net_set_params(ccmg_net *N, const float *d_params) {
    if (!N || !d_params) return CCMG_EINVAL;
    hipError_t e = hipMemcpyAsync(N->w(), d_params, sizeof(float) * kNetParams, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess) e = hipMemsetAsync(N->at<float>(N->L.m), 0, sizeof(float) * kNetParams, N->stream);
    if (e == hipSuccess) e = hipMemsetAsync(N->at<float>(N->L.v), 0, sizeof(float) * kNetParams, N->stream);
    if (e == hipSuccess) e = refresh_bf16(N);
    N->step = 0;
    return hs(e);
}

int ccmg_net_state_count(void) { return 3 * kNetParams; }

int ccmg_net_get_state(ccmg_net *N, float *d_state, int *step) {
    if (!N || !d_state || !step) return CCMG_EINVAL;
    const size_t b = sizeof(float) * kNetParams;
    hipError_t e = hipMemcpyAsync(d_state, N->w(), b, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_state + kNetParams, N->at<float>(N->L.m), b, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_state + 2 * kNetParams, N->at<float>(N->L.v), b, hipMemcpyDeviceToDevice, N->stream);
    *step = N->step;
    return hs(e);
}

int ccmg_net_set_state(ccmg_net *N, const float *d_state, int step) {
    if (!N || !d_state || step < 0) return CCMG_EINVAL;
    const size_t b = sizeof(float) * kNetParams;
    hipError_t e = hipMemcpyAsync(N->w(), d_state, b, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(N->at<float>(N->L.m), d_state + kNetParams, b, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(N->at<float>(N->L.v), d_state + 2 * kNetParams, b, hipMemcpyDeviceToDevice, N->stream);
    if (e == hipSuccess) e = refresh_bf16(N);
    if (e == hipSuccess) N->step = step;
    return hs(e);
}

int ccmg_net_get_params(ccmg_net *N, float *d_params) {
    if (!N || !d_params) return CCMG_EINVAL;
    return hs(hipMemcpyAsync(d_params, N->w(), sizeof(float) * kNetParams, hipMemcpyDeviceToDevice, N->stream));
}

int ccmg_net_forward(ccmg_net *N, const float *d_x, float *d_y, int nb) {
    if (!N || !d_x || !d_y || nb < 1 || nb > N->batch) return CCMG_EINVAL;
    return hs(forward(N, d_x, d_y, nb));
}

int ccmg_net_loss_grad(ccmg_net *N, const float *d_x, const float *d_t, int nb, float *d_grad, float *loss) {
    if (!N || !d_x || !d_t || nb < 1 || nb > N->batch) return CCMG_EINVAL;
    hipError_t e = forward(N, d_x, N->at<float>(N->L.y), nb);
    if (e == hipSuccess) e = backward(N, d_x, d_t, nb);
    if (e == hipSuccess && d_grad)
        e = hipMemcpyAsync(d_grad, N->at<float>(N->L.grad), sizeof(float) * kNetParams, hipMemcpyDeviceToDevice,
                           N->stream);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, N->at<float>(N->L.loss), sizeof(float), hipMemcpyDeviceToHost, N->stream);
    if (e == hipSuccess && loss) e = hipStreamSynchronize(N->stream);
    return hs(e);
}

int ccmg_net_train_step(ccmg_net *N, const float *d_x, const float *d_t, int nb, float lr, float *loss) {
    if (!N || !d_x || !d_t || nb < 1 || nb > N->batch || !(lr > 0)) return CCMG_EINVAL;
    int st = ccmg_net_loss_grad(N, d_x, d_t, nb, nullptr, nullptr);
    if (st != CCMG_OK) return st;
    N->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)N->step), c2 = 1.f - std::pow(b2, (float)N->step);
    hipLaunchKernelGGL(k_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, N->stream, N->w(),
                       N->at<float>(N->L.grad), N->at<float>(N->L.m), N->at<float>(N->L.v), N->w16(), kNetParams, lr,
                       b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = refresh_bf16(N);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, N->at<float>(N->L.loss), sizeof(float), hipMemcpyDeviceToHost, N->stream);
    if (e == hipSuccess && loss) e = hipStreamSynchronize(N->stream);
    return hs(e);
}

// Encoder: block means of `a` (n x n, ghosted FP64) on the G x G grid, divided
// by the RMS of `scale_src` (the right-hand side the sample belongs to).
int ccmg_net_encode(ccmg_net *N, const double *d_a, ptrdiff_t pitch, int n, const double *d_scale_src,
                    ptrdiff_t scale_pitch, float *d_x) {
    if (!N || !d_a || !d_scale_src || !d_x || n < kNetG || n > N->nmax || (n & (n - 1)) || pitch < n + 2 ||
        scale_pitch < n + 2)
        return CCMG_EINVAL;
    double *stats = N->at<double>(N->L.stats);
    hipError_t e = launch_fstats(d_scale_src, scale_pitch, n, N->at<double>(N->L.fpart), 512, stats, N->stream);
    if (e != hipSuccess) return CCMG_EHIP;
    hipLaunchKernelGGL(k_encode, dim3(kNetG / 64, kNetG), dim3(256), 0, N->stream, d_a, (long)pitch, n, stats + 2,
                       d_x);
    return hs(hipGetLastError());
}

// The initial guess for f (n x n, ghosted FP64): encode, network, relaxation
// on the network's grid, prolongations to n x n, the last one into the valid
// cells of d_phi (the solver applies the
// side rules itself and removes the mean of singular problems).  The network
// is linear without biases, so the RMS normalisation used in training cancels
// here and is skipped: net(x / s) s = net(x).
int ccmg_net_guess(ccmg_net *N, const double *d_f, ptrdiff_t pitch, int n, double length, int coarse_iters,
                   double *d_phi, ptrdiff_t phi_pitch) {
    if (!N || !d_f || !d_phi || n < 2 * kNetG || n > N->nmax || (n & (n - 1)) || pitch < n + 2 ||
        phi_pitch < n + 2 || !(length > 0) || !std::isfinite(length) || coarse_iters < 0 || coarse_iters > 64)
        return CCMG_EINVAL;
    hipStream_t s = N->stream;
    float *x1 = N->at<float>(N->L.x1), *y1 = N->at<float>(N->L.y1);
    hipLaunchKernelGGL(k_encode, dim3(kNetG / 64, kNetG), dim3(256), 0, s, d_f, (long)pitch, n,
                       (const double *)nullptr, x1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = forward(N, x1, y1, 1);
    double *bufs[2] = {N->at<double>(N->L.dec0), N->at<double>(N->L.dec1)};
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_coarse_relax, dim3(1), dim3(kRelaxThreads), 0, s, y1, x1, (const double *)nullptr, n,
                           length, coarse_iters, bufs[1]);
        e = hipGetLastError();
    }
    const double *src = bufs[1];
    for (int nc = kNetG, k = 0; e == hipSuccess && nc < n; nc *= 2, ++k) {
        const bool last = 2 * nc == n;
        double *dst = last ? d_phi : bufs[k & 1];
        hipLaunchKernelGGL(k_decode_step, dim3((4 * nc * nc + 255) / 256), dim3(256), 0, s, src, nc, dst,
                           last ? (long)phi_pitch : (long)(2 * nc), last ? 1 : 0);
        e = hipGetLastError();
        src = dst;
    }
    return hs(e);
}

// Learned solve: guess, then plain multigrid from it to the plan's tolerance;
// a guess that is not finite or absurdly large is replaced by zero.
int ccmg_solve_learned(ccmg_plan *P, ccmg_net *N, const double *d_f, double *d_phi, ptrdiff_t pitch,
                       int coarse_iters, ccmg_result *out, int *guess_used) {
    ccmg_result local;
    ccmg_result *R = out ? out : &local;
    std::memset(R, 0, sizeof(*R));
    if (guess_used) *guess_used = 0;
    if (!P || !N || !d_f || !d_phi) return R->status = CCMG_EINVAL;
    const int n = plan_n(P);
    const ccmg_problem *pr = plan_problem(P);
    const double lx = pr->xmax - pr->xmin, ly = pr->ymax - pr->ymin;
    // the network is trained on doubly periodic Poisson problems (circular
    // padding, periodic decoder): nothing else is accepted
    bool periodic = true;
    for (int q = 0; q < 4; ++q) periodic = periodic && pr->bc[q] == CCMG_BC_PERIODIC;
    if (plan_stream(P) != N->stream || n < 2 * kNetG || n > N->nmax || pr->alpha != 0.0 || pr->beta != -1.0 ||
        std::fabs(lx - ly) > 1e-12 * lx || !periodic)
        return R->status = CCMG_EINVAL;
    hipError_t e = hipEventRecord(N->ev0, N->stream);
    int st = e == hipSuccess ? ccmg_net_guess(N, d_f, pitch, n, lx, coarse_iters, d_phi, pitch) : CCMG_EHIP;
    if (st != CCMG_OK) return R->status = st;
    st = solve_impl(P, d_f, d_phi, pitch, 1, R, kGuessReject);
    if (st == kGuessRejected) {
        const double rho_guess = R->rel_resid0;
        st = ccmg_solve(P, d_f, d_phi, pitch, 0, R);
        R->rel_resid0 = rho_guess;
    } else if (guess_used) {
        *guess_used = 1;
    }
    if (st == CCMG_EHIP || st == CCMG_EINVAL) return st;
    e = hipEventRecord(N->ev1, N->stream);
    if (e == hipSuccess) e = hipEventSynchronize(N->ev1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, N->ev0, N->ev1);
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    R->ms = ms;
    return st;
}

}  // extern "C"
