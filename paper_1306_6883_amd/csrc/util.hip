// util.hip -- small kernels around the V-cycle: ghost cells of the output,
// statistics of the right-hand side, and the fixed-order reductions that turn
// per-tile partial sums into the residual norm and the mean of phi.
#include "internal.h"

namespace ccmg {

namespace {
constexpr int kRed = 256;  // threads of the reduction kernels

__device__ double block_sum256(double v, double *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double side_sign(int b) { return b == CCMG_BC_DIRICHLET ? -1.0 : 1.0; }
}  // namespace

// Ghost cells from the valid cells: Dirichlet -v, Neumann +v, periodic the
// opposite valid cell.  One thread per boundary position k in [0, n): it writes
// the four ghosts (x-lo, x-hi of row k; y-lo, y-hi of column k).  When `shift`
// is given the valid cells were shifted by the caller's mean first.
__global__ void k_fill_ghosts(double *a, long pitch, int n, int b0, int b1, int b2, int b3) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double *row = a + (long)(k + 1) * pitch;
    const double lo = row[1], hi = row[n];
    row[0] = b0 == CCMG_BC_PERIODIC ? hi : side_sign(b0) * lo;
    row[n + 1] = b1 == CCMG_BC_PERIODIC ? lo : side_sign(b1) * hi;
    const double clo = a[pitch + 1 + k], chi = a[(long)n * pitch + 1 + k];
    a[1 + k] = b2 == CCMG_BC_PERIODIC ? chi : side_sign(b2) * clo;
    a[(long)(n + 1) * pitch + 1 + k] = b3 == CCMG_BC_PERIODIC ? clo : side_sign(b3) * chi;
}

// a[valid] -= *shift (singular problems: the zero-mean representative).
__global__ void k_shift(double *a, long pitch, int n, const double *shift) {
    const double m = *shift;
    const long total = (long)n * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const long y = i / n, x = i - y * n;
        a[(y + 1) * pitch + 1 + x] -= m;
    }
}

hipError_t launch_fill_ghosts_f64(double *a, long pitch, int n, const int bc[4], const double *shift,
                                  hipStream_t s) {
    if (shift) {
        const long total = (long)n * n;
        int blocks = (int)((total + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_shift, dim3(blocks), dim3(256), 0, s, a, pitch, n, shift);
    }
    hipLaunchKernelGGL(k_fill_ghosts, dim3((n + 255) / 256), dim3(256), 0, s, a, pitch, n, bc[0], bc[1],
                       bc[2], bc[3]);
    return hipGetLastError();
}

// End of a cycle (see internal.h).
__global__ __launch_bounds__(kRed) void k_cycle_end(const double *p, int count, int n, int singular,
                                                    const double *f2, double rtol, double *rho_out,
                                                    double *phi_mean, int *done, double *host_rho) {
    __shared__ double red[4];
    if (done && *done) return;  // uniform
    double s0 = 0.0, s1 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kRed < count; i += 4 * kRed) {  // four pairs in flight, added in order
        double2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const double2 *>(p + 2 * (i + k * kRed));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s0 += v[k].x;
            s1 += v[k].y;
        }
    }
    for (; i < count; i += kRed) {
        s0 += p[2 * i];
        s1 += p[2 * i + 1];
    }
    s0 = block_sum256(s0, red);
    s1 = block_sum256(s1, red);
    if (threadIdx.x == 0) {
        const double rho = sqrt(s0) / sqrt(*f2);
        *rho_out = rho;
        if (host_rho) *host_rho = rho;  // host-mapped: read by the host after the cycle's event
        *phi_mean = singular ? s1 / ((double)n * (double)n) : 0.0;
        if (done && (rho <= rtol || !isfinite(rho))) *done = 1;
    }
}

hipError_t launch_cycle_end(const double *partial, int count, int n, int singular, const double *f2,
                            double rtol, double *rho_out, double *phi_mean, int *done, double *host_rho,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_end, dim3(1), dim3(kRed), 0, s, partial, count, n, singular, f2, rtol,
                       rho_out, phi_mean, done, host_rho);
    return hipGetLastError();
}

// Statistics of f over valid cells: sum f, sum |f|, sum f^2, and the count of
// non-finite values.  Grid-stride over rows; per-block partials in out[4*block].
__global__ __launch_bounds__(kRed) void k_fstats(const double *f, long pitch, int n, double *out) {
    __shared__ double red[4];
    double s = 0.0, sa = 0.0, s2 = 0.0, bad = 0.0;
    auto add = [&](double v) {
        if (!isfinite(v)) {
            bad += 1.0;
            return;
        }
        s += v;
        sa += fabs(v);
        s2 += v * v;
    };
    for (int y = blockIdx.x; y < n; y += gridDim.x) {
        const double *row = f + (long)(y + 1) * pitch + 1;
        int x = threadIdx.x;
        for (; x + 3 * kRed < n; x += 4 * kRed) {  // four loads in flight, added in column order
            const double v0 = row[x], v1 = row[x + kRed], v2 = row[x + 2 * kRed], v3 = row[x + 3 * kRed];
            add(v0);
            add(v1);
            add(v2);
            add(v3);
        }
        for (; x < n; x += kRed) add(row[x]);
    }
    s = block_sum256(s, red);
    sa = block_sum256(sa, red);
    s2 = block_sum256(s2, red);
    bad = block_sum256(bad, red);
    if (threadIdx.x == 0) {
        out[4 * blockIdx.x + 0] = s;
        out[4 * blockIdx.x + 1] = sa;
        out[4 * blockIdx.x + 2] = s2;
        out[4 * blockIdx.x + 3] = bad;
    }
}

// The same statistics, and the four-cell restriction of f into `coarse`
// (level 1, pitch pc) from the same loads: grid-stride over coarse rows, each
// thread one coarse cell (two 16-byte loads per fine row pair), the mean
// formed in the order ((f(2I,2J) + f(2I+1,2J)) + f(2I,2J+1)) + f(2I+1,2J+1).
__global__ __launch_bounds__(kRed) void k_fstats_restrict(const double *f, long pitch, int n, double *out,
                                                          double *coarse, long pc) {
    __shared__ double red[4];
    double s = 0.0, sa = 0.0, s2 = 0.0, bad = 0.0;
    auto add = [&](double v) {
        if (!isfinite(v)) {
            bad += 1.0;
            return;
        }
        s += v;
        sa += fabs(v);
        s2 += v * v;
    };
    const int nc = n >> 1;
    for (int J = blockIdx.x; J < nc; J += gridDim.x) {
        const double *r0 = f + (long)(2 * J + 1) * pitch + 1;
        const double *r1 = r0 + pitch;
        double *c = coarse + (long)(J + 1) * pc + 1;
        for (int I = threadIdx.x; I < nc; I += kRed) {
            const double a = r0[2 * I], b = r0[2 * I + 1], d = r1[2 * I], e = r1[2 * I + 1];
            add(a);
            add(b);
            add(d);
            add(e);
            c[I] = 0.25 * (((a + b) + d) + e);
        }
    }
    s = block_sum256(s, red);
    sa = block_sum256(sa, red);
    s2 = block_sum256(s2, red);
    bad = block_sum256(bad, red);
    if (threadIdx.x == 0) {
        out[4 * blockIdx.x + 0] = s;
        out[4 * blockIdx.x + 1] = sa;
        out[4 * blockIdx.x + 2] = s2;
        out[4 * blockIdx.x + 3] = bad;
    }
}

__global__ __launch_bounds__(kRed) void k_reduce4(const double *p, int count, double *out4) {
    __shared__ double red[4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * kRed < count; i += 4 * kRed) {  // four quadruples in flight, added in order
        double4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const double4 *>(p + 4 * (i + k * kRed));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[0] += v[k].x;
            s[1] += v[k].y;
            s[2] += v[k].z;
            s[3] += v[k].w;
        }
    }
    for (; i < count; i += kRed)
        for (int q = 0; q < 4; ++q) s[q] += p[4 * i + q];
    for (int q = 0; q < 4; ++q) {
        const double t = block_sum256(s[q], red);
        if (threadIdx.x == 0) out4[q] = t;
    }
}

hipError_t launch_reduce4(const double *partial, int count, double *out4, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce4, dim3(1), dim3(kRed), 0, s, partial, count, out4);
    return hipGetLastError();
}

hipError_t launch_fstats(const double *f, long pitch, int n, double *partial, int blocks, double *out4,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_fstats, dim3(blocks), dim3(kRed), 0, s, f, pitch, n, partial);
    hipLaunchKernelGGL(k_reduce4, dim3(1), dim3(kRed), 0, s, partial, blocks, out4);
    return hipGetLastError();
}

hipError_t launch_fstats_restrict(const double *f, long pitch, int n, double *partial, int blocks, double *out4,
                                  double *coarse, long pc, hipStream_t s) {
    hipLaunchKernelGGL(k_fstats_restrict, dim3(blocks), dim3(kRed), 0, s, f, pitch, n, partial, coarse, pc);
    hipLaunchKernelGGL(k_reduce4, dim3(1), dim3(kRed), 0, s, partial, blocks, out4);
    return hipGetLastError();
}

// Write constant values into a few device words (no memset nodes).
__global__ void k_set(double *p, int count, double v) {
    const int i = threadIdx.x;
    if (i < count) p[i] = v;
}
hipError_t launch_set(double *p, int count, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, p, count, v);
    return hipGetLastError();
}
__global__ void k_set_int(int *p, int count, int v) {
    const int i = threadIdx.x;
    if (i < count) p[i] = v;
}
hipError_t launch_set_int(int *p, int count, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, count, v);
    return hipGetLastError();
}

}  // namespace ccmg

namespace ccmg {

// Streaming probe: c = a + b over `count` doubles (count even, 16-byte
// aligned arrays), the access pattern of a launch that reads two arrays and
// writes one.  Grid-stride over 16-byte pairs; NT: nontemporal loads and
// stores (streaming hints), else ordinary ones.
typedef double probe_v2 __attribute__((ext_vector_type(2)));
hipError_t launch_probe_stream(const double *a, const double *b, double *c, long count, int blocks, bool nt,
                               hipStream_t s);
template <bool NT>
__global__ __launch_bounds__(256) void k_probe_stream(const probe_v2 *__restrict__ a, const probe_v2 *__restrict__ b,
                                                      probe_v2 *__restrict__ c, long pairs) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < pairs; i += stride) {
        if constexpr (NT) {
            const probe_v2 x = __builtin_nontemporal_load(a + i), y = __builtin_nontemporal_load(b + i);
            __builtin_nontemporal_store(x + y, c + i);
        } else {
            c[i] = a[i] + b[i];
        }
    }
}

hipError_t launch_probe_stream(const double *a, const double *b, double *c, long count, int blocks, hipStream_t s) {
    return launch_probe_stream(a, b, c, count, blocks, false, s);
}

hipError_t launch_probe_stream(const double *a, const double *b, double *c, long count, int blocks, bool nt,
                               hipStream_t s) {
    const probe_v2 *pa = reinterpret_cast<const probe_v2 *>(a), *pb = reinterpret_cast<const probe_v2 *>(b);
    probe_v2 *pc = reinterpret_cast<probe_v2 *>(c);
    if (nt) hipLaunchKernelGGL(k_probe_stream<true>, dim3(blocks), dim3(256), 0, s, pa, pb, pc, count / 2);
    else hipLaunchKernelGGL(k_probe_stream<false>, dim3(blocks), dim3(256), 0, s, pa, pb, pc, count / 2);
    return hipGetLastError();
}

}  // namespace ccmg

namespace ccmg {

// Four-cell average of a fine level into the coarse level below it (valid
// cells only): coarse(I, J) = 1/4 of the fine cells (2I, 2J), (2I+1, 2J),
// (2I, 2J+1), (2I+1, 2J+1), added in that order.  One thread per coarse cell;
// blockIdx.y is the coarse row.
__global__ __launch_bounds__(256) void k_restrict(const double *__restrict__ fine, long pf, double *__restrict__ coarse,
                                                  long pc, int nc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y;
    if (I >= nc) return;
    const double *r0 = fine + (long)(2 * J + 1) * pf + 1 + 2 * I;
    const double *r1 = r0 + pf;
    coarse[(long)(J + 1) * pc + 1 + I] = 0.25 * (((r0[0] + r0[1]) + r1[0]) + r1[1]);
}

hipError_t launch_restrict(const double *fine, long pf, double *coarse, long pc, int nc, hipStream_t s) {
    hipLaunchKernelGGL(k_restrict, dim3((nc + 255) / 256, nc), dim3(256), 0, s, fine, pf, coarse, pc, nc);
    return hipGetLastError();
}

}  // namespace ccmg
