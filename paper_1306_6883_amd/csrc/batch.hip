// batch.hip -- per-problem kernels of batched solves: one workgroup (or a row
// of workgroups) per problem, all problems in one launch.  The heavy lifting
// (relaxation, restriction, prolongation, the FP64 update) is the row-march
// work-list launch of march_impl.h and the one-workgroup tail of coarse.hip.
#include "batch.h"

namespace ccmg {

namespace {
constexpr int kRed = 256;

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

// grid (kStatBlocksPerProblem, m): partial statistics of f for each problem.
__global__ __launch_bounds__(kRed) void k_batch_fstats(const BatchProb *__restrict__ probs) {
    __shared__ double red[4];
    const BatchProb &p = probs[blockIdx.y];
    double s = 0.0, sa = 0.0, s2 = 0.0, bad = 0.0;
    for (int y = blockIdx.x; y < p.n; y += gridDim.x) {
        const double *row = p.f + (long)(y + 1) * p.pf + 1;
        for (int x = threadIdx.x; x < p.n; x += kRed) {
            const double v = row[x];
            if (!isfinite(v)) {
                bad += 1.0;
                continue;
            }
            s += v;
            sa += fabs(v);
            s2 += v * v;
        }
    }
    s = block_sum256(s, red);
    sa = block_sum256(sa, red);
    s2 = block_sum256(s2, red);
    bad = block_sum256(bad, red);
    if (threadIdx.x == 0) {
        double *o = p.stat_part + 4 * blockIdx.x;
        o[0] = s;
        o[1] = sa;
        o[2] = s2;
        o[3] = bad;
    }
}

// one workgroup per problem: totals of the statistics, flags and counters reset.
__global__ __launch_bounds__(kRed) void k_batch_fstats_reduce(const BatchProb *__restrict__ probs, int blocks) {
    __shared__ double red[4];
    const BatchProb &p = probs[blockIdx.x];
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < blocks; i += kRed)
        for (int q = 0; q < 4; ++q) t[q] += p.stat_part[4 * i + q];
    for (int q = 0; q < 4; ++q) t[q] = block_sum256(t[q], red);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) p.scal[q] = t[q];  // sum f, sum |f|, sum f^2, non-finite count
        p.scal[S_PHIMEAN] = 0.0;
        *p.done = 0;
        *p.cycles = 0;
        p.host[2] = 0.0;
    }
}

// End of a batched step (or of the starting residual pass when `start`): per
// problem, the relative residual of the FP64 iterate and the mean of phi from
// the per-tile partial sums, the history, the cycle count and the done flag.
__global__ __launch_bounds__(kRed) void k_batch_cycle_end(const BatchProb *__restrict__ probs, int start) {
    __shared__ double red[4];
    const BatchProb &p = probs[blockIdx.x];
    if (*p.done) return;  // uniform over the workgroup
    const int count = *p.norm_count;
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < count; i += kRed) {
        s0 += p.normpart[2 * i];
        s1 += p.normpart[2 * i + 1];
    }
    s0 = block_sum256(s0, red);
    s1 = block_sum256(s1, red);
    if (threadIdx.x == 0) {
        const double rho = sqrt(s0) / sqrt(p.scal[S_F2]);
        const int c = start ? 0 : *p.cycles + 1;
        *p.cycles = c;
        if (c < CCMG_HISTORY) p.hist[c] = rho;
        p.scal[S_PHIMEAN] = p.singular ? s1 / ((double)p.n * (double)p.n) : 0.0;
        const bool fin = rho <= p.rtol || !isfinite(rho) || c >= p.max_cycles;
        if (fin) *p.done = 1;
        // host-mapped summary: rho, cycles, done
        p.host[0] = rho;
        p.host[1] = (double)c;
        p.host[2] = fin ? 1.0 : 0.0;
    }
}

// grid (rows, m): the returned field.  Valid cells: copy from where the last
// step left the iterate (if that is not the caller's array) and remove the
// mean of singular problems; zeros for a zero right-hand side (whatever the
// guess was), as a single solve returns.
__global__ __launch_bounds__(kRed) void k_batch_finish_valid(const BatchFinish *__restrict__ fin) {
    const BatchFinish &q = fin[blockIdx.y];
    const double m = q.shift ? *q.shift : 0.0;
    for (int y = blockIdx.x; y < q.n; y += gridDim.x) {
        const double *src = q.src + (long)(y + 1) * q.psrc + 1;
        double *dst = q.dst + (long)(y + 1) * q.pdst + 1;
        if (q.zero) {
            for (int x = threadIdx.x; x < q.n; x += kRed) dst[x] = 0.0;
        } else {
            for (int x = threadIdx.x; x < q.n; x += kRed) dst[x] = src[x] - m;
        }
    }
}

// grid (ceil(n_max / 256), m): ghost cells of the returned field.
__global__ __launch_bounds__(kRed) void k_batch_finish_ghosts(const BatchFinish *__restrict__ fin) {
    const BatchFinish &q = fin[blockIdx.y];
    const int k = blockIdx.x * kRed + threadIdx.x;
    if (k >= q.n) return;
    double *a = q.dst;
    const long pitch = q.pdst;
    const int n = q.n;
    double *row = a + (long)(k + 1) * pitch;
    const double lo = row[1], hi = row[n];
    row[0] = q.bc[0] == CCMG_BC_PERIODIC ? hi : side_sign(q.bc[0]) * lo;
    row[n + 1] = q.bc[1] == CCMG_BC_PERIODIC ? lo : side_sign(q.bc[1]) * hi;
    const double clo = a[pitch + 1 + k], chi = a[(long)n * pitch + 1 + k];
    a[1 + k] = q.bc[2] == CCMG_BC_PERIODIC ? chi : side_sign(q.bc[2]) * clo;
    a[(long)(n + 1) * pitch + 1 + k] = q.bc[3] == CCMG_BC_PERIODIC ? clo : side_sign(q.bc[3]) * chi;
}

hipError_t launch_batch_fstats(const BatchProb *probs, int m, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_fstats, dim3(blocks, m), dim3(kRed), 0, s, probs);
    hipLaunchKernelGGL(k_batch_fstats_reduce, dim3(m), dim3(kRed), 0, s, probs, blocks);
    return hipGetLastError();
}

hipError_t launch_batch_cycle_end(const BatchProb *probs, int m, int start, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_cycle_end, dim3(m), dim3(kRed), 0, s, probs, start);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchFinish *fin, int m, int nmax, hipStream_t s) {
    const int rows = nmax < 1024 ? nmax : 1024;
    hipLaunchKernelGGL(k_batch_finish_valid, dim3(rows, m), dim3(kRed), 0, s, fin);
    hipLaunchKernelGGL(k_batch_finish_ghosts, dim3((nmax + kRed - 1) / kRed, m), dim3(kRed), 0, s, fin);
    return hipGetLastError();
}

// Instantiations of the work-list row march used by batches (V(2,2)).
template hipError_t launch_list_variant<float, 2, false, false, POST_RESTRICT>(const MarchArgs<float> *,
                                                                               const WorkItem *, int, int,
                                                                               hipStream_t);
template hipError_t launch_list_variant<float, 2, true, true, POST_NONE>(const MarchArgs<float> *,
                                                                         const WorkItem *, int, int, hipStream_t);
template hipError_t launch_list_variant<float, 2, true, true, POST_IR>(const MarchArgs<float> *, const WorkItem *,
                                                                       int, int, hipStream_t);
template hipError_t launch_list_variant<float, 0, true, false, POST_IR>(const MarchArgs<float> *,
                                                                        const WorkItem *, int, int, hipStream_t);
template hipError_t launch_list_variant<double, 0, false, false, POST_R32>(const MarchArgs<double> *,
                                                                           const WorkItem *, int, int,
                                                                           hipStream_t);
template hipError_t launch_list_variant<double, 0, true, false, POST_R32>(const MarchArgs<double> *,
                                                                          const WorkItem *, int, int,
                                                                          hipStream_t);

}  // namespace ccmg
