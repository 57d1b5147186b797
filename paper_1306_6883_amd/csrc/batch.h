// batch.h -- device-side descriptors of batched solves (see batch.hip, batch.cpp).
#pragma once
#include "march_impl.h"

namespace ccmg {

// Per-problem state read by the batch kernels.
struct BatchProb {
    const double *f;      // caller's right-hand side (FP64, ghosted)
    long pf;
    int n;
    int singular;
    double rtol;
    int max_cycles;
    double *scal;         // S_FSUM .. S_FBAD statistics of f, S_PHIMEAN
    double *hist;         // relative residual after each step (CCMG_HISTORY)
    int *done;            // skip flag of every launch of this problem
    int *cycles;          // steps performed
    const double *normpart;  // per-tile (sum r^2, sum phi) of the last FP64 residual pass
    const int *norm_count;   // how many tiles wrote them
    double *stat_part;    // per-block statistics of f
    double *host;         // host-mapped [rho, cycles, done]
};

// Per-problem description of the returned field.
struct BatchFinish {
    const double *src;    // where the last step left the FP64 iterate
    long psrc;
    double *dst;          // the caller's phi
    long pdst;
    int n;
    int bc[4];
    const double *shift;  // mean removed from singular problems (or null)
    int zero;             // f == 0: the returned field is 0 (valid and ghost cells)
};

hipError_t launch_batch_fstats(const BatchProb *probs, int m, int blocks, hipStream_t s);
hipError_t launch_batch_cycle_end(const BatchProb *probs, int m, int start, hipStream_t s);
hipError_t launch_batch_finish(const BatchFinish *fin, int m, int nmax, hipStream_t s);

}  // namespace ccmg
