// The fused finest-level row march: post-smoothing of one V-cycle, its
// residual norm, and the pre-smoothing and restriction of the next (double:
// plain solves; float: the inner cycles of a mixed-precision step); and its
// form for the end of a solve's first cycle from zero, which recomputes that
// cycle's pre-smoothing instead of reading it.
#include "march_impl.h"

namespace ccmg {
hipError_t dispatch_fused(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<double, 4, true, true, POST_FUSED>(a, sh, s, nt);
}
hipError_t dispatch_fused(const MarchArgs<float> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<float, 4, true, true, POST_FUSED>(a, sh, s, nt);
}
hipError_t dispatch_fused0(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<double, 6, false, true, POST_FUSED0>(a, sh, s, nt);
}
}  // namespace ccmg
