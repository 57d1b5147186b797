// A level's whole visit in one row march (levels below the finest, whose
// correction starts from zero): the pre-smoothing recomputed from zero, the
// prolongation of the coarse correction, the post-smoothing (double: plain
// solves; float: the inner cycles of a mixed-precision step).
#include "march_impl.h"

namespace ccmg {
hipError_t dispatch_visit(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<double, 4, false, true, POST_VISIT>(a, sh, s, nt);
}
hipError_t dispatch_visit(const MarchArgs<float> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<float, 4, false, true, POST_VISIT>(a, sh, s, nt);
}
}  // namespace ccmg
