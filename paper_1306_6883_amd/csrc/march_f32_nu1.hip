// Row-march kernels (march_impl.h) with 1 fused red-black iterations, float.
#include "march_impl.h"

namespace ccmg {
template hipError_t dispatch_nu<float, 1>(const MarchArgs<float> &, bool, bool, int, MarchShape, hipStream_t,
                                          int *);
}  // namespace ccmg
