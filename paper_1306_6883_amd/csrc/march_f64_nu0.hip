// Row-march kernels (march_impl.h) with 0 fused red-black iterations, double.
#include "march_impl.h"

namespace ccmg {
template hipError_t dispatch_nu<double, 0>(const MarchArgs<double> &, bool, bool, int, MarchShape, hipStream_t,
                                          int *);
}  // namespace ccmg
