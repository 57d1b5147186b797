// Row-march kernels (march_impl.h) with 2 fused red-black iterations, double.
#include "march_impl.h"

namespace ccmg {
template hipError_t dispatch_nu<double, 2>(const MarchArgs<double> &, bool, bool, int, MarchShape, hipStream_t,
                                          int *);
}  // namespace ccmg
