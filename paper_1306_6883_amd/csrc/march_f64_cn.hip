// The first pre-smoothing launch of a Crank-Nicolson step: the right-hand
// side phi + beta Lap phi of the old level (the loaded iterate) is formed in
// the row march and written out, instead of being read.
#include "march_impl.h"

namespace ccmg {
hipError_t dispatch_cnpre(const MarchArgs<double> &a, MarchShape sh, hipStream_t s, int *nt) {
    return go<double, 2, true, false, POST_CNPRE>(a, sh, s, nt);
}
}  // namespace ccmg
