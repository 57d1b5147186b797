// march.hip -- host entry of the row-march kernels: picks the variant with the
// requested number of fused red-black iterations (see march_impl.h).
#include <type_traits>

#include "internal.h"

namespace ccmg {

template <typename T>
hipError_t launch_march(const MarchArgs<T> &a, int nu, bool load_phi, bool prolong, int post,
                        MarchShape shape, hipStream_t s, int *nt) {
    if (post == POST_FUSED) {
        if (nu == 4 && load_phi && prolong && shape.ty >= 2 && !(shape.ty & 1) && shape.wpb >= 1 && shape.wpb <= 4)
            return dispatch_fused(a, shape, s, nt);
        return hipErrorInvalidValue;
    }
    if (post == POST_CNPRE) {
        if constexpr (std::is_same<T, double>::value) {
            if (nu == 2 && load_phi && !prolong && shape.ty >= 2 && !(shape.ty & 1) && shape.wpb >= 1 &&
                shape.wpb <= 4)
                return dispatch_cnpre(a, shape, s, nt);
        }
        return hipErrorInvalidValue;
    }
    if (post == POST_FUSED0) {
        if constexpr (std::is_same<T, double>::value) {
            if (nu == 6 && !load_phi && prolong && shape.ty >= 2 && !(shape.ty & 1) && shape.wpb >= 1 &&
                shape.wpb <= 4)
                return dispatch_fused0(a, shape, s, nt);
        }
        return hipErrorInvalidValue;
    }
    if (post == POST_VISIT) {
        if (nu == 4 && !load_phi && prolong && shape.ty >= 2 && !(shape.ty & 1) && shape.wpb >= 1 && shape.wpb <= 4)
            return dispatch_visit(a, shape, s, nt);
        return hipErrorInvalidValue;
    }
    if (shape.ty == 0) return launch_tile<T>(a, nu, load_phi, prolong, post, s, nt);
    if (shape.ty < 2 || (shape.ty & 1) || shape.wpb < 1 || shape.wpb > 4) return hipErrorInvalidValue;
    switch (nu) {
        case 0: return dispatch_nu<T, 0>(a, load_phi, prolong, post, shape, s, nt);
        case 1: return dispatch_nu<T, 1>(a, load_phi, prolong, post, shape, s, nt);
        case 2: return dispatch_nu<T, 2>(a, load_phi, prolong, post, shape, s, nt);
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_march<double>(const MarchArgs<double> &, int, bool, bool, int, MarchShape,
                                         hipStream_t, int *);
template hipError_t launch_march<float>(const MarchArgs<float> &, int, bool, bool, int, MarchShape,
                                        hipStream_t, int *);

}  // namespace ccmg
