// FP8 instantiation of the reduced-precision GEMM (kernel and tiling in tk_lowp_gemm.h).
#include "tk_lowp_gemm.h"

namespace tk {

hipError_t gemm_lp_fp8(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s) {
    if (ob != KM) return hipErrorInvalidValue;   // FP8 only for the products over a tensor
    return by_out<LP_FP8, KM>(g, outp, vec, s);
}

hipError_t gemm_lp_grouped_fp8(const LpGroupArgs& a, Orient ob, int outp, bool vec, hipStream_t s) {
    if (ob != KM) return hipErrorInvalidValue;
    return by_out_grouped<LP_FP8, KM>(a, outp, vec, s);
}

}  // namespace tk
