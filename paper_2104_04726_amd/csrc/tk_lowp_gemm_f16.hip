// F16 instantiation of the reduced-precision GEMM (kernel and tiling in tk_lowp_gemm.h).
#include "tk_lowp_gemm.h"

namespace tk {

hipError_t gemm_lp_f16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s) {
    return ob == KM ? by_out<LP_F16, KM>(g, outp, vec, s) : by_out<LP_F16, MK>(g, outp, vec, s);
}

hipError_t gemm_lp_grouped_f16(const LpGroupArgs& a, Orient ob, int outp, bool vec, hipStream_t s) {
    return ob == KM ? by_out_grouped<LP_F16, KM>(a, outp, vec, s) : by_out_grouped<LP_F16, MK>(a, outp, vec, s);
}

}  // namespace tk
