// BF16 instantiation of the reduced-precision GEMM (kernel and tiling in tk_lowp_gemm.h).
#include "tk_lowp_gemm.h"

namespace tk {

hipError_t gemm_lp_bf16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s) {
    return ob == KM ? by_out<LP_BF16, KM>(g, outp, vec, s) : by_out<LP_BF16, MK>(g, outp, vec, s);
}

}  // namespace tk
