// Reduced-precision (BF16 / FP16 / FP8-e4m3) contraction kernels of the HOOI sweep.
#pragma once
#include "tk_common.h"

namespace tk {

// storage types (numbered as tucker_precision); LP_F32OUT selects a float output
enum { LP_F32OUT = 0, LP_BF16 = 1, LP_F16 = 2, LP_FP8 = 3 };

struct LpGemmArgs {
    Desc a, b, c;
    int64_t M, N, K;
    double alpha;
    int64_t k_split;      // multiple of 64 (or == K)
    int64_t c_zstride;    // element offset between split outputs
    int lower_only;
    const float* sa;      // per-row output scale (nullable)
    const float* sb;      // per-column output scale, index n % sb_mod (nullable)
    int64_t sb_mod;
    int64_t c_valid;      // > 0: columns n with n % c.seg >= c_valid are padding and not written
};

// C = alpha diag(sa) (A B) diag(sb): A k-contiguous (desc rows m, columns k); B n-contiguous
// (ob == KM: desc rows k, columns n) or k-contiguous (ob == MK: desc rows n, columns k).
// Operands in the storage type prec; output float (outp == LP_F32OUT) or BF16/FP16.
// FP8 is provided for ob == KM with a BF16 output (the full-tensor product).
// Outputs: float, or the 16-bit type of the sweep's intermediates (BF16 for BF16 and FP8 operands,
// FP16 for FP16 operands); other combinations return hipErrorInvalidValue.
hipError_t gemm_lp(const LpGemmArgs& g, int prec, Orient ob, int outp, hipStream_t s);

// k step of the GEMM's tiles (k_split must be a multiple of it or cover all of K)
constexpr int kLpGemmK = 64;
// the per-type instantiations behind gemm_lp (vec: 8-element vector loads are legal)
hipError_t gemm_lp_bf16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_f16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_fp8(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);

// out[i] = enc(x[i] / scale[i % L]) (scale nullable)
hipError_t to_lowp(const float* x, int64_t n, int prec, int L, const float* scale, void* out, hipStream_t s);
// out[i] = dec(in[i]) * scale[i % L] (scale nullable)
hipError_t from_lowp(const void* in, int64_t n, int prec, int L, const float* scale, float* out, hipStream_t s);
// scale[l] = max_a |x[a][l]| / 448 (1 where the slice is zero); partial: nblocks * L floats
hipError_t slice_scales(const float* x, int64_t A, int L, float* partial, int nblocks, float* scale, hipStream_t s);
// Ut[r][k] = enc(U[k][r] / scale[r]) for k < rows, 0 up to ldk; scale (FP8 only) = amax of column r / 448
hipError_t factor_lowp(const float* U, int64_t rows, int64_t R, int64_t ldk, int prec, float* scale, void* Ut,
                       hipStream_t s);
// out[a][r R4 + t] = sum_{c,i} U3[c][r] U4[i][t] dec(in[a][c q + i]) scale[c q + i], rows of ldo
// 16-bit outp elements, the tail of each row zero.  u3_identity: U3 is the p x p identity (a mode
// kept at full rank), which lets the fixed-shape kernels skip its product.
hipError_t pair_lowp(const void* in, int64_t A, int p, int q, const float* U3, int R3, const float* U4, int R4,
                     int prec, const float* scale, int outp, int ldo, void* out, hipStream_t s,
                     bool u3_identity = false);

}  // namespace tk
