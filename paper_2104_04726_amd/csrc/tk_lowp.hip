// Reduced-precision contractions of the HOOI sweep (BF16, FP16, FP8-e4m3) on gfx950 matrix cores.
//
// The operands of the dense contractions (eq. (8) mode products and the mode Grams) are stored in
// a 16- or 8-bit type and multiplied by the v_mfma_f32_16x16x32_{bf16,f16,fp8_fp8} instructions with
// FP32 accumulation.  Every other part of the sweep (orthogonal iteration, norms, the small modes)
// stays in FP32/FP64.
//
// Encodings: BF16 and FP16 by round-to-nearest-even from FP32.  FP8 is the OCP E4M3 ("fn") format
// (bias 7, no infinities, largest finite 448); values are divided by a per-slice FP32 scale
// (amax / 448) before the RNE conversion, with saturation at +-448.
//
// The GEMM itself lives in tk_lowp_gemm.h (one translation unit per storage type).
#include "tk_lowp_impl.h"

namespace tk {
namespace {

// Vector (8-element) loads are legal when every 8-aligned run of a k-contiguous operand (or an
// n-contiguous B) lies inside one segment and starts on a 16- (8-) byte boundary.
bool desc_vec_ok(const Desc& d, int es) {
    const int64_t vb = 8 * es;
    const bool segok = d.seg >= (int64_t(1) << 61) || (d.seg % 8 == 0 && d.segstride % 8 == 0);
    return segok && d.ld % 8 == 0 && (((uintptr_t)d.ptr) % vb) == 0;
}

// ---------------------------------------------------------------------------- conversions
template <int P>
__global__ __launch_bounds__(256) void to_lp_kernel(const float* __restrict__ x, int64_t n, int L,
                                                    const float* __restrict__ scale,
                                                    typename Codec<P>::S* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float v = x[i];
        if (scale) v = v / scale[i % L];
        out[i] = Codec<P>::enc(v);
    }
}

// rows of L values -> rows of Lp >= L encoded values, the Lp - L tail of each row zero
template <int P>
__global__ __launch_bounds__(256) void to_lp_padded_kernel(const float* __restrict__ x, int64_t rows, int L, int Lp,
                                                           typename Codec<P>::S* __restrict__ out) {
    const int64_t n = rows * Lp;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / Lp;
        const int j = (int)(i - r * Lp);
        out[i] = j < L ? Codec<P>::enc(x[r * L + j]) : (typename Codec<P>::S)0;
    }
}

// amax over fibres per position l of a (A, L) matrix -> partial[block][l]
__global__ __launch_bounds__(256) void slice_amax_kernel(const float* __restrict__ x, int64_t A, int L,
                                                         float* __restrict__ partial) {
    __shared__ float red[256];
    for (int l = 0; l < L; ++l) {
        float m = 0.f;
        for (int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x; a < A; a += (int64_t)gridDim.x * 256)
            m = fmaxf(m, fabsf(x[a * L + l]));
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * L + l] = red[0];
        __syncthreads();
    }
}
__global__ void slice_scale_kernel(const float* __restrict__ partial, int nb, int L, float* __restrict__ scale) {
    const int l = threadIdx.x;
    if (l >= L) return;
    float m = 0.f;
    for (int b = 0; b < nb; ++b) m = fmaxf(m, partial[(int64_t)b * L + l]);
    scale[l] = (m > 0.f) ? m / 448.0f : 1.0f;
}

// Ut[r][k] = U[k][r] (U: s x R FP32) in the low-precision type, rows padded to ldk with zeros.
// With scale != nullptr (FP8) each row r is divided by scale[r] = amax_k |U[k][r]| / 448.
template <int P>
__global__ __launch_bounds__(256) void factor_lp_kernel(const float* __restrict__ U, int64_t s, int64_t R,
                                                        int64_t ldk, float* __restrict__ scale,
                                                        typename Codec<P>::S* __restrict__ Ut) {
    const int64_t r = blockIdx.x;
    __shared__ float red[256];
    float sc = 1.f;
    if (scale) {
        float m = 0.f;
        for (int64_t k = threadIdx.x; k < s; k += 256) m = fmaxf(m, fabsf(U[k * R + r]));
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        sc = (red[0] > 0.f) ? red[0] / 448.0f : 1.0f;
        if (threadIdx.x == 0) scale[r] = sc;
    }
    for (int64_t k = threadIdx.x; k < ldk; k += 256) {
        const float v = (k < s) ? U[k * R + r] : 0.f;
        Ut[r * ldk + k] = Codec<P>::enc(scale ? v / sc : v);
    }
}

template <int P>
__global__ __launch_bounds__(256) void from_lp_kernel(const typename Codec<P>::S* __restrict__ in, int64_t n,
                                                      int L, const float* __restrict__ scale, float* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float v = Codec<P>::dec(in[i]);
        if (scale) v *= scale[i % L];
        out[i] = v;
    }
}

// ---------------------------------------------------------------------------- two-mode pass
// Fixed-shape version of the pass below (P x Q fibres, ranks R3, R4, output rows of LDO): the
// chunk of 256 fibres is read with 16-byte coalesced loads prefetched one chunk ahead, mapped one
// fibre per thread with U3 in registers and U4 in LDS, and written back with 16-byte stores.
// ID3: U3 is the identity (a mode kept at full rank), so its product is skipped.  16-bit storage:
// each thread decodes the elements of its 16-byte vectors into an FP32 copy of the chunk in LDS
// (one division per vector; fibre and position advance by increments).  FP8 (16 elements per
// vector, slice scales): that decode wrote LDS with 16-way bank conflicts, so the chunk is stored
// to LDS as it is (16-byte stores, consecutive lanes on consecutive addresses) and each thread
// decodes and scales its own fibre from there, two elements per 2-byte read and conversion.
template <int P, int OUTP, int PP, int QQ, int R3, int R4, int LDO, bool ID3>
__global__ __launch_bounds__(256) void pair_lp_fixed(const typename Codec<P>::S* __restrict__ in, int64_t A,
                                                     const float* __restrict__ U3, const float* __restrict__ U4,
                                                     const float* __restrict__ scale, uint16_t* __restrict__ out) {
    typedef typename Codec<P>::S S;
    constexpr int ES = (int)sizeof(S);
    constexpr int LIN = PP * QQ, SIN = LIN | 1;
    constexpr int FPB = 256;
    constexpr int EPV = 16 / ES;                        // elements per 16-byte vector
    constexpr int NV_IN = FPB * LIN / EPV;              // vectors per full chunk
    constexpr int VPT = (NV_IN + 255) / 256;
    constexpr int NV_OUT = FPB * LDO * 2 / 16;
    constexpr bool SCALED = (P == LP_FP8);
    constexpr bool RAW = (ES == 1);                     // stage the chunk as stored, decode per fibre
    static_assert((FPB * LIN) % EPV == 0 && (FPB * LDO * 2) % 16 == 0, "chunk not a whole number of vectors");
    static_assert(!ID3 || PP == R3, "an identity U3 keeps the mode's size");
    static_assert(EPV <= LIN || RAW, "a vector spans at most two fibres");
    static_assert(!RAW || LIN % 2 == 0, "FP8 fibres are read two elements at a time");
    constexpr int NFIN = RAW ? 1 : FPB * SIN;
    constexpr int NRAW = RAW ? FPB * LIN : 16;
    __shared__ float fin[NFIN];
    __shared__ __attribute__((aligned(16))) S raw[NRAW];
    __shared__ __attribute__((aligned(16))) uint16_t fout[FPB * LDO];
    __shared__ float sc[LIN];
    __shared__ float u4[QQ * R4];
    if (SCALED)
        for (int i = threadIdx.x; i < LIN; i += 256) sc[i] = scale ? scale[i] : 1.0f;
    for (int i = threadIdx.x; i < QQ * R4; i += 256) u4[i] = U4[i];
    float u3[PP * R3];
#pragma unroll
    for (int i = 0; i < PP * R3; ++i) u3[i] = ID3 ? 0.f : U3[i];

    const int64_t nchunks = (A + FPB - 1) / FPB;
    const int64_t full = A / FPB;
    uint4 pre[VPT];
    auto prefetch = [&](int64_t ch) {
        if (ch < full) {
            const uint4* src = (const uint4*)(in + ch * FPB * LIN);
#pragma unroll
            for (int u = 0; u < VPT; ++u) {
                const int i = threadIdx.x + 256 * u;
                if (i < NV_IN) pre[u] = src[i];
            }
        }
    };
    int64_t ch = blockIdx.x;
    prefetch(ch);
    for (; ch < nchunks; ch += gridDim.x) {
        const int64_t f0 = ch * FPB;
        const int nf = (int)((A - f0) < FPB ? (A - f0) : FPB);
        __syncthreads();
        if constexpr (RAW) {
            if (ch < full) {
#pragma unroll
                for (int u = 0; u < VPT; ++u) {
                    const int i = threadIdx.x + 256 * u;
                    if (i < NV_IN) ((uint4*)raw)[i] = pre[u];
                }
            } else {
                const S* src = in + f0 * LIN;
                for (int g = threadIdx.x; g < nf * LIN; g += 256) raw[g] = src[g];
            }
        } else if (ch < full) {
#pragma unroll
            for (int u = 0; u < VPT; ++u) {
                const int i = threadIdx.x + 256 * u;
                if (i < NV_IN) {
                    const S* e = (const S*)&pre[u];
                    const int g0 = EPV * i;
                    const int fb = g0 / LIN;
                    int l = g0 - fb * LIN;
                    float* dst = fin + fb * SIN;
#pragma unroll
                    for (int j = 0; j < EPV; ++j) {
                        dst[l] = Codec<P>::dec(e[j]);
                        ++l;
                        if (l == LIN) {
                            l = 0;
                            dst += SIN;
                        }
                    }
                }
            }
        } else {
            const S* src = in + f0 * LIN;
            for (int g = threadIdx.x; g < nf * LIN; g += 256) fin[(g / LIN) * SIN + g % LIN] = Codec<P>::dec(src[g]);
        }
        __syncthreads();
        prefetch(ch + gridDim.x);
        const int f = threadIdx.x;
        if (f < nf) {
            float xv[RAW ? LIN : 1];
            if constexpr (RAW) {
                const uint16_t* xp = (const uint16_t*)(raw + f * LIN);
#pragma unroll
                for (int h = 0; h < LIN / 2; ++h) {
                    // the hardware conversion of both bytes of the 16-bit word (element 2h in the low byte)
                    const auto v2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)xp[h], false);
                    xv[2 * h] = v2[0] * sc[2 * h];
                    xv[2 * h + 1] = v2[1] * sc[2 * h + 1];
                }
            }
            const float* x = fin + f * SIN;
            auto elem = [&](int l) { return RAW ? xv[RAW ? l : 0] : x[l]; };
            float tmp[PP][R4];
#pragma unroll
            for (int c = 0; c < PP; ++c)
#pragma unroll
                for (int t = 0; t < R4; ++t) tmp[c][t] = 0.f;
#pragma unroll
            for (int i = 0; i < QQ; ++i) {
                float xc[PP];
#pragma unroll
                for (int c = 0; c < PP; ++c) xc[c] = elem(c * QQ + i);
#pragma unroll
                for (int t = 0; t < R4; ++t) {
                    const float w = u4[i * R4 + t];
#pragma unroll
                    for (int c = 0; c < PP; ++c) tmp[c][t] = fmaf(xc[c], w, tmp[c][t]);
                }
            }
            uint16_t* y = fout + f * LDO;
#pragma unroll
            for (int r = 0; r < R3; ++r)
#pragma unroll
                for (int t = 0; t < R4; ++t) {
                    float acc;
                    if (ID3) {
                        acc = tmp[r][t];
                    } else {
                        acc = 0.f;
#pragma unroll
                        for (int c = 0; c < PP; ++c) acc = fmaf(u3[c * R3 + r], tmp[c][t], acc);
                    }
                    y[r * R4 + t] = (OUTP == LP_BF16) ? enc_bf16(acc) : enc_f16(acc);
                }
#pragma unroll
            for (int o = R3 * R4; o < LDO; ++o) y[o] = 0;
        }
        __syncthreads();
        if (nf == FPB) {
            uint4* dst = (uint4*)(out + f0 * LDO);
            const uint4* s4 = (const uint4*)fout;
            for (int i = threadIdx.x; i < NV_OUT; i += 256) dst[i] = s4[i];
        } else {
            uint16_t* dst = out + f0 * LDO;
            for (int g = threadIdx.x; g < nf * LDO; g += 256) dst[g] = fout[g];
        }
    }
}

template <int P, int OUTP, int PP, int QQ, int R3, int R4, int LDO>
bool try_pair_lp(const void* in, int64_t A, int p, int q, const float* U3, int r3, const float* U4, int r4,
                 const float* scale, int ldo, bool u3_identity, void* out, hipStream_t s, hipError_t* err) {
    if (p != PP || q != QQ || r3 != R3 || r4 != R4 || ldo != LDO) return false;
    if ((((uintptr_t)in) & 15) != 0 || (((uintptr_t)out) & 15) != 0) return false;
    const int64_t nchunks = (A + 255) / 256;
    const unsigned grid = (unsigned)(nchunks < 1024 ? nchunks : 1024);
    if (u3_identity && PP == R3)
        hipLaunchKernelGGL((pair_lp_fixed<P, OUTP, PP, QQ, R3, R4, LDO, PP == R3>), dim3(grid), dim3(256), 0, s,
                           (const typename Codec<P>::S*)in, A, U3, U4, scale, (uint16_t*)out);
    else
        hipLaunchKernelGGL((pair_lp_fixed<P, OUTP, PP, QQ, R3, R4, LDO, false>), dim3(grid), dim3(256), 0, s,
                           (const typename Codec<P>::S*)in, A, U3, U4, scale, (uint16_t*)out);
    *err = hipGetLastError();
    return true;
}

template <int P, int OUTP>
bool pair_lp_any_fixed(const void* in, int64_t A, int p, int q, const float* U3, int r3, const float* U4, int r4,
                       const float* scale, int ldo, bool u3_identity, void* out, hipStream_t s, hipError_t* err) {
    // the image-stack fibre shapes: 3 colour channels x 2E images, R4 = 2E - 1 or the reduced ranks
    return try_pair_lp<P, OUTP, 3, 14, 3, 8, 24>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s, err) ||
           try_pair_lp<P, OUTP, 3, 10, 3, 6, 24>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s, err) ||
           try_pair_lp<P, OUTP, 3, 6, 3, 4, 16>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s, err) ||
           try_pair_lp<P, OUTP, 3, 6, 3, 5, 16>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s, err) ||
           try_pair_lp<P, OUTP, 3, 10, 3, 9, 32>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s, err) ||
           try_pair_lp<P, OUTP, 3, 14, 3, 13, 40>(in, A, p, q, U3, r3, U4, r4, scale, ldo, u3_identity, out, s,
                                                   err);
}

// ---------------------------------------------------------------------------- two-mode pass (generic)
// T34[a][r][t] (row stride ldo >= R3 R4, padding written as zero) = sum_{c,i} U3[c][r] U4[i][t] x[a][c][i]
// where x[a][c][i] = dec(in[a][c][i]) * (scale ? scale[c q + i] : 1).  One thread per fibre; the
// fibres of a 256-fibre chunk are staged through LDS with coalesced loads; output in OUTP.
template <int P, int OUTP>
__global__ __launch_bounds__(256) void pair_lp_kernel(const typename Codec<P>::S* __restrict__ in, int64_t A,
                                                      int p, int q, const float* __restrict__ U3, int R3,
                                                      const float* __restrict__ U4, int R4,
                                                      const float* __restrict__ scale, int ldo,
                                                      uint16_t* __restrict__ out) {
    typedef typename Codec<P>::S S;
    constexpr int FPB = 256;
    const int L = p * q;
    const int SL = L | 1;
    __shared__ float u3[4 * 4];
    __shared__ float u4[16 * 16];
    __shared__ float sc[64];
    __shared__ float fin[FPB * 65];
    __shared__ uint16_t fout[FPB * 64];
    for (int i = threadIdx.x; i < p * R3; i += 256) u3[i] = U3[i];
    for (int i = threadIdx.x; i < q * R4; i += 256) u4[i] = U4[i];
    for (int i = threadIdx.x; i < L; i += 256) sc[i] = scale ? scale[i] : 1.0f;
    const int64_t nchunks = (A + FPB - 1) / FPB;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t f0 = ch * FPB;
        const int nf = (int)((A - f0) < FPB ? (A - f0) : FPB);
        __syncthreads();
        const S* src = in + f0 * L;
        for (int g = threadIdx.x; g < nf * L; g += 256) {
            const int l = g % L;
            fin[(g / L) * SL + l] = Codec<P>::dec(src[g]) * sc[l];
        }
        __syncthreads();
        const int f = threadIdx.x;
        if (f < nf) {
            const float* x = fin + f * SL;
            float tmp[4][16];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c >= p) break;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    if (t >= R4) break;
                    float acc = 0.f;
                    for (int i = 0; i < q; ++i) acc = fmaf(x[c * q + i], u4[i * R4 + t], acc);
                    tmp[c][t] = acc;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (r >= R3) break;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    if (t >= R4) break;
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (c >= p) break;
                        acc = fmaf(u3[c * R3 + r], tmp[c][t], acc);
                    }
                    fout[f * ldo + r * R4 + t] = (OUTP == LP_BF16) ? enc_bf16(acc) : enc_f16(acc);
                }
            }
            for (int o = R3 * R4; o < ldo; ++o) fout[f * ldo + o] = 0;
        }
        __syncthreads();
        uint16_t* dst = out + f0 * ldo;
        for (int g = threadIdx.x; g < nf * ldo; g += 256) dst[g] = fout[g];
    }
}

}  // namespace

// ============================================================================ launchers
hipError_t gemm_lp(const LpGemmArgs& gin, int prec, Orient ob, int outp, hipStream_t s) {
    LpGemmArgs g = gin;
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.k_split <= 0 || g.k_split > g.K) g.k_split = g.K > 0 ? g.K : 1;
    if (g.k_split % kLpGemmK != 0 && g.k_split != g.K) return hipErrorInvalidValue;
    if (g.sb && g.sb_mod <= 0) return hipErrorInvalidValue;
    const int es = (prec == LP_FP8) ? 1 : 2;
    bool vec = desc_vec_ok(g.a, es) && desc_vec_ok(g.b, es);
    if (prec == LP_BF16) return gemm_lp_bf16(g, ob, outp, vec, s);
    if (prec == LP_F16) return gemm_lp_f16(g, ob, outp, vec, s);
    if (prec == LP_FP8) return gemm_lp_fp8(g, ob, outp, vec, s);
    return hipErrorInvalidValue;
}

hipError_t gemm_lp_grouped(const LpGemmArgs* gin, int n, int prec, Orient ob, int outp, unsigned* ctr,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > kLpGroupMax || !ctr) return hipErrorInvalidValue;
    const int es = (prec == LP_FP8) ? 1 : 2;
    LpGroupArgs a{};
    a.n = 0;
    a.ctr = ctr;
    a.start[0] = 0;
    bool vec = true;
    for (int i = 0; i < n; ++i) {
        LpGemmArgs g = gin[i];
        if (g.M <= 0 || g.N <= 0) continue;
        if (g.k_split <= 0 || g.k_split > g.K) g.k_split = g.K > 0 ? g.K : 1;
        if (g.k_split % kLpGemmK != 0 && g.k_split != g.K) return hipErrorInvalidValue;
        if (g.sb && g.sb_mod <= 0) return hipErrorInvalidValue;
        vec = vec && desc_vec_ok(g.a, es) && desc_vec_ok(g.b, es);
        a.p[a.n] = g;
        a.start[a.n + 1] = a.start[a.n] + lp_work_items(g);
        ++a.n;
    }
    if (a.n == 0) return hipSuccess;
    if (prec == LP_BF16) return gemm_lp_grouped_bf16(a, ob, outp, vec, s);
    if (prec == LP_F16) return gemm_lp_grouped_f16(a, ob, outp, vec, s);
    if (prec == LP_FP8) return gemm_lp_grouped_fp8(a, ob, outp, vec, s);
    return hipErrorInvalidValue;
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

hipError_t to_lowp(const float* x, int64_t n, int prec, int L, const float* scale, void* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (prec == LP_BF16)
        hipLaunchKernelGGL(to_lp_kernel<LP_BF16>, dim3(grid_for(n)), dim3(256), 0, s, x, n, L, scale, (uint16_t*)out);
    else if (prec == LP_F16)
        hipLaunchKernelGGL(to_lp_kernel<LP_F16>, dim3(grid_for(n)), dim3(256), 0, s, x, n, L, scale, (uint16_t*)out);
    else if (prec == LP_FP8)
        hipLaunchKernelGGL(to_lp_kernel<LP_FP8>, dim3(grid_for(n)), dim3(256), 0, s, x, n, L, scale, (uint8_t*)out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t to_lowp_padded(const float* x, int64_t rows, int L, int Lp, int prec, void* out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (Lp < L) return hipErrorInvalidValue;
    const unsigned g = grid_for(rows * Lp);
    if (prec == LP_BF16)
        hipLaunchKernelGGL(to_lp_padded_kernel<LP_BF16>, dim3(g), dim3(256), 0, s, x, rows, L, Lp, (uint16_t*)out);
    else if (prec == LP_F16)
        hipLaunchKernelGGL(to_lp_padded_kernel<LP_F16>, dim3(g), dim3(256), 0, s, x, rows, L, Lp, (uint16_t*)out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t from_lowp(const void* in, int64_t n, int prec, int L, const float* scale, float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (prec == LP_BF16)
        hipLaunchKernelGGL(from_lp_kernel<LP_BF16>, dim3(grid_for(n)), dim3(256), 0, s, (const uint16_t*)in, n, L,
                           scale, out);
    else if (prec == LP_F16)
        hipLaunchKernelGGL(from_lp_kernel<LP_F16>, dim3(grid_for(n)), dim3(256), 0, s, (const uint16_t*)in, n, L,
                           scale, out);
    else if (prec == LP_FP8)
        hipLaunchKernelGGL(from_lp_kernel<LP_FP8>, dim3(grid_for(n)), dim3(256), 0, s, (const uint8_t*)in, n, L,
                           scale, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t slice_scales(const float* x, int64_t A, int L, float* partial, int nblocks, float* scale, hipStream_t s) {
    if (L > 256 || L < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(slice_amax_kernel, dim3(nblocks), dim3(256), 0, s, x, A, L, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(slice_scale_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, L, scale);
    return hipGetLastError();
}

hipError_t factor_lowp(const float* U, int64_t rows, int64_t R, int64_t ldk, int prec, float* scale, void* Ut,
                       hipStream_t s) {
    if (R == 0) return hipSuccess;
    if (prec == LP_BF16)
        hipLaunchKernelGGL(factor_lp_kernel<LP_BF16>, dim3((unsigned)R), dim3(256), 0, s, U, rows, R, ldk, nullptr,
                           (uint16_t*)Ut);
    else if (prec == LP_F16)
        hipLaunchKernelGGL(factor_lp_kernel<LP_F16>, dim3((unsigned)R), dim3(256), 0, s, U, rows, R, ldk, nullptr,
                           (uint16_t*)Ut);
    else if (prec == LP_FP8)
        hipLaunchKernelGGL(factor_lp_kernel<LP_FP8>, dim3((unsigned)R), dim3(256), 0, s, U, rows, R, ldk, scale,
                           (uint8_t*)Ut);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t pair_lowp(const void* in, int64_t A, int p, int q, const float* U3, int R3, const float* U4, int R4,
                     int prec, const float* scale, int outp, int ldo, void* out, hipStream_t s, bool u3_identity) {
    if (p < 1 || p > 4 || q < 1 || q > 16 || R3 > p || R4 > q || ldo < R3 * R4 || ldo > 64) return hipErrorInvalidValue;
    if (outp != LP_BF16 && outp != LP_F16) return hipErrorInvalidValue;
    if (A == 0) return hipSuccess;
    {
        hipError_t e = hipSuccess;
        bool done = false;
        if (prec == LP_BF16 && outp == LP_BF16)
            done = pair_lp_any_fixed<LP_BF16, LP_BF16>(in, A, p, q, U3, R3, U4, R4, scale, ldo, u3_identity, out, s,
                                                          &e);
        else if (prec == LP_F16 && outp == LP_F16)
            done = pair_lp_any_fixed<LP_F16, LP_F16>(in, A, p, q, U3, R3, U4, R4, scale, ldo, u3_identity, out, s,
                                                          &e);
        else if (prec == LP_FP8 && outp == LP_BF16)
            done = pair_lp_any_fixed<LP_FP8, LP_BF16>(in, A, p, q, U3, R3, U4, R4, scale, ldo, u3_identity, out, s,
                                                          &e);
        if (done) return e;
    }
    const int64_t nchunks = (A + 255) / 256;
    const unsigned grid = (unsigned)(nchunks < 2048 ? nchunks : 2048);
#define TK_PAIR(PP, OO)                                                                                          \
    hipLaunchKernelGGL((pair_lp_kernel<PP, OO>), dim3(grid), dim3(256), 0, s, (const typename Codec<PP>::S*)in, A, \
                       p, q, U3, R3, U4, R4, scale, ldo, (uint16_t*)out)
    if (prec == LP_BF16) {
        if (outp == LP_BF16) TK_PAIR(LP_BF16, LP_BF16);
        else TK_PAIR(LP_BF16, LP_F16);
    } else if (prec == LP_F16) {
        if (outp == LP_BF16) TK_PAIR(LP_F16, LP_BF16);
        else TK_PAIR(LP_F16, LP_F16);
    } else if (prec == LP_FP8) {
        if (outp == LP_BF16) TK_PAIR(LP_FP8, LP_BF16);
        else TK_PAIR(LP_FP8, LP_F16);
    } else {
        return hipErrorInvalidValue;
    }
#undef TK_PAIR
    return hipGetLastError();
}

}  // namespace tk
