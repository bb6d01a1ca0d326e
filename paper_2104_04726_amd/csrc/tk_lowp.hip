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
// GEMM tiling: 256 threads = 4 waves in a 2x2 grid over a 128 x 128 output tile; each wave owns
// 4 x 4 MFMA tiles of 16 x 16 and steps k by 32.  Both operands sit in LDS with k contiguous
// ([row][k], rows padded by 16 bytes), so a lane's eight consecutive k values are one 16-byte
// (8-byte for FP8) LDS read.  A is always k-contiguous in memory (transposed factor copies, Gram
// operands).  B is either k-contiguous (Grams) or n-contiguous (mode products over a tensor): the
// latter is loaded as 4 (k) x 8 (n) register blocks and transposed on the way into LDS.  The next
// k-tile is prefetched into registers while the current one is multiplied.
#include "tk_common.h"
#include "tk_lowp.h"

namespace tk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------- encodings
__device__ __forceinline__ uint16_t enc_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // RNE
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float dec_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t enc_f16(float x) {
    _Float16 h = (_Float16)x;                 // RNE conversion instruction
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float dec_f16(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// OCP E4M3: s eeee mmm, bias 7; exponent field 0 is subnormal (m * 2^-9); 0x7f / 0xff is NaN
__device__ __forceinline__ uint8_t enc_e4m3(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    const float a = fabsf(x);
    if (!(a == a)) return sign | 0x7f;
    if (a >= 464.0f) return sign | 0x7e;                 // saturate (448 and above round to 448)
    if (a < 0.015625f) {                                 // below 2^-6: subnormal grid of 2^-9
        const int m = (int)rintf(a * 512.0f);            // 0..8 (8 is the smallest normal, 0x08)
        return sign | (uint8_t)m;
    }
    const uint32_t ua = __float_as_uint(a);
    int e = (int)((ua >> 23) & 0xffu) - 127;
    uint32_t mant = ua & 0x7fffffu;
    const uint32_t r = mant + 0x7ffffu + ((mant >> 20) & 1u);   // RNE to 3 mantissa bits
    uint32_t m3 = (r >> 20) & 7u;
    if (r & 0x800000u) {
        ++e;
        m3 = 0;
    }
    const int E = e + 7;                                  // 1..15 here (a < 464)
    return sign | (uint8_t)(E << 3) | (uint8_t)m3;
}
// decode by the hardware conversion (v_cvt_f32_fp8), which reads gfx950's FP8 bytes as OCP E4M3 like
// the matrix instructions do; exact (every E4M3 value is a binary32 value)
__device__ __forceinline__ float dec_e4m3(uint8_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

template <int P> struct Codec;
template <> struct Codec<LP_BF16> {
    typedef uint16_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_bf16(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_bf16(h); }
};
template <> struct Codec<LP_F16> {
    typedef uint16_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_f16(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_f16(h); }
};
template <> struct Codec<LP_FP8> {
    typedef uint8_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_e4m3(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_e4m3(h); }
};

// eight consecutive elements: 16 bytes for 16-bit types, 8 bytes for FP8
template <int P> struct Vec8 { typedef uint4 T; };
template <> struct Vec8<LP_FP8> { typedef uint2 T; };

template <int P>
__device__ __forceinline__ f32x4 mfma32(const typename Vec8<P>::T& a, const typename Vec8<P>::T& b, f32x4 c);
template <>
__device__ __forceinline__ f32x4 mfma32<LP_BF16>(const uint4& a, const uint4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma32<LP_F16>(const uint4& a, const uint4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma32<LP_FP8>(const uint2& a, const uint2& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0,
                                                      0, 0);
}

__device__ __forceinline__ int64_t coloff(const Desc& d, int64_t c) {
    return (c / d.seg) * d.segstride + (c % d.seg);
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    if (G < 16) return b;
    const int64_t q = G / 8, r = G % 8;
    const int64_t x = b % 8, idx = b / 8;
    return x * q + (x < r ? x : r) + idx;
}

// ---------------------------------------------------------------------------- GEMM
// C(m, n) = alpha * sa[m] * sb[n % sb_mod] * sum_k A(m, k) B(k, n)
// A: k-contiguous (desc rows m, columns k).  B: OB == KN -> desc rows k, columns n (n contiguous);
// OB == MK (NK) -> desc rows n, columns k.  Output element type: float, or the 16-bit storage type
// OUTP (LP_BF16 / LP_F16) of the sweep's intermediates.
constexpr int LBM = 128, LBN = 128, LBK = 64;

template <int P, int OB, int OUTP, bool VEC>
__global__ __launch_bounds__(256, 2) void gemm_lp_kernel(LpGemmArgs g) {
    typedef typename Codec<P>::S S;
    typedef typename Vec8<P>::T V8;
    constexpr int ES = (int)sizeof(S);
    constexpr int PADK = 16 / ES;                  // 16-byte row padding
    constexpr int LDK = LBK + PADK;                // LDS row stride in elements
    __shared__ __attribute__((aligned(16))) S As[LBM * LDK];
    __shared__ __attribute__((aligned(16))) S Bs[LBN * LDK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    const int64_t tilesM = (g.M + LBM - 1) / LBM;
    const int64_t tilesN = (g.N + LBN - 1) / LBN;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t tm, tn;
    if (g.lower_only) {
        tm = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
        while (tm * (tm + 1) / 2 > t) --tm;
        tn = t - tm * (tm + 1) / 2;
    } else {
        tm = t % tilesM;
        tn = t / tilesM;
    }
    if (tn >= tilesN || tm >= tilesM) return;
    const int64_t m0 = tm * LBM, n0 = tn * LBN;
    const int64_t kbeg = (int64_t)blockIdx.z * g.k_split;
    const int64_t kend = (kbeg + g.k_split < g.K) ? kbeg + g.k_split : g.K;

    const S* __restrict__ pa = (const S*)g.a.ptr;
    const S* __restrict__ pb = (const S*)g.b.ptr;

    // k-contiguous loader (A, and B when OB == MK): 128 rows x 64 k = 1024 vectors of 8,
    // thread -> k-vector kv = tid % 8, rows tid / 8 + 32 u
    const int kv = tid & 7;
    const int rr = tid >> 3;
    // n-contiguous loader (B when OB == KN): 64 k x 128 n as 4 x 8 blocks,
    // thread -> k rows 4 * (tid % 16) .. +3, n columns 8 * (tid / 16) .. +7
    const int bkq = tid & 15;
    const int bng = tid >> 4;

    V8 ra[4], rb[4];
    S rbt[4][8];   // KN blocks: [k][n]

    // k-contiguous operand column state: the 8-run at k = kcur (advanced by LBK per tile) sits at
    // element offset kq * segstride + kr; one division at the start, increments afterwards
    struct KCol {
        int64_t kq, kr;
    };
    auto kcol_init = [&](const Desc& d, int64_t k) { return KCol{k / d.seg, k % d.seg}; };
    auto kcol_next = [&](const Desc& d, KCol& c) {
        c.kr += LBK;
        while (c.kr >= d.seg) {
            c.kr -= d.seg;
            ++c.kq;
        }
    };
    KCol ca = kcol_init(g.a, kbeg + 8 * kv);
    KCol cb = kcol_init(g.b, kbeg + 8 * kv);
    const int64_t bn_fix = (OB == KM && n0 + 8 * bng < g.N) ? coloff(g.b, n0 + 8 * bng) : 0;

    auto load_kc = [&](const S* p, const Desc& d, const KCol& c, int64_t rows, int64_t row0, int64_t k0, V8* dst) {
        const int64_t k = k0 + 8 * kv;
        const int64_t co = c.kq * d.segstride + c.kr;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + rr + 32 * u;
            V8 v;
            if (VEC && row < rows && k + 8 <= kend) {
                v = *(const V8*)(p + row * d.ld + co);
            } else {
                S e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    e[j] = (row < rows && k + j < kend) ? p[row * d.ld + coloff(d, k + j)] : (S)0;
                v = __builtin_bit_cast(V8, e);
            }
            dst[u] = v;
        }
    };
    auto load_kn = [&](int64_t k0) {
        const int64_t n = n0 + 8 * bng;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = k0 + 4 * bkq + q;
            if (VEC && k < kend && n + 8 <= g.N) {
                const V8 v = *(const V8*)(pb + k * g.b.ld + bn_fix);
                const auto e = __builtin_bit_cast(S __attribute__((ext_vector_type(8))), v);
#pragma unroll
                for (int j = 0; j < 8; ++j) rbt[q][j] = e[j];
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    rbt[q][j] = (k < kend && n + j < g.N) ? pb[k * g.b.ld + coloff(g.b, n + j)] : (S)0;
            }
        }
    };
    auto load_tiles = [&](int64_t k0) {
        load_kc(pa, g.a, ca, g.M, m0, k0, ra);
        kcol_next(g.a, ca);
        if (OB == KM) {
            load_kn(k0);
        } else {
            load_kc(pb, g.b, cb, g.N, n0, k0, rb);
            kcol_next(g.b, cb);
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int u = 0; u < 4; ++u) *(V8*)(As + (rr + 32 * u) * LDK + 8 * kv) = ra[u];
        if (OB == KM) {
            // column n of the block -> Bs[n][4 bkq .. 4 bkq + 3]
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                S e[4] = {rbt[0][j], rbt[1][j], rbt[2][j], rbt[3][j]};
                S* dst = Bs + (8 * bng + j) * LDK + 4 * bkq;
                if constexpr (ES == 2) *(uint2*)dst = __builtin_bit_cast(uint2, e);
                else *(uint32_t*)dst = __builtin_bit_cast(uint32_t, e);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) *(V8*)(Bs + (rr + 32 * u) * LDK + 8 * kv) = rb[u];
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15;
    const int fk = lane >> 4;          // which 8-wide k group of the 32-wide step
    const int wbm = wm * 64, wbn = wn * 64;

    if (kbeg < kend) {
        load_tiles(kbeg);
        store_tiles();
        __syncthreads();
        for (int64_t k0 = kbeg; k0 < kend; k0 += LBK) {
            const bool more = (k0 + LBK) < kend;
            if (more) load_tiles(k0 + LBK);
#pragma unroll
            for (int ks = 0; ks < LBK / 32; ++ks) {
                V8 av[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = *(const V8*)(As + (wbm + i * 16 + fr) * LDK + ks * 32 + 8 * fk);
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = *(const V8*)(Bs + (wbn + j * 16 + fr) * LDK + ks * 32 + 8 * fk);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mfma32<P>(av[i], bv[j], acc[i][j]);
            }
            __syncthreads();
            if (more) {
                store_tiles();
                __syncthreads();
            }
        }
    }

    // epilogue: lane holds column (lane & 15), rows 4 * (lane >> 4) + v of each 16 x 16 tile
    char* cbase = (char*)g.c.ptr;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t n = n0 + wbn + j * 16 + fr;
        if (n >= g.N) continue;
        if (g.c_valid > 0 && (n % g.c.seg) >= g.c_valid) continue;   // padding columns of a folded output
        const int64_t co = coloff(g.c, n);
        const float cs = (float)g.alpha * (g.sb ? g.sb[n % g.sb_mod] : 1.0f);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wbm + i * 16 + 4 * fk + v;
                if (m >= g.M) continue;
                float val = acc[i][j][v] * cs;
                if (g.sa) val *= g.sa[m];
                const int64_t off = (int64_t)blockIdx.z * g.c_zstride + m * g.c.ld + co;
                if (OUTP == LP_F32OUT) ((float*)cbase)[off] = val;
                else if (OUTP == LP_BF16) ((uint16_t*)cbase)[off] = enc_bf16(val);
                else ((uint16_t*)cbase)[off] = enc_f16(val);
            }
        }
    }
}

template <int P, int OB, int OUTP>
hipError_t launch_lp(const LpGemmArgs& g, bool vec, hipStream_t s) {
    const int64_t tilesM = (g.M + LBM - 1) / LBM;
    const int64_t tilesN = (g.N + LBN - 1) / LBN;
    const int64_t tiles = g.lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
    const int64_t splits = (g.K + g.k_split - 1) / g.k_split;
    if (tiles == 0) return hipSuccess;
    dim3 grid((unsigned)tiles, 1, (unsigned)(splits > 0 ? splits : 1));
    if (vec) hipLaunchKernelGGL((gemm_lp_kernel<P, OB, OUTP, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_lp_kernel<P, OB, OUTP, false>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

template <int P, int OB>
hipError_t by_out(const LpGemmArgs& g, int outp, bool vec, hipStream_t s) {
    if (outp == LP_F32OUT) return launch_lp<P, OB, LP_F32OUT>(g, vec, s);
    if (outp == LP_BF16) return launch_lp<P, OB, LP_BF16>(g, vec, s);
    if (outp == LP_F16) return launch_lp<P, OB, LP_F16>(g, vec, s);
    return hipErrorInvalidValue;
}

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
// chunk of 256 fibres is read with 16-byte coalesced loads prefetched one chunk ahead, decoded
// into LDS, mapped one fibre per thread with U3 in registers and U4 in LDS, and written back with
// 16-byte stores.  ID3: U3 is the identity (a mode kept at full rank), so its product is skipped.  Only FP8
// carries slice scales.  The decode walks each 16-byte vector's elements with one division per
// vector (fibre and position advance by increments).
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
    static_assert((FPB * LIN) % EPV == 0 && (FPB * LDO * 2) % 16 == 0, "chunk not a whole number of vectors");
    static_assert(!ID3 || PP == R3, "an identity U3 keeps the mode's size");
    static_assert(EPV <= LIN, "a vector spans at most two fibres");
    __shared__ float fin[FPB * SIN];
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
        if (ch < full) {
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
                        const float v = Codec<P>::dec(e[j]);
                        dst[l] = SCALED ? v * sc[l] : v;
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
            for (int g = threadIdx.x; g < nf * LIN; g += 256) {
                const int l = g % LIN;
                const float v = Codec<P>::dec(src[g]);
                fin[(g / LIN) * SIN + l] = SCALED ? v * sc[l] : v;
            }
        }
        __syncthreads();
        prefetch(ch + gridDim.x);
        const int f = threadIdx.x;
        if (f < nf) {
            const float* x = fin + f * SIN;
            float tmp[PP][R4];
#pragma unroll
            for (int c = 0; c < PP; ++c)
#pragma unroll
                for (int t = 0; t < R4; ++t) tmp[c][t] = 0.f;
#pragma unroll
            for (int i = 0; i < QQ; ++i) {
                float xc[PP];
#pragma unroll
                for (int c = 0; c < PP; ++c) xc[c] = x[c * QQ + i];
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
    if (g.k_split % LBK != 0 && g.k_split != g.K) return hipErrorInvalidValue;
    if (g.sb && g.sb_mod <= 0) return hipErrorInvalidValue;
    const int es = (prec == LP_FP8) ? 1 : 2;
    bool vec = desc_vec_ok(g.a, es) && desc_vec_ok(g.b, es);
    if (prec == LP_BF16) {
        return ob == KM ? by_out<LP_BF16, KM>(g, outp, vec, s) : by_out<LP_BF16, MK>(g, outp, vec, s);
    }
    if (prec == LP_F16) {
        return ob == KM ? by_out<LP_F16, KM>(g, outp, vec, s) : by_out<LP_F16, MK>(g, outp, vec, s);
    }
    if (prec == LP_FP8) {
        if (ob != KM) return hipErrorInvalidValue;   // FP8 only for the products over a tensor
        if (outp == LP_BF16) return launch_lp<LP_FP8, KM, LP_BF16>(g, vec, s);
        if (outp == LP_F32OUT) return launch_lp<LP_FP8, KM, LP_F32OUT>(g, vec, s);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

int64_t gemm_lp_blocks(const LpGemmArgs& g) {
    const int64_t tilesM = (g.M + LBM - 1) / LBM;
    const int64_t tilesN = (g.N + LBN - 1) / LBN;
    const int64_t tiles = g.lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
    const int64_t ks = (g.k_split <= 0 || g.k_split > g.K) ? g.K : g.k_split;
    return tiles * ((g.K + ks - 1) / (ks > 0 ? ks : 1));
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
