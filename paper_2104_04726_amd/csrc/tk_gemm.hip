// Dense contractions of the HOOI sweep on CDNA4 matrix cores (gfx950).
//
// One kernel template computes C(m,n) = alpha * sum_k A(m,k) B(k,n) for operands described
// by tk::Desc (row-major with an optional folded column index).  This single form covers
// every dense contraction of a sweep (Sec. III-B, eq. (8) and the Gram of the text after it):
//   * mode-n products  Y = T x_n U^T : A = U (KM), B = T viewed (A, s_n, B) (KN, folded);
//   * mode-n Grams     S = Y_(n) Y_(n)^T : A = B = Y viewed (A, s_n, B) (MK/NK, folded k);
//   * orthogonal iteration Z = S U, and the FP64 CholeskyQR products W = Z^T Z, Q = Z T^T.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid; each wave owns a (BM/2) x (BN/2) block of
// 16x16 MFMA tiles (v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64).  Operand tiles are staged
// through LDS in the orientation they have in memory ([k][m] for KM, [m][k] for MK), padded so
// that the fragment reads of the 16x16x4 layout hit distinct banks.  The next k-tile is
// prefetched into registers while the current one is multiplied.  Block ids are remapped so
// that consecutive logical tiles (same N-tile, different M-tiles) run on the same XCD and share
// its L2.
#include <atomic>

#include "tk_common.h"

// k-tile depths of the FP32 (128 x 128 tiles) and FP64 (64 x 64 tiles) kernels
#ifndef TK_F32_BK
#define TK_F32_BK 32
#endif
#ifndef TK_F64_BK
#define TK_F64_BK 16
#endif
// two LDS stages for the vector-load FP32 kernels as well (1) or only for the scalar-load ones (0)
#ifndef TK_F32_DB_VEC
#define TK_F32_DB_VEC 0
#endif

namespace tk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 V;
    static __device__ __forceinline__ V run(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef f64x4 V;
    static __device__ __forceinline__ V run(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ int64_t coloff(const Desc& d, int64_t c) {
    return (c / d.seg) * d.segstride + (c % d.seg);
}

// logical tile index for hardware block b, so that each XCD gets a contiguous range
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    if (G < 16) return b;
    const int64_t q = G / 8, r = G % 8;
    const int64_t x = b % 8, idx = b / 8;
    return x * q + (x < r ? x : r) + idx;
}

template <typename T, typename TA, typename TB, int OA, int OB, int EPI, bool ACC64, int BM, int BN,
          int BK, int VEC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    constexpr int PADKM = (sizeof(T) == 4) ? 16 : 8;   // row stride of [k][x] tiles
    constexpr int PADMK = (sizeof(T) == 4) ? 4 : 2;    // row stride of [x][k] tiles
    constexpr int LDA = (OA == KM) ? (BM + PADKM) : (BK + PADMK);
    constexpr int LDB = (OB == KM) ? (BN + PADKM) : (BK + PADMK);
    constexpr int ASZ = (OA == KM) ? BK * LDA : BM * LDA;
    constexpr int BSZ = (OB == KM) ? BK * LDB : BN * LDB;
    constexpr int EA = BM * BK / 256;   // elements of A each thread loads per k-tile
    constexpr int EB = BN * BK / 256;
    constexpr int TM = BM / 32;         // 16x16 tiles per wave along m
    constexpr int TN = BN / 32;
    typedef typename Mfma<T>::V V;

    // FP32 tiles with scalar loads use two LDS stages (the next k-tile is stored into one while the
    // other is multiplied, one barrier per k-tile); measured slower for the vector-load and FP64
    // variants, which keep one stage (barrier, store, barrier)
    constexpr bool DB = (VEC == 0 || (VEC == 4 && TK_F32_DB_VEC)) && sizeof(T) == 4;
    constexpr int NST = DB ? 2 : 1;
    __shared__ __attribute__((aligned(16))) T As2[NST * ASZ];
    __shared__ __attribute__((aligned(16))) T Bs2[NST * BSZ];
    T* As = As2;     // stage written by store_tiles
    T* Bs = Bs2;
    // VEC: both operands k-major (KM) FP32 with 4-aligned contiguous column runs; each thread moves
    // 4 consecutive columns per row as one 16-byte load and one 16-byte LDS store
    // VECK: both operands k-contiguous (MK) FP32 data with 4-aligned k runs; each operand tile is 128
    // float4 vectors, loaded by one half of the workgroup (threads 0..127 A, 128..255 B)
    constexpr bool VECK = VEC == 4 && OA == MK;
    // V2K: k-contiguous FP32 operands whose k runs are only 2-aligned (e.g. 42-long pixel fibres):
    // 8-byte vectors, two of each operand per thread (1024-element tiles)
    constexpr bool V2K = VEC == 2;
    // V4K: k-contiguous (MK) FP32 operands with 4-aligned k runs on large tiles: 16-byte vectors,
    // BM*BK/1024 of A and BN*BK/1024 of B per thread (vector tid + 256 u: row tid / (BK/4) + u 256 / (BK/4),
    // k quad tid % (BK/4)); both operands share the k position (equal segment lengths)
    constexpr bool V4K = VEC == 5;
    static_assert(VEC != 5 || (OA == MK && OB == MK && sizeof(TA) == 4 && sizeof(TB) == 4 && (BM * BK) % 1024 == 0 &&
                               (BN * BK) % 1024 == 0),
                  "16-byte k-vectors need k-contiguous FP32 operands and whole vectors per thread");
    constexpr int V4A = V4K ? BM * BK / 1024 : 1, V4B = V4K ? BN * BK / 1024 : 1;
    static_assert(VEC != 2 || (OA == MK && OB == MK && sizeof(TA) == 4 && sizeof(TB) == 4 && BM == BN &&
                               BM * BK == 1024),
                  "8-byte vector loads need k-contiguous FP32 operands and 1024-element tiles");
    static_assert(VEC != 4 || (OA == KM && OB == KM && sizeof(TA) == 4 && sizeof(TB) == 4 &&
                           (BM * BK) % 1024 == 0 && (BN * BK) % 1024 == 0) ||
                      (OA == MK && OB == MK && sizeof(TA) == 4 && sizeof(TB) == 4 && BM == BN &&
                       (BM * BK == 512 || BM * BK == 1024)),
                  "vector loads need whole float4 per thread");
    constexpr bool VK2 = VECK && BM * BK == 1024;   // every thread loads one vector of A and one of B
    // KMV: both operands k-major (KM) FP32 with contiguous column runs of KW (VEC 4: runs of 4 as 16-byte
    // loads; VEC 3: runs only 2-aligned, e.g. 42-long folded pixel fibres, as 8-byte loads)
    constexpr bool KMV = (VEC == 4 || VEC == 3) && OA == KM;
    constexpr int KW = (VEC == 3) ? 2 : 4;
    static_assert(VEC != 3 || (OA == KM && OB == KM && sizeof(TA) == 4 && sizeof(TB) == 4 &&
                               (BM * BK) % 512 == 0 && (BN * BK) % 512 == 0),
                  "8-byte k-major loads need FP32 operands and whole float2 per thread");
    // D2: FP64 operands with 2-aligned contiguous runs (64 x 64 x 16 tiles): 16-byte loads of two
    // doubles, two per operand per thread.  KM tile (16 k-rows x 64): row tid / 32 + 8 u, column
    // pair tid % 32; MK tile (64 rows x 16 k): row tid / 8 + 32 u, k pair tid % 8.
    constexpr bool D2 = VEC == 8;
    static_assert(!D2 || (sizeof(T) == 8 && sizeof(TA) == 8 && sizeof(TB) == 8 && BM == 64 && BN == 64 && BK == 16),
                  "two-double loads need FP64 operands and 64 x 64 x 16 tiles");
    if (g.run_if && *g.run_if == 0) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // ---- tile coordinates
    const int64_t tilesM = (g.M + BM - 1) / BM;
    const int64_t tilesN = (g.N + BN - 1) / BN;
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
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
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * g.k_split;
    int64_t kend = (kbeg + g.k_split < g.K) ? kbeg + g.k_split : g.K;
    if (g.k_upto_n && n0 + BN < kend) kend = n0 + BN;   // triangular B: the rest of k contributes zero

    const TA* __restrict__ pa = (const TA*)g.a.ptr;
    const TB* __restrict__ pb = (const TB*)g.b.ptr;

    // ---- per-thread load coordinates
    // KM tile: BK rows (k) x BM cols (m): thread -> col c = tid % BM, rows r0 + step*u
    // MK tile: BM rows (m) x BK cols (k): thread -> col c = tid % BK, rows r0 + step*u
    const int a_c = (OA == KM) ? (tid % BM) : (tid % BK);
    const int a_r0 = (OA == KM) ? (tid / BM) : (tid / BK);
    constexpr int a_step = (OA == KM) ? (256 / BM) : (256 / BK);
    const int b_c = (OB == KM) ? (tid % BN) : (tid % BK);
    const int b_r0 = (OB == KM) ? (tid / BN) : (tid / BK);
    constexpr int b_step = (OB == KM) ? (256 / BN) : (256 / BK);

    // KM: the column (m or n) is fixed for the whole K loop
    int64_t a_fix = 0, b_fix = 0;
    bool a_colok = true, b_colok = true;
    if (OA == KM && !KMV) {
        a_colok = (m0 + a_c) < g.M;
        a_fix = a_colok ? coloff(g.a, m0 + a_c) : 0;
    }
    if (OB == KM && !KMV) {
        b_colok = (n0 + b_c) < g.N;
        b_fix = b_colok ? coloff(g.b, n0 + b_c) : 0;
    }
    // VECK mapping: 512-element tiles: half h = tid / 128 (0: A, 1: B), row = (tid % 128) / (BK / 4);
    // 1024-element tiles (VK2): every thread one vector of each operand, row = tid / (BK / 4)
    const int vk_half = VK2 ? 0 : (tid >> 7);
    const int vk_row = VK2 ? tid / (BK / 4) : (tid & 127) / (BK / 4);
    const int vk_k4 = tid % (BK / 4);
    struct KCol4 {
        int64_t kq, kr;
    };
    KCol4 vkc{0, 0};
    if constexpr (VECK) {
        const Desc& d = vk_half ? g.b : g.a;
        const int64_t k = kbeg + 4 * vk_k4;
        vkc = KCol4{k / d.seg, k % d.seg};
    }
    float4 vk_reg = make_float4(0.f, 0.f, 0.f, 0.f), vk_reg2 = make_float4(0.f, 0.f, 0.f, 0.f);
    // V2K mapping: vector index tid + 256 u (u = 0, 1) -> row (tid / (BK/2)) + 32 u, k pair tid % (BK/2)
    constexpr int v2_rstep = 256 / (BK / 2 > 0 ? BK / 2 : 1);
    const int v2_row = tid / (BK / 2 > 0 ? BK / 2 : 1);
    const int v2_kw = tid % (BK / 2 > 0 ? BK / 2 : 1);
    KCol4 v2c{0, 0};
    if constexpr (V2K) {
        const int64_t k = kbeg + 2 * v2_kw;
        v2c = KCol4{k / g.a.seg, k % g.a.seg};
    }
    float2 v2a[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    constexpr int v4_rstep = 256 / (BK / 4 > 0 ? BK / 4 : 1);
    const int v4_row = tid / (BK / 4 > 0 ? BK / 4 : 1);
    const int v4_k4 = tid % (BK / 4 > 0 ? BK / 4 : 1);
    KCol4 v4c{0, 0};
    if constexpr (V4K) {
        const int64_t k = kbeg + 4 * v4_k4;
        v4c = KCol4{k / g.a.seg, k % g.a.seg};
    }
    float4 v4a[V4A], v4b[V4B];
    float2 v2b[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    auto ld2 = [&](const Desc& d, int64_t rows, int64_t row, int64_t k) {
        float2 v = make_float2(0.f, 0.f);
        if (row < rows) {
            const TA* src = (const TA*)d.ptr + row * d.ld + v2c.kq * d.segstride + v2c.kr;
            if (k + 2 <= kend) {
                v = *(const float2*)src;
            } else if (k < kend) {
                v.x = src[0];
            }
        }
        return v;
    };
    // KMV mapping: thread -> column group c4 (KW columns), rows r0 + step * u
    constexpr int A4 = BM / KW, B4 = BN / KW;
    constexpr int av_step = 256 / A4, bv_step = 256 / B4;
    const int av_c4 = tid % A4, av_r0 = tid / A4;
    const int bv_c4 = tid % B4, bv_r0 = tid / B4;
    int64_t av_fix = 0, bv_fix = 0;
    int av_n = 0, bv_n = 0;      // valid columns of the thread's group (0..KW)
    if (KMV) {
        const int64_t ca = m0 + KW * av_c4, cb = n0 + KW * bv_c4;
        av_n = (int)((g.M - ca) < KW ? ((g.M - ca) > 0 ? (g.M - ca) : 0) : KW);
        bv_n = (int)((g.N - cb) < KW ? ((g.N - cb) > 0 ? (g.N - cb) : 0) : KW);
        av_fix = av_n > 0 ? coloff(g.a, ca) : 0;
        bv_fix = bv_n > 0 ? coloff(g.b, cb) : 0;
    }

    T ra[EA], rb[EB];

    // D2 coordinates: fixed column offset (KM) or incremental k position (MK) per operand
    struct D2Op {
        int64_t fix;     // KM: offset of the thread's column pair
        bool colok;      // KM: the pair is inside the matrix
        int64_t kq, kr;  // MK: segment and offset of the thread's k pair
    };
    D2Op d2o[2] = {{0, false, 0, 0}, {0, false, 0, 0}};
    double2 d2v[2][2];
    if constexpr (D2) {
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const Desc& d = o ? g.b : g.a;
            const int orient = o ? OB : OA;
            const int64_t x0 = o ? n0 : m0, ext = o ? g.N : g.M;
            if (orient == KM) {
                const int64_t c = x0 + 2 * (tid % 32);
                d2o[o].colok = c < ext;
                d2o[o].fix = d2o[o].colok ? coloff(d, c) : 0;
            } else {
                const int64_t k = kbeg + 2 * (tid % 8);
                d2o[o].kq = k / d.seg;
                d2o[o].kr = k % d.seg;
            }
        }
    }
    auto d2_load = [&](int o, int64_t k0) {
        const Desc& d = o ? g.b : g.a;
        const int orient = o ? OB : OA;
        const double* base = (const double*)d.ptr;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            double2 v = make_double2(0.0, 0.0);
            if (orient == KM) {
                const int64_t k = k0 + tid / 32 + 8 * u;
                if (d2o[o].colok && k < kend) v = *(const double2*)(base + k * d.ld + d2o[o].fix);
            } else {
                const int64_t row = (o ? n0 : m0) + tid / 8 + 32 * u;
                const int64_t k = k0 + 2 * (tid % 8);
                if (row < (o ? g.N : g.M) && k < kend) {
                    const double* src = base + row * d.ld + d2o[o].kq * d.segstride + d2o[o].kr;
                    if (k + 2 <= kend) {
                        v = *(const double2*)src;
                    } else {
                        v.x = src[0];
                    }
                }
            }
            d2v[o][u] = v;
        }
        if (orient == MK) {
            d2o[o].kr += BK;
            while (d2o[o].kr >= d.seg) {
                d2o[o].kr -= d.seg;
                ++d2o[o].kq;
            }
        }
    };

    // MK operands: the column offset of k = kbeg + (thread's k column) advances by BK per k-tile;
    // one division at the start, increments afterwards (loads always advance tile by tile)
    struct KCol {
        int64_t kq, kr;
    };
    auto kcol_next = [&](const Desc& d, KCol& c) {
        c.kr += BK;
        while (c.kr >= d.seg) {
            c.kr -= d.seg;
            ++c.kq;
        }
    };
    KCol kca{0, 0}, kcb{0, 0};
    if (OA == MK) kca = KCol{(kbeg + a_c) / g.a.seg, (kbeg + a_c) % g.a.seg};
    if (OB == MK) kcb = KCol{(kbeg + b_c) / g.b.seg, (kbeg + b_c) % g.b.seg};

    auto load_vec = [&](const TA* p, const Desc& d, int64_t fix, int nvalid, int r0, int step, int64_t k0, T* dst,
                        int count) {
        for (int u = 0; u < count; ++u) {
            const int64_t k = k0 + r0 + step * u;
            if constexpr (KW == 4) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k < kend && nvalid > 0) {
                    const TA* src = p + k * d.ld + fix;
                    if (nvalid == 4) {
                        v = *(const float4*)src;
                    } else {
                        v.x = src[0];
                        if (nvalid > 1) v.y = src[1];
                        if (nvalid > 2) v.z = src[2];
                    }
                }
                dst[4 * u + 0] = v.x;
                dst[4 * u + 1] = v.y;
                dst[4 * u + 2] = v.z;
                dst[4 * u + 3] = v.w;
            } else {
                float2 v = make_float2(0.f, 0.f);
                if (k < kend && nvalid > 0) {
                    const TA* src = p + k * d.ld + fix;
                    if (nvalid == 2) v = *(const float2*)src;
                    else v.x = src[0];
                }
                dst[2 * u + 0] = v.x;
                dst[2 * u + 1] = v.y;
            }
        }
    };
    auto load_tiles = [&](int64_t k0) {
        if constexpr (D2) {
            d2_load(0, k0);
            d2_load(1, k0);
            return;
        }
        if constexpr (VECK) {
            auto ld4 = [&](const Desc& d, int64_t rows, int64_t row, int64_t k) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (row < rows) {
                    const TA* src = (const TA*)d.ptr + row * d.ld + vkc.kq * d.segstride + vkc.kr;
                    if (k + 4 <= kend) {
                        v = *(const float4*)src;
                    } else {
                        if (k < kend) v.x = src[0];
                        if (k + 1 < kend) v.y = src[1];
                        if (k + 2 < kend) v.z = src[2];
                    }
                }
                return v;
            };
            const int64_t k = k0 + 4 * vk_k4;
            // A and B share the k position (same segment structure is required of VK2 operands)
            if (VK2) {
                vk_reg = ld4(g.a, g.M, m0 + vk_row, k);
                vk_reg2 = ld4(g.b, g.N, n0 + vk_row, k);
            } else {
                vk_reg = vk_half ? ld4(g.b, g.N, n0 + vk_row, k) : ld4(g.a, g.M, m0 + vk_row, k);
            }
            const Desc& d = vk_half ? g.b : g.a;
            vkc.kr += BK;
            while (vkc.kr >= d.seg) {
                vkc.kr -= d.seg;
                ++vkc.kq;
            }
            return;
        }
        if constexpr (V4K) {
            auto ld4 = [&](const Desc& d, int64_t rows, int64_t row, int64_t k) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (row < rows) {
                    const TA* src = (const TA*)d.ptr + row * d.ld + v4c.kq * d.segstride + v4c.kr;
                    if (k + 4 <= kend) {
                        v = *(const float4*)src;
                    } else {
                        if (k < kend) v.x = src[0];
                        if (k + 1 < kend) v.y = src[1];
                        if (k + 2 < kend) v.z = src[2];
                    }
                }
                return v;
            };
            const int64_t k = k0 + 4 * v4_k4;
#pragma unroll
            for (int u = 0; u < V4A; ++u) v4a[u] = ld4(g.a, g.M, m0 + v4_row + v4_rstep * u, k);
#pragma unroll
            for (int u = 0; u < V4B; ++u) v4b[u] = ld4(g.b, g.N, n0 + v4_row + v4_rstep * u, k);
            v4c.kr += BK;
            while (v4c.kr >= g.a.seg) {
                v4c.kr -= g.a.seg;
                ++v4c.kq;
            }
            return;
        }
        if constexpr (V2K) {
            const int64_t k = k0 + 2 * v2_kw;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int row = v2_row + v2_rstep * u;
                v2a[u] = ld2(g.a, g.M, m0 + row, k);
                v2b[u] = ld2(g.b, g.N, n0 + row, k);
            }
            v2c.kr += BK;
            while (v2c.kr >= g.a.seg) {
                v2c.kr -= g.a.seg;
                ++v2c.kq;
            }
            return;
        }
        if constexpr (KMV) {
            load_vec((const TA*)pa, g.a, av_fix, av_n, av_r0, av_step, k0, ra, EA / KW);
            load_vec((const TA*)pb, g.b, bv_fix, bv_n, bv_r0, bv_step, k0, rb, EB / KW);
            return;
        }
        if (OA == KM) {
#pragma unroll
            for (int u = 0; u < EA; ++u) {
                const int64_t k = k0 + a_r0 + a_step * u;
                ra[u] = (a_colok && k < kend) ? (T)pa[k * g.a.ld + a_fix] : (T)0;
            }
        } else {
            const int64_t k = k0 + a_c;
            const bool kok = k < kend;
            const int64_t ko = kca.kq * g.a.segstride + kca.kr;
#pragma unroll
            for (int u = 0; u < EA; ++u) {
                const int64_t m = m0 + a_r0 + a_step * u;
                ra[u] = (kok && m < g.M) ? (T)pa[m * g.a.ld + ko] : (T)0;
            }
            kcol_next(g.a, kca);
        }
        if (OB == KM) {
#pragma unroll
            for (int u = 0; u < EB; ++u) {
                const int64_t k = k0 + b_r0 + b_step * u;
                rb[u] = (b_colok && k < kend) ? (T)pb[k * g.b.ld + b_fix] : (T)0;
            }
        } else {
            const int64_t k = k0 + b_c;
            const bool kok = k < kend;
            const int64_t ko = kcb.kq * g.b.segstride + kcb.kr;
#pragma unroll
            for (int u = 0; u < EB; ++u) {
                const int64_t n = n0 + b_r0 + b_step * u;
                rb[u] = (kok && n < g.N) ? (T)pb[n * g.b.ld + ko] : (T)0;
            }
            kcol_next(g.b, kcb);
        }
    };
    auto store_tiles = [&]() {
        if constexpr (D2) {
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                T* dst = o ? Bs : As;
                const int ld = o ? LDB : LDA;
                const int orient = o ? OB : OA;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int idx = (orient == KM) ? (tid / 32 + 8 * u) * ld + 2 * (tid % 32)
                                                   : (tid / 8 + 32 * u) * ld + 2 * (tid % 8);
                    *(double2*)&dst[idx] = d2v[o][u];
                }
            }
            return;
        }
        if constexpr (VECK) {
            T* dst = (vk_half ? Bs : As) + vk_row * (vk_half ? LDB : LDA) + 4 * vk_k4;
            dst[0] = (T)vk_reg.x;
            dst[1] = (T)vk_reg.y;
            dst[2] = (T)vk_reg.z;
            dst[3] = (T)vk_reg.w;
            if (VK2) {
                T* d2 = Bs + vk_row * LDB + 4 * vk_k4;
                d2[0] = (T)vk_reg2.x;
                d2[1] = (T)vk_reg2.y;
                d2[2] = (T)vk_reg2.z;
                d2[3] = (T)vk_reg2.w;
            }
            return;
        }
        if constexpr (V4K) {
#pragma unroll
            for (int u = 0; u < V4A; ++u) *(float4*)&As[(v4_row + v4_rstep * u) * LDA + 4 * v4_k4] = v4a[u];
#pragma unroll
            for (int u = 0; u < V4B; ++u) *(float4*)&Bs[(v4_row + v4_rstep * u) * LDB + 4 * v4_k4] = v4b[u];
            return;
        }
        if constexpr (V2K) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int row = v2_row + v2_rstep * u;
                T* da = As + row * LDA + 2 * v2_kw;
                da[0] = (T)v2a[u].x;
                da[1] = (T)v2a[u].y;
                T* db = Bs + row * LDB + 2 * v2_kw;
                db[0] = (T)v2b[u].x;
                db[1] = (T)v2b[u].y;
            }
            return;
        }
        if constexpr (VEC == 3 && OA == KM) {
#pragma unroll
            for (int u = 0; u < EA / 2; ++u) {
                T* d = &As[(av_r0 + av_step * u) * LDA + 2 * av_c4];
                if constexpr (sizeof(T) == 4) *(float2*)d = make_float2(ra[2 * u], ra[2 * u + 1]);
                else *(double2*)d = make_double2(ra[2 * u], ra[2 * u + 1]);
            }
#pragma unroll
            for (int u = 0; u < EB / 2; ++u) {
                T* d = &Bs[(bv_r0 + bv_step * u) * LDB + 2 * bv_c4];
                if constexpr (sizeof(T) == 4) *(float2*)d = make_float2(rb[2 * u], rb[2 * u + 1]);
                else *(double2*)d = make_double2(rb[2 * u], rb[2 * u + 1]);
            }
            return;
        }
        if constexpr (VEC == 4 && OA == KM) {
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int u = 0; u < EA / 4; ++u)
                    *(float4*)&As[(av_r0 + av_step * u) * LDA + 4 * av_c4] =
                        make_float4(ra[4 * u], ra[4 * u + 1], ra[4 * u + 2], ra[4 * u + 3]);
#pragma unroll
                for (int u = 0; u < EB / 4; ++u)
                    *(float4*)&Bs[(bv_r0 + bv_step * u) * LDB + 4 * bv_c4] =
                        make_float4(rb[4 * u], rb[4 * u + 1], rb[4 * u + 2], rb[4 * u + 3]);
            } else {
                // FP64 tiles of FP32 data: the 4 converted values as two 16-byte LDS stores
#pragma unroll
                for (int u = 0; u < EA / 4; ++u) {
                    double2* d = (double2*)&As[(av_r0 + av_step * u) * LDA + 4 * av_c4];
                    d[0] = make_double2(ra[4 * u], ra[4 * u + 1]);
                    d[1] = make_double2(ra[4 * u + 2], ra[4 * u + 3]);
                }
#pragma unroll
                for (int u = 0; u < EB / 4; ++u) {
                    double2* d = (double2*)&Bs[(bv_r0 + bv_step * u) * LDB + 4 * bv_c4];
                    d[0] = make_double2(rb[4 * u], rb[4 * u + 1]);
                    d[1] = make_double2(rb[4 * u + 2], rb[4 * u + 3]);
                }
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < EA; ++u) As[(a_r0 + a_step * u) * LDA + a_c] = ra[u];
#pragma unroll
        for (int u = 0; u < EB; ++u) Bs[(b_r0 + b_step * u) * LDB + b_c] = rb[u];
    };

    V acc[TM][TN];
    double acc64[ACC64 ? TM : 1][ACC64 ? TN : 1][ACC64 ? 4 : 1];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            acc[i][j] = V{0, 0, 0, 0};
            if (ACC64) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[ACC64 ? i : 0][ACC64 ? j : 0][ACC64 ? v : 0] = 0.0;
            }
        }

    const int fr = lane & 15;       // row (m or n) inside a 16x16 tile
    const int fk = lane >> 4;       // k inside a 4-wide k-step
    const int wbm = wm * (BM / 2), wbn = wn * (BN / 2);

    if (kbeg < kend) {
        load_tiles(kbeg);
        store_tiles();
        __syncthreads();
        int stage = 0;
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            const bool more = (k0 + BK) < kend;
            if (more) load_tiles(k0 + BK);
            const T* Ac = As2 + stage * ASZ;
            const T* Bc = Bs2 + stage * BSZ;
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                const int k = kk * 4 + fk;
                T av[TM], bv[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int m = wbm + i * 16 + fr;
                    av[i] = (OA == KM) ? Ac[k * LDA + m] : Ac[m * LDA + k];
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int n = wbn + j * 16 + fr;
                    bv[j] = (OB == KM) ? Bc[k * LDB + n] : Bc[n * LDB + k];
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::run(av[i], bv[j], acc[i][j]);
            }
            if (ACC64) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc64[ACC64 ? i : 0][ACC64 ? j : 0][ACC64 ? v : 0] += (double)acc[i][j][v];
                        acc[i][j] = V{0, 0, 0, 0};
                    }
            }
            if constexpr (DB) {
                // the other stage was last read before the previous barrier: store into it, then
                // one barrier makes it readable and frees this stage for the store after next
                if (more) {
                    stage ^= 1;
                    As = As2 + stage * ASZ;
                    Bs = Bs2 + stage * BSZ;
                    store_tiles();
                }
                __syncthreads();
            } else {
                __syncthreads();
                if (more) {
                    store_tiles();
                    __syncthreads();
                }
            }
        }
    }

    // ---- epilogue.  16x16x4 output layout: lane holds column (lane & 15); its 4 accumulator
    // entries are rows 4*(lane>>4)+v for the f32 instruction and rows (lane>>4)+4*v for f64.
    T* __restrict__ pc = (T*)g.c.ptr + (int64_t)blockIdx.z * g.c_zstride;
    double rsum = 0.0;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wbn + j * 16 + fr;
        if (n >= g.N) continue;
        const int64_t co = coloff(g.c, n);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wbm + i * 16 + (sizeof(T) == 4 ? 4 * fk + v : fk + 4 * v);
                if (m >= g.M) continue;
                const double val =
                    ACC64 ? acc64[ACC64 ? i : 0][ACC64 ? j : 0][ACC64 ? v : 0] : (double)acc[i][j][v];
                T* dst = pc + m * g.c.ld + co;
                if (EPI == EPI_STORE && sizeof(T) == 8 && g.c_f32) {
                    ((float*)g.c.ptr)[(int64_t)blockIdx.z * g.c_zstride + m * g.c.ld + co] = (float)(g.alpha * val);
                } else if (EPI == EPI_STORE) {
                    *dst = (T)(g.alpha * val);
                } else if (EPI == EPI_ADD) {
                    *dst = (T)(g.alpha * val + (double)*dst);
                } else {
                    const double d = (double)*dst - (double)(T)(g.alpha * val);
                    rsum += d * d;
                }
            }
        }
    }
    if (EPI == EPI_RESID) {
        __shared__ double red[256];
        red[tid] = rsum;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0)
            g.resid_partial[(int64_t)blockIdx.z * gridDim.x + blockIdx.x] = red[0];
    }
}

template <typename T, int BM, int BN>
dim3 grid_of(const GemmArgs& g) {
    const int64_t tilesM = (g.M + BM - 1) / BM;
    const int64_t tilesN = (g.N + BN - 1) / BN;
    const int64_t tiles = g.lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
    const int64_t splits = (g.K + g.k_split - 1) / (g.k_split > 0 ? g.k_split : 1);
    return dim3((unsigned)tiles, 1, (unsigned)(splits > 0 ? splits : 1));
}

// k-major FP32 operand whose rows are read as aligned runs of 4 contiguous columns
bool km_vec_ok(const Desc& d) {
    const bool segok = d.seg >= (int64_t(1) << 61) || (d.seg % 4 == 0 && d.segstride % 4 == 0);
    return segok && d.ld % 4 == 0 && (((uintptr_t)d.ptr) & 15) == 0;
}

template <typename T, typename TA, typename TB, int OA, int OB, int EPI, bool ACC64, int BM, int BN,
          int BK>
hipError_t launch_one(const GemmArgs& g, hipStream_t s) {
    dim3 grid = grid_of<T, BM, BN>(g);
    if (grid.x == 0) return hipSuccess;
    constexpr bool can_vec = (OA == KM && OB == KM && sizeof(TA) == 4 && sizeof(TB) == 4 &&
                              (BM * BK) % 1024 == 0 && (BN * BK) % 1024 == 0) ||
                             (OA == MK && OB == MK && sizeof(TA) == 4 && sizeof(TB) == 4 && BM == BN &&
                              (BM * BK == 512 || BM * BK == 1024));
    if constexpr (can_vec) {
        // the 1024-element form advances one k position for both operands: equal segment lengths
        // (each operand keeps its own segment stride)
        const bool same_seg = !(OA == MK && BM * BK == 1024) || g.a.seg == g.b.seg;
        if (km_vec_ok(g.a) && km_vec_ok(g.b) && same_seg && (OA == KM || g.k_split % 4 == 0)) {
            hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 4>), grid, dim3(256), 0, s,
                               g);
            return hipGetLastError();
        }
    }
    constexpr bool can_km2 = OA == KM && OB == KM && sizeof(TA) == 4 && sizeof(TB) == 4 && (BM * BK) % 512 == 0 &&
                             (BN * BK) % 512 == 0;
    if constexpr (can_km2) {
        // k-major rows read as 2-aligned runs of 2 columns (8-byte loads), e.g. 42-long folded fibres
        auto ok2 = [](const Desc& d) {
            const bool segok = d.seg >= (int64_t(1) << 61) || (d.seg % 2 == 0 && d.segstride % 2 == 0);
            return segok && d.ld % 2 == 0 && (((uintptr_t)d.ptr) & 7) == 0;
        };
        if (ok2(g.a) && ok2(g.b)) {
            hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 3>), grid, dim3(256), 0, s,
                               g);
            return hipGetLastError();
        }
    }
    constexpr bool can_vec2 = OA == MK && OB == MK && sizeof(TA) == 4 && sizeof(TB) == 4 && BM == BN &&
                              BM * BK == 1024;
    if constexpr (can_vec2) {
        auto ok2 = [](const Desc& d) {
            const bool segok = d.seg >= (int64_t(1) << 61) || (d.seg % 2 == 0 && d.segstride % 2 == 0);
            return segok && d.ld % 2 == 0 && (((uintptr_t)d.ptr) & 7) == 0;
        };
        // one k position for both operands: equal segment lengths (each keeps its own stride)
        if (ok2(g.a) && ok2(g.b) && g.a.seg == g.b.seg && g.k_split % 2 == 0) {
            hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 2>), grid, dim3(256), 0, s,
                               g);
            return hipGetLastError();
        }
    }
    constexpr bool can_v4k = OA == MK && OB == MK && sizeof(T) == 4 && sizeof(TA) == 4 && sizeof(TB) == 4 && !ACC64 &&
                             (BM * BK) % 1024 == 0 && (BN * BK) % 1024 == 0 && BM * BK > 1024;
    if constexpr (can_v4k) {
        // 16-byte k-vectors on large FP32 tiles: both operands 4-aligned k runs of equal segment length
        if (km_vec_ok(g.a) && km_vec_ok(g.b) && g.a.seg == g.b.seg && g.k_split % 4 == 0) {
            hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 5>), grid, dim3(256), 0, s,
                               g);
            return hipGetLastError();
        }
    }
    constexpr bool can_d2 = sizeof(T) == 8 && sizeof(TA) == 8 && sizeof(TB) == 8 && BM == 64 && BN == 64 && BK == 16;
    if constexpr (can_d2) {
        // 16-byte loads: runs of the contiguous index are 2-aligned and (KM) the extent is even
        auto okd = [](const Desc& d, int orient, int64_t ext) {
            const bool segok = d.seg >= (int64_t(1) << 61) || (d.seg % 2 == 0 && d.segstride % 2 == 0);
            return segok && d.ld % 2 == 0 && (((uintptr_t)d.ptr) & 15) == 0 && (orient == MK || ext % 2 == 0);
        };
        if (okd(g.a, OA, g.M) && okd(g.b, OB, g.N) && g.k_split % 2 == 0) {
            hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 8>), grid, dim3(256), 0, s,
                               g);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, OA, OB, EPI, ACC64, BM, BN, BK, 0>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

template <typename T, typename TA, typename TB, int EPI, bool ACC64, int BM, int BN, int BK>
hipError_t by_orient(const GemmArgs& g, Orient oa, Orient ob, hipStream_t s) {
    if (oa == KM && ob == KM) return launch_one<T, TA, TB, KM, KM, EPI, ACC64, BM, BN, BK>(g, s);
    if (oa == KM && ob == MK) return launch_one<T, TA, TB, KM, MK, EPI, ACC64, BM, BN, BK>(g, s);
    if (oa == MK && ob == KM) return launch_one<T, TA, TB, MK, KM, EPI, ACC64, BM, BN, BK>(g, s);
    return launch_one<T, TA, TB, MK, MK, EPI, ACC64, BM, BN, BK>(g, s);
}

// 128 x 64 instead of 128 x 128 output tiles for an FP32 product when the wide tiles leave the CUs
// unevenly loaded (average over maximum tiles per CU more than 5% better with narrow tiles) or
// under-filled (fewer than 1.5 wide tiles per CU): measured 405 -> 376 us for 609 wide tiles and
// 215 -> 203 us for 252, and slower where the wide tiles already balance.
bool narrow_tiles_pay(const GemmArgs& g) {
    const int64_t cus = device_cu_count();
    const int64_t tm = (g.M + 127) / 128;
    const int64_t t128 = tm * ((g.N + 127) / 128) * ((g.K + g.k_split - 1) / g.k_split);
    const int64_t t64 = tm * ((g.N + 63) / 64) * ((g.K + g.k_split - 1) / g.k_split);
    auto balance = [&](int64_t t) { return ((double)t / cus) / (double)((t + cus - 1) / cus); };
    return 2 * t128 < 3 * cus || balance(t64) > 1.05 * balance(t128);
}

GemmArgs normalised(const GemmArgs& in) {
    GemmArgs g = in;
    if (g.k_split <= 0 || g.k_split > g.K) g.k_split = g.K > 0 ? g.K : 1;
    return g;
}

}  // namespace

int64_t gemm_grid_blocks(const GemmArgs& gin, bool f64) {
    GemmArgs g = normalised(gin);
    dim3 d = f64 ? grid_of<double, 64, 64>(g) : grid_of<float, 128, 128>(g);
    return (int64_t)d.x * d.z;
}

hipError_t gemm_f32(const GemmArgs& gin, Orient oa, Orient ob, Epilogue epi, bool acc64,
                    hipStream_t s) {
    GemmArgs g = normalised(gin);
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (epi == EPI_STORE) {
        if (acc64) return by_orient<float, float, float, EPI_STORE, true, 128, 128, TK_F32_BK>(g, oa, ob, s);
        // output tile 128 x 128 (0) or 128 x 64 (1): the same sums in the same order either way, so the
        // choice is left to the autotuner (the load-balance heuristic without it)
        auto launch = [&](int c) {
            return c == 1 ? by_orient<float, float, float, EPI_STORE, false, 128, 64, TK_F32_BK>(g, oa, ob, s)
                          : by_orient<float, float, float, EPI_STORE, false, 128, 128, TK_F32_BK>(g, oa, ob, s);
        };
        const int64_t shape[5] = {g.M, g.N, g.K, g.k_split,
                                  (int64_t)oa * 4 + (int64_t)ob * 2 + (g.b.seg < (int64_t(1) << 61) ? 1 : 0)};
        hipError_t e = hipSuccess;
        const int c = tune_choose(kTuneF32Tile, shape, 2, narrow_tiles_pay(g) ? 1 : 0, s, launch, &e);
        if (e != hipSuccess) return e;
        return launch(c);
    }
    if (epi == EPI_ADD) return by_orient<float, float, float, EPI_ADD, false, 128, 128, TK_F32_BK>(g, oa, ob, s);
    return by_orient<float, float, float, EPI_RESID, false, 128, 128, TK_F32_BK>(g, oa, ob, s);
}

hipError_t gemm_f64(const GemmArgs& gin, Orient oa, Orient ob, Epilogue epi, bool a_is_f32,
                    bool b_is_f32, hipStream_t s) {
    GemmArgs g = normalised(gin);
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (epi != EPI_STORE) return hipErrorInvalidValue;
    if (a_is_f32 && b_is_f32) return by_orient<double, float, float, EPI_STORE, false, 64, 64, TK_F64_BK>(g, oa, ob, s);
    if (a_is_f32) return by_orient<double, float, double, EPI_STORE, false, 64, 64, 16>(g, oa, ob, s);
    if (b_is_f32) return by_orient<double, double, float, EPI_STORE, false, 64, 64, 16>(g, oa, ob, s);
    return by_orient<double, double, double, EPI_STORE, false, 64, 64, 16>(g, oa, ob, s);
}

int device_cu_count() {
    static std::atomic<int> cached{0};
    int c = cached.load(std::memory_order_relaxed);
    if (c > 0) return c;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
        c = 256;
    cached.store(c, std::memory_order_relaxed);
    return c;
}

int gram_f64_blocks_per_cu() {
    int per = 0;
    const void* k = reinterpret_cast<const void*>(&gemm_kernel<double, float, float, MK, MK, EPI_STORE, false, 64, 64,
                                                               TK_F64_BK, 4>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 256, 0) != hipSuccess) return 0;
    return per;
}

}  // namespace tk
