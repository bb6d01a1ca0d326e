// The reduced-precision GEMM kernel and its launch variants (internal: each of the per-type
// translation units tk_lowp_gemm_{bf16,f16,fp8}.hip includes this and instantiates one storage type,
// so that the variants compile in parallel).
//
// GEMM tiling: 256 threads = 4 waves in a 2x2 grid over a 128 x 128 output tile; each wave owns
// 4 x 4 MFMA tiles of 16 x 16 and steps k by 32.  Both operands sit in LDS with k contiguous
// ([row][k], rows padded by 16 bytes), so a lane's eight consecutive k values are one 16-byte
// (8-byte for FP8) LDS read.  A is always k-contiguous in memory (transposed factor copies, Gram
// operands).  B is either k-contiguous (Grams) or n-contiguous (mode products over a tensor): the
// latter is loaded as 4 (k) x 8 (n) register blocks and transposed on the way into LDS.  The next
// k-tile is prefetched into registers while the current one is multiplied.
#pragma once
#include <algorithm>
#include <type_traits>

#include "tk_lowp_impl.h"

namespace tk {
namespace {

// ---------------------------------------------------------------------------- GEMM
// C(m, n) = alpha * sa[m] * sb[n % sb_mod] * sum_k A(m, k) B(k, n)
// A: k-contiguous (desc rows m, columns k).  B: OB == KN -> desc rows k, columns n (n contiguous);
// OB == MK (NK) -> desc rows n, columns k.  Output element type: float, or the 16-bit storage type
// OUTP (LP_BF16 / LP_F16) of the sweep's intermediates.
constexpr int LBN = 128, LBK = kLpGemmK;

// NST: LDS stages (2: the next k-tile is stored into the other stage while this one is multiplied, one
// barrier per k-tile).  OCC: workgroups per CU the register budget is sized for.  Neither changes any
// output element's sum or its order, so the variants give identical results and are left to the
// autotuner.
//
// Workgroups whose 128 x 128 output tile lies inside C (and whose operands allow vector loads) run
// their full 64-wide k-tiles through a loader without bounds checks; the last, partial k-tile and
// the edge tiles take the checked loader.
// One output tile (logical tile index t, k split z) of C; every thread of the workgroup calls it.
template <int P, int OB, int OUTP, bool VEC, int NST>
__device__ __forceinline__ void gemm_lp_tile(const LpGemmArgs& g, int64_t t, int64_t z) {
    typedef typename Codec<P>::S S;
    typedef typename Vec8<P>::T V8;
    constexpr int ES = (int)sizeof(S);
    constexpr int PADK = 16 / ES;                  // 16-byte row padding
    constexpr int LDK = LBK + PADK;                // LDS row stride in elements
    constexpr int BMT = 128;
    __shared__ __attribute__((aligned(16))) S As2[NST * BMT * LDK];
    __shared__ __attribute__((aligned(16))) S Bs2[NST * LBN * LDK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    const int64_t tilesM = (g.M + BMT - 1) / BMT;
    const int64_t tilesN = (g.N + LBN - 1) / LBN;
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
    const int64_t m0 = tm * BMT, n0 = tn * LBN;
    const int64_t kbeg = z * g.k_split;
    const int64_t kend = (kbeg + g.k_split < g.K) ? kbeg + g.k_split : g.K;
    const bool full = VEC && m0 + BMT <= g.M && n0 + LBN <= g.N;

    const S* __restrict__ pa = (const S*)g.a.ptr;
    const S* __restrict__ pb = (const S*)g.b.ptr;

    // k-contiguous loader (A, and B when OB == MK): 128 rows x 64 k as vectors of 8,
    // thread -> k-vector kv = tid % 8, rows tid / 8 + 32 u
    const int kv = tid & 7;
    const int rr = tid >> 3;
    // n-contiguous loader (B when OB == KN): 64 k x 128 n as 4 x 8 blocks,
    // thread -> k rows 4 * (tid % 16) .. +3, n columns 8 * (tid / 16) .. +7
    const int bkq = tid & 15;
    const int bng = tid >> 4;

    V8 ra[4], rb[4];   // rb: k-contiguous B rows, or (OB == KN) the four 8-wide n runs of rows k

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
    // row bases of the k-contiguous loads
    const S* __restrict__ pa_row = pa + (m0 + rr) * g.a.ld;
    const S* __restrict__ pb_row = pb + (n0 + rr) * g.b.ld;
    const int64_t a_step = 32 * g.a.ld, b_step = 32 * g.b.ld;

    // With VEC every aligned 8-run of a k-contiguous operand (and of an n-contiguous B) lies inside
    // one segment, so a partial run is read element by element from contiguous addresses.
    auto masked8 = [&](const S* p, int valid) {
        S e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = (j < valid) ? p[j] : (S)0;
        return __builtin_bit_cast(V8, e);
    };
    auto load_kc = [&](const S* p, const Desc& d, const KCol& c, int64_t rows, int64_t row0, int64_t k0, V8* dst) {
        const int64_t k = k0 + 8 * kv;
        const int64_t co = c.kq * d.segstride + c.kr;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + rr + 32 * u;
            V8 v;
            if (VEC) {
                const int64_t valid = row < rows ? kend - k : 0;
                if (valid >= 8) v = *(const V8*)(p + row * d.ld + co);
                else v = masked8(p + row * d.ld + co, (int)(valid > 0 ? valid : 0));
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
            if (VEC) {
                const int64_t valid = k < kend ? g.N - n : 0;
                if (valid >= 8) rb[q] = *(const V8*)(pb + k * g.b.ld + bn_fix);
                else rb[q] = masked8(pb + k * g.b.ld + bn_fix, (int)(valid > 0 ? valid : 0));
            } else {
                S e[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    e[j] = (k < kend && n + j < g.N) ? pb[k * g.b.ld + coloff(g.b, n + j)] : (S)0;
                rb[q] = __builtin_bit_cast(V8, e);
            }
        }
    };
    // checked loader (edge tiles, the partial k-tile)
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
    // unchecked loader: the tile is inside C and [k0, k0 + 64) inside [kbeg, kend)
    auto load_fast = [&](int64_t k0) {
        {
            const S* p = pa_row + (ca.kq * g.a.segstride + ca.kr);
#pragma unroll
            for (int u = 0; u < 4; ++u) ra[u] = *(const V8*)(p + u * a_step);
            kcol_next(g.a, ca);
        }
        if (OB == KM) {
            const S* p = pb + (k0 + 4 * bkq) * g.b.ld + bn_fix;
#pragma unroll
            for (int q = 0; q < 4; ++q) rb[q] = *(const V8*)(p + q * g.b.ld);
        } else {
            const S* p = pb_row + (cb.kq * g.b.segstride + cb.kr);
#pragma unroll
            for (int u = 0; u < 4; ++u) rb[u] = *(const V8*)(p + u * b_step);
            kcol_next(g.b, cb);
        }
    };
    auto store_tiles = [&](S* Ad, S* Bd) {
#pragma unroll
        for (int u = 0; u < 4; ++u) *(V8*)(Ad + (rr + 32 * u) * LDK + 8 * kv) = ra[u];
        if (OB == KM) {
            // column n of the block -> Bd[n][4 bkq .. 4 bkq + 3]
            typedef S SV8 __attribute__((ext_vector_type(8)));
            const SV8 r0 = __builtin_bit_cast(SV8, rb[0]), r1 = __builtin_bit_cast(SV8, rb[1]);
            const SV8 r2 = __builtin_bit_cast(SV8, rb[2]), r3 = __builtin_bit_cast(SV8, rb[3]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                S e[4] = {r0[j], r1[j], r2[j], r3[j]};
                S* dst = Bd + (8 * bng + j) * LDK + 4 * bkq;
                if constexpr (ES == 2) *(uint2*)dst = __builtin_bit_cast(uint2, e);
                else *(uint32_t*)dst = __builtin_bit_cast(uint32_t, e);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) *(V8*)(Bd + (rr + 32 * u) * LDK + 8 * kv) = rb[u];
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

    auto compute = [&](const S* Ac, const S* Bc) {
#pragma unroll
        for (int ks = 0; ks < LBK / 32; ++ks) {
            V8 bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = *(const V8*)(Bc + (wbn + j * 16 + fr) * LDK + ks * 32 + 8 * fk);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const V8 av = *(const V8*)(Ac + (wbm + i * 16 + fr) * LDK + ks * 32 + 8 * fk);
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma32<P>(av, bv[j], acc[i][j]);
            }
        }
    };
    // one k-tile: prefetch the next (fast or checked), multiply the current, rotate the stages
    int cur = 0;
    auto step = [&](bool more, auto&& prefetch) {
        if (more) prefetch();
        compute(As2 + cur * BMT * LDK, Bs2 + cur * LBN * LDK);
        if (NST == 2) {
            if (more) store_tiles(As2 + (cur ^ 1) * BMT * LDK, Bs2 + (cur ^ 1) * LBN * LDK);
            __syncthreads();
            cur ^= 1;
        } else {
            __syncthreads();
            if (more) {
                store_tiles(As2, Bs2);
                __syncthreads();
            }
        }
    };

    if (kbeg < kend) {
        // full k-tiles [kbeg, kfe) of an interior tile take the unchecked loader
        const int64_t kfe = full ? kbeg + ((kend - kbeg) / LBK) * LBK : kbeg;
        if (kfe > kbeg) load_fast(kbeg);
        else load_tiles(kbeg);
        store_tiles(As2, Bs2);
        __syncthreads();
        int64_t k0 = kbeg;
        for (; k0 + LBK < kfe; k0 += LBK) step(true, [&] { load_fast(k0 + LBK); });
        for (; k0 < kend; k0 += LBK) step(k0 + LBK < kend, [&] { load_tiles(k0 + LBK); });
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
                const int64_t off = z * g.c_zstride + m * g.c.ld + co;
                if (OUTP == LP_F32OUT) ((float*)cbase)[off] = val;
                else if (OUTP == LP_BF16) ((uint16_t*)cbase)[off] = enc_bf16(val);
                else ((uint16_t*)cbase)[off] = enc_f16(val);
            }
        }
    }
}

template <int P, int OB, int OUTP, bool VEC, int NST, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_lp_kernel(LpGemmArgs g) {
    gemm_lp_tile<P, OB, OUTP, VEC, NST>(g, xcd_remap(blockIdx.x, gridDim.x), blockIdx.z);
}

// Persistent grouped launch: each workgroup claims work items (tile, split) of the group's products
// from a device counter until none is left; items are numbered product by product.  The last
// workgroup to finish clears both counters for the next launch on the stream.
template <int P, int OB, int OUTP, bool VEC, int NST, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_lp_grouped_kernel(LpGroupArgs a) {
    __shared__ int64_t claim;
    for (;;) {
        if (threadIdx.x == 0) claim = (int64_t)atomicAdd(a.ctr, 1u);
        __syncthreads();
        const int64_t w = claim;
        __syncthreads();
        if (w >= a.start[a.n]) break;
        int p = 0;
        while (p + 1 < a.n && a.start[p + 1] <= w) ++p;
        const int64_t local = w - a.start[p];
        const int64_t tilesM = (a.p[p].M + 127) / 128;
        const int64_t tilesN = (a.p[p].N + LBN - 1) / LBN;
        const int64_t tiles = a.p[p].lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
        gemm_lp_tile<P, OB, OUTP, VEC, NST>(a.p[p], local % tiles, local / tiles);
    }
    if (threadIdx.x == 0 && atomicAdd(a.ctr + 1, 1u) == gridDim.x - 1) {
        atomicExch(a.ctr, 0u);
        atomicExch(a.ctr + 1, 0u);
    }
}

template <int P, int OB, int OUTP, int NST, int OCC>
hipError_t launch_lp_v(const LpGemmArgs& g, bool vec, hipStream_t s) {
    const int64_t tilesM = (g.M + 127) / 128;
    const int64_t tilesN = (g.N + LBN - 1) / LBN;
    const int64_t tiles = g.lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
    const int64_t splits = (g.K + g.k_split - 1) / g.k_split;
    if (tiles == 0) return hipSuccess;
    dim3 grid((unsigned)tiles, 1, (unsigned)(splits > 0 ? splits : 1));
    if (vec) hipLaunchKernelGGL((gemm_lp_kernel<P, OB, OUTP, true, NST, OCC>), grid, dim3(256), 0, s, g);
    // element-wise loads (operands that do not allow vector loads) need more registers: two per CU
    else hipLaunchKernelGGL((gemm_lp_kernel<P, OB, OUTP, false, NST, 2>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// candidates: 0 = one LDS stage (three workgroups per CU fit in registers and LDS), 1 = two stages
// (two per CU).  On the products of a sweep the first measured faster: more resident workgroups hide
// more of the load latency than the second stage does.
template <int P, int OB, int OUTP>
hipError_t launch_lp(const LpGemmArgs& g, bool vec, hipStream_t s) {
    auto launch = [&](int c) -> hipError_t {
        return c == 1 ? launch_lp_v<P, OB, OUTP, 2, 2>(g, vec, s) : launch_lp_v<P, OB, OUTP, 1, 3>(g, vec, s);
    };
    const int64_t shape[5] = {g.M, g.N, g.K, g.k_split,
                              1000 * P + 100 * OB + 10 * OUTP + (vec ? 1 : 0) + (g.lower_only ? 10000 : 0)};
    hipError_t e = hipSuccess;
    const int c = tune_choose(kTuneLpTile, shape, 2, 0, s, launch, &e);
    return e != hipSuccess ? e : launch(c);
}

// the grouped form of launch_lp: the LDS staging is the one kept for the first product's shape (or the
// heuristic's, never measured here), the grid is what stays resident (three workgroups per CU)
template <int P, int OB, int OUTP, int NST>
hipError_t launch_lp_grouped_v(const LpGroupArgs& a, bool vec, hipStream_t s) {
    const int64_t items = a.start[a.n];
    if (items == 0) return hipSuccess;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus <= 0)
        cus = 256;
    const int64_t per = (NST == 2 || !vec) ? 2 : 3;
    const unsigned grid = (unsigned)std::min<int64_t>(items, per * cus);
    if (vec) {
        if (NST == 2) hipLaunchKernelGGL((gemm_lp_grouped_kernel<P, OB, OUTP, true, 2, 2>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((gemm_lp_grouped_kernel<P, OB, OUTP, true, 1, 3>), dim3(grid), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((gemm_lp_grouped_kernel<P, OB, OUTP, false, NST, 2>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <int P, int OB, int OUTP>
hipError_t launch_lp_grouped(const LpGroupArgs& a, bool vec, hipStream_t s) {
    const LpGemmArgs& g = a.p[0];
    const int64_t shape[5] = {g.M, g.N, g.K, g.k_split,
                              1000 * P + 100 * OB + 10 * OUTP + (vec ? 1 : 0) + (g.lower_only ? 10000 : 0)};
    hipError_t e = hipSuccess;
    const bool was = tune_enabled();
    tune_set_enabled(false);
    const int c = tune_choose(kTuneLpTile, shape, 2, 0, s, [](int) { return hipSuccess; }, &e);
    tune_set_enabled(was);
    if (e != hipSuccess) return e;
    return c == 1 ? launch_lp_grouped_v<P, OB, OUTP, 2>(a, vec, s) : launch_lp_grouped_v<P, OB, OUTP, 1>(a, vec, s);
}

// outputs: FP32, or the 16-bit type of the sweep's intermediates (BF16 for BF16 and FP8 operands, FP16
// for FP16 operands)
template <int P, int OB>
hipError_t by_out(const LpGemmArgs& g, int outp, bool vec, hipStream_t s) {
    constexpr int LP16 = (P == LP_F16) ? LP_F16 : LP_BF16;
    if (outp == LP_F32OUT) return launch_lp<P, OB, LP_F32OUT>(g, vec, s);
    if (outp == LP16) return launch_lp<P, OB, LP16>(g, vec, s);
    return hipErrorInvalidValue;
}
template <int P, int OB>
hipError_t by_out_grouped(const LpGroupArgs& a, int outp, bool vec, hipStream_t s) {
    constexpr int LP16 = (P == LP_F16) ? LP_F16 : LP_BF16;
    if (outp == LP_F32OUT) return launch_lp_grouped<P, OB, LP_F32OUT>(a, vec, s);
    if (outp == LP16) return launch_lp_grouped<P, OB, LP16>(a, vec, s);
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace tk
