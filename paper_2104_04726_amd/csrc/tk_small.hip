// Memory-bound and small-mode kernels of the HOOI sweep (gfx950, wave64).
//
//  * sumsq        ||x||^2 in FP64 by a fixed-grid two-stage tree (deterministic, no atomics):
//                 ||X||^2 once and ||G||^2 per sweep for the fit.
//  * pair_ttm     the full-tensor pass over the two trailing (small) modes:
//                 T34 = X x_3 U3^T x_4 U4^T (eq. (8), the chain shared by modes 1 and 2),
//                 the core G = T12 x_3 U3^T x_4 U4^T, and the expanding product of eq. (1).
//                 Each block stages a contiguous run of fibres in LDS with coalesced 16-byte
//                 loads; each thread maps one fibre through the two small factors held in LDS.
//  * fibre_gram   sum over fibres of x x^T for fibres of length <= 64, from which the Grams of
//                 both trailing modes follow for any U3/U4 (pair_mode_gram).
//  * small_ttm / small_gram: one-mode products and Grams for modes of size <= 64.
#include "tk_common.h"

namespace tk {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ __launch_bounds__(256) void sumsq_stage1(const T* __restrict__ x, int64_t n,
                                                    double* __restrict__ partial) {
    __shared__ double red[kThreads];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = (double)x[i];
        acc += v * v;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// vectorised fp32 variant: 16-byte loads when x is 16-byte aligned
__global__ __launch_bounds__(256) void sumsq_stage1_v4(const float4* __restrict__ x, int64_t n4,
                                                       const float* __restrict__ tail, int ntail,
                                                       double* __restrict__ partial) {
    __shared__ double red[kThreads];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = x[i];
        acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) {
        const double v = tail[threadIdx.x];
        acc += v * v;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partial, int64_t n,
                                                     double* __restrict__ out) {
    __shared__ double red[kThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------- small one-mode product
__global__ __launch_bounds__(256) void small_ttm_kernel(const float* __restrict__ in, int64_t A,
                                                        int64_t K, int64_t B,
                                                        const float* __restrict__ U, int64_t R,
                                                        int expand, float* __restrict__ out) {
    extern __shared__ float Us[];          // K*R factor entries, as Mk[k][r]
    for (int64_t i = threadIdx.x; i < K * R; i += blockDim.x) {
        const int64_t k = i / R, r = i % R;
        Us[i] = expand ? U[r * K + k] : U[k * R + r];
    }
    __syncthreads();
    const int64_t total = A * R * B;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += stride) {
        const int64_t b = o % B;
        const int64_t r = (o / B) % R;
        const int64_t a = o / (B * R);
        const float* src = in + a * K * B + b;
        float acc = 0.f;
        for (int64_t k = 0; k < K; ++k) acc = fmaf(Us[k * R + r], src[k * B], acc);
        out[o] = acc;
    }
}

// ---------------------------------------------------------------- fused two-trailing-mode pass
// Fibres are the (p x q) trailing blocks (contiguous, length L = p*q).  One block handles FPB
// fibres per iteration; each thread one fibre.  LDS rows are padded to an odd stride.
constexpr int kPairMaxP = 4, kPairMaxQ = 16;
constexpr int kPairFPB = 256;

template <bool EXPAND>
__global__ __launch_bounds__(256) void pair_ttm_kernel(const float* __restrict__ in, int64_t A,
                                                       int p, int q, const float* __restrict__ U3,
                                                       int R3, const float* __restrict__ U4, int R4,
                                                       float* __restrict__ out) {
    // input fibre (len Lin) -> output fibre (len Lout)
    const int Lin = EXPAND ? R3 * R4 : p * q;
    const int Lout = EXPAND ? p * q : R3 * R4;
    const int SIN = Lin | 1, SOUT = Lout | 1;     // odd strides: conflict-free column access
    extern __shared__ float lds[];
    float* u3 = lds;                              // p x R3
    float* u4 = u3 + kPairMaxP * kPairMaxP;       // q x R4
    float* fin = u4 + kPairMaxQ * kPairMaxQ;      // FPB x SIN
    float* fout = fin + kPairFPB * SIN;           // FPB x SOUT
    for (int i = threadIdx.x; i < p * R3; i += blockDim.x) u3[i] = U3[i];
    for (int i = threadIdx.x; i < q * R4; i += blockDim.x) u4[i] = U4[i];

    const int64_t nchunks = (A + kPairFPB - 1) / kPairFPB;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t f0 = ch * kPairFPB;
        const int nf = (int)((A - f0) < kPairFPB ? (A - f0) : kPairFPB);
        const int64_t nin = (int64_t)nf * Lin;
        const float* src = in + f0 * Lin;
        __syncthreads();
        // coalesced copy of nf fibres into padded LDS rows
        if ((((uintptr_t)src) & 15) == 0) {
            const int64_t n4 = nin / 4;
            const float4* s4 = (const float4*)src;
            for (int64_t i = threadIdx.x; i < n4; i += blockDim.x) {
                const float4 v = s4[i];
                const int64_t e = i * 4;
                const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t g = e + j;
                    fin[(g / Lin) * SIN + (g % Lin)] = vv[j];
                }
            }
            for (int64_t g = n4 * 4 + threadIdx.x; g < nin; g += blockDim.x)
                fin[(g / Lin) * SIN + (g % Lin)] = src[g];
        } else {
            for (int64_t g = threadIdx.x; g < nin; g += blockDim.x)
                fin[(g / Lin) * SIN + (g % Lin)] = src[g];
        }
        __syncthreads();
        const int f = threadIdx.x;
        if (f < nf) {
            const float* x = fin + f * SIN;
            float* y = fout + f * SOUT;
            if (!EXPAND) {
                // tmp[c][t] = sum_i x[c][i] U4[i][t];  y[r][t] = sum_c U3[c][r] tmp[c][t]
                float tmp[kPairMaxP][kPairMaxQ];
#pragma unroll
                for (int c = 0; c < kPairMaxP; ++c) {
                    if (c >= p) break;
#pragma unroll
                    for (int t = 0; t < kPairMaxQ; ++t) {
                        if (t >= R4) break;
                        float acc = 0.f;
#pragma unroll
                        for (int i = 0; i < kPairMaxQ; ++i) {
                            if (i >= q) break;
                            acc = fmaf(x[c * q + i], u4[i * R4 + t], acc);
                        }
                        tmp[c][t] = acc;
                    }
                }
#pragma unroll
                for (int r = 0; r < kPairMaxP; ++r) {
                    if (r >= R3) break;
#pragma unroll
                    for (int t = 0; t < kPairMaxQ; ++t) {
                        if (t >= R4) break;
                        float acc = 0.f;
#pragma unroll
                        for (int c = 0; c < kPairMaxP; ++c) {
                            if (c >= p) break;
                            acc = fmaf(u3[c * R3 + r], tmp[c][t], acc);
                        }
                        y[r * R4 + t] = acc;
                    }
                }
            } else {
                // tmp[r][i] = sum_t x[r][t] U4[i][t];  y[c][i] = sum_r U3[c][r] tmp[r][i]
                float tmp[kPairMaxP][kPairMaxQ];
#pragma unroll
                for (int r = 0; r < kPairMaxP; ++r) {
                    if (r >= R3) break;
#pragma unroll
                    for (int i = 0; i < kPairMaxQ; ++i) {
                        if (i >= q) break;
                        float acc = 0.f;
#pragma unroll
                        for (int t = 0; t < kPairMaxQ; ++t) {
                            if (t >= R4) break;
                            acc = fmaf(x[r * R4 + t], u4[i * R4 + t], acc);
                        }
                        tmp[r][i] = acc;
                    }
                }
#pragma unroll
                for (int c = 0; c < kPairMaxP; ++c) {
                    if (c >= p) break;
#pragma unroll
                    for (int i = 0; i < kPairMaxQ; ++i) {
                        if (i >= q) break;
                        float acc = 0.f;
#pragma unroll
                        for (int r = 0; r < kPairMaxP; ++r) {
                            if (r >= R3) break;
                            acc = fmaf(u3[c * R3 + r], tmp[r][i], acc);
                        }
                        y[c * q + i] = acc;
                    }
                }
            }
        }
        __syncthreads();
        // coalesced write-back
        const int64_t nout = (int64_t)nf * Lout;
        float* dst = out + f0 * Lout;
        for (int64_t g = threadIdx.x; g < nout; g += blockDim.x) dst[g] = fout[(g / Lout) * SOUT + (g % Lout)];
    }
}

// ---------------------------------------------------------------- specialised two-mode pass
// Same product as pair_ttm_kernel for a compile-time fibre shape: factors live in registers (U3)
// and LDS (U4 rows read as 16-byte vectors), all index arithmetic is by constants, and the next
// chunk's 16-byte coalesced loads are issued into registers before the current chunk is mapped,
// so HBM reads overlap the arithmetic.
template <int P, int Q, int R3, int R4, bool EXPAND, bool ID3>
__global__ __launch_bounds__(256) void pair_ttm_fixed(const float* __restrict__ in, int64_t A,
                                                      const float* __restrict__ U3,
                                                      const float* __restrict__ U4,
                                                      float* __restrict__ out) {
    constexpr int LIN = EXPAND ? R3 * R4 : P * Q;
    constexpr int LOUT = EXPAND ? P * Q : R3 * R4;
    constexpr int SIN = LIN | 1, SOUT = LOUT | 1;
    constexpr int FPB = 256;
    constexpr int NV_IN = (FPB * LIN) / 4;          // float4 per full chunk (LIN*256 divisible by 4)
    constexpr int NV_OUT = (FPB * LOUT) / 4;
    constexpr int VPT_IN = (NV_IN + 255) / 256;     // float4 loads per thread
    __shared__ float fin[FPB * SIN];
    __shared__ float fout[FPB * SOUT];
    static_assert(!ID3 || P == R3, "an identity U3 keeps the mode's size");
    __shared__ float u4s[Q * R4];
    for (int i = threadIdx.x; i < Q * R4; i += 256) u4s[i] = U4[i];
    float u3[P * R3];
#pragma unroll
    for (int i = 0; i < P * R3; ++i) u3[i] = ID3 ? 0.f : U3[i];

    const int64_t nchunks = (A + FPB - 1) / FPB;
    const int64_t full_chunks = A / FPB;
    float4 pre[VPT_IN];
    auto prefetch = [&](int64_t ch) {
        if (ch < full_chunks) {
            const float4* src = (const float4*)(in + ch * FPB * LIN);
#pragma unroll
            for (int u = 0; u < VPT_IN; ++u) {
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
        if (ch < full_chunks) {
#pragma unroll
            for (int u = 0; u < VPT_IN; ++u) {
                const int i = threadIdx.x + 256 * u;
                if (i < NV_IN) {
                    // one division per vector; position and fibre advance by increments (LIN >= 4)
                    const float vv[4] = {pre[u].x, pre[u].y, pre[u].z, pre[u].w};
                    const int fb = (4 * i) / LIN;
                    int l = 4 * i - fb * LIN;
                    float* dst = fin + fb * SIN;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        dst[l] = vv[j];
                        ++l;
                        if (l == LIN) {
                            l = 0;
                            dst += SIN;
                        }
                    }
                }
            }
        } else {
            const float* src = in + f0 * LIN;
            for (int g = threadIdx.x; g < nf * LIN; g += 256) fin[(g / LIN) * SIN + (g % LIN)] = src[g];
        }
        __syncthreads();
        prefetch(ch + gridDim.x);
        const int f = threadIdx.x;
        if (f < nf) {
            const float* x = fin + f * SIN;
            float* y = fout + f * SOUT;
            if (!EXPAND) {
                float tmp[P][R4];
#pragma unroll
                for (int c = 0; c < P; ++c)
#pragma unroll
                    for (int t = 0; t < R4; ++t) tmp[c][t] = 0.f;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    float xc[P];
#pragma unroll
                    for (int c = 0; c < P; ++c) xc[c] = x[c * Q + i];
#pragma unroll
                    for (int t = 0; t < R4; ++t) {
                        const float w = u4s[i * R4 + t];
#pragma unroll
                        for (int c = 0; c < P; ++c) tmp[c][t] = fmaf(xc[c], w, tmp[c][t]);
                    }
                }
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
                            for (int c = 0; c < P; ++c) acc = fmaf(u3[c * R3 + r], tmp[c][t], acc);
                        }
                        y[r * R4 + t] = acc;
                    }
            } else {
                float tmp[R3][Q];
#pragma unroll
                for (int r = 0; r < R3; ++r)
#pragma unroll
                    for (int i = 0; i < Q; ++i) tmp[r][i] = 0.f;
#pragma unroll
                for (int t = 0; t < R4; ++t) {
                    float xr[R3];
#pragma unroll
                    for (int r = 0; r < R3; ++r) xr[r] = x[r * R4 + t];
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const float w = u4s[i * R4 + t];
#pragma unroll
                        for (int r = 0; r < R3; ++r) tmp[r][i] = fmaf(xr[r], w, tmp[r][i]);
                    }
                }
#pragma unroll
                for (int c = 0; c < P; ++c)
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        float acc;
                        if (ID3) {
                            acc = tmp[c][i];
                        } else {
                            acc = 0.f;
#pragma unroll
                            for (int r = 0; r < R3; ++r) acc = fmaf(u3[c * R3 + r], tmp[r][i], acc);
                        }
                        y[c * Q + i] = acc;
                    }
            }
        }
        __syncthreads();
        float* dst = out + f0 * LOUT;
        if (nf == FPB && ((((uintptr_t)dst) & 15) == 0)) {
            float4* d4 = (float4*)dst;
            for (int i = threadIdx.x; i < NV_OUT; i += 256) {
                float v[4];
                const int fb = (4 * i) / LOUT;
                int l = 4 * i - fb * LOUT;
                const float* src = fout + fb * SOUT;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = src[l];
                    ++l;
                    if (l == LOUT) {
                        l = 0;
                        src += SOUT;
                    }
                }
                d4[i] = make_float4(v[0], v[1], v[2], v[3]);
            }
        } else {
            for (int g = threadIdx.x; g < nf * LOUT; g += 256) dst[g] = fout[(g / LOUT) * SOUT + (g % LOUT)];
        }
    }
}

// ---------------------------------------------------------------- fibre Gram (L <= 64)
// F = sum_f x_f x_f^T over the fibres x_f (rows of length L <= 64) is a Gram with a long contraction
// (the fibre index), run on the FP64 matrix cores: the L columns are covered by NB blocks of 16, and
// each wave accumulates the NB (NB + 1) / 2 lower 16 x 16 blocks over groups of 4 fibres
// (v_mfma_f64_16x16x4: lane l holds x_(f0 + l/16)[16 I + l%16] as the A operand of block row I and as
// the B operand of block column J).  Products of FP32 values are exact in FP64.  The fibre groups go
// to the waves round-robin; the four waves of a block add their sums in wave order in LDS, and the
// block writes its lower triangle as one partial.
typedef double f64x4_fg __attribute__((ext_vector_type(4)));
template <int NB>
__global__ __launch_bounds__(256) void fibre_gram_kernel(const float* __restrict__ in, int64_t A, int L,
                                                         double* __restrict__ partial) {
    constexpr int NT = NB * (NB + 1) / 2, LD = 16 * NB, UNR = 4;
    __shared__ double red[LD * LD];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kk = lane >> 4;
    f64x4_fg acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f64x4_fg{0.0, 0.0, 0.0, 0.0};
    const int64_t ngroups = (A + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * 4;
    for (int64_t g0 = (int64_t)blockIdx.x * 4 + wave; g0 < ngroups; g0 += stride * UNR) {
        double xv[UNR][NB];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t f = (g0 + u * stride) * 4 + kk;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c = 16 * b + r;
                xv[u][b] = (f < A && c < L) ? (double)in[f * L + c] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            int t = 0;
#pragma unroll
            for (int I = 0; I < NB; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[u][I], xv[u][J], acc[t], 0, 0, 0);
        }
    }
    // lane l holds rows l/16 + 4 v, column l % 16 of each block
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
            int t = 0;
#pragma unroll
            for (int I = 0; I < NB; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J, ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = (16 * I + kk + 4 * v) * LD + 16 * J + r;
                        red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[t][v];
                    }
        }
        __syncthreads();
    }
    double* dst = partial + (int64_t)blockIdx.x * L * L;
    for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
        const int i = e / L, j = e - (e / L) * L;
        if (j <= i) dst[i * L + j] = red[i * LD + j];
    }
}

// F (symmetric) = sum over the nblocks partial lower triangles.  A team of 32 lanes per entry:
// lane l adds partials l, l + 32, ... in order, then a fixed butterfly adds the 32 lane sums, so
// the result does not depend on timing.
__global__ __launch_bounds__(256) void fibre_gram_reduce(const double* __restrict__ partial, int nblocks,
                                                         int L, double* __restrict__ F) {
    const int npairs = L * (L + 1) / 2;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int idx = (int)(gt >> 5), l = (int)(gt & 31);
    const bool valid = idx < npairs;
    int i = 0, j = 0;
    if (valid) {
        i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= idx) ++i;
        while (i * (i + 1) / 2 > idx) --i;
        j = idx - i * (i + 1) / 2;
    }
    double s = 0.0;
    if (valid) {
        const int64_t st = (int64_t)L * L, off = (int64_t)i * L + j;
#pragma unroll 4
        for (int b = l; b < nblocks; b += 32) s += partial[(int64_t)b * st + off];
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    if (valid && l == 0) {
        F[i * L + j] = s;
        F[j * L + i] = s;
    }
}

// S3/S4 from the fibre Gram and the projector of the other trailing mode
__global__ __launch_bounds__(256) void pair_mode_gram_kernel(const double* __restrict__ F, int p, int q,
                                                             const double* __restrict__ U, int R,
                                                             int which, double* __restrict__ S) {
    const int L = p * q;
    const int n = (which == 3) ? p : q;
    const int o = (which == 3) ? q : p;      // size of the other mode
    __shared__ double P[64 * 64];
    for (int e = threadIdx.x; e < o * o; e += blockDim.x) {
        const int a = e / o, b = e % o;
        double v = 0.0;
        if (U) {
            for (int r = 0; r < R; ++r) v += U[a * R + r] * U[b * R + r];
        } else {
            v = (a == b) ? 1.0 : 0.0;
        }
        P[e] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int x = e / n, y = e % n;
        double acc = 0.0;
        for (int a = 0; a < o; ++a)
            for (int b = 0; b < o; ++b) {
                const double pv = P[a * o + b];
                if (pv == 0.0) continue;
                // which==3: F[(x,a),(y,b)]  (fibre index c*q+i);  which==4: F[(a,x),(b,y)]
                const int r = (which == 3) ? x * q + a : a * q + x;
                const int c = (which == 3) ? y * q + b : b * q + y;
                acc += F[r * L + c] * pv;
            }
        S[e] = acc;
    }
}

// ---------------------------------------------------------------- small Gram (s <= 64)
// S[i][j] = sum_{a,b} Y[a][i][b] Y[a][j][b]; each block takes a range of (a, b) columns.
__global__ __launch_bounds__(256) void small_gram_kernel(const float* __restrict__ in, int64_t A,
                                                         int64_t sdim, int64_t B,
                                                         double* __restrict__ partial) {
    __shared__ float cs[64 * 65];     // 64 columns x sdim rows, column-major with stride 65
    const int s = (int)sdim;
    const int npairs = s * (s + 1) / 2;
    int pi[9], pj[9];
    double accd[9];
    for (int u = 0; u < 9; ++u) {
        const int idx = threadIdx.x + u * blockDim.x;
        if (idx < npairs) {
            int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            while ((i + 1) * (i + 2) / 2 <= idx) ++i;
            while (i * (i + 1) / 2 > idx) --i;
            pi[u] = i;
            pj[u] = idx - i * (i + 1) / 2;
        } else {
            pi[u] = -1;
            pj[u] = 0;
        }
        accd[u] = 0.0;
    }
    const int64_t ncols = A * B;
    const int64_t nchunks = (ncols + 63) / 64;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t c0 = ch * 64;
        const int nc = (int)((ncols - c0) < 64 ? (ncols - c0) : 64);
        __syncthreads();
        for (int e = threadIdx.x; e < nc * s; e += blockDim.x) {
            const int cc = e % nc, i = e / nc;
            const int64_t col = c0 + cc;
            const int64_t a = col / B, b = col % B;
            cs[cc * 65 + i] = in[(a * sdim + i) * B + b];
        }
        __syncthreads();
        for (int u = 0; u < 9; ++u) {
            if (pi[u] < 0) continue;
            double acc = 0.0;
            for (int cc = 0; cc < nc; ++cc) acc = fma((double)cs[cc * 65 + pi[u]], (double)cs[cc * 65 + pj[u]], acc);
            accd[u] += acc;
        }
    }
    double* dst = partial + (int64_t)blockIdx.x * s * s;
    for (int u = 0; u < 9; ++u)
        if (pi[u] >= 0) dst[pi[u] * s + pj[u]] = accd[u];
}

// ---------------------------------------------------------------- split-K Gram reduction
// S(i, j) = S(j, i) = sum_z P_z(i, j) for i >= j, summed in split order in FP64 (the partials hold the
// lower triangle of n x n row-major Grams, zstride apart).  One 32 x 32 lower tile (I >= J) per block:
// the partials are read once and row-wise, the tile is written as it is and, through LDS, transposed,
// so that every load and store is coalesced.
template <typename TP>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const TP* __restrict__ P, int nsplit, int64_t n,
                                                          int64_t zstride, float* __restrict__ S32,
                                                          double* __restrict__ S64) {
    __shared__ double tile[32][33];
    const int64_t b = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int64_t J = b - I * (I + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        const int64_t i = 32 * I + r, j = 32 * J + tx;
        double s = 0.0;
        if (i < n && j < n && (I != J || r >= tx)) {
            const int64_t src = i * n + j;
            int z = 0;
            for (; z + 4 <= nsplit; z += 4) {
                const TP a0 = P[(int64_t)z * zstride + src], a1 = P[(int64_t)(z + 1) * zstride + src];
                const TP a2 = P[(int64_t)(z + 2) * zstride + src], a3 = P[(int64_t)(z + 3) * zstride + src];
                s += (double)a0;
                s += (double)a1;
                s += (double)a2;
                s += (double)a3;
            }
            for (; z < nsplit; ++z) s += (double)P[(int64_t)z * zstride + src];
            if (S32) S32[src] = (float)s;
            if (S64) S64[src] = s;
        }
        tile[r][tx] = s;
    }
    __syncthreads();
    // the mirror: S(32 J + r, 32 I + c) = tile[c][r], strictly above the diagonal
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        const int64_t i = 32 * J + r, j = 32 * I + tx;
        if (i < n && j < n && (I != J || tx > r)) {
            const double v = tile[tx][r];
            if (S32) S32[i * n + j] = (float)v;
            if (S64) S64[i * n + j] = v;
        }
    }
}

// ---------------------------------------------------------------- elementwise helpers
__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void f32_to_f64_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}
template <typename T>
__global__ void identity_kernel(T* __restrict__ out, int64_t rows, int64_t cols) {
    const int64_t n = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (i / cols == i % cols) ? (T)1 : (T)0;
}
__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
// SplitMix64 (Steele, Lea & Flood, 2014): a counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void random_kernel(float* __restrict__ out, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t h = splitmix64(seed + (uint64_t)i);
        out[i] = (float)((double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
    }
}
__global__ void fit_norms_kernel(const double* nx2, const double* ng2, double* fit) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double a = *nx2;
        if (!(a > 0.0)) {
            *fit = 1.0;
            return;
        }
        const double d = a - *ng2;
        *fit = 1.0 - sqrt(d < 0.0 ? 0.0 : d) / sqrt(a);     // a NaN difference stays NaN
    }
}
__global__ void fit_resid_kernel(const double* nx2, const double* r2, double* fit) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double a = *nx2;
        const double r = *r2;
        *fit = (a > 0.0) ? 1.0 - sqrt(r < 0.0 ? 0.0 : r) / sqrt(a) : 1.0;   // NaN propagates
    }
}

unsigned grid_for(int64_t n, int64_t cap = 4096) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t sumsq_f32(const float* x, int64_t n, double* partial, int nblocks, double* result,
                     hipStream_t s) {
    if ((((uintptr_t)x) & 15) == 0 && n >= 4) {
        const int64_t n4 = n / 4;
        const int ntail = (int)(n - n4 * 4);
        hipLaunchKernelGGL(sumsq_stage1_v4, dim3(nblocks), dim3(kThreads), 0, s, (const float4*)x, n4,
                           x + n4 * 4, ntail, partial);
    } else {
        hipLaunchKernelGGL(sumsq_stage1<float>, dim3(nblocks), dim3(kThreads), 0, s, x, n, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_f64(partial, nblocks, result, s);
}

hipError_t sumsq_f64(const double* x, int64_t n, double* partial, int nblocks, double* result,
                     hipStream_t s) {
    hipLaunchKernelGGL(sumsq_stage1<double>, dim3(nblocks), dim3(kThreads), 0, s, x, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_f64(partial, nblocks, result, s);
}

hipError_t reduce_f64(const double* partial, int64_t n, double* result, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partial, n, result);
    return hipGetLastError();
}

hipError_t small_ttm(const float* in, int64_t A, int64_t K, int64_t B, const float* U, int64_t R,
                     bool expand, float* out, hipStream_t s) {
    const int64_t total = A * R * B;
    if (total == 0) return hipSuccess;
    const size_t shm = (size_t)K * R * sizeof(float);
    hipLaunchKernelGGL(small_ttm_kernel, dim3(grid_for(total, 8192)), dim3(256), shm, s, in, A, K, B, U, R,
                       expand ? 1 : 0, out);
    return hipGetLastError();
}

bool pair_ttm_supported(int p, int q) { return p >= 1 && p <= kPairMaxP && q >= 1 && q <= kPairMaxQ; }

namespace {
template <int P, int Q, int R3, int R4>
bool try_fixed(const float* in, int64_t A, int p, int q, const float* U3, int r3, const float* U4, int r4,
               bool expand, bool u3_identity, float* out, hipStream_t s, hipError_t* err) {
    if (p != P || q != Q || r3 != R3 || r4 != R4) return false;
    // float4 staging needs 16-byte aligned chunk starts: 256 * LIN * 4 bytes is a multiple of 16
    if ((((uintptr_t)in) & 15) != 0) return false;
    const int64_t nchunks = (A + 255) / 256;
    const unsigned grid = (unsigned)(nchunks < 1024 ? nchunks : 1024);
    constexpr bool CAN_ID = (P == R3);
    if (expand) {
        if (CAN_ID && u3_identity)
            hipLaunchKernelGGL((pair_ttm_fixed<P, Q, R3, R4, true, CAN_ID>), dim3(grid), dim3(256), 0, s, in, A, U3, U4,
                               out);
        else
            hipLaunchKernelGGL((pair_ttm_fixed<P, Q, R3, R4, true, false>), dim3(grid), dim3(256), 0, s, in, A, U3, U4,
                               out);
    } else {
        if (CAN_ID && u3_identity)
            hipLaunchKernelGGL((pair_ttm_fixed<P, Q, R3, R4, false, CAN_ID>), dim3(grid), dim3(256), 0, s, in, A, U3,
                               U4, out);
        else
            hipLaunchKernelGGL((pair_ttm_fixed<P, Q, R3, R4, false, false>), dim3(grid), dim3(256), 0, s, in, A, U3, U4,
                               out);
    }
    *err = hipGetLastError();
    return true;
}
}  // namespace

hipError_t pair_ttm(const float* in, int64_t A, int p, int q, const float* U3, int R3, const float* U4,
                    int R4, bool expand, float* out, hipStream_t s, bool u3_identity) {
    if (!pair_ttm_supported(p, q) || R3 > p || R4 > q) return hipErrorInvalidValue;
    if (A == 0) return hipSuccess;
    {
        // fibre shapes of the multi-exposure stacks: 3 colour channels x 2E images, R4 = 2E - 1,
        // and the reduced ranks used by the large stacks
        hipError_t e = hipSuccess;
        if (try_fixed<3, 14, 3, 8>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e) ||
            try_fixed<3, 10, 3, 6>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e) ||
            try_fixed<3, 6, 3, 4>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e) ||
            try_fixed<3, 6, 3, 5>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e) ||
            try_fixed<3, 10, 3, 9>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e) ||
            try_fixed<3, 14, 3, 13>(in, A, p, q, U3, R3, U4, R4, expand, u3_identity, out, s, &e))
            return e;
    }
    const int Lin = expand ? R3 * R4 : p * q;
    const int Lout = expand ? p * q : R3 * R4;
    const size_t shm = sizeof(float) * (kPairMaxP * kPairMaxP + kPairMaxQ * kPairMaxQ +
                                        (size_t)kPairFPB * ((Lin | 1) + (Lout | 1)));
    const int64_t nchunks = (A + kPairFPB - 1) / kPairFPB;
    const unsigned grid = (unsigned)(nchunks < 2048 ? nchunks : 2048);
    hipError_t e;
    if (expand) {
        e = hipFuncSetAttribute((const void*)pair_ttm_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pair_ttm_kernel<true>, dim3(grid), dim3(256), shm, s, in, A, p, q, U3, R3, U4, R4, out);
    } else {
        e = hipFuncSetAttribute((const void*)pair_ttm_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pair_ttm_kernel<false>, dim3(grid), dim3(256), shm, s, in, A, p, q, U3, R3, U4, R4, out);
    }
    return hipGetLastError();
}

hipError_t fibre_gram(const float* in, int64_t A, int L, double* partial, int nblocks, double* F,
                      hipStream_t s) {
    if (L < 1 || L > 64) return hipErrorInvalidValue;
    const int nb = (L + 15) / 16;
    if (nb == 1) hipLaunchKernelGGL(fibre_gram_kernel<1>, dim3(nblocks), dim3(256), 0, s, in, A, L, partial);
    else if (nb == 2) hipLaunchKernelGGL(fibre_gram_kernel<2>, dim3(nblocks), dim3(256), 0, s, in, A, L, partial);
    else if (nb == 3) hipLaunchKernelGGL(fibre_gram_kernel<3>, dim3(nblocks), dim3(256), 0, s, in, A, L, partial);
    else hipLaunchKernelGGL(fibre_gram_kernel<4>, dim3(nblocks), dim3(256), 0, s, in, A, L, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fibre_gram_reduce, dim3((unsigned)((L * (L + 1) / 2 * 32 + 255) / 256)), dim3(256), 0, s,
                       partial, nblocks, L, F);
    return hipGetLastError();
}

hipError_t pair_mode_gram(const double* F, int p, int q, const double* U, int R, int which, double* S,
                          hipStream_t s) {
    if (p * q > 64 || (which != 3 && which != 4)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pair_mode_gram_kernel, dim3(1), dim3(256), 0, s, F, p, q, U, R, which, S);
    return hipGetLastError();
}

hipError_t small_gram(const float* in, int64_t A, int64_t sdim, int64_t B, double* partial, int nblocks,
                      double* S, hipStream_t s) {
    if (sdim < 1 || sdim > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(small_gram_kernel, dim3(nblocks), dim3(256), 0, s, in, A, sdim, B, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fibre_gram_reduce, dim3((unsigned)((sdim * (sdim + 1) / 2 * 32 + 255) / 256)), dim3(256), 0,
                       s, partial, nblocks, (int)sdim, S);
    return hipGetLastError();
}

static unsigned gram_reduce_blocks(int64_t n) {
    const int64_t t = (n + 31) / 32;
    return (unsigned)(t * (t + 1) / 2);
}

hipError_t gram_reduce(const float* P, int nsplit, int64_t n, int64_t zstride, float* S32, double* S64,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(gram_reduce_blocks(n)), dim3(256), 0, s, P, nsplit, n,
                       zstride, S32, S64);
    return hipGetLastError();
}

hipError_t gram_reduce64(const double* P, int nsplit, int64_t n, int64_t zstride, double* S64, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(gram_reduce_blocks(n)), dim3(256), 0, s, P, nsplit, n,
                       zstride, nullptr, S64);
    return hipGetLastError();
}

hipError_t f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t fill_identity_f32(float* out, int64_t rows, int64_t cols, hipStream_t s) {
    hipLaunchKernelGGL(identity_kernel<float>, dim3(grid_for(rows * cols)), dim3(256), 0, s, out, rows, cols);
    return hipGetLastError();
}
hipError_t fill_identity_f64(double* out, int64_t rows, int64_t cols, hipStream_t s) {
    hipLaunchKernelGGL(identity_kernel<double>, dim3(grid_for(rows * cols)), dim3(256), 0, s, out, rows, cols);
    return hipGetLastError();
}
hipError_t fill_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}
hipError_t fill_random(float* out, int64_t n, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(random_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, n, seed);
    return hipGetLastError();
}
hipError_t fit_from_norms(const double* nx2, const double* ng2, double* fit, hipStream_t s) {
    hipLaunchKernelGGL(fit_norms_kernel, dim3(1), dim3(64), 0, s, nx2, ng2, fit);
    return hipGetLastError();
}
hipError_t fit_from_resid(const double* nx2, const double* r2, double* fit, hipStream_t s) {
    hipLaunchKernelGGL(fit_resid_kernel, dim3(1), dim3(64), 0, s, nx2, r2, fit);
    return hipGetLastError();
}

}  // namespace tk
