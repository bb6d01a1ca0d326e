// Kernels of the codec hand-off: the kept block of an ordered core and its uniform quantisation.
//
// The paper adjusts the bit rate of the representation through the rank of the core and its
// quantisation (Abstract; Sec. I).  After the factors have been rotated so that the core is
// all-orthogonal with energy-ordered slices, keeping the leading k_n slices of every mode is the rank
// knob, and a uniform mid-tread quantiser of the kept core is the quantisation knob:
//   step = max|G| / (2^(b-1) - 1),  code = round-half-even(G / step) clamped to +-(2^(b-1) - 1),
//   dequantised = code * step,
// each a single correctly rounded binary32 operation, so the codes depend only on the core's values.
#include <cstdint>

#include "tk_common.h"

namespace tk {
namespace {

// out[j] = in[offset of the j-th index of the leading block keep[0] x ... x keep[N-1]]
__global__ __launch_bounds__(256) void gather_block_kernel(const float* __restrict__ in, int N, DimPack dims,
                                                           DimPack keep, int64_t total, float* __restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < total; j += (int64_t)gridDim.x * 256) {
        int64_t rem = j, off = 0, stride = 1;
        for (int n = N - 1; n >= 0; --n) {
            const int64_t i = rem % keep.v[n];
            rem /= keep.v[n];
            off += i * stride;
            stride *= dims.v[n];
        }
        out[j] = in[off];
    }
}

__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
    __shared__ float red[256];
    float m = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmaxf(m, fabsf(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ __launch_bounds__(256) void quantize_kernel(const float* __restrict__ x, int64_t n, const float* amax,
                                                       float levels, int32_t* __restrict__ codes,
                                                       float* __restrict__ deq, float* __restrict__ step_out) {
    const float a = *amax;
    const float step = a / levels;
    if (blockIdx.x == 0 && threadIdx.x == 0) *step_out = (a > 0.f) ? step : 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float q = 0.f;
        if (a > 0.f) {
            q = rintf(x[i] / step);
            q = fminf(fmaxf(q, -levels), levels);
        }
        codes[i] = (int32_t)q;
        deq[i] = (a > 0.f) ? q * step : 0.f;
    }
}

__global__ __launch_bounds__(256) void sqrt_clamp_kernel(const double* __restrict__ lam, int64_t n,
                                                         double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = sqrt(fmax(lam[i], 0.0));
}

unsigned grid_of(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

}  // namespace

hipError_t gather_block(const float* in, int N, const int64_t* dims, const int64_t* keep, float* out, hipStream_t s) {
    DimPack d{}, k{};
    int64_t total = 1;
    for (int n = 0; n < N; ++n) {
        d.v[n] = dims[n];
        k.v[n] = keep[n];
        total *= keep[n];
    }
    hipLaunchKernelGGL(gather_block_kernel, dim3(grid_of(total)), dim3(256), 0, s, in, N, d, k, total, out);
    return hipGetLastError();
}

hipError_t quantize_uniform(const float* x, int64_t n, int bits, float* amax_scratch, int32_t* codes, float* deq,
                            float* step, hipStream_t s) {
    hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(256), 0, s, x, n, amax_scratch);
    const float levels = (float)((1 << (bits - 1)) - 1);
    hipLaunchKernelGGL(quantize_kernel, dim3(grid_of(n)), dim3(256), 0, s, x, n, amax_scratch, levels, codes, deq,
                       step);
    return hipGetLastError();
}

hipError_t sqrt_clamp(const double* lam, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sqrt_clamp_kernel, dim3(grid_of(n)), dim3(256), 0, s, lam, n, out);
    return hipGetLastError();
}

}  // namespace tk

// ---------------------------------------------------------------- elementwise helpers of the
// pairwise-perturbation sweep (Sec. III-B, eq. (11)) and its factor alignment
namespace tk {
namespace {
__global__ __launch_bounds__(256) void axpy_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] += x[i];
}
__global__ __launch_bounds__(256) void diff_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                   float* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) out[i] = a[i] - b[i];
}
// D = 1.5 I - 0.5 B (n x n), the Newton-Schulz step matrix of the polar factor
__global__ __launch_bounds__(256) void ns_step_kernel(const double* __restrict__ B, double* __restrict__ D, int64_t n) {
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / n, j = e % n;
        D[e] = (i == j ? 1.5 : 0.0) - 0.5 * B[e];
    }
}
unsigned grid_n(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}
}  // namespace

hipError_t axpy_f32(const float* x, float* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_n(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}
hipError_t diff_f32(const float* a, const float* b, float* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(diff_kernel, dim3(grid_n(n)), dim3(256), 0, s, a, b, out, n);
    return hipGetLastError();
}
hipError_t ns_step(const double* B, double* D, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(ns_step_kernel, dim3(grid_n(n * n)), dim3(256), 0, s, B, D, n);
    return hipGetLastError();
}
}  // namespace tk
