// Symmetric eigen-decomposition of an n x n FP64 matrix, n <= 1024, by two-sided block Jacobi.
//
// The matrix is padded to np (a multiple of 64) and split into T = np / 32 blocks of 32 rows.  A sweep
// runs T - 1 rounds of the round-robin tournament over the blocks; in a round every pair (p, q) of
// blocks is independent: one workgroup diagonalises the 64 x 64 principal submatrix on the rows of
// blocks p and q exactly (cyclic Jacobi with the parallel round-robin ordering, Golub & Van Loan
// Alg. 8.4.3, in LDS) and stores its rotation Q_pq; then A <- J^T A J and V <- V J, where J applies
// each Q_pq to its two blocks, in two passes over the matrix (rows, then columns).  Sweeps repeat
// until the off-diagonal mass is below np 2^-100 of the total (in squares), checked on the host after
// each sweep: the sub-problems leave each off-diagonal pair below 2^-53 sqrt(|a_ii a_jj|), at most
// np 2^-106 of the total in squares, so the test stops the sweeps once every pair is decoupled to
// rounding (a factor 64 of margin).  Padding rows and columns start decoupled (zero off-diagonal, a diagonal below every
// eigenvalue by Gershgorin's bound) and stay exactly decoupled, so the n largest diagonal entries at
// the end are the eigenvalues.
#include <algorithm>
#include <cmath>

#include "tk_common.h"

namespace tk {
namespace {

constexpr int EB = 32;            // block rows
constexpr int SP = 2 * EB;        // sub-problem order
constexpr int SLD = SP + 1;       // LDS row stride

// -(1 + max_i sum_j |A_ij|): below every eigenvalue of A (Gershgorin)
__global__ __launch_bounds__(256) void pad_value_kernel(const double* __restrict__ A, int n, double* out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += fabs(A[(int64_t)i * n + j]);
        m = fmax(m, s);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = -(1.0 + red[0]);
}

// Ap (np x np) = A symmetrised, padded; V = I
__global__ __launch_bounds__(256) void eig_init_kernel(const double* __restrict__ A, int n, int np,
                                                       const double* __restrict__ padv, double* __restrict__ Ap,
                                                       double* __restrict__ V) {
    const double pv = *padv;
    const int64_t total = (int64_t)np * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / np), j = (int)(e % np);
        double v;
        if (i < n && j < n) v = 0.5 * (A[(int64_t)i * n + j] + A[(int64_t)j * n + i]);
        else v = (i == j) ? pv : 0.0;
        Ap[e] = v;
        V[e] = (i == j) ? 1.0 : 0.0;
    }
}

// Round r of the tournament over T blocks (T even): pair k holds blocks (first, second).
__device__ __forceinline__ void pair_of(int T, int r, int k, int& p, int& q) {
    auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (T - 1)); };
    p = player(k);
    q = player(T - 1 - k);
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}
// block -> (pair, position) in round r
__device__ __forceinline__ void slot_of(int T, int r, int blk, int& k, int& pos) {
    int pp;
    if (blk == 0) {
        pp = 0;
    } else {
        pp = ((blk - 1 - r) % (T - 1) + (T - 1)) % (T - 1) + 1;
    }
    // position pp in the circle: pairs are (pp, T-1-pp)
    k = pp < T / 2 ? pp : T - 1 - pp;
    int p, q;
    pair_of(T, r, k, p, q);
    pos = (blk == p) ? 0 : 1;
}

// One workgroup per block pair: the 64 x 64 principal submatrix on blocks (p, q) is diagonalised by
// cyclic Jacobi in LDS; Q (row-major 64 x 64, columns = eigenvectors of the submatrix) to Qbuf[k].
// Threshold rule: the rotation of (i, j) is skipped when |a_ij| <= 2^-53 sqrt(|a_ii a_jj|) (the pair is
// decoupled to the rounding of its diagonal), a round without rotations skips its updates, and the
// sub-problem ends after a sweep without rotations.
__global__ __launch_bounds__(256) void bj_solve_kernel(const double* __restrict__ Ap, int np, int T, int r,
                                                       double* __restrict__ Qbuf) {
    __shared__ double A[SP * SLD], Q[SP * SLD];
    __shared__ double cs[SP / 2], sn[SP / 2];
    __shared__ int pp_[SP / 2], qq_[SP / 2];
    __shared__ int rot[SP];
    const int tid = threadIdx.x;
    const int k = blockIdx.x;
    int bp, bq;
    pair_of(T, r, k, bp, bq);
    auto grow = [&](int l) { return (l < EB) ? bp * EB + l : bq * EB + (l - EB); };
    for (int e = tid; e < SP * SP; e += 256) {
        const int i = e / SP, j = e % SP;
        A[i * SLD + j] = Ap[(int64_t)grow(i) * np + grow(j)];
        Q[i * SLD + j] = (i == j) ? 1.0 : 0.0;
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (tid < SP) rot[tid] = 0;
        __syncthreads();
        bool any = false;
        for (int rr = 0; rr < SP - 1; ++rr) {
            if (tid < SP / 2) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + rr) % (SP - 1)); };
                int p = player(tid), q = player(SP - 1 - tid);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                const double apq = A[p * SLD + q];
                const double app = A[p * SLD + p], aqq = A[q * SLD + q];
                if (fabs(apq) > 0x1p-53 * sqrt(fabs(app) * fabs(aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    rot[rr] = 1;
                }
                pp_[tid] = p;
                qq_[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            if (rot[rr] == 0) continue;     // the same value in every thread: no barrier is skipped unevenly
            any = true;
            for (int e = tid; e < (SP / 2) * SP; e += 256) {     // rows: A <- J^T A
                const int kk = e / SP, col = e % SP;
                const int p = pp_[kk], q = qq_[kk];
                const double c = cs[kk], s = sn[kk];
                const double ap = A[p * SLD + col], aq = A[q * SLD + col];
                A[p * SLD + col] = c * ap - s * aq;
                A[q * SLD + col] = s * ap + c * aq;
            }
            __syncthreads();
            for (int e = tid; e < (SP / 2) * SP; e += 256) {     // columns: A <- A J, Q <- Q J
                const int kk = e / SP, row = e % SP;
                const int p = pp_[kk], q = qq_[kk];
                const double c = cs[kk], s = sn[kk];
                const double ap = A[row * SLD + p], aq = A[row * SLD + q];
                A[row * SLD + p] = c * ap - s * aq;
                A[row * SLD + q] = s * ap + c * aq;
                const double vp = Q[row * SLD + p], vq = Q[row * SLD + q];
                Q[row * SLD + p] = c * vp - s * vq;
                Q[row * SLD + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        if (!any) break;
    }
    double* out = Qbuf + (int64_t)k * SP * SP;
    for (int e = tid; e < SP * SP; e += 256) out[e] = Q[(e / SP) * SLD + (e % SP)];
}

// B = J^T A (rows): row i of block I (pair k, position pos, local row li) becomes
// sum_l Q_k[l][pos*32 + li] A[row of l in pair k][j]
__global__ __launch_bounds__(256) void bj_rows_kernel(const double* __restrict__ A, int np, int T, int r,
                                                      const double* __restrict__ Qbuf, double* __restrict__ B) {
    const int64_t total = (int64_t)np * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / np), j = (int)(e % np);
        const int blk = i / EB, li = i % EB;
        int k, pos, p, q;
        slot_of(T, r, blk, k, pos);
        pair_of(T, r, k, p, q);
        const double* Qk = Qbuf + (int64_t)k * SP * SP;
        const int col = pos * EB + li;
        double acc = 0.0;
#pragma unroll 8
        for (int l = 0; l < EB; ++l) acc = fma(Qk[l * SP + col], A[(int64_t)(p * EB + l) * np + j], acc);
#pragma unroll 8
        for (int l = 0; l < EB; ++l) acc = fma(Qk[(EB + l) * SP + col], A[(int64_t)(q * EB + l) * np + j], acc);
        B[e] = acc;
    }
}

// C = B J (columns), for the matrix and for the eigenvector basis
__global__ __launch_bounds__(256) void bj_cols_kernel(const double* __restrict__ B, int np, int T, int r,
                                                      const double* __restrict__ Qbuf, double* __restrict__ C) {
    const int64_t total = (int64_t)np * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / np), j = (int)(e % np);
        const int blk = j / EB, lj = j % EB;
        int k, pos, p, q;
        slot_of(T, r, blk, k, pos);
        pair_of(T, r, k, p, q);
        const double* Qk = Qbuf + (int64_t)k * SP * SP;
        const int col = pos * EB + lj;
        const double* brow = B + (int64_t)i * np;
        double acc = 0.0;
#pragma unroll 8
        for (int l = 0; l < EB; ++l) acc = fma(brow[p * EB + l], Qk[l * SP + col], acc);
#pragma unroll 8
        for (int l = 0; l < EB; ++l) acc = fma(brow[q * EB + l], Qk[(EB + l) * SP + col], acc);
        C[e] = acc;
    }
}

// off-diagonal and total squared mass of A (np x np), one workgroup per row slice, then one fold
__global__ __launch_bounds__(256) void offnorm_kernel(const double* __restrict__ A, int np, double* partial) {
    __shared__ double r1[256], r2[256];
    double off = 0.0, tot = 0.0;
    const int64_t total = (int64_t)np * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const double v = A[e];
        tot += v * v;
        if (e / np != e % np) off += v * v;
    }
    r1[threadIdx.x] = off;
    r2[threadIdx.x] = tot;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r1[0];
        partial[2 * blockIdx.x + 1] = r2[0];
    }
}
__global__ void offnorm_fold_kernel(const double* partial, int nb, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nb; ++i) {
            a += partial[2 * i];
            b += partial[2 * i + 1];
        }
        out[0] = a;
        out[1] = b;
    }
}

// rank of every diagonal entry in descending order (ties by index); the n largest are the eigenvalues,
// lam[0..n); then U (n x r, row-major; and/or U32) = the eigenvectors of the first r
__global__ __launch_bounds__(256) void eig_sort_kernel(const double* __restrict__ A, int n, int np,
                                                       int* __restrict__ rank, double* __restrict__ lam) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < np; i += gridDim.x * 256) {
        const double li = A[(int64_t)i * np + i];
        int k = 0;
        for (int j = 0; j < np; ++j) {
            const double lj = A[(int64_t)j * np + j];
            if (lj > li || (lj == li && j < i)) ++k;
        }
        rank[i] = k;
        if (k < n && lam) lam[k] = li;
    }
}
__global__ __launch_bounds__(256) void eig_gather_kernel(const double* __restrict__ V, const int* __restrict__ rank,
                                                         int n, int np, int r, double* __restrict__ U,
                                                         float* __restrict__ U32) {
    const int64_t total = (int64_t)n * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int row = (int)(e / np), i = (int)(e % np);
        const int k = rank[i];
        if (k < r) {
            const double v = V[(int64_t)row * np + i];
            if (U) U[(int64_t)row * r + k] = v;
            if (U32) U32[(int64_t)row * r + k] = (float)v;
        }
    }
}

unsigned grid_for_elems(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

}  // namespace

int64_t sym_eig_work_doubles(int n) {
    const int64_t np = (int64_t)((n + 63) / 64) * 64;
    const int64_t T = np / EB;
    return 3 * np * np + (T / 2) * SP * SP + 2 * 1024 + 16 + np;   // Ap, V, tmp, Q blocks, partials, scalars, ranks
}

hipError_t sym_eig_blocked(const double* A, int n, int r, double* lam, double* U, float* U32, double* work,
                           hipStream_t s, int* sweeps_out) {
    if (n < 1 || n > 1024 || r < 1 || r > n) return hipErrorInvalidValue;
    const int np = ((n + 63) / 64) * 64;
    const int T = np / EB;
    double* Ap = work;
    double* V = Ap + (int64_t)np * np;
    double* tmp = V + (int64_t)np * np;
    double* Qbuf = tmp + (int64_t)np * np;
    double* partial = Qbuf + (int64_t)(T / 2) * SP * SP;
    double* scal = partial + 2 * 1024;
    int* rank = reinterpret_cast<int*>(scal + 16);
    hipLaunchKernelGGL(pad_value_kernel, dim3(1), dim3(256), 0, s, A, n, scal + 2);
    hipLaunchKernelGGL(eig_init_kernel, dim3(grid_for_elems((int64_t)np * np)), dim3(256), 0, s, A, n, np, scal + 2,
                       Ap, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned g2 = grid_for_elems((int64_t)np * np);
    const int nbo = (int)std::min<unsigned>(g2, 1024);
    int sweeps = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        hipLaunchKernelGGL(offnorm_kernel, dim3(nbo), dim3(256), 0, s, Ap, np, partial);
        hipLaunchKernelGGL(offnorm_fold_kernel, dim3(1), dim3(64), 0, s, partial, nbo, scal);
        double h[2] = {0.0, 0.0};
        e = hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (!(h[0] > (double)np * 0x1p-100 * h[1])) break;
        for (int rr = 0; rr < T - 1; ++rr) {
            hipLaunchKernelGGL(bj_solve_kernel, dim3(T / 2), dim3(256), 0, s, Ap, np, T, rr, Qbuf);
            hipLaunchKernelGGL(bj_rows_kernel, dim3(g2), dim3(256), 0, s, Ap, np, T, rr, Qbuf, tmp);
            hipLaunchKernelGGL(bj_cols_kernel, dim3(g2), dim3(256), 0, s, tmp, np, T, rr, Qbuf, Ap);
            hipLaunchKernelGGL(bj_cols_kernel, dim3(g2), dim3(256), 0, s, V, np, T, rr, Qbuf, tmp);
            std::swap(V, tmp);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ++sweeps;
    }
    hipLaunchKernelGGL(eig_sort_kernel, dim3((np + 255) / 256), dim3(256), 0, s, Ap, n, np, rank, lam);
    hipLaunchKernelGGL(eig_gather_kernel, dim3(grid_for_elems((int64_t)n * np)), dim3(256), 0, s, V, rank, n, np, r,
                       U, U32);
    if (sweeps_out) *sweeps_out = sweeps;
    return hipGetLastError();
}

}  // namespace tk
