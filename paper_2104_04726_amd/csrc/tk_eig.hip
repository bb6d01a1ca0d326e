// Symmetric eigen-decomposition of an n x n FP64 matrix, n <= 1024, by two-sided block Jacobi.
//
// The matrix is padded to np (a multiple of 64) and split into T = np / 16 blocks of 16 rows.  A sweep
// runs T - 1 rounds of the round-robin tournament over the blocks; in a round every pair (p, q) of
// blocks is independent: one workgroup diagonalises the 32 x 32 principal submatrix on the rows of
// blocks p and q exactly (cyclic Jacobi with the parallel round-robin ordering, Golub & Van Loan
// Alg. 8.4.3, in LDS) and stores its rotation Q_pq; then A <- J^T A J and V <- V J, where J applies
// each Q_pq to its two blocks, in one launch that updates every block pair of A and every block of V
// in place (small sub-problems: their Jacobi sweeps are latency-bound, so 16-row blocks give twice
// the rounds of 32-row blocks at about a quarter of the cost each).  Sweeps repeat
// until the off-diagonal mass is below np 2^-100 of the total (in squares), checked on the host after
// each sweep: once every pair is below the sub-problems' rotation threshold 2^-53 sqrt(|a_ii a_jj|), the
// off-diagonal mass is at most np 2^-106 of the total, so the test stops the sweeps there (a factor 64
// of margin).  Padding rows and columns start decoupled (zero off-diagonal, a diagonal of
// -(1 + ||A||_F), below every eigenvalue) and stay exactly decoupled, so the n largest diagonal entries
// at the end are the eigenvalues.
#include <algorithm>
#include <cmath>

#include "tk_common.h"

namespace tk {
namespace {

constexpr int EB = 16;            // block rows
constexpr int SP = 2 * EB;        // sub-problem order
constexpr int SLD = SP + 1;       // LDS row stride
constexpr int kSubSweeps = 1;     // Jacobi sweeps of a sub-problem per round

// Ap (np x np) = A symmetrised, padded; V = I.  The padding diagonal is -(1 + ||A||_F), below every
// eigenvalue (|lam| <= ||sym(A)||_F <= ||A||_F); fro2[1] holds ||A||_F^2.
__global__ __launch_bounds__(256) void eig_init_kernel(const double* __restrict__ A, int n, int np,
                                                       const double* __restrict__ fro2, double* __restrict__ Ap,
                                                       double* __restrict__ V) {
    const double pv = -(1.0 + sqrt(fro2[1]));
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

// One workgroup per block pair: one cyclic Jacobi sweep in LDS over the SP x SP principal submatrix on
// blocks (p, q); the accumulated rotation Q (row-major SP x SP) to Qbuf[k].  A single sweep per round,
// not the sub-problem solved to convergence: the outer sweeps needed barely change (11 -> 12 for a
// dense graded 128 x 128 matrix, emulated), while each round's latency falls several-fold.
// Within a round the SP/2 rotations act on disjoint index pairs, so A' = J^T A J is updated one 2 x 2
// block at a time: the block on rows {p_a, q_a} and columns {p_b, q_b} becomes J_a^T A_blk J_b, read
// and written by one thread (one phase, one barrier), and the diagonal blocks' couplings are stored
// as zero (exact in exact arithmetic; their rounding residue, up to 2^-53 max(|a_pp|, |a_qq|), would
// otherwise re-trigger rotations when the diagonal is graded).  Threshold rule: the rotation of (p, q)
// is skipped when a_pq^2 <= 2^-106 |a_pp a_qq| (decoupled to the rounding of its diagonal), and a
// round without rotations skips its update.  Rotation (Golub & Van Loan Alg. 8.4.2, the smaller angle,
// written with one square root and one reciprocal square root): d = a_qq - a_pp, h = 2 a_pq,
// r = sqrt(d^2 + h^2), u = r + |d|, c = u / sqrt(2 r u), s = sign(d) h / sqrt(2 r u) (so that
// t = s / c = sign(d) h / (|d| + r)).
__global__ __launch_bounds__(256) void bj_solve_kernel(const double* __restrict__ Ap, int np, int T, int r,
                                                       double* __restrict__ Qbuf) {
    constexpr int HP = SP / 2;
    __shared__ double A[SP * SLD], Q[SP * SLD];
    __shared__ double cs[HP], sn[HP];
    __shared__ int pp_[HP], qq_[HP];
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
    for (int sweep = 0; sweep < kSubSweeps; ++sweep) {
        if (tid < SP) rot[tid] = 0;
        __syncthreads();
        for (int rr = 0; rr < SP - 1; ++rr) {
            if (tid < HP) {
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
                if (apq * apq > 0x1p-106 * fabs(app * aqq)) {
                    const double d = aqq - app, h = 2.0 * apq;
                    const double rad = sqrt(fma(d, d, h * h));
                    const double u = rad + fabs(d);
                    const double w = rsqrt(2.0 * rad * u);
                    c = u * w;
                    s = (d < 0.0 ? -h : h) * w;
                    rot[rr] = 1;
                }
                pp_[tid] = p;
                qq_[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            if (rot[rr] == 0) continue;     // the same value in every thread: no barrier is skipped unevenly
            for (int e = tid; e < HP * HP; e += 256) {           // A <- J^T A J, one 2 x 2 block each
                const int ka = e / HP, kb = e % HP;
                const int pa = pp_[ka], qa = qq_[ka], pb = pp_[kb], qb = qq_[kb];
                const double ca = cs[ka], sa = sn[ka], cb = cs[kb], sb = sn[kb];
                const double x00 = A[pa * SLD + pb], x01 = A[pa * SLD + qb];
                const double x10 = A[qa * SLD + pb], x11 = A[qa * SLD + qb];
                const double y00 = ca * x00 - sa * x10, y01 = ca * x01 - sa * x11;
                const double y10 = sa * x00 + ca * x10, y11 = sa * x01 + ca * x11;
                A[pa * SLD + pb] = cb * y00 - sb * y01;
                A[pa * SLD + qb] = (ka == kb) ? 0.0 : sb * y00 + cb * y01;
                A[qa * SLD + pb] = (ka == kb) ? 0.0 : cb * y10 - sb * y11;
                A[qa * SLD + qb] = sb * y10 + cb * y11;
            }
            for (int e = tid; e < HP * SP; e += 256) {           // Q <- Q J
                const int kb = e / SP, row = e % SP;
                const int pb = pp_[kb], qb = qq_[kb];
                const double cb = cs[kb], sb = sn[kb];
                const double vp = Q[row * SLD + pb], vq = Q[row * SLD + qb];
                Q[row * SLD + pb] = cb * vp - sb * vq;
                Q[row * SLD + qb] = sb * vp + cb * vq;
            }
            __syncthreads();
        }
    }
    double* out = Qbuf + (int64_t)k * SP * SP;
    for (int e = tid; e < SP * SP; e += 256) out[e] = Q[(e / SP) * SLD + (e % SP)];
}

// One round's rotation J applied in place.  A <- J^T A J on the (T/2)(T/2+1)/2 block pairs (ki, kj),
// ki <= kj: the SP x SP block on the rows of pair ki's two blocks and the columns of pair kj's becomes
// Q_ki^T A_blk Q_kj, and its transpose is stored in the mirrored block (so A stays exactly symmetric).
// V <- V J on (np / SP) x (T/2) blocks: the SP rows of a row chunk on the columns of pair kj become
// V_blk Q_kj.  Every block is read and written by its own workgroup only.
__global__ __launch_bounds__(256) void bj_apply_kernel(double* __restrict__ A, double* __restrict__ V, int np, int T,
                                                       int r, const double* __restrict__ Qbuf) {
    __shared__ double M[SP * SLD], Qa[SP * SLD], Qb[SP * SLD];
    constexpr int PER = SP * SP / 256;            // outputs per thread
    const int tid = threadIdx.x;
    const int half = T / 2;
    const int nA = half * (half + 1) / 2;
    int b = blockIdx.x;
    int ki = 0, kj = 0, rb = 0;
    const bool onA = b < nA;
    if (onA) {
        while (b >= half - ki) {
            b -= half - ki;
            ++ki;
        }
        kj = ki + b;
    } else {
        b -= nA;
        kj = b % half;
        rb = b / half;
    }
    int pi = 0, qi = 0, pj, qj;
    if (onA) pair_of(T, r, ki, pi, qi);
    pair_of(T, r, kj, pj, qj);
    auto rowg = [&](int l) { return onA ? ((l < EB) ? pi * EB + l : qi * EB + (l - EB)) : rb * SP + l; };
    auto colg = [&](int l) { return (l < EB) ? pj * EB + l : qj * EB + (l - EB); };
    double* __restrict__ X = onA ? A : V;
    const double* Qj = Qbuf + (int64_t)kj * SP * SP;
    const double* Qi = Qbuf + (int64_t)ki * SP * SP;
    for (int e = tid; e < SP * SP; e += 256) {
        const int i = e / SP, j = e % SP;
        M[i * SLD + j] = X[(int64_t)rowg(i) * np + colg(j)];
        Qb[i * SLD + j] = Qj[e];
        if (onA) Qa[i * SLD + j] = Qi[e];
    }
    __syncthreads();
    double acc[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {                // C = M Q_kj
        const int e = tid + 256 * t, i = e / SP, j = e % SP;
        double v = 0.0;
#pragma unroll 8
        for (int l = 0; l < SP; ++l) v = fma(M[i * SLD + l], Qb[l * SLD + j], v);
        acc[t] = v;
    }
    if (!onA) {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + 256 * t, i = e / SP, j = e % SP;
            X[(int64_t)rowg(i) * np + colg(j)] = acc[t];
        }
        return;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = tid + 256 * t;
        M[(e / SP) * SLD + (e % SP)] = acc[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {                // A' = Q_ki^T C
        const int e = tid + 256 * t, i = e / SP, j = e % SP;
        double v = 0.0;
#pragma unroll 8
        for (int l = 0; l < SP; ++l) v = fma(Qa[l * SLD + i], M[l * SLD + j], v);
        X[(int64_t)rowg(i) * np + colg(j)] = v;
        if (ki != kj) X[(int64_t)colg(j) * np + rowg(i)] = v;
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
// fold of the nb partial pairs by one workgroup, in a fixed order
__global__ __launch_bounds__(256) void offnorm_fold_kernel(const double* __restrict__ partial, int nb, double* out) {
    __shared__ double r1[256], r2[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r1[0];
        out[1] = r2[0];
    }
}

// rank of every diagonal entry in descending order (ties by index); the n largest are the eigenvalues,
// lam[0..n); then U (n x r, row-major; and/or U32) = the eigenvectors of the first r
__global__ __launch_bounds__(256) void eig_sort_kernel(const double* __restrict__ A, int n, int np,
                                                       int* __restrict__ rank, double* __restrict__ lam) {
    __shared__ double dg[1024];
    for (int j = threadIdx.x; j < np; j += 256) dg[j] = A[(int64_t)j * np + j];
    __syncthreads();
    for (int i = blockIdx.x * 256 + threadIdx.x; i < np; i += gridDim.x * 256) {
        const double li = dg[i];
        int k = 0;
        for (int j = 0; j < np; ++j) {
            const double lj = dg[j];
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
    return 2 * np * np + (T / 2) * SP * SP + 2 * 1024 + 16 + np;   // Ap, V, Q blocks, partials, scalars, ranks
}

hipError_t sym_eig_blocked(const double* A, int n, int r, double* lam, double* U, float* U32, double* work,
                           hipStream_t s, int* sweeps_out) {
    if (n < 1 || n > 1024 || r < 1 || r > n) return hipErrorInvalidValue;
    const int np = ((n + 63) / 64) * 64;
    const int T = np / EB;
    double* Ap = work;
    double* V = Ap + (int64_t)np * np;
    double* Qbuf = V + (int64_t)np * np;
    double* partial = Qbuf + (int64_t)(T / 2) * SP * SP;
    double* scal = partial + 2 * 1024;
    int* rank = reinterpret_cast<int*>(scal + 16);
    const unsigned g2 = grid_for_elems((int64_t)np * np);
    const int nbo = (int)std::min<unsigned>(g2, 64);
    hipLaunchKernelGGL(offnorm_kernel, dim3(nbo), dim3(256), 0, s, A, n, partial);      // ||A||_F^2 to scal[3]
    hipLaunchKernelGGL(offnorm_fold_kernel, dim3(1), dim3(256), 0, s, partial, nbo, scal + 2);
    hipLaunchKernelGGL(eig_init_kernel, dim3(g2), dim3(256), 0, s, A, n, np, scal + 2, Ap, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned napply = (unsigned)((T / 2) * (T / 2 + 1) / 2 + (np / SP) * (T / 2));
    int sweeps = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        hipLaunchKernelGGL(offnorm_kernel, dim3(nbo), dim3(256), 0, s, Ap, np, partial);
        hipLaunchKernelGGL(offnorm_fold_kernel, dim3(1), dim3(256), 0, s, partial, nbo, scal);
        double h[2] = {0.0, 0.0};
        e = hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (!(h[0] > (double)np * 0x1p-100 * h[1])) break;
        for (int rr = 0; rr < T - 1; ++rr) {
            hipLaunchKernelGGL(bj_solve_kernel, dim3(T / 2), dim3(256), 0, s, Ap, np, T, rr, Qbuf);
            hipLaunchKernelGGL(bj_apply_kernel, dim3(napply), dim3(256), 0, s, Ap, V, np, T, rr, Qbuf);
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

// ---- the same eigensolver in steps (SymEigRun, tk_common.h)
namespace {
struct EigLayout {
    int np, T, nbo;
    unsigned g2, napply;
    double *Ap, *V, *Qbuf, *partial, *scal;
    int* rank;
};
EigLayout eig_layout(int n, double* work) {
    EigLayout L;
    L.np = ((n + 63) / 64) * 64;
    L.T = L.np / EB;
    L.Ap = work;
    L.V = L.Ap + (int64_t)L.np * L.np;
    L.Qbuf = L.V + (int64_t)L.np * L.np;
    L.partial = L.Qbuf + (int64_t)(L.T / 2) * SP * SP;
    L.scal = L.partial + 2 * 1024;
    L.rank = reinterpret_cast<int*>(L.scal + 16);
    L.g2 = grid_for_elems((int64_t)L.np * L.np);
    L.nbo = (int)std::min<unsigned>(L.g2, 64);
    L.napply = (unsigned)((L.T / 2) * (L.T / 2 + 1) / 2 + (L.np / SP) * (L.T / 2));
    return L;
}
// the convergence test of the current matrix: off-diagonal and total mass to the pinned host pair
hipError_t eig_check(const SymEigRun& j, const EigLayout& L) {
    hipLaunchKernelGGL(offnorm_kernel, dim3(L.nbo), dim3(256), 0, j.s, L.Ap, L.np, L.partial);
    hipLaunchKernelGGL(offnorm_fold_kernel, dim3(1), dim3(256), 0, j.s, L.partial, L.nbo, L.scal);
    hipError_t e = hipMemcpyAsync(j.host, L.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, j.s);
    if (e == hipSuccess) e = hipEventRecord(j.ev, j.s);
    return e;
}
}  // namespace

hipError_t sym_eig_start(SymEigRun& j) {
    if (j.n < 1 || j.n > 1024 || j.r < 1 || j.r > j.n || !j.host || !j.ev) return hipErrorInvalidValue;
    const EigLayout L = eig_layout(j.n, j.work);
    j.sweeps = 0;
    j.done = false;
    hipLaunchKernelGGL(offnorm_kernel, dim3(L.nbo), dim3(256), 0, j.s, j.A, j.n, L.partial);
    hipLaunchKernelGGL(offnorm_fold_kernel, dim3(1), dim3(256), 0, j.s, L.partial, L.nbo, L.scal + 2);
    hipLaunchKernelGGL(eig_init_kernel, dim3(L.g2), dim3(256), 0, j.s, j.A, j.n, L.np, L.scal + 2, L.Ap, L.V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return eig_check(j, L);
}

hipError_t sym_eig_step(SymEigRun& j) {
    if (j.done) return hipSuccess;
    const EigLayout L = eig_layout(j.n, j.work);
    hipError_t e = hipEventSynchronize(j.ev);
    if (e != hipSuccess) return e;
    const bool converged = !(j.host[0] > (double)L.np * 0x1p-100 * j.host[1]);
    if (converged || j.sweeps >= 40) {
        hipLaunchKernelGGL(eig_sort_kernel, dim3((L.np + 255) / 256), dim3(256), 0, j.s, L.Ap, j.n, L.np, L.rank,
                           j.lam);
        hipLaunchKernelGGL(eig_gather_kernel, dim3(grid_for_elems((int64_t)j.n * L.np)), dim3(256), 0, j.s, L.V,
                           L.rank, j.n, L.np, j.r, j.U, j.U32);
        j.done = true;
        return hipGetLastError();
    }
    for (int rr = 0; rr < L.T - 1; ++rr) {
        hipLaunchKernelGGL(bj_solve_kernel, dim3(L.T / 2), dim3(256), 0, j.s, L.Ap, L.np, L.T, rr, L.Qbuf);
        hipLaunchKernelGGL(bj_apply_kernel, dim3(L.napply), dim3(256), 0, j.s, L.Ap, L.V, L.np, L.T, rr, L.Qbuf);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ++j.sweeps;
    return eig_check(j, L);
}

}  // namespace tk
