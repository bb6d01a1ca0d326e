// FP64 dense linear algebra for orthogonal iteration and the small modes (gfx950).
//
// chol_inv_scaled: W~ = D^-1 W D^-1 (D = sqrt(diag W)) is factored W~ = L L^T and T = L^-1 D^-1 is
//   produced, so that Q = Z T^T has orthonormal columns when W = Z^T Z (one CholeskyQR pass).
//   The n x n problem is split into TB x TB tiles (TB = kCholTile) and run as one launch of a tiled
//   task graph:
//   factor tasks in column-major order, then inverse tasks (i,j), i > j.  The diagonal task (j,j)
//   also forms the sub-diagonal tile L(j,j-1) as soon as the inverse of L(j-1,j-1) is published
//   and applies its update from LDS, so the critical path crosses one flag per column.
//   Each workgroup claims the next task with an atomic ticket, so every task it waits for was
//   claimed earlier by a running workgroup: the graph cannot deadlock whatever the residency.
//   Waits are bounded spins; a wait that gives up raises an error flag instead of hanging, and the
//   epilogue counts it in a word the host reads back (the call then fails with a device error).
//   Producer: coherent stores, barrier, agent-scope release store of the flag.
//   Consumer: agent-scope acquire load of the flag, barrier, coherent loads.
//
// jacobi_eig: cyclic two-sided Jacobi (Golub & Van Loan, Alg. 8.4.3, with the parallel
//   round-robin ordering) on a symmetric matrix of order <= 64 held in LDS.
#include <algorithm>
#include <utility>

#include "tk_common.h"

namespace tk {
namespace {

constexpr int TB = kCholTile;
constexpr int TS = TB + 1;                  // padded LDS row stride
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr long long kMaxSpin = 1ll << 24;   // default bound of a wait (x ~64 cycles of sleep each)

struct CholArgs {
    double* W;
    int64_t n;
    int T;
    double shift;          // added to the diagonal of the scaled matrix
    bool scale;            // scale by D^-1 on both sides (D = sqrt(diag W)); else D = I
    double* dsc;           // out: 1/sqrt(W_ii) (or 1), written by the diagonal tasks
    double* Tout;
    int* ticket;
    int* flagL;
    int* flagI;
    int* shifts;
    int* err;
    const int* run_if;
    long long max_spin;    // bound of every wait, in sleep steps
};

// Shared tiles are accessed with agent-scope relaxed atomics, which are coherent across the XCDs.
// Flags carry the ordering: the producer's tile stores happen before the workgroup barrier, which
// happens before thread 0's agent-scope release store of the flag; the consumer's thread 0 reads
// the flag with an agent-scope acquire load, and the barrier after it orders every thread's tile
// loads after that acquire.
__device__ __forceinline__ int ld_flag(int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __attribute__((always_inline)) void wait_flags(int* f1, int* f2, int* err, long long max_spin) {
    if (threadIdx.x == 0) {
        long long it = 0;
        bool ready;
        while (!(ready = (ld_flag(f1) != 0 && (!f2 || ld_flag(f2) != 0))) && it < max_spin) {
            __builtin_amdgcn_s_sleep(1);
            ++it;
        }
        if (!ready) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
}

__device__ __attribute__((always_inline)) void release_flag(int* f) {
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0) st_flag(f, 1);
}

// tile (ti,tj) of an n x n row-major matrix -> LDS t; out-of-range -> 0 (or 1 on the diagonal
// when pad_diag), optionally scaled by dr[r] dc[c] (LDS, local row / column) and shifted on the diagonal.  Every thread
// issues all of its TB*TB/256 coherent loads before the first use, so their latencies overlap.
constexpr int kTileVals = TB * TB / 256;

__device__ __attribute__((always_inline)) void load_tile(const double* M, int64_t n, int ti, int tj, double* t, const double* dr,
                          const double* dc, bool pad_diag, double shift = 0.0) {
    double v[kTileVals];
#pragma unroll
    for (int u = 0; u < kTileVals; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int r = e / TB, c = e % TB;
        const int64_t gr = (int64_t)ti * TB + r, gc = (int64_t)tj * TB + c;
        v[u] = 0.0;
        if (gr < n && gc < n) v[u] = ld_coh(&M[gr * n + gc]);
    }
#pragma unroll
    for (int u = 0; u < kTileVals; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int r = e / TB, c = e % TB;
        const int64_t gr = (int64_t)ti * TB + r, gc = (int64_t)tj * TB + c;
        double x;
        if (gr < n && gc < n) {
            x = v[u];
            if (dr) x *= dr[r] * dc[c];
            if (gr == gc) x += shift;
        } else {
            x = (pad_diag && gr == gc) ? 1.0 : 0.0;
        }
        t[r * TS + c] = x;
    }
}

__device__ __attribute__((always_inline)) void store_tile(double* M, int64_t n, int ti, int tj, const double* t) {
#pragma unroll
    for (int u = 0; u < kTileVals; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int r = e / TB, c = e % TB;
        const int64_t gr = (int64_t)ti * TB + r, gc = (int64_t)tj * TB + c;
        if (gr < n && gc < n) st_coh(&M[gr * n + gc], t[r * TS + c]);
    }
}

// C = beta*C + alpha * A * op(B), op(B) = B^T when transB, on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  256 threads = 4 waves; wave w owns the TB/2 x TB/2 quadrant at rows
// TB/2 (w & 1), columns TB/2 (w >> 1) as 16 x 16 tiles.  Fragment layouts: A lane l holds
// (row l % 16, k l / 16), B lane l holds (k l / 16, column l % 16), the result lane l holds
// column l % 16 and rows l / 16 + 4 v.  C may alias A or B (results are written after a barrier).
__device__ __attribute__((always_inline)) void tile_gemm(double* C, const double* A, const double* B, bool transB,
                                                         double alpha, double beta) {
    constexpr int H = TB / 2, NT = TB / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = H * (wave & 1), col0 = H * (wave >> 1);
    const int fr = lane & 15, fk = lane >> 4;
    f64x4_t acc[NT][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < TB; k0 += 4) {
        const int k = k0 + fk;
        double av[NT], bv[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) av[i] = A[(row0 + 16 * i + fr) * TS + k];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int c = col0 + 16 * j + fr;
            bv[j] = transB ? B[c * TS + k] : B[k * TS + c];
        }
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();   // C may alias A or B
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* d = &C[(row0 + 16 * i + fk + 4 * v) * TS + col0 + 16 * j + fr];
                *d = (beta == 0.0 ? 0.0 : beta * *d) + alpha * acc[i][j][v];
            }
    __syncthreads();
}

// ---- TB x TB tile factorisation and inversion, blocked by 16: the sequential parts are 16 x 16
// problems solved inside one wave's registers (row r in lane r, column entries broadcast across
// lanes, no barriers); the rest is parallel over the workgroup with a barrier per phase.
constexpr int SB = 16;   // inner block
static_assert(TB == 32 || TB == 64, "the tile kernels assume 32 x 32 or 64 x 64 tiles and 256 threads");

__device__ __forceinline__ double safe_pivot(double d) { return (d > 1e-13) ? d : 1e-13; }

// 1/d for d > 0: the hardware reciprocal estimate refined by two Newton steps y <- y (2 - d y)
// (each step squares the relative error; the result is within a few ulp).  Keeps the long-latency
// IEEE division off the sequential pivot chains below.
__device__ __forceinline__ double rcp_nr(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = fma(fma(-d, y, 1.0), y, y);
    y = fma(fma(-d, y, 1.0), y, y);
    return y;
}

// ---- 16 x 16 diagonal blocks in one wave.  Lane r holds row r of the block (a[j] = A_rj) and
// column r of its inverse (x[i] = X_ir); the four 16-lane rows of the wave repeat the same problem.
// Column entries are broadcast within each 16-lane row with DPP row_newbcast, one instruction per
// double.  A broadcast must run with every lane of the row active (a masked-off source lane reads
// as zero), so it is never placed inside a lane-dependent branch.
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xF, 0xF, true);
}

// Elimination of column K (L D L^T form, pivot d = A_KK): for rows j > K,
//   A_rj -= (A_rK / d) A_jK   and, for the unit-lower inverse, x_j -= (A_jK / d) x_K.
template <int K, int... J>
__device__ __forceinline__ void ldl_eliminate(double (&a)[SB], double (&x)[SB], double c, double ci, double t,
                                              std::integer_sequence<int, J...>) {
    ((a[K + 1 + J] = fma(-ci, row_bcast<K + 1 + J>(c), a[K + 1 + J]),
      x[K + 1 + J] = fma(-row_bcast<K + 1 + J>(c), t, x[K + 1 + J])), ...);
}

template <int K>
__device__ __forceinline__ void ldl_steps(double (&a)[SB], double (&x)[SB], double& dmine, int r, int& bad) {
    if constexpr (K < SB) {
        const double d = row_bcast<K>(a[K]);           // pivot of column K
        if (r == K) dmine = d;
        bad += (d > 1e-13) ? 0 : 1;
        const double rinv = rcp_nr(safe_pivot(d));
        const double c = a[K];
        ldl_eliminate<K>(a, x, c, c * rinv, x[K] * rinv, std::make_integer_sequence<int, SB - 1 - K>{});
        // the inverse columns feed nothing until the end; without this (empty) register constraint
        // the compiler postpones their updates and parks every broadcast in spare registers
#pragma unroll
        for (int j = K + 1; j < SB; ++j) asm volatile("" : "+v"(x[j]));
        ldl_steps<K + 1>(a, x, dmine, r, bad);
    }
}

// L = L~ D^1/2 (L_rj = A_rj / sqrt(d_j) below the diagonal, sqrt(d_r) on it, 0 above) and
// L^-1 = D^-1/2 L~^-1 (row i of the inverse scaled by 1/sqrt(d_i)).
template <int J>
__device__ __forceinline__ void ldl_finish1(double (&a)[SB], double (&x)[SB], double sq, double rs, int r) {
    const double b = row_bcast<J>(rs);
    const double v = a[J] * b;
    a[J] = (J < r) ? v : ((J == r) ? sq : 0.0);
    x[J] *= b;
}
template <int... J>
__device__ __forceinline__ void ldl_finish(double (&a)[SB], double (&x)[SB], double sq, double rs, int r,
                                           std::integer_sequence<int, J...>) {
    (ldl_finish1<J>(a, x, sq, rs, r), ...);
}

// One wave (all 64 lanes active): Cholesky of the 16 x 16 diagonal block at (o, o) of A (LDS, row
// stride TS), in place (lower L, upper zeroed), and L^-1 into X (LDS, row stride ldx, zeros above
// the diagonal).  Pivots <= 1e-13 are replaced by 1e-13 and counted in *shifts.
__device__ __attribute__((always_inline)) void wave_potrf16(double* A, int o, double* X, int ldx, int* shifts) {
    const int lane = threadIdx.x & 63, r = lane & 15;
    double a[SB], x[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        a[j] = A[(o + r) * TS + o + j];
        x[j] = (j == r) ? 1.0 : 0.0;
    }
    double dmine = 1.0;
    int bad = 0;
    ldl_steps<0>(a, x, dmine, r, bad);
    const double sq = sqrt(safe_pivot(dmine));
    const double rs = rcp_nr(sq);
    ldl_finish(a, x, sq, rs, r, std::make_integer_sequence<int, SB>{});
    if (lane < SB) {
#pragma unroll
        for (int j = 0; j < SB; ++j) {
            A[(o + r) * TS + o + j] = a[j];
            X[j * ldx + r] = x[j];
        }
    }
    if (lane == 0 && bad) atomicAdd(shifts, bad);
}

// In-LDS Cholesky of the TB x TB tile A (lower; upper zeroed); the inverses of its TB/16 diagonal
// 16 x 16 blocks go to the diagonal blocks of X (row stride TS).  Right-looking over the 16-wide
// block columns: wave 0 factors and inverts the diagonal block; the block column below,
// L_ib = A_ib L_bb^-T, and the trailing update A_ij -= L_ib L_jb^T (i >= j, 16 x 16 tiles) run on
// the FP64 matrix cores, one 16 x 16 tile per wave.
__device__ __attribute__((always_inline)) void tile_potrf(double* A, double* X, int* shifts) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int fr = lane & 15, fk = lane >> 4;
    for (int b = 0; b < TB / SB; ++b) {
        const int o = b * SB;
        if (tid < 64) wave_potrf16(A, o, X + o * TS + o, TS, shifts);
        __syncthreads();
        const int nt = (TB - o - SB) / SB;      // 16-row tiles below the diagonal block
        if (nt > 0) {
            if (wave < nt) {
                // L_ic = sum_k A_ik Y_ck (Y = L_bb^-1): A fragment (row fr, k), B fragment (k, column fr) = Y[fr][k]
                const int r0 = o + SB + SB * wave;
                f64x4_t acc = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < SB / 4; ++st) {
                    const int k = 4 * st + fk;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(r0 + fr) * TS + o + k], X[(o + fr) * TS + o + k],
                                                               acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) A[(r0 + fk + 4 * v) * TS + o + fr] = acc[v];
            }
            __syncthreads();
            // trailing lower triangle by 16 x 16 tile pairs (I >= J)
            const int npairs = nt * (nt + 1) / 2;
            for (int pidx = wave; pidx < npairs; pidx += 4) {
                int I = 0;
                while ((I + 1) * (I + 2) / 2 <= pidx) ++I;
                const int J = pidx - I * (I + 1) / 2;
                const int ri = o + SB + SB * I, rj = o + SB + SB * J;
                f64x4_t acc = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < SB / 4; ++st) {
                    const int k = 4 * st + fk;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(ri + fr) * TS + o + k], A[(rj + fr) * TS + o + k],
                                                               acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) A[(ri + fk + 4 * v) * TS + rj + fr] -= acc[v];
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < TB * TB; e += blockDim.x) {
        const int i = e / TB, j = e % TB;
        if (j > i) A[i * TS + j] = 0.0;
    }
    __syncthreads();
}

// Inverse of the lower-triangular TB x TB tile L (LDS) into X (LDS), given the inverses of the
// diagonal 16 x 16 blocks in X and zeros above them: block forward substitution over the block
// rows, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj, on the FP64 matrix cores.
__device__ __attribute__((always_inline)) void tile_trtri(const double* L, double* X) {
    __shared__ double Tm[3 * SB * SB];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int fr = lane & 15, fk = lane >> 4;
    for (int bi = 1; bi < TB / SB; ++bi) {
        // wave j < bi: T_j = sum_{k=j}^{bi-1} L_{bi,k} X_{k,j}
        if (wave < bi) {
            const int bj = wave;
            f64x4_t acc = f64x4_t{0.0, 0.0, 0.0, 0.0};
            for (int bk = bj; bk < bi; ++bk)
#pragma unroll
                for (int st = 0; st < SB / 4; ++st) {
                    const int k = bk * SB + 4 * st + fk;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(L[(bi * SB + fr) * TS + k], X[k * TS + bj * SB + fr],
                                                               acc, 0, 0, 0);
                }
#pragma unroll
            for (int v = 0; v < 4; ++v) Tm[bj * SB * SB + (fk + 4 * v) * SB + fr] = acc[v];
        }
        __syncthreads();
        // wave j < bi: X_{bi,j} = -X_{bi,bi} T_j
        if (wave < bi) {
            const int bj = wave;
            f64x4_t acc = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < SB / 4; ++st) {
                const int k = 4 * st + fk;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[(bi * SB + fr) * TS + bi * SB + k],
                                                           Tm[bj * SB * SB + k * SB + fr], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) X[(bi * SB + fk + 4 * v) * TS + bj * SB + fr] = -acc[v];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void chol_graph(CholArgs a) {
    __shared__ double At[TB * TS], Bt[TB * TS], Ct[TB * TS], Dt[TB * TS];
    __shared__ int task_s;
    if (a.run_if && *a.run_if == 0) return;
    if (threadIdx.x == 0) task_s = atomicAdd(a.ticket, 1);
    __syncthreads();
    const int task = task_s;
    const int T = a.T;
    // factor tasks, column by column: the diagonal task (j, j) (which also forms the sub-diagonal
    // tile L(j, j-1)), then (i, j) for i >= j + 2; then the inverse tasks
    const int nf = T * (T + 1) / 2 - (T - 1);
    if (task >= nf + T * (T - 1) / 2) return;
    auto fL = [&](int i, int j) { return a.flagL + i * T + j; };
    auto fI = [&](int i, int j) { return a.flagI + i * T + j; };

    if (task < nf) {
        int j = 0, rem = task;
        while (rem >= ((j < T - 1) ? T - j - 1 : 1)) {
            rem -= (j < T - 1) ? T - j - 1 : 1;
            ++j;
        }
        const int i = (rem == 0) ? j : j + 1 + rem;
        const bool diag = i == j;
        const bool sub = diag && j > 0;
        // D^-1 for the rows of tile i, the columns of tile j and (sub) those of tile j - 1, from the
        // diagonal of W (the diagonal tiles of W are never overwritten: L_jj is not stored back)
        __shared__ double dr[TB], dc[TB], dp[TB];
        if (threadIdx.x < 3 * TB) {
            const int grp = threadIdx.x / TB, l = threadIdx.x % TB;
            const int tile = grp == 0 ? i : (grp == 1 ? j : j - 1);
            const int64_t g = (int64_t)tile * TB + l;
            double v = 1.0;
            if (tile >= 0 && g < a.n && a.scale) {
                const double d = a.W[g * a.n + g];
                v = (d > 0.0) ? 1.0 / sqrt(d) : 1.0;
                if (diag && grp == 0) {
                    a.dsc[g] = v;
                    if (!(d > 0.0)) atomicAdd(a.shifts, 1);
                }
            } else if (tile >= 0 && g < a.n && diag && grp == 0) {
                a.dsc[g] = 1.0;
            }
            (grp == 0 ? dr : (grp == 1 ? dc : dp))[l] = v;
        }
        __syncthreads();
        load_tile(a.W, a.n, i, j, At, dr, dc, diag, diag ? a.shift : 0.0);
        if (sub) load_tile(a.W, a.n, j, j - 1, Ct, dr, dp, false);
        __syncthreads();   // the whole tile is in LDS before wave 0 may factor it (j == 0)
        if (sub) {
            // A_jj -= L_jk L_jk^T and A_j,j-1 -= L_jk L_j-1,k^T for k < j - 1
            for (int k = 0; k < j - 1; ++k) {
                wait_flags(fL(j, k), fL(j - 1, k), a.err, a.max_spin);
                load_tile(a.W, a.n, j, k, Bt, nullptr, nullptr, false);
                load_tile(a.W, a.n, j - 1, k, Dt, nullptr, nullptr, false);
                __syncthreads();
                tile_gemm(At, Bt, Bt, true, -1.0, 1.0);
                tile_gemm(Ct, Bt, Dt, true, -1.0, 1.0);
            }
            // L_j,j-1 = A_j,j-1 Linv_j-1^T; A_jj -= L_j,j-1 L_j,j-1^T from LDS while its stores drain
            wait_flags(fI(j - 1, j - 1), nullptr, a.err, a.max_spin);
            load_tile(a.Tout, a.n, j - 1, j - 1, Bt, nullptr, nullptr, false);
            __syncthreads();
            tile_gemm(Dt, Ct, Bt, true, 1.0, 0.0);
            store_tile(a.W, a.n, j, j - 1, Dt);
            tile_gemm(At, Dt, Dt, true, -1.0, 1.0);   // overlaps the stores of L_j,j-1
            release_flag(fL(j, j - 1));
        } else {
            for (int k = 0; k < j; ++k) {
                wait_flags(fL(i, k), fL(j, k), a.err, a.max_spin);
                load_tile(a.W, a.n, i, k, Bt, nullptr, nullptr, false);
                if (!diag) load_tile(a.W, a.n, j, k, Ct, nullptr, nullptr, false);
                __syncthreads();
                tile_gemm(At, Bt, diag ? Bt : Ct, true, -1.0, 1.0);
            }
        }
        if (diag) {
            for (int e = threadIdx.x; e < TB * TS; e += blockDim.x) Bt[e] = 0.0;
            __syncthreads();
            tile_potrf(At, Bt, a.shifts);
            tile_trtri(At, Bt);
            store_tile(a.Tout, a.n, j, j, Bt);     // L_jj itself is not needed by any later task
            stores_done();
            __syncthreads();
            if (threadIdx.x == 0) {
                st_flag(fL(j, j), 1);
                st_flag(fI(j, j), 1);
            }
        } else {
            wait_flags(fL(j, j), nullptr, a.err, a.max_spin);
            load_tile(a.Tout, a.n, j, j, Bt, nullptr, nullptr, false);
            __syncthreads();
            tile_gemm(Ct, At, Bt, true, 1.0, 0.0);       // L_ij = A_ij Linv_jj^T
            store_tile(a.W, a.n, i, j, Ct);
            release_flag(fL(i, j));
        }
    } else {
        int rem = task - nf, j = 0;
        while (rem >= T - 1 - j) {
            rem -= T - 1 - j;
            ++j;
        }
        const int i = j + 1 + rem;
        for (int e = threadIdx.x; e < TB * TS; e += blockDim.x) Ct[e] = 0.0;
        __syncthreads();
        for (int k = j; k < i; ++k) {
            wait_flags(fL(i, k), fI(k, j), a.err, a.max_spin);
            load_tile(a.W, a.n, i, k, At, nullptr, nullptr, false);
            load_tile(a.Tout, a.n, k, j, Bt, nullptr, nullptr, false);
            __syncthreads();
            tile_gemm(Ct, At, Bt, false, 1.0, 1.0);       // acc += L_ik Linv_kj
        }
        wait_flags(fI(i, i), nullptr, a.err, a.max_spin);
        load_tile(a.Tout, a.n, i, i, At, nullptr, nullptr, false);
        __syncthreads();
        tile_gemm(Bt, At, Ct, false, -1.0, 0.0);          // Linv_ij = -Linv_ii acc
        store_tile(a.Tout, a.n, i, j, Bt);
        release_flag(fI(i, j));
    }
}

// T <- lower(T) * D^-1 (column scaling), upper triangle zeroed.  Block 0 also counts a call of the
// task graph in which a wait gave up (shifts[kWaitTimeoutSlot]) and then clears the graph's
// counters for the next call.
__global__ __launch_bounds__(256) void chol_epilogue(double* Tm, int64_t n, const double* dsc, int* counters,
                                                     int nctr, int* shifts, const int* run_if) {
    if (run_if && *run_if == 0) return;
    if (blockIdx.x == 0) {
        __shared__ int err;
        if (threadIdx.x == 0) err = counters[1];
        __syncthreads();
        if (threadIdx.x == 0 && err) atomicAdd(shifts + kWaitTimeoutSlot, 1);
        for (int e = threadIdx.x; e < nctr; e += blockDim.x) counters[e] = 0;
    }
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e % n;
        Tm[e] = (r >= c) ? Tm[e] * dsc[c] : 0.0;
    }
}

// Deviation of a Gram Q^T Q from the identity, max_ij |W_ij - delta_ij|: per-block maxima, then
// one block folds them and writes need = (max > tol) (NaN counts as needed) and counts the passes.
constexpr int kOrthBlocks = 128;
// max_ij |W_ij - delta_ij| > tol -> *need = 1 (and ++*count), else *need = 0, in one launch: each
// block reduces its share, and the last block to finish (ticket in *sync, cleared afterwards) takes
// the maximum of the block maxima, which does not depend on their order.
__global__ __launch_bounds__(256) void orth_check_kernel(const double* __restrict__ W, int64_t n, double tol,
                                                         double* partial, int* need, int* count, int* sync) {
    __shared__ double red[256];
    __shared__ int last;
    double m = 0.0;
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t row = e / n, col = e - row * n;
        if (col > row) continue;            // the lower triangle (W symmetric; only it is formed)
        const double a = fabs(W[e] - ((row == col) ? 1.0 : 0.0));
        m = (a > m || a != a) ? a : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(&partial[blockIdx.x], red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int t = __hip_atomic_fetch_add(sync, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    // the last block: one block maximum per thread, then the same tree as above
    double mx = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 256) {
        const double o = __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (o > mx || o != o) mx = o;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int nd = !(red[0] <= tol);
        *need = nd;
        if (nd && count) atomicAdd(count, 1);
        __hip_atomic_store(sync, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// *need: the second pass ran and U64 holds its result -> U32 = U64; else U64 = U32 = Q1
__global__ __launch_bounds__(256) void finish_factor_kernel(const int* need, const double* __restrict__ Q1,
                                                            double* __restrict__ U64, float* __restrict__ U32,
                                                            int64_t n) {
    const bool second = *need != 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = second ? U64[i] : Q1[i];
        if (!second) U64[i] = v;
        if (U32) U32[i] = (float)v;
    }
}

// ---------------------------------------------------------------- Jacobi
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ S, int n, int r,
                                                     double* __restrict__ U64, float* __restrict__ U32,
                                                     double* __restrict__ lam, double* __restrict__ Vio,
                                                     int warm) {
    constexpr int NM = 64, LD = 65;
    __shared__ double A[NM * LD], V[NM * LD], Tw[NM * LD];
    __shared__ double cs[NM / 2], sn[NM / 2];
    __shared__ int pp[NM / 2], qq[NM / 2];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int n2 = n + (n & 1);
    for (int e = tid; e < n2 * n2; e += blockDim.x) {
        const int i = e / n2, j = e % n2;
        double v = 0.0;
        if (i < n && j < n) v = 0.5 * (S[i * n + j] + S[j * n + i]);
        A[i * LD + j] = v;
        double w = (i == j) ? 1.0 : 0.0;
        if (warm && i < n && j < n) w = Vio[i * n + j];
        V[i * LD + j] = w;
    }
    __syncthreads();
    if (warm) {
        // start from the previous eigenvector basis V0: A <- V0^T S V0 (nearly diagonal when S has
        // changed little), the rotations then accumulate onto V0
        for (int e = tid; e < n2 * n2; e += blockDim.x) {
            const int i = e / n2, j = e % n2;
            double t = 0.0;
            for (int k = 0; k < n2; ++k) t = fma(A[i * LD + k], V[k * LD + j], t);
            Tw[i * LD + j] = t;
        }
        __syncthreads();
        for (int e = tid; e < n2 * n2; e += blockDim.x) {
            const int i = e / n2, j = e % n2;
            if (j > i) continue;
            double t = 0.0, u = 0.0;
            for (int k = 0; k < n2; ++k) {
                t = fma(V[k * LD + i], Tw[k * LD + j], t);
                u = fma(V[k * LD + j], Tw[k * LD + i], u);
            }
            const double v = 0.5 * (t + u);
            A[i * LD + j] = v;
            A[j * LD + i] = v;
        }
        __syncthreads();
    }
    const int npair = n2 / 2;
    for (int sweep = 0; sweep < 40 && n2 > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < n2 * n2; e += blockDim.x) {
            const int i = e / n2, j = e % n2;
            const double v = A[i * LD + j];
            tot += v * v;
            if (i != j) off += v * v;
        }
        red[tid] = off;
        __syncthreads();
        for (int w = (int)blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        const double offs = red[0];
        __syncthreads();
        red[tid] = tot;
        __syncthreads();
        for (int w = (int)blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        const double tots = red[0];
        __syncthreads();
        if (!(offs > 1e-30 * tots)) break;
        for (int rr = 0; rr < n2 - 1; ++rr) {
            if (tid < npair) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + rr) % (n2 - 1)); };
                int p = player(tid), q = player(n2 - 1 - tid);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                const double apq = A[p * LD + q];
                if (q < n && apq != 0.0) {
                    const double app = A[p * LD + p], aqq = A[q * LD + q];
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                pp[tid] = p;
                qq[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            for (int e = tid; e < npair * n2; e += blockDim.x) {     // rows: A <- J^T A
                const int k = e / n2, col = e % n2;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = A[p * LD + col], aq = A[q * LD + col];
                A[p * LD + col] = c * ap - s * aq;
                A[q * LD + col] = s * ap + c * aq;
            }
            __syncthreads();
            for (int e = tid; e < npair * n2; e += blockDim.x) {     // cols: A <- A J, V <- V J
                const int k = e / n2, row = e % n2;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = A[row * LD + p], aq = A[row * LD + q];
                A[row * LD + p] = c * ap - s * aq;
                A[row * LD + q] = s * ap + c * aq;
                const double vp = V[row * LD + p], vq = V[row * LD + q];
                V[row * LD + p] = c * vp - s * vq;
                V[row * LD + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // rank = number of larger eigenvalues (ties by index): descending order
    __shared__ int rank[NM];
    if (tid < n) {
        const double li = A[tid * LD + tid];
        int k = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j * LD + j];
            if (lj > li || (lj == li && j < tid)) ++k;
        }
        rank[tid] = k;
        if (lam) lam[k] = li;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int row = e / n, i = e % n;
        const int k = rank[i];
        const double v = V[row * LD + i];
        if (k < r) {
            U64[row * r + k] = v;
            if (U32) U32[row * r + k] = (float)v;
        }
        if (Vio) Vio[row * n + k] = v;     // the whole sorted basis, for the next warm start
    }
}

}  // namespace

int64_t chol_counter_ints(int64_t n) {
    const int64_t T = (n + TB - 1) / TB;
    return 2 + 2 * T * T;
}

hipError_t chol_inv_scaled(double* W, int64_t n, bool scale, double shift, double* Tout, int* counters,
                           double* dsc, int* shifts, hipStream_t s, const int* run_if, long long max_spin) {
    if (n <= 0) return hipSuccess;
    if (max_spin <= 0) max_spin = kMaxSpin;
    const int T = (int)((n + TB - 1) / TB);
    // counters: [0] ticket, [1] error, then flagL (T*T), flagI (T*T); zero on entry, cleared again
    // by the epilogue
    const int nctr = (int)chol_counter_ints(n);
    CholArgs a{W, n, T, shift, scale, dsc, Tout, counters, counters + 2, counters + 2 + T * T, shifts, counters + 1,
               run_if, max_spin};
    hipLaunchKernelGGL(chol_graph, dim3((unsigned)(T * T - T + 1)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = n * n;
    hipLaunchKernelGGL(chol_epilogue, dim3((unsigned)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096)),
                       dim3(256), 0, s, Tout, n, dsc, counters, nctr, shifts, run_if);
    return hipGetLastError();
}

int orth_check_partials() { return kOrthBlocks; }

hipError_t orth_check(const double* W, int64_t n, double tol, double* partial, int* need, int* count, int* sync,
                      hipStream_t s) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kOrthBlocks, (n * n + 255) / 256));
    hipLaunchKernelGGL(orth_check_kernel, dim3(nb), dim3(256), 0, s, W, n, tol, partial, need, count, sync);
    return hipGetLastError();
}

hipError_t finish_factor(const int* need, const double* Q1, double* U64, float* U32, int64_t n, hipStream_t s) {
    const int64_t g = std::min<int64_t>(2048, (n + 255) / 256);
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_factor_kernel, dim3((unsigned)g), dim3(256), 0, s, need, Q1, U64, U32, n);
    return hipGetLastError();
}

// out (cols x rows) = in^T for a row-major FP32 in (rows x cols), through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void transpose_f32_kernel(const float* __restrict__ in, int64_t rows, int64_t cols,
                                                            float* __restrict__ out) {
    __shared__ float t[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) t[k][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < cols && r < rows) out[c * rows + r] = t[tx][k];
    }
}

hipError_t transpose_f32(const float* in, int64_t rows, int64_t cols, float* out, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if ((rows + 31) / 32 > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(transpose_f32_kernel, grid, dim3(256), 0, s, in, rows, cols, out);
    return hipGetLastError();
}

hipError_t jacobi_eig(const double* S, int n, int r, double* U64, float* U32, double* lam, hipStream_t s,
                      double* Vio, bool warm) {
    if (n < 1 || n > 64 || r < 1 || r > n) return hipErrorInvalidValue;
    if (warm && !Vio) return hipErrorInvalidValue;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(256), 0, s, S, n, r, U64, U32, lam, Vio, warm ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tk
