// Internal declarations shared by the HIP translation units of the Tucker-ALS library.
// Every kernel launcher returns hipError_t and enqueues on the stream it is given.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

namespace tk {

// ---------------------------------------------------------------------------------------
// Strided operand descriptor.  Element (r, c) of a logical matrix lives at
//   ptr[r * ld + (c / seg) * segstride + (c % seg)]
// so one descriptor covers plain row-major matrices (seg >= #cols) and the (A, K, B)
// views of a row-major tensor whose "column" index folds two modes (seg = B).
// ---------------------------------------------------------------------------------------
struct Desc {
    const void* ptr;
    int64_t ld;
    int64_t seg;
    int64_t segstride;
};

inline Desc plain(const void* p, int64_t ld) { return Desc{p, ld, int64_t(1) << 62, 0}; }
inline Desc folded(const void* p, int64_t ld, int64_t seg, int64_t segstride) {
    return Desc{p, ld, seg, segstride};
}

// Operand orientation: for A, KM means element (m,k) is desc(r=k, c=m); MK means desc(r=m, c=k).
// For B, KN means (k,n) is desc(r=k, c=n); NK means desc(r=n, c=k).
enum Orient { KM = 0, MK = 1 };

enum Epilogue {
    EPI_STORE = 0,      // C(m,n) = alpha * acc
    EPI_ADD = 1,        // C(m,n) = alpha * acc + C(m,n)
    EPI_RESID = 2       // sum over tile of (X(m,n) - alpha*acc)^2 into one double per block
};

struct GemmArgs {
    Desc a, b, c;       // c: output (or, for EPI_RESID, the reference tensor X)
    int64_t M, N, K;
    double alpha;
    int64_t k_split;    // K elements per split (grid.z splits); == K when not split
    int64_t c_zstride;  // element offset between split outputs
    int lower_only;     // enumerate only tiles with tile_m >= tile_n (Gram / SYRK)
    double* resid_partial;   // EPI_RESID: one double per block
    const int* run_if;       // nullable: the launch does nothing when *run_if == 0
    int c_f32;               // FP64 kernels, EPI_STORE: write c as float (rounded once)
    int k_upto_n;            // B(k, n) = 0 for k > n: a tile's k range ends at its last column
};

// fp32 MFMA GEMM (operands fp32, accumulation fp32; acc64 = FP64 accumulation across k-tiles)
hipError_t gemm_f32(const GemmArgs& g, Orient oa, Orient ob, Epilogue epi, bool acc64,
                    hipStream_t s);
// fp64 MFMA GEMM; a_is_f32/b_is_f32 select float operands converted to double on load
hipError_t gemm_f64(const GemmArgs& g, Orient oa, Orient ob, Epilogue epi, bool a_is_f32,
                    bool b_is_f32, hipStream_t s);
// workgroups of the FP64 Gram kernel (FP32 operands, both k-contiguous) resident per CU (0 if unknown)
int gram_f64_blocks_per_cu();
// compute units of the current device (queried once per process; 256 when no device answers)
int device_cu_count();
// number of blocks gemm_* launches for these arguments (for EPI_RESID partial sizing)
int64_t gemm_grid_blocks(const GemmArgs& g, bool f64);

// ---------------------------------------------------------------------------------------
// Small / memory-bound kernels (tk_small.hip)
// ---------------------------------------------------------------------------------------
// partial[b] = sum of squares of a grid-stride share; then result = sum(partial) (fp64).
hipError_t sumsq_f32(const float* x, int64_t n, double* partial, int nblocks, double* result,
                     hipStream_t s);
hipError_t sumsq_f64(const double* x, int64_t n, double* partial, int nblocks, double* result,
                     hipStream_t s);
hipError_t reduce_f64(const double* partial, int64_t n, double* result, hipStream_t s);
constexpr int kSumsqBlocks = 1024;

// Mode product on a (A, K, B) view with a small K and R:
//   expand == false: out[a][r][b] = sum_k U[k*R + r] * in[a][k][b]   (U is K x R)
//   expand == true : out[a][r][b] = sum_k U[r*K + k] * in[a][k][b]   (U is R x K)
hipError_t small_ttm(const float* in, int64_t A, int64_t K, int64_t B, const float* U,
                     int64_t R, bool expand, float* out, hipStream_t s);

// Fused product over the two trailing modes of a (A, p, q) view (p <= 4, q <= 16):
//   expand == false: out[a][r][t] = sum_{c,i} U3[c*R3+r] U4[i*R4+t] in[a][c][i]
//   expand == true : out[a][c][i] = sum_{r,t} U3[c*R3+r] U4[i*R4+t] in[a][r][t]
//   (U3 is p x R3, U4 is q x R4 in both cases)
//   u3_identity: U3 is the p x p identity (a mode kept at full rank); its product is skipped
hipError_t pair_ttm(const float* in, int64_t A, int p, int q, const float* U3, int R3,
                    const float* U4, int R4, bool expand, float* out, hipStream_t s, bool u3_identity = false);
bool pair_ttm_supported(int p, int q);

// Fibre Gram of a (A, L) row-major matrix (L <= 64): F = sum_a x_a x_a^T (fp64, L x L),
// two-stage deterministic.  partial: nblocks * L * L doubles.
hipError_t fibre_gram(const float* in, int64_t A, int L, double* partial, int nblocks,
                      double* F, hipStream_t s);
constexpr int kFibreGramBlocks = 512;

// Given the fibre Gram F over (p x q) fibres and projectors P3 = U3 U3^T (p x p),
// P4 = U4 U4^T (q x q) (fp64 factors), produce the mode Grams:
//   which == 3: S3[c][c'] = sum_{i,i'} F[(c,i),(c',i')] P4[i][i']
//   which == 4: S4[i][i'] = sum_{c,c'} F[(c,i),(c',i')] P3[c][c']
// A null projector means the identity.  Output fp64 (n x n).
hipError_t pair_mode_gram(const double* F, int p, int q, const double* U, int R, int which,
                          double* S, hipStream_t s);

// Mode Gram of a (A, s, B) view with s <= 64 by vector FMAs; fp64 result.
hipError_t small_gram(const float* in, int64_t A, int64_t sdim, int64_t B, double* partial,
                      int nblocks, double* S, hipStream_t s);

// Split-K Gram reduction: S[i][j] = sum_z P[z][max(i,j)][min(i,j)] (fp64 sum, symmetric fill).
hipError_t gram_reduce(const float* P, int nsplit, int64_t n, int64_t zstride, float* S32,
                       double* S64, hipStream_t s);

hipError_t gram_reduce64(const double* P, int nsplit, int64_t n, int64_t zstride, double* S64, hipStream_t s);

hipError_t f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s);
hipError_t fill_identity_f32(float* out, int64_t rows, int64_t cols, hipStream_t s);
hipError_t fill_identity_f64(double* out, int64_t rows, int64_t cols, hipStream_t s);
hipError_t fill_zero(void* p, int64_t bytes, hipStream_t s);
// counter-based start basis: out[i] = uniform(-1,1) from splitmix64(seed + i)
hipError_t fill_random(float* out, int64_t n, uint64_t seed, hipStream_t s);
// fit = 1 - sqrt(max(nx2 - ng2, 0)) / sqrt(nx2)   (single thread)
hipError_t fit_from_norms(const double* nx2, const double* ng2, double* fit, hipStream_t s);
hipError_t fit_from_resid(const double* nx2, const double* r2, double* fit, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Dense linear algebra (tk_linalg.hip)
// ---------------------------------------------------------------------------------------
// Column-scaled Cholesky W~ + shift I = L L^T of W (n x n fp64, lower triangle read; W~ =
// D^-1 W D^-1, D = sqrt(diag W) when scale) by a tiled task graph, then T = L^-1 D^-1 (lower
// triangular) to Tout.  W's off-diagonal tiles are overwritten by L; its diagonal tiles are kept.
// counters: chol_counter_ints(n) ints that must be zero on entry; they are zero again when the
// call's kernels have finished.  dsc: n doubles of scratch (the diagonal scale).
// shifts: at least kWaitTimeoutSlot + 1 ints; shifts[0] is incremented for every pivot that needed
// the shifted fallback, shifts[kWaitTimeoutSlot] for every call in which a wait of the task graph
// gave up after max_spin sleep steps (<= 0: the default bound, about half a second); such a call's
// result is garbage and the caller must report an error.
// run_if (nullable): every kernel of the call returns at once when *run_if == 0.
constexpr int kWaitTimeoutSlot = 5;
// tile edge of the Cholesky task graph (32: a shorter critical path per block column than 64 on
// gfx950, whose FP64 matrix rate makes the 64 x 64 tile products the slow link)
constexpr int kCholTile = 32;
hipError_t chol_inv_scaled(double* W, int64_t n, bool scale, double shift, double* Tout, int* counters,
                           double* dsc, int* shifts, hipStream_t s, const int* run_if = nullptr,
                           long long max_spin = 0);
// need[0] = 1 (and ++count[0]) when max_{i>=j} |W_ij - delta_ij| > tol, else 0 (n x n FP64, symmetric:
// only the lower triangle is read), in one
// launch.  partial: orth_check_partials() doubles of scratch; sync: an int that is zero on entry
// (and zero again afterwards).
hipError_t orth_check(const double* W, int64_t n, double tol, double* partial, int* need, int* count, int* sync,
                      hipStream_t s);
int orth_check_partials();
// *need != 0: U32 = (float)U64; else U64 = Q1 and U32 = (float)Q1 (n values)
hipError_t finish_factor(const int* need, const double* Q1, double* U64, float* U32, int64_t n, hipStream_t s);
int64_t chol_counter_ints(int64_t n);

// Eigen-decomposition of a symmetric n x n FP64 matrix A (row-major, read-only), n <= 1024, by two-sided
// block Jacobi (tk_eig.hip): all eigenvalues descending to lam (nullable, n doubles), the eigenvectors
// of the r largest to U (nullable, n x r FP64) and U32 (nullable, FP32).  work: sym_eig_work_doubles(n)
// doubles of scratch.  Synchronises the stream once per sweep (convergence test); *sweeps_out (nullable)
// receives the sweep count.
int64_t sym_eig_work_doubles(int n);
hipError_t sym_eig_blocked(const double* A, int n, int r, double* lam, double* U, float* U32, double* work,
                           hipStream_t s, int* sweeps_out = nullptr);
// The same eigensolver in steps, so that several can run on different streams side by side:
// sym_eig_start enqueues the set-up and the first convergence test (its two sums copied to the
// pinned host pair `host`, completion marked by `ev`); each sym_eig_step waits for the pending test,
// then enqueues either one sweep and the next test or (converged, or 40 sweeps) the final sort and
// gather, and sets done.  The caller owns host (pinned, 2 doubles) and ev.
struct SymEigRun {
    const double* A = nullptr;
    int n = 0, r = 0;
    double* lam = nullptr;
    double* U = nullptr;
    float* U32 = nullptr;
    double* work = nullptr;
    hipStream_t s = nullptr;
    double* host = nullptr;
    hipEvent_t ev = nullptr;
    int sweeps = 0;
    bool done = false;
};
hipError_t sym_eig_start(SymEigRun& j);
hipError_t sym_eig_step(SymEigRun& j);

// ---------------------------------------------------------------------------------------
// Autotuner (tk_tune.hip): measured launch choices cached per (operation, shape, device)
// ---------------------------------------------------------------------------------------
enum TuneOp { kTuneF32Tile = 1, kTuneGramSplit = 2, kTuneLpTile = 3 };
void tune_set_enabled(bool on);     // this thread's calls may time new keys
bool tune_enabled();
// The cached choice for (op, device, shape), else, when tuning is enabled and the stream is not
// capturing, candidates 0..ncand-1 launched (three times each, the last two timed) and the fastest
// cached unless `heuristic` is within the operation's tie margin of it; otherwise `heuristic`.  launch(c) enqueues candidate c on s.
int tune_choose(int op, const int64_t shape[5], int ncand, int heuristic, hipStream_t s,
                const std::function<hipError_t(int)>& launch, hipError_t* err);
std::string tune_dump();
void tune_clear();
// candidate `choice` for every later call of op (< 0: none); false for an unknown op
bool tune_force(int op, int choice);
size_t tune_size();
// RAII: tuning on for this thread while in scope (restores the previous state)
struct TuneScope {
    bool prev;
    explicit TuneScope(bool on) : prev(tune_enabled()) { tune_set_enabled(on); }
    ~TuneScope() { tune_set_enabled(prev); }
};

// ---------------------------------------------------------------------------------------
// Codec hand-off (tk_codec.hip)
// ---------------------------------------------------------------------------------------
struct DimPack {
    int64_t v[8];
};
// out (prod keep) = the leading keep[0] x ... x keep[N-1] block of in (dims), row-major
hipError_t gather_block(const float* in, int N, const int64_t* dims, const int64_t* keep, float* out, hipStream_t s);
// uniform mid-tread quantiser of n floats with 2^(bits-1) - 1 levels per sign: codes, dequantised
// values and the step (device float); amax_scratch: one device float
hipError_t quantize_uniform(const float* x, int64_t n, int bits, float* amax_scratch, int32_t* codes, float* deq,
                            float* step, hipStream_t s);
// out[i] = sqrt(max(lam[i], 0))
hipError_t sqrt_clamp(const double* lam, int64_t n, double* out, hipStream_t s);
// y += x; out = a - b (FP32); D = 1.5 I - 0.5 B (FP64, n x n)
hipError_t axpy_f32(const float* x, float* y, int64_t n, hipStream_t s);
hipError_t diff_f32(const float* a, const float* b, float* out, int64_t n, hipStream_t s);
hipError_t ns_step(const double* B, double* D, int64_t n, hipStream_t s);

// Jacobi eigen-decomposition of a symmetric n x n (n <= 64) fp64 matrix; writes the leading
// r eigenvectors (descending) to U64 (n x r fp64) and U32 (n x r fp32, nullable), all
// eigenvalues descending to lam (nullable).  Vio (nullable, n x n): receives the whole sorted
// eigenvector basis; with warm, it also supplies the starting basis (a previous result).
// out (cols x rows) = in^T, in row-major FP32 (rows x cols)
hipError_t transpose_f32(const float* in, int64_t rows, int64_t cols, float* out, hipStream_t s);
hipError_t jacobi_eig(const double* S, int n, int r, double* U64, float* U32, double* lam,
                      hipStream_t s, double* Vio = nullptr, bool warm = false);

}  // namespace tk
