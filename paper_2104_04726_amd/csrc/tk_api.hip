// Host driver and C ABI of the Tucker-ALS (HOOI) library.
//
// Algorithm (Sharma & Grover, arXiv 2104.04726, Sec. III-B):
//   * T-HOSVD start (Sec. III-B.1, eq. (3)-(7)): U_n = leading R_n eigenvectors of X_(n) X_(n)^T.
//   * ALS sweeps (eq. (8)): for n = 1..N in order, Y = X x_{m != n} U_m^T with the newest factors,
//     U_n <- leading R_n eigenvectors of Y_(n) Y_(n)^T (the Gram route the paper takes to avoid
//     a large SVD); the core G = Y x_N U_N^T closes the sweep.
// Realisation on one GPU:
//   * modes with R_n = s_n keep their (orthonormal) factor: any basis of R^{s_n} is optimal;
//   * modes with s_n <= 64: the Gram is diagonalised exactly by Jacobi in FP64;
//   * larger modes: orthogonal iteration warm-started from the previous U_n: Z = S U (FP32 MFMA),
//     U <- CholeskyQR2(Z) in FP64 (cold start from a counter-based random basis for the T-HOSVD);
//   * order-4 tensors whose two trailing modes are small (the image stacks: H, W, channel, image)
//     use a dimension tree: T34 = X x_3 U_3^T x_4 U_4^T serves modes 1 and 2, T12 = X x_1 U_1^T x_2 U_2^T
//     serves modes 3, 4 and the core; other shapes contract each chain directly;
//   * fit: ||X||^2 - ||G||^2 per sweep (FP64 sums), and at the end 1 - ||X - Xhat|| / ||X|| from the
//     explicit residual, fused into the last expanding product.
#include <algorithm>
#include <atomic>
#include <functional>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tk_common.h"
#include "tk_lowp.h"
#include "../../include/tucker.h"

using namespace tk;

hipError_t tk_sum_splits_f64(const double* P, int nsplit, int64_t n, int64_t zstride, double* out, hipStream_t s);
hipError_t tk_sum_splits_to_f32(const double* P, int nsplit, int64_t n, int64_t zstride, float* out, hipStream_t s);
template <typename TO>
hipError_t tk_sum_splits_f32p(const float* P, int nsplit, int64_t n, int64_t zstride, TO* out, hipStream_t s);
hipError_t tk_set_int(int* p, int v, hipStream_t s);
hipError_t tk_fit_push(const double* src, int* counter, double* fits, hipStream_t s);
hipError_t tk_resid_sumsq(const float* X, const float* Xh, int64_t n, double* partial, int nblocks, double* out,
                          hipStream_t s);
hipError_t tk_diff_sumsq_f64(const double* A, const double* B, int64_t n, double* partial, int nblocks, double* out,
                             hipStream_t s);

// ---- the allocation-free CholeskyQR half (tucker_chol_inv_noalloc): its scratch is one file-scope
// device array per GPU.  In host code `scratch` names a host-side stand-in, never the device memory:
// its device address is looked up once per device at context creation and kept in g_scratch.
constexpr int64_t kNoAllocMaxN = 512;
constexpr size_t kNoAllocAlign = 256;
constexpr size_t align_up(size_t v) { return (v + kNoAllocAlign - 1) / kNoAllocAlign * kNoAllocAlign; }
constexpr size_t kNoAllocW = 0;                                                     // n x n doubles
constexpr size_t kNoAllocCtr = align_up(kNoAllocW + sizeof(double) * kNoAllocMaxN * kNoAllocMaxN);
constexpr size_t kNoAllocCtrInts = 2 + 2 * ((kNoAllocMaxN + kCholTile - 1) / kCholTile) * ((kNoAllocMaxN + kCholTile - 1) / kCholTile);
constexpr size_t kNoAllocDsc = align_up(kNoAllocCtr + sizeof(int) * kNoAllocCtrInts);     // n doubles
constexpr size_t kNoAllocShifts = align_up(kNoAllocDsc + sizeof(double) * kNoAllocMaxN);  // 8 ints
constexpr size_t kNoAllocBytes = align_up(kNoAllocShifts + 8 * sizeof(int));

static __device__ __align__(256) char scratch[kNoAllocBytes];

struct tucker_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tucker_options opt{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    tucker_stats stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> pool;   // stage timer events (created on first use)
    bool async_alloc = false;       // workspace from the stream-ordered allocator (server slots)
    hipStream_t aux = nullptr;      // second stream: the cold start of mode 1 beside that of mode 2
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    double* eig_host = nullptr;     // pinned convergence sums of two interleaved eigensolver runs
    hipEvent_t eig_ev[2] = {nullptr, nullptr};
};

namespace {

constexpr int64_t kSmallMode = 64;       // modes up to this size are diagonalised exactly

struct Fail {
    tucker_status st;
    std::string msg;
};

#define TK_HIP(expr)                                                                      \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            throw Fail{TUCKER_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

int64_t prod(const int64_t* d, int a, int b) {
    int64_t p = 1;
    for (int i = a; i < b; ++i) p *= d[i];
    return p;
}

// ------------------------------------------------------------------ bump arena over one block
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    size_t cap = 0;     // 0 while sizing
    template <typename T>
    T* take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        if (base && off > cap) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "workspace plan overflow"};
        return p;
    }
};

enum ModeKind { FIXED = 0, SMALL = 1, LARGE = 2 };

// ------------------------------------------------------------------ plan and buffers
struct Plan {
    int N = 0;
    int64_t s[TUCKER_MAX_ORDER]{}, R[TUCKER_MAX_ORDER]{};
    int64_t Rc[TUCKER_MAX_ORDER]{};     // columns of the cold start (R_n + oversampling, at most s_n)
    ModeKind kind[TUCKER_MAX_ORDER]{};
    bool tree = false;
    int max_iters = 0;
    int refine = 0;          // FP32 sweeps after reduced-precision ones
    // reduced-precision sweeps (tree shapes): storage type of X (prec) and of the intermediates (ip)
    int prec = 0, ip = 0;
    int64_t R23p = 0;        // R3 R4 rounded up to 8: padded fibre length of T34 / Y0 / Y1
    int64_t Lp = 0;          // s3 s4 rounded up to 8: padded fibre length of T1 (zero padding)
    bool lp_start = false;   // reduced-precision runs: the start's Grams of X from a padded copy in T34
    void *Xlp = nullptr, *T34lp = nullptr, *Y0lp = nullptr, *Y1lp = nullptr, *T1lp = nullptr;
    void *U1t = nullptr, *U2t = nullptr, *U1t8 = nullptr;   // transposed factor copies (rows padded to 8)
    float *xscale = nullptr, *u1scale = nullptr, *spart = nullptr;
    float* Pf = nullptr;     // FP32 Gram partials
    int64_t Pf_elems = 0;
    float* S32 = nullptr;    // FP32 copy of the sweep Grams (reduced-precision sweeps)

    float* U32[TUCKER_MAX_ORDER]{};
    bool ident[TUCKER_MAX_ORDER]{};     // U_n is exactly the identity (a full-rank mode started from it)
    double* Vsm[TUCKER_MAX_ORDER]{};    // small modes: the whole eigenvector basis of the last update
    bool vsm_valid[TUCKER_MAX_ORDER]{};
    double* U64[TUCKER_MAX_ORDER]{};
    // tree buffers
    float *T34 = nullptr, *Y0 = nullptr, *Y1 = nullptr, *T1 = nullptr, *T12 = nullptr;
    // generic chain buffers
    float *Ya = nullptr, *Yb = nullptr;
    float* G = nullptr;
    // Gram / OI
    double* S64 = nullptr;
    double* P = nullptr;
    int64_t P_elems = 0;
    double* Z = nullptr;
    double* Q1 = nullptr;
    double* W = nullptr;
    double* Wpart = nullptr;
    int64_t Wpart_elems = 0;
    double* Tm = nullptr;
    void* chol_ws = nullptr;     // task-graph counters of the Cholesky (zero between calls)
    double* chol_dsc = nullptr;
    int64_t chol_cap = 0;        // largest order the counters are sized for
    // second orthogonal-iteration scratch set (Gram, products, CholeskyQR, counters), so that the
    // cold starts of the two large modes of a tree shape can run on two streams; swap_oi exchanges
    // it with the first
    bool has_alt = false;
    double *S64b = nullptr, *Wpartb = nullptr, *Zb = nullptr, *Q1b = nullptr, *Wb = nullptr, *Tmb = nullptr;
    double *chol_dscb = nullptr, *redb = nullptr;
    void* chol_wsb = nullptr;
    int* shiftsb = nullptr;
    int64_t Wpartb_elems = 0, chol_capb = 0;
    // capacities (elements) of S64 and Z in the active set and the other one, checked before a
    // Gram or an orthogonal iteration writes them (0: not tracked)
    int64_t S64_elems = 0, S64b_elems = 0, Z_elems = 0, Zb_elems = 0;
    double* F = nullptr;
    double* Fpart = nullptr;
    // norms and fits
    double* red = nullptr;       // kSumsqBlocks partials
    double* rpart = nullptr;     // residual partials (one per GEMM block)
    int64_t rpart_elems = 0;
    double* scal = nullptr;      // [0] nx2 [1] ng2 [2] r2 [3] fit_exact
    double* fits = nullptr;      // max_iters + 1
    int* shifts = nullptr;
    float* Xh = nullptr;         // explicit reconstruction when the residual cannot be fused
    // pairwise perturbation (tree shapes): operators at the reference factors, the reference
    // factors, their changes, and the scratch of the factor alignment
    bool pp = false;
    float *Y0p = nullptr, *Y1p = nullptr, *T12p = nullptr, *Zp = nullptr, *PPtmp = nullptr;
    float* U32p[TUCKER_MAX_ORDER]{};
    double* U64p[TUCKER_MAX_ORDER]{};
    double* U64prev[TUCKER_MAX_ORDER]{};
    float* dU[TUCKER_MAX_ORDER]{};
    double *NS_X = nullptr, *NS_B = nullptr, *NS_D = nullptr, *NS_T = nullptr, *NS_U = nullptr;
    double* ppdist = nullptr;    // squared Frobenius norms of U^T V, one per mode
};

int64_t max_large_s(const Plan& p) {
    int64_t m = 0;
    for (int n = 0; n < p.N; ++n)
        if (p.kind[n] == LARGE) m = std::max(m, p.s[n]);
    return m;
}
int64_t max_large_sR(const Plan& p) {
    int64_t m = 0;
    for (int n = 0; n < p.N; ++n)
        if (p.kind[n] == LARGE) m = std::max(m, p.s[n] * p.Rc[n]);
    return m;
}
int64_t max_large_R(const Plan& p) {
    int64_t m = 0;
    for (int n = 0; n < p.N; ++n)
        if (p.kind[n] == LARGE) m = std::max(m, p.Rc[n]);
    return m;
}

// largest intermediate of the direct chains (generic path), including reconstruction chains
int64_t chain_max(const Plan& p) {
    int64_t mx = 0;
    for (int n = 0; n < p.N; ++n) {
        int64_t d[TUCKER_MAX_ORDER];
        for (int i = 0; i < p.N; ++i) d[i] = p.s[i];
        for (int m = 0; m < p.N; ++m) {
            if (m == n) continue;
            d[m] = p.R[m];
            mx = std::max(mx, prod(d, 0, p.N));
        }
    }
    // core chain and reconstruction chain (from the core up)
    int64_t d[TUCKER_MAX_ORDER];
    for (int i = 0; i < p.N; ++i) d[i] = p.R[i];
    for (int m = p.N - 1; m >= 0; --m) {
        d[m] = p.s[m];
        mx = std::max(mx, prod(d, 0, p.N));
    }
    return mx;
}

constexpr int64_t kGramFallbackCapacity = 768;
constexpr double kGramSplitOverheadK = 256.0;   // fixed cost of a workgroup, in k steps
constexpr int kLpScaleBlocks = 256;
constexpr int kRefineInner = 4;
constexpr int64_t kRitzMaxOrder = 1024;   // largest Rayleigh-Ritz matrix (block-Jacobi eigensolver)
constexpr int64_t kZSplitK = 128;         // longest FP32-accumulated k range of the one-step S U product
constexpr int kLpGramTargetBlocks = 512;

// split-K of a reduced-precision Gram (128 x 128 tiles, lower triangle; k_split a multiple of 64)
int64_t lp_gram_ksplit(int64_t s, int64_t K) {
    const int64_t t = (s + 127) / 128;
    const int64_t tiles = t * (t + 1) / 2;
    int64_t sp = std::max<int64_t>(1, (kLpGramTargetBlocks + tiles - 1) / tiles);
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / 512));
    int64_t ks = (K + sp - 1) / sp;
    return (ks + 63) / 64 * 64;
}
int64_t lp_gram_partials(int64_t s, int64_t K) {
    const int64_t ks = lp_gram_ksplit(s, K);
    return ((K + ks - 1) / ks) * s * s;
}

// Workgroups of the FP64 Gram kernel that are resident on the device at once (CUs x occupancy),
// queried once per process on the current device; 768 (256 CUs x 3) when no device answers.
int64_t gram_capacity() {
    static std::atomic<int64_t> cached{0};
    int64_t c = cached.load(std::memory_order_relaxed);
    if (c > 0) return c;
    int dev = 0, cus = 0;
    const int per = gram_f64_blocks_per_cu();
    if (per > 0 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        c = (int64_t)cus * per;
    else
        c = kGramFallbackCapacity;
    cached.store(c, std::memory_order_relaxed);
    return c;
}

// Split-K of the FP64 Gram (64 x 64 lower-triangle tiles): the count minimising
// rounds x (K / splits + overhead), where a round is one set of resident workgroups, so that the
// last round is not left mostly empty; ties go to fewer splits (less partial-sum traffic).
int gram_splits(int64_t s, int64_t K) {
    const int64_t t = (s + 63) / 64;
    const int64_t tiles = t * (t + 1) / 2;
    const int64_t cap = gram_capacity();
    const int64_t maxsp = std::min<int64_t>(64, std::max<int64_t>(1, K / 256));
    int64_t best = 1;
    double best_cost = 0.0;
    for (int64_t sp = 1; sp <= maxsp; ++sp) {
        const int64_t rounds = (tiles * sp + cap - 1) / cap;
        const double cost = (double)rounds * ((double)K / (double)sp + kGramSplitOverheadK);
        if (sp == 1 || cost < best_cost * 0.999) {
            best = sp;
            best_cost = cost;
        }
    }
    return (int)best;
}

void build_plan(Plan& p, Arena& a) {
    const int N = p.N;
    for (int n = 0; n < N; ++n) {
        p.U32[n] = a.take<float>(p.s[n] * p.R[n]);
        if (p.kind[n] == SMALL) p.Vsm[n] = a.take<double>(p.s[n] * p.s[n]);
        p.U64[n] = a.take<double>(p.s[n] * p.Rc[n]);
    }
    const int64_t Xn = prod(p.s, 0, N);
    if (p.tree) {
        const int64_t s0 = p.s[0], s1 = p.s[1], L = p.s[2] * p.s[3], R23 = p.R[2] * p.R[3];
        p.T34 = a.take<float>(s0 * s1 * R23);
        p.Y0 = a.take<float>(s0 * p.R[1] * R23);
        p.Y1 = a.take<float>(p.R[0] * s1 * R23);
        p.T1 = a.take<float>(p.R[0] * s1 * L);
        p.T12 = a.take<float>(p.R[0] * p.R[1] * L);
        p.F = a.take<double>(64 * 64);
        p.Fpart = a.take<double>(std::max<int64_t>((int64_t)kFibreGramBlocks * L * L, 64 * 64 * 64));
        if (p.prec != 0) {
            const int es = (p.prec == TUCKER_FP8_E4M3) ? 1 : 2;
            const int64_t R0 = p.R[0], R1 = p.R[1];
            const int64_t s0p = (s0 + 7) / 8 * 8, s1p = (s1 + 7) / 8 * 8;
            p.R23p = (R23 + 7) / 8 * 8;
            p.Xlp = a.take<char>(Xn * es);
            p.xscale = a.take<float>(L);
            p.spart = a.take<float>(kLpScaleBlocks * L);
            p.T34lp = a.take<uint16_t>(s0 * s1 * p.R23p);
            p.Y0lp = a.take<uint16_t>(s0 * R1 * p.R23p);
            p.Y1lp = a.take<uint16_t>(R0 * s1 * p.R23p);
            p.Lp = (L + 7) / 8 * 8;
            p.T1lp = a.take<uint16_t>(R0 * s1 * p.Lp);
            p.U1t = a.take<uint16_t>(R0 * s0p);
            p.U2t = a.take<uint16_t>(R1 * s1p);
            p.U1t8 = a.take<uint8_t>(R0 * s0p);
            p.u1scale = a.take<float>(R0);
            p.Pf_elems = std::max(lp_gram_partials(s0, R1 * p.R23p), lp_gram_partials(s1, R0 * p.R23p));
            // the start's Grams of X in the sweeps' reduced precision: a copy of X with zero-padded
            // fibres (16-bit, Lp long) fits where the FP32 T34 goes, which the start does not use
            p.lp_start = p.kind[0] == LARGE && p.kind[1] == LARGE && 2 * p.Lp <= 4 * R23;
            if (p.lp_start)
                p.Pf_elems = std::max(p.Pf_elems, std::max(lp_gram_partials(s0, s1 * p.Lp), lp_gram_partials(s1, s0 * p.Lp)));
            p.Pf = a.take<float>(p.Pf_elems);
            p.S32 = a.take<float>(std::max(s0 * s0, s1 * s1));
        }
    } else {
        const int64_t cm = chain_max(p);
        p.Ya = a.take<float>(cm);
        p.Yb = a.take<float>(cm);
    }
    p.G = a.take<float>(prod(p.R, 0, N));
    // Grams: largest split-K partial buffer over the large modes, init (X) and sweep shapes
    int64_t maxs = 0, pmax = 0, maxsmall = 1;
    for (int n = 0; n < N; ++n) {
        if (p.kind[n] == LARGE) {
            const int64_t sn = p.s[n];
            maxs = std::max(maxs, sn);
            const int64_t Kx = Xn / sn;
            int64_t Ky = prod(p.R, 0, N) / p.R[n];   // sweep Gram inner size
            const int64_t K = std::max(Kx, Ky);
            pmax = std::max(pmax, (int64_t)gram_splits(sn, K) * sn * sn);
        } else {
            maxsmall = std::max(maxsmall, p.s[n]);
        }
    }
    if (p.tree) pmax = std::max(pmax, prod(p.R, 0, N));   // W of the direct warm update (R_n x A x B)
    p.S64_elems = std::max<int64_t>(std::max(maxs, maxsmall) * std::max(maxs, maxsmall), 64 * 64);
    p.S64 = a.take<double>(p.S64_elems);
    p.P = a.take<double>(pmax);
    p.P_elems = pmax;
    const int64_t sR = max_large_sR(p), Rm = max_large_R(p);
    p.Z = a.take<double>(sR);
    p.Z_elems = sR;
    p.Q1 = a.take<double>(sR);
    p.W = a.take<double>(Rm * Rm);
    p.Wpart_elems = std::max<int64_t>(16 * Rm * Rm, 8 * sR);
    if (Rm > 0 && Rm <= 1024) p.Wpart_elems = std::max(p.Wpart_elems, sym_eig_work_doubles((int)Rm));
    p.Wpart = a.take<double>(p.Wpart_elems);
    p.Tm = a.take<double>(Rm * Rm);
    p.chol_ws = a.take<int>(chol_counter_ints(Rm));
    p.chol_dsc = a.take<double>(Rm);
    p.chol_cap = Rm;
    if (!p.tree) {
        p.F = a.take<double>(64 * 64);
        p.Fpart = a.take<double>(64 * 64 * 64);
    }
    p.red = a.take<double>(kSumsqBlocks);
    p.rpart_elems = std::max<int64_t>(4096, (Xn / (128 * 128)) + 4096);
    p.rpart = a.take<double>(p.rpart_elems);
    p.scal = a.take<double>(8);
    p.fits = a.take<double>(p.max_iters + p.refine + 2);
    p.shifts = a.take<int>(8);
    if (!p.tree) p.Xh = (p.kind[0] == LARGE && p.s[0] > kSmallMode) ? nullptr : a.take<float>(Xn);
    if (p.pp) {
        const int64_t s0 = p.s[0], s1 = p.s[1], L = p.s[2] * p.s[3], R23 = p.R[2] * p.R[3];
        p.Y0p = a.take<float>(s0 * p.R[1] * R23);
        p.Y1p = a.take<float>(p.R[0] * s1 * R23);
        p.T12p = a.take<float>(p.R[0] * p.R[1] * L);
        p.Zp = a.take<float>(s0 * p.R[1] * L);
        p.PPtmp = a.take<float>(std::max(s0 * p.R[1] * R23, p.R[0] * s1 * R23));
        int64_t rr = 1, sr = 1;
        for (int n = 0; n < N; ++n) {
            p.U32p[n] = a.take<float>(p.s[n] * p.R[n]);
            p.U64p[n] = a.take<double>(p.s[n] * p.R[n]);
            p.U64prev[n] = a.take<double>(p.s[n] * p.R[n]);
            p.dU[n] = a.take<float>(p.s[n] * p.R[n]);
            rr = std::max(rr, p.R[n] * p.R[n]);
            sr = std::max(sr, p.s[n] * p.R[n]);
        }
        p.NS_X = a.take<double>(rr);
        p.NS_B = a.take<double>(rr);
        p.NS_D = a.take<double>(rr);
        p.NS_T = a.take<double>(rr);
        p.NS_U = a.take<double>(sr);
        p.ppdist = a.take<double>(2 * TUCKER_MAX_ORDER + kSumsqBlocks);
    }
    p.has_alt = p.tree && p.kind[0] == LARGE && p.kind[1] == LARGE;
    if (p.has_alt) {
        const int64_t s0 = p.s[0], R0 = p.Rc[0];
        p.S64b = a.take<double>(s0 * s0);
        p.S64b_elems = s0 * s0;
        p.Zb = a.take<double>(s0 * R0);
        p.Zb_elems = s0 * R0;
        p.Q1b = a.take<double>(s0 * R0);
        p.Wb = a.take<double>(R0 * R0);
        p.Wpartb_elems = std::max<int64_t>(16 * R0 * R0, 8 * s0 * R0);
        if (R0 > 0 && R0 <= 1024) p.Wpartb_elems = std::max(p.Wpartb_elems, sym_eig_work_doubles((int)R0));
        p.Wpartb = a.take<double>(p.Wpartb_elems);
        p.Tmb = a.take<double>(R0 * R0);
        p.chol_wsb = a.take<int>(chol_counter_ints(R0));
        p.chol_dscb = a.take<double>(R0);
        p.chol_capb = R0;
        p.redb = a.take<double>(kSumsqBlocks);
        p.shiftsb = a.take<int>(8);
    }
}

void swap_oi(Plan& p) {
    std::swap(p.S64, p.S64b);
    std::swap(p.S64_elems, p.S64b_elems);
    std::swap(p.Z_elems, p.Zb_elems);
    std::swap(p.Wpart, p.Wpartb);
    std::swap(p.Wpart_elems, p.Wpartb_elems);
    std::swap(p.Z, p.Zb);
    std::swap(p.Q1, p.Q1b);
    std::swap(p.W, p.Wb);
    std::swap(p.Tm, p.Tmb);
    std::swap(p.chol_ws, p.chol_wsb);
    std::swap(p.chol_dsc, p.chol_dscb);
    std::swap(p.chol_cap, p.chol_capb);
    std::swap(p.red, p.redb);
    std::swap(p.shifts, p.shiftsb);
}

// ------------------------------------------------------------------ driver state
struct Run {
    tucker_ctx* ctx;
    Plan p;
    hipStream_t st;
    const float* X = nullptr;
    struct Mark {
        int stage, b, e;
    };
    std::vector<Mark> marks;
    size_t next_ev = 0;
    int inner_override = 0;     // orthogonal-iteration steps per update in refinement sweeps
    double orth_tol = 1e-12;    // CholeskyQR second-pass threshold on max |Q^T Q - I|
    int oi_steps_init = 0, oi_steps_sweeps = 0;   // orthogonal-iteration steps taken (host count)
    double oi_resid_max = 0.0;  // inner_tol > 0: largest final relative residual of an update
    int rr_sweeps = 0;          // block-Jacobi sweeps of the Rayleigh-Ritz steps (oversampled starts)
    bool defer_ritz = false;    // an oversampled cold start leaves its Rayleigh-Ritz step to the caller
    bool lp_su = false;         // reduced-precision sweep: warm S U from the FP32 copy of S
    double* fit0_slot = nullptr;  // set: the start's fit is still to be written here, by the first
                                  // sweep's mode-1 update (its W = Y0 x_1 U1^T is the start's core)

    long long spin() const { return (long long)ctx->opt.wait_spin_limit; }
    double inner_tol() const { return ctx->opt.inner_tol; }

    int record() {
        if (next_ev >= ctx->pool.size()) {
            hipEvent_t e;
            TK_HIP(hipEventCreate(&e));
            ctx->pool.push_back(e);
        }
        TK_HIP(hipEventRecord(ctx->pool[next_ev], st));
        return (int)next_ev++;
    }
};

// HIP-event timer of one sweep stage, active when tucker_options.timing is set
struct StageTimer {
    Run& r;
    int stage;
    int b = -1;
    StageTimer(Run& run, int s) : r(run), stage(s) {
        const uint32_t mask = r.ctx->opt.timing_stages;
        if (r.ctx->opt.timing && stage >= 0 && (mask == 0 || ((mask >> stage) & 1u))) b = r.record();
    }
    ~StageTimer() {
        if (b >= 0) {
            try {
                const int e = r.record();
                r.marks.push_back({stage, b, e});
            } catch (...) {
            }
        }
    }
};

// out = in x_n U^T (contract, U: dims[n] x R)  or  in x_n U (expand, U: s x dims[n], result dim s)
// dims: current dims of `in` (order N); the new size of mode n is newdim.
// When resid_ref is set (only for an expanding GEMM), the product is not stored: the squared
// difference against resid_ref (same layout as the product) is summed into rpart.  Ut (optional, an
// expanding product over an inner mode): U^T (dims[n] x newdim), read as the k-major operand, so that
// both operands take 16-byte vector loads.
void ttm(Run& r, const float* in, const int64_t* dims, int N, int n, const float* U, int64_t newdim,
         bool expand, float* out, const float* resid_ref = nullptr, int64_t* nblocks = nullptr,
         const float* Ut = nullptr) {
    const int64_t A = prod(dims, 0, n), K = dims[n], B = prod(dims, n + 1, N);
    const int64_t R = newdim;
    if (!resid_ref && K <= kSmallMode && R <= kSmallMode) {
        TK_HIP(small_ttm(in, A, K, B, U, R, expand, out, r.st));
        return;
    }
    GemmArgs g{};
    g.alpha = 1.0;
    g.k_split = 0;
    g.c_zstride = 0;
    g.lower_only = 0;
    Orient oa, ob;
    if (B == 1) {
        // C(m = a, n = r) = sum_k in[a][k] * Uop(k, r)
        g.M = A;
        g.N = R;
        g.K = K;
        g.a = plain(in, K);
        oa = MK;
        if (!expand) {
            g.b = plain(U, R);   // U[k][r]
            ob = KM;
        } else {
            g.b = plain(U, K);   // U[r][k]: (k, n=r) at r*K + k
            ob = MK;
        }
        g.c = plain(resid_ref ? (const void*)resid_ref : (const void*)out, R);
    } else {
        g.M = R;
        g.N = A * B;
        g.K = K;
        if (!expand) {
            g.a = plain(U, R);   // A(m=r, k) = U[k][r]
            oa = KM;
        } else if (Ut) {
            g.a = plain(Ut, R);  // A(m=i, k=r) = Ut[r][i]
            oa = KM;
        } else {
            g.a = plain(U, K);   // A(m=i, k=r) = U[i][r]
            oa = MK;
        }
        g.b = folded(in, B, B, K * B);
        ob = KM;
        g.c = folded(resid_ref ? (const void*)resid_ref : (const void*)out, B, B, R * B);
    }
    if (resid_ref) {
        const int64_t nb = gemm_grid_blocks(g, false);
        if (nb > r.p.rpart_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "residual partial buffer too small"};
        g.resid_partial = r.p.rpart;
        TK_HIP(gemm_f32(g, oa, ob, EPI_RESID, false, r.st));
        if (nblocks) *nblocks = nb;
    } else {
        TK_HIP(gemm_f32(g, oa, ob, EPI_STORE, false, r.st));
    }
}

// Mode-n Gram of `in` (dims, order N) into S64 (FP64, s x s, symmetric).  Large modes use the
// FP64 MFMA kernel on the FP32 data (every product exact, FP64 accumulation; a FP32-accumulated
// Gram loses the directions next to the rank boundary of strongly decaying spectra), split over K
// with FP64 partials summed in a fixed order; small modes use the vector kernel.
void gram(Run& r, const float* in, const int64_t* dims, int N, int n, int stage = -1) {
    Plan& p = r.p;
    const int64_t A = prod(dims, 0, n), s = dims[n], B = prod(dims, n + 1, N);
    if (p.S64_elems > 0 && s * s > p.S64_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "Gram output buffer too small"};
    if (s <= kSmallMode) {
        StageTimer t(r, stage);
        TK_HIP(small_gram(in, A, s, B, p.Fpart, kFibreGramBlocks / 8, p.S64, r.st));
        return;
    }
    GemmArgs g{};
    g.alpha = 1.0;
    g.lower_only = 1;
    g.M = s;
    g.N = s;
    Orient oa, ob;
    if (B == 1) {
        g.K = A;
        g.a = plain(in, s);   // (m=i, k=a) at a*s + i
        g.b = plain(in, s);
        oa = KM;
        ob = KM;
    } else {
        g.K = A * B;
        g.a = folded(in, B, B, s * B);   // (m=i, k=(a,b)) at i*B + a*s*B + b
        g.b = g.a;
        oa = MK;
        ob = MK;
    }
    // split count: the occupancy heuristic, or the autotuner's pick among it, half and double of it
    // (each one fixed reduction order) within the capacity of the partial buffer
    const int h = gram_splits(s, g.K);
    std::vector<int> cand{h};
    for (int c : {std::max(1, h / 2), 2 * h, std::max(1, h / 4)}) {
        int64_t ks = ((g.K + c - 1) / c + 15) / 16 * 16;
        const int64_t ns = (g.K + ks - 1) / ks;
        if (ns * s * s <= p.P_elems && std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
    auto plan_split = [&](int splits, int64_t& ks) {
        ks = ((g.K + splits - 1) / splits + 15) / 16 * 16;
        return (int)((g.K + ks - 1) / ks);
    };
    g.c = plain(p.P, s);
    g.c_zstride = s * s;
    auto launch = [&](int c) {
        GemmArgs gc = g;
        int64_t ks = 0;
        const int nsplit = plan_split(cand[c], ks);
        gc.k_split = ks;
        hipError_t e = gemm_f64(gc, oa, ob, EPI_STORE, true, true, r.st);
        return e != hipSuccess ? e : gram_reduce64(p.P, nsplit, s, s * s, p.S64, r.st);
    };
    const int64_t shape[5] = {s, g.K, A, B, p.P_elems / (s * s)};
    hipError_t te = hipSuccess;
    const int choice = tune_choose(kTuneGramSplit, shape, (int)cand.size(), 0, r.st, launch, &te);
    TK_HIP(te);
    int64_t ks = 0;
    const int nsplit = plan_split(cand[std::min<int>(choice, (int)cand.size() - 1)], ks);
    if ((int64_t)nsplit * s * s > p.P_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "Gram partial buffer too small"};
    g.k_split = ks;
    {
        StageTimer t(r, stage);
        TK_HIP(gemm_f64(g, oa, ob, EPI_STORE, true, true, r.st));
    }
    StageTimer t(r, stage >= 0 ? TUCKER_STAGE_REDUCE : -1);
    TK_HIP(gram_reduce64(p.P, nsplit, s, s * s, p.S64, r.st));
}

// W = A^T A (FP64) for A (rows x cols), A float or double, split over rows
// W = A^T A (cols x cols, FP64); lower: only the tiles on and below the diagonal are formed (the
// Cholesky and the orthogonality check read only the lower triangle)
void gram_tn64(Run& r, const void* A, bool a32, int64_t rows, int64_t cols, double* W, bool lower = false) {
    Plan& p = r.p;
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = cols;
    g.N = cols;
    g.lower_only = lower ? 1 : 0;
    g.K = rows;
    g.a = plain(A, cols);
    g.b = plain(A, cols);
    const int64_t t = (cols + 63) / 64;
    const int64_t tiles = lower ? t * (t + 1) / 2 : t * t;
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>(16, (512 + tiles - 1) / tiles));
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, rows / 64));
    int64_t ks = (rows + splits - 1) / splits;
    ks = (ks + 15) / 16 * 16;
    const int nsplit = (int)((rows + ks - 1) / ks);
    g.k_split = ks;
    if ((int64_t)nsplit * cols * cols > p.Wpart_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "W partial buffer"};
    if (nsplit == 1) {
        g.c = plain(W, cols);
        TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, a32, a32, r.st));
        return;
    }
    g.c = plain(p.Wpart, cols);
    g.c_zstride = cols * cols;
    TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, a32, a32, r.st));
    TK_HIP(tk_sum_splits_f64(p.Wpart, nsplit, cols * cols, cols * cols, W, r.st));
}

// Q = A T^T (A rows x cols float/double, T cols x cols lower-triangular fp64) -> Q fp64
// Every call that factors starts with zeroed counters: p.shifts (pivot shifts, second-pass count,
// the second-pass flag, the fit counter, the orthogonality-check ticket) and the Cholesky task-graph
// counters, which each factorisation leaves zeroed for the next.
void reset_counters(Run& r) {
    TK_HIP(fill_zero(r.p.shifts, 8 * (int64_t)sizeof(int), r.st));
    if (r.p.chol_ws) TK_HIP(fill_zero(r.p.chol_ws, chol_counter_ints(r.p.chol_cap) * (int64_t)sizeof(int), r.st));
    if (r.p.has_alt) {
        TK_HIP(fill_zero(r.p.shiftsb, 8 * (int64_t)sizeof(int), r.st));
        TK_HIP(fill_zero(r.p.chol_wsb, chol_counter_ints(r.p.chol_capb) * (int64_t)sizeof(int), r.st));
    }
}

// work enqueued after fork_aux on ctx->aux (under OnAux) runs after everything queued on the main
// stream so far; join_aux makes the main stream wait for it
void fork_aux(Run& r) {
    TK_HIP(hipEventRecord(r.ctx->fork_ev, r.st));
    TK_HIP(hipStreamWaitEvent(r.ctx->aux, r.ctx->fork_ev, 0));
}
void join_aux(Run& r) {
    TK_HIP(hipEventRecord(r.ctx->join_ev, r.ctx->aux));
    TK_HIP(hipStreamWaitEvent(r.st, r.ctx->join_ev, 0));
}
struct OnAux {
    Run& r;
    hipStream_t main;
    explicit OnAux(Run& run) : r(run), main(run.st) { r.st = r.ctx->aux; }
    ~OnAux() { r.st = main; }
};

void apply_tri(Run& r, const void* A, bool a32, int64_t rows, int64_t cols, const double* Tm, double* Q,
               const int* run_if = nullptr) {
    GemmArgs g{};
    g.run_if = run_if;
    g.alpha = 1.0;
    g.M = rows;
    g.N = cols;
    g.K = cols;
    g.a = plain(A, cols);      // (m=row, k) at row*cols + k
    g.b = plain(Tm, cols);     // (k, n) = T[n][k] -> NK; T lower triangular: zero for k > n
    g.c = plain(Q, cols);
    g.k_split = 0;
    g.k_upto_n = 1;
    TK_HIP(gemm_f64(g, MK, MK, EPI_STORE, a32, false, r.st));
}

// U64/U32 <- orthonormal basis of span(Z) by CholeskyQR in FP64 with column scaling.
// cold: shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020): the first pass
// factors the scaled Gram plus s I, s = 11 (m n + n (n+1)) u ||W~||_2 with ||W~||_2 <= n (unit
// diagonal), which cannot break down for a numerically full-rank Z and leaves Q1 well conditioned;
// two plain passes follow.  warm (Z = S U with U near the invariant subspace): CholeskyQR2, whose
// second pass runs only when the first left max_ij |(Q1^T Q1 - I)_ij| above kOrthTol: the test and
// the skip happen on the device (the second pass's kernels return at once), so nothing waits on
// the host.  Column scaling makes the first pass nearly exact when the columns of Z are close to
// orthogonal, which is the case once the leading columns have settled.  mid (an intermediate step
// of a multi-step iteration): one plain pass into U64 only, which carries span(Z) into the next
// product.  Each pass maps the basis by an invertible triangular factor, so the column space is that
// of Z.  U32 (nullable) receives the FP32 copy of the final basis.
constexpr double kOrthTol = 1e-12;     // FP32 sweeps: the factors are orthonormal to FP64 rounding
constexpr double kOrthTolLowp = 1e-6;  // reduced-precision sweeps: far below the 2^-8..2^-4 rounding of
                                       // the factor copies their products use

void orthonormalize(Run& r, const void* Z, bool z32, int64_t rows, int64_t cols, double* U64, float* U32,
                    bool cold, bool mid = false) {
    Plan& p = r.p;
    if (mid) {
        // an intermediate step of the cold start: one CholeskyQR pass gives a basis of span(Z),
        // all that the next product S U needs; the last step delivers the orthonormal factor
        gram_tn64(r, Z, z32, rows, cols, p.W, true);
        TK_HIP(chol_inv_scaled(p.W, cols, true, 0.0, p.Tm, (int*)p.chol_ws, p.chol_dsc, p.shifts, r.st,
                               nullptr, r.spin()));
        apply_tri(r, Z, z32, rows, cols, p.Tm, U64);
        return;
    }
    const double u = std::ldexp(1.0, -53);
    const double shift = cold ? 11.0 * ((double)rows * cols + (double)cols * (cols + 1)) * u * (double)cols : 0.0;
    // pass 1: Z -> Q1
    gram_tn64(r, Z, z32, rows, cols, p.W, true);
    TK_HIP(chol_inv_scaled(p.W, cols, true, shift, p.Tm, (int*)p.chol_ws, p.chol_dsc, p.shifts, r.st,
                               nullptr, r.spin()));
    apply_tri(r, Z, z32, rows, cols, p.Tm, p.Q1);
    gram_tn64(r, p.Q1, false, rows, cols, p.W, true);
    if (!cold) {
        // pass 2 only where needed: need = p.shifts[2], counted in p.shifts[1]
        int* need = p.shifts + 2;
        TK_HIP(orth_check(p.W, cols, r.orth_tol, p.red, need, p.shifts + 1, p.shifts + 4, r.st));
        TK_HIP(chol_inv_scaled(p.W, cols, true, 0.0, p.Tm, (int*)p.chol_ws, p.chol_dsc, p.shifts, r.st,
                               need, r.spin()));
        apply_tri(r, p.Q1, false, rows, cols, p.Tm, U64, need);
        TK_HIP(finish_factor(need, p.Q1, U64, U32, rows * cols, r.st));
        return;
    } else {
        TK_HIP(chol_inv_scaled(p.W, cols, true, 0.0, p.Tm, (int*)p.chol_ws, p.chol_dsc, p.shifts, r.st,
                               nullptr, r.spin()));
        apply_tri(r, p.Q1, false, rows, cols, p.Tm, U64);
        gram_tn64(r, U64, false, rows, cols, p.W, true);
        TK_HIP(chol_inv_scaled(p.W, cols, true, 0.0, p.Tm, (int*)p.chol_ws, p.chol_dsc, p.shifts, r.st,
                               nullptr, r.spin()));
        apply_tri(r, U64, false, rows, cols, p.Tm, p.Q1);
        TK_HIP(hipMemcpyAsync(U64, p.Q1, rows * cols * sizeof(double), hipMemcpyDeviceToDevice, r.st));
    }
    if (U32) TK_HIP(f64_to_f32(U64, U32, rows * cols, r.st));
}

// ||Z - U (U^T Z)||_F for Z = S U in p.Z (s x R) and orthonormal U (FP64): the residual of span(U) as an
// invariant subspace of S.  B = U^T Z goes to p.W, Z - U B to p.Q1; synchronises the stream.
double subspace_residual(Run& r, const double* U, int64_t s, int64_t R) {
    Plan& p = r.p;
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = R;
    g.N = R;
    g.K = s;
    g.a = plain(U, R);          // A(m, k) = U[k][m]
    g.b = plain(p.Z, R);        // B(k, n) = Z[k][n]
    g.c = plain(p.W, R);
    g.k_split = s;
    TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, false, false, r.st));
    GemmArgs h{};
    h.alpha = 1.0;
    h.M = s;
    h.N = R;
    h.K = R;
    h.a = plain(U, R);          // A(m, k) = U[m][k]
    h.b = plain(p.W, R);        // B(k, n) = B[k][n]
    h.c = plain(p.Q1, R);
    h.k_split = R;
    TK_HIP(gemm_f64(h, MK, KM, EPI_STORE, false, false, r.st));
    double e2 = 0.0;
    TK_HIP(tk_diff_sumsq_f64(p.Z, p.Q1, s * R, p.red, kSumsqBlocks - 8, p.red + kSumsqBlocks - 3, r.st));
    TK_HIP(hipMemcpyAsync(&e2, p.red + kSumsqBlocks - 3, sizeof(double), hipMemcpyDeviceToHost, r.st));
    TK_HIP(hipStreamSynchronize(r.st));
    return std::sqrt(e2);
}

// Z = S U for the Gram S64 (s x s) and the basis U64[n] (s x cols), into p.Z.  The product has few
// output tiles ((s/64) x (cols/64)); K is split so that the grid fills the chip, the FP64 partials
// summed in a fixed order.  Split count: the best per-CU balance of workgroups (average over maximum
// per CU), counting fewer than two per CU as under-filled; ties go to fewer splits (less partial-sum
// traffic).
void su_product(Run& r, int n, int64_t cols) {
    Plan& p = r.p;
    const int64_t s = p.s[n], R = cols;
    const int64_t tiles = ((s + 63) / 64) * ((R + 63) / 64);
    const int64_t cus = device_cu_count();
    const int64_t maxsp = std::max<int64_t>(1, std::min<int64_t>(
                                                   std::min<int64_t>(16, s / 128), p.Wpart_elems / std::max<int64_t>(1, s * R)));
    int64_t splits = 1;
    double best = -1.0;
    for (int64_t sp = 1; sp <= maxsp; ++sp) {
        const int64_t b = tiles * sp;
        const double score = ((double)b / cus) / (double)((b + cus - 1) / cus) * std::min(1.0, (double)b / (2.0 * cus));
        if (score > best + 1e-9) {
            best = score;
            splits = sp;
        }
    }
    int64_t ks = (s + splits - 1) / splits;
    ks = (ks + 15) / 16 * 16;
    const int nsplit = (int)((s + ks - 1) / ks);
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = s;
    g.N = R;
    g.K = s;
    g.a = plain(p.S64, s);      // A(m, k) = S[k][m] (symmetric)
    g.b = plain(p.U64[n], R);
    if (nsplit > 1) {
        g.k_split = ks;
        g.c = plain(p.Wpart, R);
        g.c_zstride = s * R;
        TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, false, false, r.st));
        TK_HIP(tk_sum_splits_f64(p.Wpart, nsplit, s * R, s * R, p.Z, r.st));
    } else {
        g.c = plain(p.Z, R);
        TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, false, false, r.st));
    }
}

// Z = S U from the FP32 copies of S (p.S32) and U (U32[n]) in a reduced-precision sweep, whose Gram
// already carries the 2^-8 .. 2^-4 rounding of its operands: FP32 MFMA, K split only as far as
// filling the chip needs, FP32 partials summed in FP64 into p.Z.
void su_product_f32(Run& r, int n, int64_t R) {
    Plan& p = r.p;
    const int64_t s = p.s[n];
    float* part = reinterpret_cast<float*>(p.Wpart);
    const int64_t part_cap = 2 * p.Wpart_elems;
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = s;
    g.N = R;
    g.K = s;
    g.a = plain(p.S32, s);      // A(m, k) = S[k][m] (symmetric)
    g.b = plain(p.U32[n], R);
    const int64_t tiles = ((s + 127) / 128) * ((R + 127) / 128);
    int64_t splits = std::max<int64_t>(1, (2 * device_cu_count() + tiles - 1) / tiles);
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, std::min<int64_t>(s / 128, part_cap / (s * R))));
    int64_t ks = (s + splits - 1) / splits;
    ks = (ks + 31) / 32 * 32;
    const int nsplit = (int)((s + ks - 1) / ks);
    g.k_split = ks;
    g.c = plain(part, R);
    g.c_zstride = s * R;
    TK_HIP(gemm_f32(g, KM, KM, EPI_STORE, false, r.st));
    TK_HIP(tk_sum_splits_f32p(part, nsplit, s * R, s * R, p.Z, r.st));
}

// Rayleigh-Ritz step closing an oversampled cold start (Rc = p.Rc[n] > R columns): with U (s x Rc,
// orthonormal) in U64[n], B = U^T S U (Rc x Rc) is diagonalised in FP64 (block Jacobi) and the
// factor becomes U V_R (s x R), V_R the eigenvectors of the R largest Ritz values, descending.  U V_R
// is orthonormal to FP64 rounding (both factors are).  In three parts: the products up to B (into
// p.W), the eigensolver (V_R into p.Tm, scratch in p.Wpart), and U V_R; the eigensolver checks its
// convergence on the host after each sweep.
void ritz_products(Run& r, int n) {
    Plan& p = r.p;
    const int64_t s = p.s[n], Rc = p.Rc[n];
    if (sym_eig_work_doubles((int)Rc) > p.Wpart_elems)
        throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "Rayleigh-Ritz scratch too small"};
    su_product(r, n, Rc);
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = Rc;
    g.N = Rc;
    g.K = s;
    g.a = plain(p.U64[n], Rc);  // A(m, k) = U[k][m]
    g.b = plain(p.Z, Rc);       // B(k, n) = (S U)[k][n]
    g.c = plain(p.W, Rc);
    g.k_split = s;
    TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, false, false, r.st));
}
void ritz_rotate(Run& r, int n) {
    Plan& p = r.p;
    const int64_t s = p.s[n], R = p.R[n], Rc = p.Rc[n];
    GemmArgs h{};
    h.alpha = 1.0;
    h.M = s;
    h.N = R;
    h.K = Rc;
    h.a = plain(p.U64[n], Rc);  // A(m, k) = U[m][k]
    h.b = plain(p.Tm, R);       // B(k, n) = V[k][n]
    h.c = plain(p.Q1, R);
    h.k_split = Rc;
    TK_HIP(gemm_f64(h, MK, KM, EPI_STORE, false, false, r.st));
    TK_HIP(hipMemcpyAsync(p.U64[n], p.Q1, s * R * sizeof(double), hipMemcpyDeviceToDevice, r.st));
    TK_HIP(f64_to_f32(p.U64[n], p.U32[n], s * R, r.st));
}
void rayleigh_ritz(Run& r, int n) {
    Plan& p = r.p;
    ritz_products(r, n);
    int sweeps = 0;
    TK_HIP(sym_eig_blocked(p.W, (int)p.Rc[n], (int)p.R[n], nullptr, p.Tm, nullptr, p.Wpart, r.st, &sweeps));
    r.rr_sweeps += sweeps;
    ritz_rotate(r, n);
}

// The Rayleigh-Ritz steps of the two large modes of a concurrent start: mode 0 on the main stream with
// the active scratch set, mode 1 on the second stream with the other set; the sweeps of their
// eigensolvers are interleaved (each waits only for its own convergence test), so the two run side by
// side.
void rayleigh_ritz_pair(Run& r) {
    Plan& p = r.p;
    tucker_ctx* ctx = r.ctx;
    if (!ctx->eig_host) {
        void* h = nullptr;
        TK_HIP(hipHostMalloc(&h, 4 * sizeof(double), hipHostMallocDefault));
        ctx->eig_host = (double*)h;
    }
    for (auto& e : ctx->eig_ev)
        if (!e) TK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    SymEigRun e[2];
    auto setup = [&](int n, int k) {
        ritz_products(r, n);
        e[k].A = p.W;
        e[k].n = (int)p.Rc[n];
        e[k].r = (int)p.R[n];
        e[k].U = p.Tm;
        e[k].work = p.Wpart;
        e[k].s = r.st;
        e[k].host = ctx->eig_host + 2 * k;
        e[k].ev = ctx->eig_ev[k];
        TK_HIP(sym_eig_start(e[k]));
    };
    setup(0, 0);
    swap_oi(p);
    {
        OnAux aux(r);
        setup(1, 1);
    }
    swap_oi(p);
    while (!e[0].done || !e[1].done)
        for (auto& j : e)
            if (!j.done) TK_HIP(sym_eig_step(j));
    r.rr_sweeps += e[0].sweeps + e[1].sweeps;
    ritz_rotate(r, 0);
    swap_oi(p);
    {
        OnAux aux(r);
        ritz_rotate(r, 1);
    }
    swap_oi(p);
}

// q steps of orthogonal iteration on S64 (s x s), from U64: Z = S U in FP64, then CholeskyQR.  With
// inner_tol > 0, q is the most steps, and the iteration stops once span(U) is invariant to the
// tolerance (checked once more after the q-th step).  An oversampled cold start iterates on p.Rc[n]
// columns and ends with the Rayleigh-Ritz step.
void orth_iter(Run& r, int n, int q, bool cold) {
    Plan& p = r.p;
    const int64_t s = p.s[n], R = cold ? p.Rc[n] : p.R[n];
    const bool ritz = cold && R > p.R[n];
    if ((p.S64_elems > 0 && s * s > p.S64_elems) || (p.Z_elems > 0 && s * R > p.Z_elems) || R > p.chol_cap)
        throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "orthogonal-iteration scratch set too small for this mode"};
    // inner_tol > 0: ||S||_F once; each step's product Z = S U first measures the residual of the
    // current U, and the iteration stops there when it is small enough
    const double tol = r.inner_tol();
    double snorm = 0.0, resid = -1.0;
    if (tol > 0.0) {
        TK_HIP(sumsq_f64(p.S64, s * s, p.red, kSumsqBlocks - 8, p.red + kSumsqBlocks - 4, r.st));
        TK_HIP(hipMemcpyAsync(&snorm, p.red + kSumsqBlocks - 4, sizeof(double), hipMemcpyDeviceToHost, r.st));
        TK_HIP(hipStreamSynchronize(r.st));
        snorm = std::sqrt(snorm);
    }
    // reduced-precision sweeps: the warm step's S U from the FP32 copy of S that their Gram wrote
    const bool su32 = r.lp_su && !cold && tol <= 0.0 && p.S32;
    for (int it = 0; it < q || (tol > 0.0 && it == q); ++it) {
        if (su32) su_product_f32(r, n, R);
        else su_product(r, n, R);
        if (tol > 0.0 && !(cold && it == 0)) {
            resid = subspace_residual(r, p.U64[n], s, R) / std::max(snorm, 1e-300);
            if (resid <= tol || it == q) break;
        }
        // cold start: shifted CholeskyQR3 for the first two steps, one pass for the intermediate
        // ones, the checked CholeskyQR2 for the last; with a tolerance every step may be the last,
        // so every step after the first two is a checked CholeskyQR2.  A warm update of several
        // steps likewise takes one pass for all but its last step (its warm basis keeps Z well
        // conditioned).  The FP32 copy is written only for a basis of the factor's own width.
        const bool mid = tol <= 0.0 && it < q - 1 && (cold ? it >= 2 : true);
        orthonormalize(r, p.Z, false, s, R, p.U64[n], ritz ? nullptr : p.U32[n], cold && it < 2, mid);
        (cold ? r.oi_steps_init : r.oi_steps_sweeps) += 1;
    }
    if (tol > 0.0) r.oi_resid_max = std::max(r.oi_resid_max, resid);
    if (ritz && !r.defer_ritz) rayleigh_ritz(r, n);
}

// factor update of mode n from the Gram in S64
void update_factor(Run& r, int n, bool cold) {
    Plan& p = r.p;
    if (p.kind[n] == FIXED) return;
    if (p.kind[n] == SMALL) {
        // warm start from the basis of the previous update once the cold start has run in this call
        TK_HIP(jacobi_eig(p.S64, (int)p.s[n], (int)p.R[n], p.U64[n], p.U32[n], nullptr, r.st, p.Vsm[n],
                          !cold && p.vsm_valid[n]));
        if (cold) p.vsm_valid[n] = true;
        return;
    }
    if (cold) {
        // the seeded random start (s x Rc), drawn in FP32 into p.Q1 when it is wider than U32
        float* u0 = p.Rc[n] > p.R[n] ? reinterpret_cast<float*>(p.Q1) : p.U32[n];
        TK_HIP(fill_random(u0, p.s[n] * p.Rc[n], r.ctx->opt.seed * 0x100000001b3ull + (uint64_t)n * 0x9e3779b9ull,
                           r.st));
        TK_HIP(f32_to_f64(u0, p.U64[n], p.s[n] * p.Rc[n], r.st));
        orth_iter(r, n, std::max(1, r.ctx->opt.init_iters), true);
    } else {
        const int q = r.inner_override > 0 ? std::max(r.inner_override, r.ctx->opt.inner_iters) : r.ctx->opt.inner_iters;
        orth_iter(r, n, std::max(1, q), false);
    }
}

// Warm single-step update of a large mode without forming its Gram.  With Y viewed (A, s, B) and
// S = Y_(n) Y_(n)^T, one orthogonal-iteration step needs S U = Y_(n) (Y_(n)^T U) = Y_(n) W_(n)^T,
// W = Y x_n U^T (R x A x B): 4 s R A B instead of s^2 A B + 2 s^2 R flops (18.1 instead of 25.5
// GFLOP for the 1920-row mode of a 1080p stack).  Both products accumulate in FP64 on the FP32
// data; W is rounded once to FP32 (from the FP32 factor), a relative error of 2^-24 against the
// FP32 rounding that Y already carries from the product chain, so both products run on the
// vector-load FP32-operand kernels.  Used when one step per sweep is asked for.
bool direct_update_ok(const Run& r, int n) {
    const Plan& p = r.p;
    return p.tree && p.kind[n] == LARGE && r.inner_override <= 0 && r.ctx->opt.inner_iters == 1 &&
           !(r.inner_tol() > 0.0);
}

// The W product of a one-step update: W = Uw^T Yw with Uw (K x Rw, FP32 factor, m = r contiguous)
// and Yw given as the k-major operand desc (k = contraction index, n = the other indices).  Stored
// to Wout (Rw x N, FP32).
struct WProduct {
    const float* U;
    int64_t R, K, N;
    Desc y;
};

void direct_update(Run& r, const float* Y, int64_t A, int64_t s, int64_t B, int n, const WProduct& wp, const Desc& wz,
                   int stage_prod, int stage_oi) {
    Plan& p = r.p;
    const int64_t R = p.R[n], AB = A * B;
    if (wp.R * wp.N > 2 * p.P_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "direct update buffer too small"};
    float* W = (float*)p.P;
    float* part = reinterpret_cast<float*>(p.Wpart);     // FP32 split partials (2 per FP64 slot)
    const int64_t part_cap = 2 * p.Wpart_elems;
    {
        StageTimer t(r, stage_prod);
        // W = U^T Y on the FP32 matrix cores, accumulated in FP32 over K = s_n like the products that
        // formed Y (their rounding, up to K u, bounds what W can carry); K split in two, FP32 partials
        // summed in FP64 and rounded once, when the output tiles alone leave the CUs unevenly loaded
        GemmArgs g{};
        g.alpha = 1.0;
        g.M = wp.R;
        g.N = wp.N;
        g.K = wp.K;
        g.a = plain(wp.U, wp.R);           // A(m = r, k = i) = U[i][r]
        g.b = wp.y;
        const int64_t cus = device_cu_count();
        const int64_t tw = ((wp.R + 127) / 128) * ((wp.N + 63) / 64);
        auto balance = [&](int64_t t) { return ((double)t / cus) / (double)((t + cus - 1) / cus); };
        const bool split_w = wp.K >= 512 && 2 * wp.R * wp.N <= part_cap && balance(2 * tw) > 1.05 * balance(tw);
        if (split_w) {
            g.k_split = (((wp.K + 1) / 2) + 31) / 32 * 32;
            g.c = plain(part, wp.N);
            g.c_zstride = wp.R * wp.N;
            TK_HIP(gemm_f32(g, KM, KM, EPI_STORE, false, r.st));
            TK_HIP(tk_sum_splits_f32p(part, (int)((wp.K + g.k_split - 1) / g.k_split), wp.R * wp.N, wp.R * wp.N, W,
                                      r.st));
        } else {
            g.c = plain(W, wp.N);
            TK_HIP(gemm_f32(g, KM, KM, EPI_STORE, false, r.st));
        }
        if (n == 0 && r.fit0_slot) {
            // first sweep, mode 1: Y0 = X x_2 U2^T x_3 U3^T x_4 U4^T with the start's factors and U1 not
            // yet updated, so W = Y0 x_1 U1^T is the start's core and ||W|| gives the start's fit
            TK_HIP(sumsq_f32(W, wp.R * wp.N, p.red, kSumsqBlocks, p.scal + 1, r.st));
            TK_HIP(fit_from_norms(p.scal + 0, p.scal + 1, r.fit0_slot, r.st));
            r.fit0_slot = nullptr;
        }
        // Z(m = i, n = r) = sum_(a,b) Y[a][i][b] W(k = (a, b), r) on the FP32 matrix cores, K split to
        // fill the chip and to at most kZSplitK per split; FP32 partials summed in FP64 into Z
        GemmArgs h{};
        h.alpha = 1.0;
        h.M = s;
        h.N = R;
        h.K = AB;
        h.a = folded(Y, B, B, s * B);      // A(m = i, k = (a, b))
        h.b = wz;                          // B(k = (a, b), n = r), same k segments as A
        const int64_t tiles = ((s + 127) / 128) * ((R + 127) / 128);
        int64_t splits = std::max<int64_t>(std::max<int64_t>(1, 2 * cus / tiles), (AB + kZSplitK - 1) / kZSplitK);
        splits = std::min<int64_t>(splits, std::max<int64_t>(1, AB / 64));
        splits = std::min<int64_t>(splits, std::max<int64_t>(1, part_cap / (s * R)));
        int64_t ks = (AB + splits - 1) / splits;
        ks = (ks + 31) / 32 * 32;
        const int nsplit = (int)((AB + ks - 1) / ks);
        h.k_split = ks;
        h.c = plain(part, R);
        h.c_zstride = s * R;
        TK_HIP(gemm_f32(h, MK, MK, EPI_STORE, false, r.st));
        TK_HIP(tk_sum_splits_f32p(part, nsplit, s * R, s * R, p.Z, r.st));
    }
    StageTimer t(r, stage_oi);
    orthonormalize(r, p.Z, false, s, R, p.U64[n], p.U32[n], false);
}

// the plain form: W = Y x_n U_n^T from the same Y (viewed (A, s, B)), stored (R, A, B)
void direct_update(Run& r, const float* Y, int64_t A, int64_t s, int64_t B, int n, int stage_prod, int stage_oi) {
    Plan& p = r.p;
    const int64_t R = p.R[n], AB = A * B;
    const WProduct wp{p.U32[n], R, s, AB, folded(Y, B, B, s * B)};
    direct_update(r, Y, A, s, B, n, wp, folded(p.P, AB, B, B), stage_prod, stage_oi);
}

void identity_factor(Run& r, int n) {
    TK_HIP(fill_identity_f32(r.p.U32[n], r.p.s[n], r.p.R[n], r.st));
    TK_HIP(fill_identity_f64(r.p.U64[n], r.p.s[n], r.p.R[n], r.st));
    r.p.ident[n] = r.p.s[n] == r.p.R[n];
}

// G = X x_1 U1^T ... x_N UN^T into p.G
void core_from_x(Run& r) {
    Plan& p = r.p;
    const int N = p.N;
    if (p.tree) {
        int64_t d[4] = {p.s[0], p.s[1], p.s[2] * p.s[3], 1};
        ttm(r, r.X, d, 3, 0, p.U32[0], p.R[0], false, p.T1);
        d[0] = p.R[0];
        ttm(r, p.T1, d, 3, 1, p.U32[1], p.R[1], false, p.T12);
        TK_HIP(pair_ttm(p.T12, p.R[0] * p.R[1], (int)p.s[2], (int)p.s[3], p.U32[2], (int)p.R[2], p.U32[3], (int)p.R[3],
                        false, p.G, r.st));
        return;
    }
    int64_t d[TUCKER_MAX_ORDER];
    for (int i = 0; i < N; ++i) d[i] = p.s[i];
    const float* cur = r.X;
    float* bufs[2] = {p.Ya, p.Yb};
    int w = 0;
    for (int m = 0; m < N; ++m) {
        float* dst = (m == N - 1) ? p.G : bufs[w];
        ttm(r, cur, d, N, m, p.U32[m], p.R[m], false, dst);
        d[m] = p.R[m];
        cur = dst;
        w ^= 1;
    }
}

void core_norm_and_fit(Run& r, double* fit_slot) {
    Plan& p = r.p;
    TK_HIP(sumsq_f32(p.G, prod(p.R, 0, p.N), p.red, kSumsqBlocks, p.scal + 1, r.st));
    TK_HIP(fit_from_norms(p.scal + 0, p.scal + 1, fit_slot, r.st));
}

// ------------------------------------------------------------------ T-HOSVD initialisation
void lp_gram(Run& r, Desc y, int64_t srows, int64_t K, int stage);

// Gram of X for the start of large mode n (0 or 1 of a tree shape): in the sweeps' reduced precision
// from the padded copy made by lp_start_copy (FP32 partial sums over k splits, summed in FP64), else in
// FP64 from the FP32 tensor
void start_gram(Run& r, int n) {
    Plan& p = r.p;
    if (!p.lp_start || n > 1) {
        gram(r, r.X, p.s, p.N, n);
        return;
    }
    const int64_t s0 = p.s[0], s1 = p.s[1], Lp = p.Lp;
    const void* xp = p.T34;
    if (n == 0) lp_gram(r, plain(xp, s1 * Lp), s0, s1 * Lp, -1);
    else lp_gram(r, folded(xp, Lp, Lp, s1 * Lp), s1, s0 * Lp, -1);
}
void lp_start_copy(Run& r) {
    Plan& p = r.p;
    if (!p.lp_start) return;
    const int64_t L = p.s[2] * p.s[3];
    TK_HIP(to_lowp_padded(r.X, p.s[0] * p.s[1], (int)L, (int)p.Lp, p.ip, p.T34, r.st));
}

void thosvd(Run& r) {
    Plan& p = r.p;
    // modes from `from` on, in order.  Tree shapes: the Grams of the two small trailing modes come
    // from the fibre Gram of X (one coalesced pass over X), F = sum_(h,w) x_(h,w) x_(h,w)^T over
    // the (s3 s4)-long fibres
    auto modes_from = [&](int from) {
        bool have_f = false;
        for (int n = from; n < p.N; ++n) {
            if (p.kind[n] == FIXED) {
                identity_factor(r, n);
                continue;
            }
            if (p.tree && n >= 2) {
                if (!have_f) {
                    TK_HIP(fibre_gram(r.X, p.s[0] * p.s[1], (int)(p.s[2] * p.s[3]), p.Fpart, kFibreGramBlocks, p.F,
                                      r.st));
                    have_f = true;
                }
                TK_HIP(pair_mode_gram(p.F, (int)p.s[2], (int)p.s[3], nullptr, 0, n == 2 ? 3 : 4, p.S64, r.st));
            } else {
                start_gram(r, n);
            }
            update_factor(r, n, true);
        }
    };
    lp_start_copy(r);
    bool ritz = false;
    for (int n = 0; n < p.N; ++n) ritz = ritz || p.Rc[n] > p.R[n];
    if (!p.has_alt || r.inner_tol() > 0.0) {
        // (with a tolerance every step waits for the host, so the two streams could not overlap)
        modes_from(0);
        return;
    }
    if (ritz) {
        // oversampled: the two cold iterations run side by side as below, then their Rayleigh-Ritz
        // steps (whose eigensolvers wait for the host) side by side, then the small modes
        start_gram(r, 1);
        fork_aux(r);
        r.defer_ritz = p.Rc[1] > p.R[1];
        {
            OnAux aux(r);
            update_factor(r, 1, true);
        }
        const bool deferred1 = r.defer_ritz;
        swap_oi(p);
        start_gram(r, 0);
        r.defer_ritz = p.Rc[0] > p.R[0] && deferred1;
        update_factor(r, 0, true);
        r.defer_ritz = false;
        if (deferred1 && p.Rc[0] > p.R[0]) rayleigh_ritz_pair(r);
        else if (deferred1) {
            swap_oi(p);
            {
                OnAux aux(r);
                rayleigh_ritz(r, 1);
            }
            swap_oi(p);
        }
        modes_from(2);
        swap_oi(p);
        join_aux(r);
        return;
    }
    // the modes start from the unprojected X independently.  Mode 2's Gram (the larger) comes first,
    // in the first scratch set (sized for the largest mode); its latency-bound cold orthogonal
    // iterations then run on the second stream with that set, while the main stream, with the
    // second set (sized for mode 1), forms mode 1's Gram (its split partials sit in a buffer the
    // iterations do not use) and runs mode 1's iterations and the small modes
    start_gram(r, 1);
    fork_aux(r);
    {
        OnAux aux(r);
        update_factor(r, 1, true);
    }
    swap_oi(p);
    start_gram(r, 0);
    update_factor(r, 0, true);
    modes_from(2);
    swap_oi(p);
    join_aux(r);
}

// ------------------------------------------------------------------ ST-HOSVD initialisation
// The sequentially truncated ("interlaced") HOSVD, the cheaper start of Sec. III-B.1: modes in
// ascending order, each factor from the Gram of the tensor already projected on the earlier
// factors, Y(n) = Y(n-1) x_n U_n^T; the last projection is the core.  Tree shapes reuse the sweep's
// buffers: T1 = X x_1 U1^T (pass C1) feeds mode 2's Gram (contracted over R1 s3 s4 instead of
// s1 s3 s4), T12 = T1 x_2 U2^T feeds the fibre Gram of the two small modes, and G closes the start.
// Leaves the core in p.G.
void sthosvd(Run& r) {
    Plan& p = r.p;
    const int N = p.N;
    auto start_mode = [&](const float* y, const int64_t* d, int nd, int n) {
        if (p.kind[n] == FIXED) {
            identity_factor(r, n);
            return;
        }
        gram(r, y, d, nd, n);
        update_factor(r, n, true);
    };
    if (p.tree) {
        const int64_t s0 = p.s[0], s1 = p.s[1], s2 = p.s[2], s3 = p.s[3], L = s2 * s3;
        int64_t d[3] = {s0, s1, L};
        start_mode(r.X, d, 3, 0);
        ttm(r, r.X, d, 3, 0, p.U32[0], p.R[0], false, p.T1);
        d[0] = p.R[0];
        start_mode(p.T1, d, 3, 1);
        ttm(r, p.T1, d, 3, 1, p.U32[1], p.R[1], false, p.T12);
        // modes 3 and 4 from the fibre Gram of T12: mode 3 with mode 4 not yet projected, then
        // mode 4 with mode 3 projected on the new U3
        TK_HIP(fibre_gram(p.T12, p.R[0] * p.R[1], (int)L, p.Fpart, kFibreGramBlocks, p.F, r.st));
        if (p.kind[2] == FIXED) {
            identity_factor(r, 2);
        } else {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, nullptr, 0, 3, p.S64, r.st));
            update_factor(r, 2, true);
        }
        if (p.kind[3] == FIXED) {
            identity_factor(r, 3);
        } else {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[2], (int)p.R[2], 4, p.S64, r.st));
            update_factor(r, 3, true);
        }
        TK_HIP(pair_ttm(p.T12, p.R[0] * p.R[1], (int)s2, (int)s3, p.U32[2], (int)p.R[2], p.U32[3], (int)p.R[3],
                        false, p.G, r.st));
        return;
    }
    int64_t d[TUCKER_MAX_ORDER];
    for (int i = 0; i < N; ++i) d[i] = p.s[i];
    const float* cur = r.X;
    float* bufs[2] = {p.Ya, p.Yb};
    int w = 0;
    for (int n = 0; n < N; ++n) {
        start_mode(cur, d, N, n);
        float* dst = (n == N - 1) ? p.G : bufs[w];
        ttm(r, cur, d, N, n, p.U32[n], p.R[n], false, dst);
        d[n] = p.R[n];
        cur = dst;
        w ^= 1;
    }
}

// ------------------------------------------------------------------ one ALS sweep
void sweep_tree(Run& r) {
    Plan& p = r.p;
    const int64_t s0 = p.s[0], s1 = p.s[1], s2 = p.s[2], s3 = p.s[3];
    const int64_t R0 = p.R[0], R1 = p.R[1], R2 = p.R[2], R3 = p.R[3];
    const int64_t R23 = R2 * R3, L = s2 * s3;
    // T34 = X x_3 U3^T x_4 U4^T (full-tensor pass, memory-bound)
    {
        StageTimer t(r, TUCKER_STAGE_PASS_A);
        TK_HIP(pair_ttm(r.X, s0 * s1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, false, p.T34, r.st,
                        p.ident[2]));
    }
    // mode 1: Y0 = T34 x_2 U2^T, S0 = Y0_(1) Y0_(1)^T
    if (p.kind[0] != FIXED) {
        int64_t d[3] = {s0, s1, R23};
        {
            StageTimer t(r, TUCKER_STAGE_TTM_Y1);
            ttm(r, p.T34, d, 3, 1, p.U32[1], R1, false, p.Y0);
        }
        if (direct_update_ok(r, 0)) {
            direct_update(r, p.Y0, 1, s0, R1 * R23, 0, TUCKER_STAGE_GRAM_1, TUCKER_STAGE_OI_1);
        } else {
            int64_t dy[3] = {s0, R1, R23};
            gram(r, p.Y0, dy, 3, 0, TUCKER_STAGE_GRAM_1);
            StageTimer t(r, TUCKER_STAGE_OI_1);
            update_factor(r, 0, false);
        }
    }
    // second full-tensor pass T1 = X x_1 U1^T: it needs only the new U1, so it runs before mode 2
    int64_t dc[3] = {s0, s1, L};
    {
        StageTimer t(r, TUCKER_STAGE_PASS_C1);
        ttm(r, r.X, dc, 3, 0, p.U32[0], R0, false, p.T1);
    }
    // mode 2: Y1 = T34 x_1 U1^T = T1 x_3 U3^T x_4 U4^T (distinct modes commute), formed from T1 by
    // the memory-bound fibre kernel instead of a product over s1
    if (p.kind[1] != FIXED) {
        {
            StageTimer t(r, TUCKER_STAGE_TTM_Y2);
            TK_HIP(pair_ttm(p.T1, R0 * s1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, false, p.Y1,
                            r.st, p.ident[2]));
        }
        if (direct_update_ok(r, 1) && p.kind[0] != FIXED) {
            // Y1^T U2 = T34 x_1 U1^T x_2 U2^T = Y0 x_1 U1^T: contracted over s1 from Y0 (still resident
            // from mode 1, computed with the same U2) instead of over s2 from Y1; W(r1, r2, c)
            const WProduct wp{p.U32[0], R0, s0, R1 * R23, plain(p.Y0, R1 * R23)};
            direct_update(r, p.Y1, R0, s1, R23, 1, wp, folded(p.P, R23, R23, R1 * R23), TUCKER_STAGE_GRAM_2,
                          TUCKER_STAGE_OI_2);
        } else if (direct_update_ok(r, 1)) {
            direct_update(r, p.Y1, R0, s1, R23, 1, TUCKER_STAGE_GRAM_2, TUCKER_STAGE_OI_2);
        } else {
            int64_t dy[3] = {R0, s1, R23};
            gram(r, p.Y1, dy, 3, 1, TUCKER_STAGE_GRAM_2);
            StageTimer t(r, TUCKER_STAGE_OI_2);
            update_factor(r, 1, false);
        }
    }
    // T12 = T1 x_2 U2^T
    {
        dc[0] = R0;
        StageTimer t(r, TUCKER_STAGE_TTM_C2);
        ttm(r, p.T1, dc, 3, 1, p.U32[1], R1, false, p.T12);
    }
    // modes 3 and 4 from the fibre Gram of T12
    if (p.kind[2] != FIXED || p.kind[3] != FIXED) {
        StageTimer t(r, TUCKER_STAGE_SMALL);
        TK_HIP(fibre_gram(p.T12, R0 * R1, (int)L, p.Fpart, kFibreGramBlocks, p.F, r.st));
        if (p.kind[2] != FIXED) {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[3], (int)R3, 3, p.S64, r.st));
            update_factor(r, 2, false);
        }
        if (p.kind[3] != FIXED) {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[2], (int)R2, 4, p.S64, r.st));
            update_factor(r, 3, false);
        }
    }
    // core G = T12 x_3 U3^T x_4 U4^T
    StageTimer t(r, TUCKER_STAGE_CORE);
    TK_HIP(pair_ttm(p.T12, R0 * R1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, false, p.G, r.st,
                    p.ident[2]));
}

// ------------------------------------------------------------------ pairwise perturbation
// Sec. III-B, eq. (9)-(13): around reference factors S_p (the factors when the sweeps had nearly
// settled), the tensor of an update is taken to first order in dS = S - S_p,
//   Y~(n) = Y_p(n) + sum_{i != n} Y_p(i,n) x_i dS(i)^T,
// with the operators Y_p(n) = X x_{l != n} S_p(l)^T and Y_p(i,n) = X x_{j not in {i,n}} S_p(j)^T formed once
// per reference point; perturbation sweeps read only them, never X.  For the image stacks (modes
// (H, W, C, I), the colour mode kept at full rank with the identity factor, so dS(3) = 0):
//   Y_p(1) = T34 x_2 S2^T (Y0p), Y_p(1,2) = T34 = X x_3 S3^T x_4 S4^T, Y_p(1,4) = Z = X x_2 S2^T,
//   Y_p(2) = T1 x_3 x_4 (Y1p), Y_p(2,4) = T1 = X x_1 S1^T, Y_p(4) = T12 = T1 x_2 S2^T,
// so Y~(1) = Y0p + T34 x_2 dS2^T + Z x_4 dS4^T, Y~(2) = Y1p + T34 x_1 dS1^T + T1 x_4 dS4^T and
// Y~(4) = T12p + Z x_1 dS1^T + T1 x_2 dS2^T.  Each new factor is represented by the orthonormal basis
// of its subspace closest to the reference (orthogonal Procrustes, the polar factor of U^T S_p by
// Newton-Schulz iteration in FP64).  The sweeps switch between ordinary and perturbation ones on the
// subspace distance d(U, V) = ||U U^T - V V^T||_F / sqrt(2R) = sqrt(1 - ||U^T V||_F^2 / R).

// out += in x_n U^T (U: dims[n] x R) by the FP32 matrix cores, accumulating into out
void ttm_add(Run& r, const float* in, const int64_t* dims, int N, int n, const float* U, int64_t R, float* out) {
    const int64_t A = prod(dims, 0, n), K = dims[n], B = prod(dims, n + 1, N);
    GemmArgs g{};
    g.alpha = 1.0;
    if (B == 1) {
        g.M = A;
        g.N = R;
        g.K = K;
        g.a = plain(in, K);
        g.b = plain(U, R);
        g.c = plain(out, R);
        TK_HIP(gemm_f32(g, MK, KM, EPI_ADD, false, r.st));
    } else {
        g.M = R;
        g.N = A * B;
        g.K = K;
        g.a = plain(U, R);
        g.b = folded(in, B, B, K * B);
        g.c = folded(out, B, B, R * B);
        TK_HIP(gemm_f32(g, KM, KM, EPI_ADD, false, r.st));
    }
}

// C (M x N, FP64) = A^T B for A (K x M) and B (K x N), FP64 row-major
void gemm_tn64(Run& r, const double* A, const double* B, int64_t K, int64_t M, int64_t N, double* C) {
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = M;
    g.N = N;
    g.K = K;
    g.a = plain(A, M);
    g.b = plain(B, N);
    g.c = plain(C, N);
    TK_HIP(gemm_f64(g, KM, KM, EPI_STORE, false, false, r.st));
}
// C (M x N) = A B for A (M x K) and B (K x N), FP64
void gemm_nn64(Run& r, const double* A, const double* B, int64_t M, int64_t K, int64_t N, double* C) {
    GemmArgs g{};
    g.alpha = 1.0;
    g.M = M;
    g.N = N;
    g.K = K;
    g.a = plain(A, K);
    g.b = plain(B, N);
    g.c = plain(C, N);
    TK_HIP(gemm_f64(g, MK, KM, EPI_STORE, false, false, r.st));
}

constexpr int kNewtonSchulzSteps = 12;   // quadratic convergence for singular values of U^T S_p above ~0.1

// U_n <- U_n Q with Q the polar factor of U_n^T S_p(n): the basis of span(U_n) closest to S_p(n)
void pp_align(Run& r, int n) {
    Plan& p = r.p;
    const int64_t s = p.s[n], R = p.R[n];
    gemm_tn64(r, p.U64[n], p.U64p[n], s, R, R, p.NS_X);
    for (int it = 0; it < kNewtonSchulzSteps; ++it) {
        gemm_tn64(r, p.NS_X, p.NS_X, R, R, R, p.NS_B);          // B = X^T X
        TK_HIP(ns_step(p.NS_B, p.NS_D, R, r.st));               // D = 1.5 I - 0.5 B
        gemm_nn64(r, p.NS_X, p.NS_D, R, R, R, p.NS_T);          // X <- X D
        std::swap(p.NS_X, p.NS_T);
    }
    gemm_nn64(r, p.U64[n], p.NS_X, s, R, R, p.NS_U);
    TK_HIP(hipMemcpyAsync(p.U64[n], p.NS_U, s * R * sizeof(double), hipMemcpyDeviceToDevice, r.st));
    TK_HIP(f64_to_f32(p.U64[n], p.U32[n], s * R, r.st));
}

// max over the modes of d(U_n, V_n) for V = the reference (against_ref) or the previous sweep's factors
double pp_distance(Run& r, bool against_ref) {
    Plan& p = r.p;
    for (int n = 0; n < p.N; ++n) {
        const int64_t s = p.s[n], R = p.R[n];
        gemm_tn64(r, p.U64[n], against_ref ? p.U64p[n] : p.U64prev[n], s, R, R, p.NS_B);
        TK_HIP(sumsq_f64(p.NS_B, R * R, p.ppdist + 2 * TUCKER_MAX_ORDER, kSumsqBlocks, p.ppdist + n, r.st));
    }
    double h[TUCKER_MAX_ORDER] = {};
    TK_HIP(hipMemcpyAsync(h, p.ppdist, p.N * sizeof(double), hipMemcpyDeviceToHost, r.st));
    TK_HIP(hipStreamSynchronize(r.st));
    double d = 0.0;
    for (int n = 0; n < p.N; ++n) d = std::max(d, std::sqrt(std::max(1.0 - h[n] / (double)p.R[n], 0.0)));
    return d;
}

// the reference point: current factors and the operators around them
void pp_init(Run& r) {
    Plan& p = r.p;
    const int64_t s0 = p.s[0], s1 = p.s[1], s2 = p.s[2], s3 = p.s[3], L = s2 * s3;
    const int64_t R0 = p.R[0], R1 = p.R[1], R2 = p.R[2], R3 = p.R[3], R23 = R2 * R3;
    if (!p.ident[2]) throw Fail{TUCKER_ERR_UNSUPPORTED, "pairwise perturbation needs the identity colour factor"};
    for (int n = 0; n < p.N; ++n) {
        TK_HIP(hipMemcpyAsync(p.U32p[n], p.U32[n], p.s[n] * p.R[n] * sizeof(float), hipMemcpyDeviceToDevice, r.st));
        TK_HIP(hipMemcpyAsync(p.U64p[n], p.U64[n], p.s[n] * p.R[n] * sizeof(double), hipMemcpyDeviceToDevice, r.st));
    }
    TK_HIP(pair_ttm(r.X, s0 * s1, (int)s2, (int)s3, p.U32p[2], (int)R2, p.U32p[3], (int)R3, false, p.T34, r.st,
                    true));
    int64_t d34[3] = {s0, s1, R23};
    ttm(r, p.T34, d34, 3, 1, p.U32p[1], R1, false, p.Y0p);
    int64_t dx[3] = {s0, s1, L};
    ttm(r, r.X, dx, 3, 0, p.U32p[0], R0, false, p.T1);
    ttm(r, r.X, dx, 3, 1, p.U32p[1], R1, false, p.Zp);
    TK_HIP(pair_ttm(p.T1, R0 * s1, (int)s2, (int)s3, p.U32p[2], (int)R2, p.U32p[3], (int)R3, false, p.Y1p, r.st,
                    true));
    int64_t d1[3] = {R0, s1, L};
    ttm(r, p.T1, d1, 3, 1, p.U32p[1], R1, false, p.T12p);
}

// one perturbation sweep: modes 1, 2 and 4 from the first-order tensors, the core from Y~(4)
void pp_sweep(Run& r) {
    Plan& p = r.p;
    const int64_t s0 = p.s[0], s1 = p.s[1], s2 = p.s[2], s3 = p.s[3], L = s2 * s3;
    const int64_t R0 = p.R[0], R1 = p.R[1], R2 = p.R[2], R3 = p.R[3], R23 = R2 * R3;
    auto delta = [&](int n) { TK_HIP(diff_f32(p.U32[n], p.U32p[n], p.dU[n], p.s[n] * p.R[n], r.st)); };
    const bool m4 = p.kind[3] != FIXED;
    delta(1);
    if (m4) delta(3);
    // mode 1: Y~(1) = Y0p + T34 x_2 dS2^T + Z x_4 dS4^T (s0, R1, R3 R4)
    TK_HIP(hipMemcpyAsync(p.Y0, p.Y0p, s0 * R1 * R23 * sizeof(float), hipMemcpyDeviceToDevice, r.st));
    {
        StageTimer t(r, TUCKER_STAGE_TTM_Y1);
        int64_t d34[3] = {s0, s1, R23};
        ttm_add(r, p.T34, d34, 3, 1, p.dU[1], R1, p.Y0);
        if (m4) {
            TK_HIP(small_ttm(p.Zp, s0 * R1 * s2, s3, 1, p.dU[3], R3, false, p.PPtmp, r.st));
            TK_HIP(axpy_f32(p.PPtmp, p.Y0, s0 * R1 * R23, r.st));
        }
    }
    direct_update(r, p.Y0, 1, s0, R1 * R23, 0, TUCKER_STAGE_GRAM_1, TUCKER_STAGE_OI_1);
    pp_align(r, 0);
    delta(0);
    // mode 2: Y~(2) = Y1p + T34 x_1 dS1^T + T1 x_4 dS4^T (R0, s1, R3 R4)
    TK_HIP(hipMemcpyAsync(p.Y1, p.Y1p, R0 * s1 * R23 * sizeof(float), hipMemcpyDeviceToDevice, r.st));
    {
        StageTimer t(r, TUCKER_STAGE_TTM_Y2);
        int64_t d34[2] = {s0, s1 * R23};
        ttm_add(r, p.T34, d34, 2, 0, p.dU[0], R0, p.Y1);
        if (m4) {
            TK_HIP(small_ttm(p.T1, R0 * s1 * s2, s3, 1, p.dU[3], R3, false, p.PPtmp, r.st));
            TK_HIP(axpy_f32(p.PPtmp, p.Y1, R0 * s1 * R23, r.st));
        }
    }
    direct_update(r, p.Y1, R0, s1, R23, 1, TUCKER_STAGE_GRAM_2, TUCKER_STAGE_OI_2);
    pp_align(r, 1);
    delta(1);
    // mode 4: Y~(4) = T12p + Z x_1 dS1^T + T1 x_2 dS2^T (R0, R1, s3 s4)
    TK_HIP(hipMemcpyAsync(p.T12, p.T12p, R0 * R1 * L * sizeof(float), hipMemcpyDeviceToDevice, r.st));
    {
        StageTimer t(r, TUCKER_STAGE_TTM_C2);
        int64_t dz[2] = {s0, R1 * L};
        ttm_add(r, p.Zp, dz, 2, 0, p.dU[0], R0, p.T12);
        int64_t d1[3] = {R0, s1, L};
        ttm_add(r, p.T1, d1, 3, 1, p.dU[1], R1, p.T12);
    }
    if (m4) {
        StageTimer t(r, TUCKER_STAGE_SMALL);
        TK_HIP(fibre_gram(p.T12, R0 * R1, (int)L, p.Fpart, kFibreGramBlocks, p.F, r.st));
        TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[2], (int)R2, 4, p.S64, r.st));
        update_factor(r, 3, false);
        pp_align(r, 3);
    }
    StageTimer t(r, TUCKER_STAGE_CORE);
    TK_HIP(pair_ttm(p.T12, R0 * R1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, false, p.G, r.st,
                    true));
}

// ------------------------------------------------------------------ reduced-precision sweep
// The same tree sweep as sweep_tree with every dense contraction on the 16-/8-bit matrix cores
// (FP32 accumulation) and the intermediates T34, Y0, Y1, T1 stored in the 16-bit type; the
// orthogonal iteration, the small modes, the core and all norms are unchanged.  X is converted
// once per decomposition (FP8: one scale per (channel, image) slice, folded back in pass A and in
// the epilogue of pass C1).

// X -> Xlp (and the FP8 slice scales)
void lp_convert_x(Run& r) {
    Plan& p = r.p;
    const int64_t L = p.s[2] * p.s[3], Xn = prod(p.s, 0, p.N);
    const float* scale = nullptr;
    if (p.prec == TUCKER_FP8_E4M3) {
        TK_HIP(slice_scales(r.X, Xn / L, (int)L, p.spart, kLpScaleBlocks, p.xscale, r.st));
        scale = p.xscale;
    }
    TK_HIP(to_lowp(r.X, Xn, p.prec, (int)L, scale, p.Xlp, r.st));
    // T1 rows are padded from L to Lp; the padding is never written and must read as zero
    if (p.Lp != L) TK_HIP(fill_zero(p.T1lp, p.R[0] * p.s[1] * p.Lp * (int64_t)sizeof(uint16_t), r.st));
}

// transposed reduced-precision copy of factor n: Ut (R x round8(s)), k contiguous
void lp_factor(Run& r, int n, int prec, void* Ut, float* scale) {
    Plan& p = r.p;
    const int64_t sp = (p.s[n] + 7) / 8 * 8;
    TK_HIP(factor_lowp(p.U32[n], p.s[n], p.R[n], sp, prec, scale, Ut, r.st));
}

// a reduced-precision product of a sweep: through the calling thread's lock-step group when it has
// one (served requests of one shape), else launched alone
hipError_t lp_launch(const LpGemmArgs& g, int prec, Orient ob, int outp, hipStream_t st) {
    if (LpGrouper* G = lp_group_current()) return G->gemm(g, prec, ob, outp, st);
    return gemm_lp(g, prec, ob, outp, st);
}

// mode product out = B x U^T on the matrix cores: A = Ut (M = R rows, K = s), B an n-contiguous view
void lp_ttm(Run& r, int prec, const void* Ut, int64_t R, int64_t K, Desc b, int64_t N, Desc c, int outp,
            const float* sa = nullptr, const float* sb = nullptr, int64_t sb_mod = 0, int64_t c_valid = 0) {
    LpGemmArgs g{};
    g.c_valid = c_valid;
    g.a = plain(Ut, (K + 7) / 8 * 8);
    g.b = b;
    g.c = c;
    g.M = R;
    g.N = N;
    g.K = K;
    g.alpha = 1.0;
    g.k_split = 0;
    g.sa = sa;
    g.sb = sb;
    g.sb_mod = sb_mod;
    TK_HIP(lp_launch(g, prec, KM, outp, r.st));
}

// S64 = Y Y^T for a k-contiguous view Y (s rows, K columns): FP32 partials over K splits, summed in FP64
void lp_gram(Run& r, Desc y, int64_t srows, int64_t K, int stage) {
    Plan& p = r.p;
    LpGemmArgs g{};
    g.a = y;
    g.b = y;
    g.M = srows;
    g.N = srows;
    g.K = K;
    g.alpha = 1.0;
    g.lower_only = 1;
    g.k_split = lp_gram_ksplit(srows, K);
    const int nsplit = (int)((K + g.k_split - 1) / g.k_split);
    if ((int64_t)nsplit * srows * srows > p.Pf_elems) throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "Gram partial buffer"};
    g.c = plain(p.Pf, srows);
    g.c_zstride = srows * srows;
    {
        StageTimer t(r, stage);
        TK_HIP(lp_launch(g, p.ip, MK, LP_F32OUT, r.st));
    }
    StageTimer t(r, stage >= 0 ? TUCKER_STAGE_REDUCE : -1);
    TK_HIP(gram_reduce(p.Pf, nsplit, srows, srows * srows, r.lp_su ? p.S32 : nullptr, p.S64, r.st));
}

void sweep_tree_lp(Run& r) {
    Plan& p = r.p;
    struct LpSu {
        Run& r;
        explicit LpSu(Run& run) : r(run) { r.lp_su = true; }
        ~LpSu() { r.lp_su = false; }
    } lp_su_scope(r);
    const int64_t s0 = p.s[0], s1 = p.s[1], s2 = p.s[2], s3 = p.s[3];
    const int64_t R0 = p.R[0], R1 = p.R[1], R2 = p.R[2], R3 = p.R[3];
    const int64_t R23p = p.R23p, L = s2 * s3;
    const int ip = p.ip;
    // T34 = X x_3 U3^T x_4 U4^T from the reduced-precision X, padded fibres of R23p
    {
        StageTimer t(r, TUCKER_STAGE_PASS_A);
        TK_HIP(pair_lowp(p.Xlp, s0 * s1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, p.prec,
                         p.prec == TUCKER_FP8_E4M3 ? p.xscale : nullptr, ip, (int)R23p, p.T34lp, r.st,
                         p.kind[2] == FIXED && p.ident[2]));
    }
    // mode 1: Y0 = T34 x_2 U2^T (k = w; n = (h, j)), S0 = Y0_(1) Y0_(1)^T
    {
        StageTimer t(r, TUCKER_STAGE_TTM_Y1);
        lp_factor(r, 1, ip, p.U2t, nullptr);
        lp_ttm(r, ip, p.U2t, R1, s1, folded(p.T34lp, R23p, R23p, s1 * R23p), s0 * R23p,
               folded(p.Y0lp, R23p, R23p, R1 * R23p), ip);
    }
    lp_gram(r, plain(p.Y0lp, R1 * R23p), s0, R1 * R23p, TUCKER_STAGE_GRAM_1);
    {
        StageTimer t(r, TUCKER_STAGE_OI_1);
        update_factor(r, 0, false);
    }
    // mode 2: Y1 = T34 x_1 U1^T (new U1), S1 from Y1 viewed (R0, s1, R23p)
    {
        StageTimer t(r, TUCKER_STAGE_TTM_Y2);
        lp_factor(r, 0, ip, p.U1t, nullptr);
        lp_ttm(r, ip, p.U1t, R0, s0, plain(p.T34lp, s1 * R23p), s1 * R23p, plain(p.Y1lp, s1 * R23p), ip);
    }
    lp_gram(r, folded(p.Y1lp, R23p, R23p, s1 * R23p), s1, R0 * R23p, TUCKER_STAGE_GRAM_2);
    {
        StageTimer t(r, TUCKER_STAGE_OI_2);
        update_factor(r, 1, false);
    }
    // T1 = X x_1 U1^T (second pass over X, rows of T1 padded to Lp), T12 = T1 x_2 U2^T in FP32
    const int64_t Lp = p.Lp;
    {
        StageTimer t(r, TUCKER_STAGE_PASS_C1);
        const Desc t1 = folded(p.T1lp, s1 * Lp, L, Lp);
        if (p.prec == TUCKER_FP8_E4M3) {
            lp_factor(r, 0, TUCKER_FP8_E4M3, p.U1t8, p.u1scale);
            lp_ttm(r, TUCKER_FP8_E4M3, p.U1t8, R0, s0, plain(p.Xlp, s1 * L), s1 * L, t1, ip, p.u1scale, p.xscale, L);
        } else {
            lp_ttm(r, p.prec, p.U1t, R0, s0, plain(p.Xlp, s1 * L), s1 * L, t1, ip);
        }
    }
    {
        StageTimer t(r, TUCKER_STAGE_TTM_C2);
        lp_factor(r, 1, ip, p.U2t, nullptr);
        lp_ttm(r, ip, p.U2t, R1, s1, folded(p.T1lp, Lp, Lp, s1 * Lp), R0 * Lp, folded(p.T12, L, Lp, R1 * L),
               LP_F32OUT, nullptr, nullptr, 0, L);
    }
    // modes 3 and 4 and the core exactly as in the FP32 sweep
    if (p.kind[2] != FIXED || p.kind[3] != FIXED) {
        StageTimer t(r, TUCKER_STAGE_SMALL);
        TK_HIP(fibre_gram(p.T12, R0 * R1, (int)L, p.Fpart, kFibreGramBlocks, p.F, r.st));
        if (p.kind[2] != FIXED) {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[3], (int)R3, 3, p.S64, r.st));
            update_factor(r, 2, false);
        }
        if (p.kind[3] != FIXED) {
            TK_HIP(pair_mode_gram(p.F, (int)s2, (int)s3, p.U64[2], (int)R2, 4, p.S64, r.st));
            update_factor(r, 3, false);
        }
    }
    StageTimer t(r, TUCKER_STAGE_CORE);
    TK_HIP(pair_ttm(p.T12, R0 * R1, (int)s2, (int)s3, p.U32[2], (int)R2, p.U32[3], (int)R3, false, p.G, r.st,
                    p.ident[2]));
}

void sweep_generic(Run& r) {
    Plan& p = r.p;
    const int N = p.N;
    float* bufs[2] = {p.Ya, p.Yb};
    int64_t d[TUCKER_MAX_ORDER];
    const float* cur = nullptr;
    for (int n = 0; n < N; ++n) {
        for (int i = 0; i < N; ++i) d[i] = p.s[i];
        cur = r.X;
        int w = 0;
        for (int m = 0; m < N; ++m) {
            if (m == n) continue;
            ttm(r, cur, d, N, m, p.U32[m], p.R[m], false, bufs[w]);
            d[m] = p.R[m];
            cur = bufs[w];
            w ^= 1;
        }
        if (p.kind[n] != FIXED) {
            gram(r, cur, d, N, n);
            update_factor(r, n, false);
        }
    }
    // core from the last chain: G = Y x_N U_N^T
    ttm(r, cur, d, N, N - 1, p.U32[N - 1], p.R[N - 1], false, p.G);
}

// ------------------------------------------------------------------ reconstruction chain
// Expands G through all factors.  With out == nullptr the last product is fused with the
// residual against X and ||X - Xhat||^2 lands in scal[2].
void expand_chain(Run& r, const float* G, float* const* U, float* out, const float* Xref) {
    Plan& p = r.p;
    const int N = p.N;
    if (p.tree) {
        const int64_t R0 = p.R[0], R1 = p.R[1], s2 = p.s[2], s3 = p.s[3];
        TK_HIP(pair_ttm(G, R0 * R1, (int)s2, (int)s3, U[2], (int)p.R[2], U[3], (int)p.R[3], true, p.T12, r.st));
        int64_t d[3] = {R0, R1, s2 * s3};
        ttm(r, p.T12, d, 3, 1, U[1], p.s[1], true, p.T1);
        d[1] = p.s[1];
        // the last product, the chain's largest, reads U1 through its transpose, kept in p.P (the Gram
        // partials and one-step W products that use p.P are consumed before any reconstruction)
        float* u0t = nullptr;
        if (p.P && p.s[0] * R0 <= 2 * p.P_elems) {
            u0t = reinterpret_cast<float*>(p.P);
            TK_HIP(transpose_f32(U[0], p.s[0], R0, u0t, r.st));
        }
        if (Xref) {
            int64_t nb = 0;
            ttm(r, p.T1, d, 3, 0, U[0], p.s[0], true, nullptr, Xref, &nb, u0t);
            TK_HIP(reduce_f64(p.rpart, nb, p.scal + 2, r.st));
        } else {
            ttm(r, p.T1, d, 3, 0, U[0], p.s[0], true, out, nullptr, nullptr, u0t);
        }
        return;
    }
    int64_t d[TUCKER_MAX_ORDER];
    for (int i = 0; i < N; ++i) d[i] = p.R[i];
    float* bufs[2] = {p.Ya, p.Yb};
    const float* cur = G;
    int w = 0;
    const bool fuse = Xref && p.Xh == nullptr;
    for (int m = N - 1; m >= 0; --m) {
        if (m == 0 && fuse) {
            int64_t nb = 0;
            ttm(r, cur, d, N, 0, U[0], p.s[0], true, nullptr, Xref, &nb);
            TK_HIP(reduce_f64(p.rpart, nb, p.scal + 2, r.st));
            return;
        }
        float* dst = (m == 0) ? (Xref ? p.Xh : out) : bufs[w];
        ttm(r, cur, d, N, m, U[m], p.s[m], true, dst);
        d[m] = p.s[m];
        cur = dst;
        w ^= 1;
    }
    if (Xref) {
        TK_HIP(tk_resid_sumsq(Xref, p.Xh, prod(p.s, 0, N), p.red, kSumsqBlocks, p.scal + 2, r.st));
    }
}

// ------------------------------------------------------------------ validation
tucker_status validate_args(int ndim, const int64_t* dims, const int64_t* ranks, int max_iters, double tol,
                            std::string& why) {
    if (!dims || !ranks) {
        why = "dims/ranks is NULL";
        return TUCKER_ERR_INVALID_ARG;
    }
    if (ndim < 2 || ndim > TUCKER_MAX_ORDER) {
        why = "ndim must be in [2, 8]";
        return TUCKER_ERR_INVALID_ARG;
    }
    long double total_r = 1;
    int64_t total = 1;
    for (int n = 0; n < ndim; ++n) {
        if (dims[n] < 1) {
            why = "dims must be >= 1";
            return TUCKER_ERR_INVALID_ARG;
        }
        if (ranks[n] < 1 || ranks[n] > dims[n]) {
            why = "ranks must be in [1, dims]";
            return TUCKER_ERR_INVALID_ARG;
        }
        if (total > (int64_t(1) << 40) / dims[n]) {
            why = "tensor too large";
            return TUCKER_ERR_INVALID_ARG;
        }
        total *= dims[n];
        total_r *= (long double)ranks[n];
    }
    for (int n = 0; n < ndim; ++n) {
        if ((long double)ranks[n] * ranks[n] > total_r) {
            why = "ranks[n] exceeds the product of the other ranks";
            return TUCKER_ERR_INVALID_ARG;
        }
    }
    if (max_iters < 0) {
        why = "max_iters must be >= 0";
        return TUCKER_ERR_INVALID_ARG;
    }
    if (!(tol >= 0.0)) {
        why = "tol must be >= 0 and not NaN";
        return TUCKER_ERR_INVALID_ARG;
    }
    return TUCKER_OK;
}

void make_plan(Plan& p, int ndim, const int64_t* dims, const int64_t* ranks, int max_iters, int prec = 0,
               int refine = 0, bool pp = false, int oversample = 0) {
    p.N = ndim;
    p.max_iters = max_iters;
    p.refine = prec ? refine : 0;
    for (int n = 0; n < ndim; ++n) {
        p.s[n] = dims[n];
        p.R[n] = ranks[n];
        p.kind[n] = (ranks[n] == dims[n]) ? FIXED : (dims[n] <= kSmallMode ? SMALL : LARGE);
        p.Rc[n] = p.kind[n] == LARGE ? std::min<int64_t>(dims[n], ranks[n] + std::max(0, oversample)) : ranks[n];
        if (p.Rc[n] > p.R[n] && p.Rc[n] > kRitzMaxOrder)
            throw Fail{TUCKER_ERR_UNSUPPORTED, "oversampled start: min(s_n, R_n + oversample) exceeds 1024"};
    }
    p.tree = (ndim == 4) && pair_ttm_supported((int)dims[2], (int)dims[3]) && dims[2] * dims[3] <= 64;
    p.prec = prec;
    p.ip = (prec == TUCKER_FP8_E4M3) ? TUCKER_BF16 : prec;
    if (prec != 0 && !(p.tree && p.kind[0] == LARGE && p.kind[1] == LARGE))
        throw Fail{TUCKER_ERR_UNSUPPORTED,
                   "reduced precision needs an order-4 tensor with two large leading modes and small trailing ones"};
    p.pp = pp;
    if (pp && !(p.tree && prec == 0 && p.kind[0] == LARGE && p.kind[1] == LARGE && p.kind[2] == FIXED))
        throw Fail{TUCKER_ERR_UNSUPPORTED,
                   "pairwise perturbation needs FP32 sweeps of an order-4 stack with two large leading modes, a "
                   "full-rank third mode and a small fourth one"};
}

size_t plan_bytes(Plan& p) {
    Arena a;
    build_plan(p, a);
    return a.off + 256;
}

void ensure_ws(tucker_ctx* ctx, size_t bytes) {
    if (ctx->opt.hbm_budget_bytes && bytes > ctx->opt.hbm_budget_bytes)
        throw Fail{TUCKER_ERR_OUT_OF_MEMORY, "workspace exceeds hbm_budget_bytes"};
    if (bytes <= ctx->ws_bytes) return;
    if (ctx->ws) {
        if (ctx->async_alloc) {
            TK_HIP(hipFreeAsync(ctx->ws, ctx->stream));
        } else {
            TK_HIP(hipStreamSynchronize(ctx->stream));
            (void)hipFree(ctx->ws);
        }
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    hipError_t e = ctx->async_alloc ? hipMallocAsync(&ctx->ws, bytes, ctx->stream) : hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        throw Fail{TUCKER_ERR_OUT_OF_MEMORY, std::string("hipMalloc workspace: ") + hipGetErrorString(e)};
    }
    ctx->ws_bytes = bytes;
    ctx->stats.workspace_bytes = bytes;
}

void bind(tucker_ctx* ctx, Plan& p) {
    const size_t need = plan_bytes(p);
    ensure_ws(ctx, need);
    Arena a;
    a.base = (char*)ctx->ws;
    a.cap = ctx->ws_bytes;
    build_plan(p, a);
}

}  // namespace

// captured sweep graph: released after the stream has drained
struct GraphHold {
    hipStream_t s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphHold() {
        if (exec || graph) (void)hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// helpers defined in this TU but called through extern declarations above
namespace {
__global__ void set_int_kernel(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
__global__ void fit_push_kernel(const double* __restrict__ src, int* counter, double* __restrict__ fits) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int k = *counter;
        fits[k] = *src;
        *counter = k + 1;
    }
}
template <typename TO, typename TP = double>
__global__ void sum_splits_kernel(const TP* __restrict__ P, int nsplit, int64_t n, int64_t zstride,
                                  TO* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        int z = 0;
        for (; z + 4 <= nsplit; z += 4) {     // four loads in flight, summed in split order
            const double a0 = P[(int64_t)z * zstride + e], a1 = P[(int64_t)(z + 1) * zstride + e];
            const double a2 = P[(int64_t)(z + 2) * zstride + e], a3 = P[(int64_t)(z + 3) * zstride + e];
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; z < nsplit; ++z) s += (double)P[(int64_t)z * zstride + e];
        out[e] = (TO)s;
    }
}
__global__ void resid_kernel(const float* __restrict__ X, const float* __restrict__ Xh, int64_t n,
                             double* __restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)X[i] - (double)Xh[i];
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
__global__ void diff_sumsq64_kernel(const double* __restrict__ A, const double* __restrict__ B, int64_t n,
                                    double* __restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = A[i] - B[i];
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
}  // namespace

hipError_t tk_set_int(int* p, int v, hipStream_t s) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}
hipError_t tk_fit_push(const double* src, int* counter, double* fits, hipStream_t s) {
    hipLaunchKernelGGL(fit_push_kernel, dim3(1), dim3(64), 0, s, src, counter, fits);
    return hipGetLastError();
}

hipError_t tk_sum_splits_f64(const double* P, int nsplit, int64_t n, int64_t zstride, double* out, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    g = std::max<int64_t>(1, std::min<int64_t>(g, 4096));
    hipLaunchKernelGGL(sum_splits_kernel<double>, dim3((unsigned)g), dim3(256), 0, s, P, nsplit, n, zstride, out);
    return hipGetLastError();
}
// the same FP64 sum, rounded once to FP32
hipError_t tk_sum_splits_to_f32(const double* P, int nsplit, int64_t n, int64_t zstride, float* out, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    g = std::max<int64_t>(1, std::min<int64_t>(g, 4096));
    hipLaunchKernelGGL(sum_splits_kernel<float>, dim3((unsigned)g), dim3(256), 0, s, P, nsplit, n, zstride, out);
    return hipGetLastError();
}
// FP32 partials summed in FP64 in split order, stored as TO
template <typename TO>
hipError_t tk_sum_splits_f32p(const float* P, int nsplit, int64_t n, int64_t zstride, TO* out, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    g = std::max<int64_t>(1, std::min<int64_t>(g, 4096));
    hipLaunchKernelGGL((sum_splits_kernel<TO, float>), dim3((unsigned)g), dim3(256), 0, s, P, nsplit, n, zstride, out);
    return hipGetLastError();
}
template hipError_t tk_sum_splits_f32p<float>(const float*, int, int64_t, int64_t, float*, hipStream_t);
template hipError_t tk_sum_splits_f32p<double>(const float*, int, int64_t, int64_t, double*, hipStream_t);
hipError_t tk_resid_sumsq(const float* X, const float* Xh, int64_t n, double* partial, int nblocks, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3(nblocks), dim3(256), 0, s, X, Xh, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_f64(partial, nblocks, out, s);
}

hipError_t tk_diff_sumsq_f64(const double* A, const double* B, int64_t n, double* partial, int nblocks, double* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(diff_sumsq64_kernel, dim3(nblocks), dim3(256), 0, s, A, B, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_f64(partial, nblocks, out, s);
}

// ======================================================================================
// C ABI
// ======================================================================================
namespace {

template <typename Fn>
tucker_status guarded(tucker_ctx* ctx, Fn fn) {
    try {
        TK_HIP(hipSetDevice(ctx->device));
        fn();
        return TUCKER_OK;
    } catch (const Fail& f) {
        ctx->err = f.msg;
        (void)hipGetLastError();
        return f.st;
    } catch (const std::exception& e) {
        ctx->err = e.what();
        return TUCKER_ERR_DEVICE;
    }
}

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return (double)ms;
}

// scratch arena for the step-level entry points
template <typename Fn>
void with_scratch(tucker_ctx* ctx, Fn layout) {
    Arena a;
    layout(a);
    ensure_ws(ctx, a.off + 256);
    Arena b;
    b.base = (char*)ctx->ws;
    b.cap = ctx->ws_bytes;
    layout(b);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Looks up this device's copy of `scratch` once (the device must be current).
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<char*>(ptr);
    return hipSuccess;
}

// After a step-level call that ran the Cholesky task graph: synchronise, record the pivot shifts and
// timed-out waits (int counters as laid out by chol_inv_scaled) and fail when a wait gave up.
void check_chol_calls(tucker_ctx* ctx, const int* shifts, hipStream_t s) {
    int h[8] = {};
    TK_HIP(hipMemcpyAsync(h, shifts, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    ctx->stats.chol_shifts = h[0];
    ctx->stats.wait_timeouts = h[kWaitTimeoutSlot];
    if (h[kWaitTimeoutSlot])
        throw Fail{TUCKER_ERR_DEVICE, "Cholesky task graph: a wait gave up (wait_spin_limit reached); the result is "
                                      "invalid"};
}

}  // namespace

extern "C" {

void tucker_default_options(tucker_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->precision = TUCKER_FP32;
    o->refine_sweeps = 1;
    o->inner_iters = 1;
    o->init_iters = 20;
    o->inner_tol = 0.0;
    o->use_graphs = 0;
    o->hbm_budget_bytes = 0;
    o->seed = 0x5eedull;
}

tucker_status tucker_validate(int ndim, const int64_t* dims, const int64_t* ranks, int max_iters, double tol) {
    std::string why;
    return validate_args(ndim, dims, ranks, max_iters, tol, why);
}

tucker_status tucker_workspace_size(int ndim, const int64_t* dims, const int64_t* ranks, tucker_precision precision,
                                    size_t* bytes) {
    std::string why;
    tucker_status st = validate_args(ndim, dims, ranks, 0, 0.0, why);
    if (st != TUCKER_OK) return st;
    if (!bytes || precision < TUCKER_FP32 || precision > TUCKER_FP8_E4M3) return TUCKER_ERR_INVALID_ARG;
    try {
        Plan p;
        make_plan(p, ndim, dims, ranks, 0, (int)precision, 1);
        *bytes = plan_bytes(p);
    } catch (const Fail& f) {
        return f.st;
    }
    return TUCKER_OK;
}

tucker_status tucker_create(const tucker_options* opts, tucker_ctx** out) {
    if (!out) return TUCKER_ERR_INVALID_ARG;
    *out = nullptr;
    tucker_options o;
    tucker_default_options(&o);
    if (opts) o = *opts;
    if (o.inner_iters < 1 || o.init_iters < 1 || o.refine_sweeps < 0 || o.precision < TUCKER_FP32 ||
        o.precision > TUCKER_FP8_E4M3 || o.device < 0 || !(o.inner_tol >= 0.0) || o.wait_spin_limit < 0 ||
        !(o.pp_tol >= 0.0) || o.oversample < 0 ||
        (o.start != TUCKER_START_THOSVD && o.start != TUCKER_START_STHOSVD))
        return TUCKER_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return TUCKER_ERR_DEVICE;
    }
    if (o.device >= count) return TUCKER_ERR_DEVICE;
    if (hipSetDevice(o.device) != hipSuccess) {
        (void)hipGetLastError();
        return TUCKER_ERR_DEVICE;
    }
    tucker_ctx* c = new tucker_ctx();
    c->device = o.device;
    c->opt = o;
    // NULL selects the device's default (null) stream, which orders with other default-stream
    // work such as a framework's copies.
    c->stream = (hipStream_t)o.stream;
    c->own_stream = false;
    for (auto& e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            tucker_destroy(c);
            return TUCKER_ERR_DEVICE;
        }
    }
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess || noalloc_setup(o.device) != hipSuccess) {
        (void)hipGetLastError();
        tucker_destroy(c);
        return TUCKER_ERR_DEVICE;
    }
    *out = c;
    return TUCKER_OK;
}

tucker_status tucker_destroy(tucker_ctx* ctx) {
    if (!ctx) return TUCKER_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->ws && ctx->async_alloc) (void)hipFreeAsync(ctx->ws, ctx->stream);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws && !ctx->async_alloc) (void)hipFree(ctx->ws);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    for (auto& e : ctx->eig_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->eig_host) (void)hipHostFree(ctx->eig_host);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return TUCKER_OK;
}

tucker_status tucker_decompose_ex(tucker_ctx* ctx, const float* tensor, int ndim, const int64_t* dims,
                                  const int64_t* ranks, int max_iters, double tol,
                                  const float* const* init_factors, float* core, float* const* factors,
                                  double* fit, double* fit_history, int* sweeps_done) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    ctx->err.clear();
    std::string why;
    tucker_status st = validate_args(ndim, dims, ranks, max_iters, tol, why);
    if (st != TUCKER_OK) {
        ctx->err = why;
        return st;
    }
    if (!tensor || !core || !factors || !fit) {
        ctx->err = "NULL tensor/core/factors/fit";
        return TUCKER_ERR_INVALID_ARG;
    }
    for (int n = 0; n < ndim; ++n) {
        if (!factors[n] || (init_factors && !init_factors[n])) {
            ctx->err = "NULL factor pointer";
            return TUCKER_ERR_INVALID_ARG;
        }
    }
    return guarded(ctx, [&]() {
        TuneScope tune(ctx->opt.autotune != 0);
        Run r{ctx, Plan{}, ctx->stream, tensor};
        Plan& p = r.p;
        ctx->stats = tucker_stats{};
        if (ctx->opt.pp_tol > 0.0 && tol > 0.0)
            throw Fail{TUCKER_ERR_UNSUPPORTED, "pairwise perturbation runs a fixed number of sweeps (tol = 0)"};
        make_plan(p, ndim, dims, ranks, max_iters, (int)ctx->opt.precision, ctx->opt.refine_sweeps,
                  ctx->opt.pp_tol > 0.0, init_factors ? 0 : ctx->opt.oversample);
        bind(ctx, p);
        const hipStream_t s = r.st;
        reset_counters(r);
        TK_HIP(hipEventRecord(ctx->ev[0], s));
        const int64_t Xn = prod(p.s, 0, p.N);
        TK_HIP(sumsq_f32(tensor, Xn, p.red, kSumsqBlocks, p.scal + 0, s));
        double nx2 = 0.0;
        TK_HIP(hipMemcpyAsync(&nx2, p.scal + 0, sizeof(double), hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        if (!std::isfinite(nx2)) throw Fail{TUCKER_ERR_NUMERICAL, "||X||^2 is not finite"};
        if (nx2 == 0.0) {
            TK_HIP(fill_zero(core, prod(p.R, 0, p.N) * (int64_t)sizeof(float), s));
            for (int n = 0; n < p.N; ++n) TK_HIP(fill_identity_f32(factors[n], p.s[n], p.R[n], s));
            TK_HIP(hipStreamSynchronize(s));
            *fit = 1.0;
            if (fit_history) fit_history[0] = 1.0;
            if (sweeps_done) *sweeps_done = 0;
            ctx->stats = tucker_stats{};
            ctx->stats.workspace_bytes = ctx->ws_bytes;
            return;
        }
        if (init_factors) {
            for (int n = 0; n < p.N; ++n) {
                TK_HIP(hipMemcpyAsync(p.U32[n], init_factors[n], p.s[n] * p.R[n] * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
                TK_HIP(f32_to_f64(p.U32[n], p.U64[n], p.s[n] * p.R[n], s));
            }
        } else if (ctx->opt.start == TUCKER_START_STHOSVD) {
            sthosvd(r);
        } else {
            thosvd(r);
        }
        // per-sweep fit: ||X||^2 - ||G||^2 (cheap; with the FP32 core its error is amplified by the
        // cancellation, about 3e-5 at 1080p), or, when a tolerance decides the stop, the explicit
        // residual ||X - Xhat|| (one more expanding pass per sweep)
        const bool exact_fits = tol > 0.0;
        auto sweep_fit = [&](double* slot) {
            if (exact_fits) {
                expand_chain(r, p.G, p.U32, nullptr, tensor);
                TK_HIP(fit_from_resid(p.scal + 0, p.scal + 2, slot, s));
            } else {
                core_norm_and_fit(r, slot);
            }
        };
        const bool graphs = ctx->opt.use_graphs && s != nullptr && !ctx->opt.timing && !(tol > 0.0) && max_iters > 0 &&
                            !(r.inner_tol() > 0.0) && !p.pp;
        // The start's core is needed only for its fit when sweeps follow.  In an FP32 tree sweep the
        // first mode-1 update forms W = Y0 x_1 U1^T from the start's factors, which is that core, so the
        // start's fit is taken from W there instead of from two more products over X (ST-HOSVD ends with
        // its core anyway).
        const bool fit0_from_w = max_iters > 0 && p.prec == 0 && p.tree && !exact_fits &&
                                 p.kind[0] != FIXED && direct_update_ok(r, 0) &&
                                 (init_factors || ctx->opt.start != TUCKER_START_STHOSVD);
        if (fit0_from_w) {
            r.fit0_slot = p.fits + 0;
        } else {
            if (init_factors || ctx->opt.start != TUCKER_START_STHOSVD) core_from_x(r);   // (ST-HOSVD ends with G)
            sweep_fit(p.fits + 0);
        }
        TK_HIP(hipEventRecord(ctx->ev[1], s));
        int done = 0;
        std::vector<double> hf(2);
        if (p.prec != 0) {
            lp_convert_x(r);
            r.orth_tol = kOrthTolLowp;
        }
        auto one_sweep = [&]() {
            if (p.prec != 0)
                sweep_tree_lp(r);
            else if (p.tree)
                sweep_tree(r);
            else
                sweep_generic(r);
        };
        // Graph replay: the first sweep runs on the stream directly (in an FP32 tree sweep it also
        // leaves the start's fit); the next sweep (and its fit) is captured from the stream once and
        // replayed for sweeps 2 .. max_iters; every node reads and writes the same workspace each
        // sweep, and the fit lands in fits[k] through a device-side counter.  Needs a capturable
        // (non-null) stream, no per-sweep host read (tol = 0) and no stage timers.
        GraphHold hold{s};
        if (graphs) {
            one_sweep();
            sweep_fit(p.fits + 1);
            if (max_iters > 1) {
                TK_HIP(tk_set_int(p.shifts + 3, 2, s));
                TK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
                try {
                    one_sweep();
                    core_norm_and_fit(r, p.scal + 4);
                    TK_HIP(tk_fit_push(p.scal + 4, p.shifts + 3, p.fits, s));
                } catch (...) {
                    hipGraph_t g2 = nullptr;
                    (void)hipStreamEndCapture(s, &g2);
                    if (g2) (void)hipGraphDestroy(g2);
                    (void)hipGetLastError();
                    throw;
                }
                TK_HIP(hipStreamEndCapture(s, &hold.graph));
                TK_HIP(hipGraphInstantiate(&hold.exec, hold.graph, nullptr, nullptr, 0));
                for (int k = 2; k <= max_iters; ++k) TK_HIP(hipGraphLaunch(hold.exec, s));
            }
            done = max_iters;
        }
        // pairwise perturbation: ordinary sweeps until the factors settle, then perturbation sweeps
        // around the reference point while they stay near it (switching on the subspace distance)
        bool pp_mode = false, last_pp = false;
        int pp_sweeps = 0, pp_refs = 0;
        for (int k = 1; k <= max_iters && !graphs; ++k) {
            if (p.pp && !pp_mode)
                for (int n = 0; n < p.N; ++n)
                    TK_HIP(hipMemcpyAsync(p.U64prev[n], p.U64[n], p.s[n] * p.R[n] * sizeof(double),
                                          hipMemcpyDeviceToDevice, s));
            if (pp_mode)
                pp_sweep(r);
            else
                one_sweep();
            sweep_fit(p.fits + k);
            last_pp = pp_mode;
            if (p.pp && k < max_iters) {
                if (pp_mode) {
                    ++pp_sweeps;
                    if (pp_distance(r, true) > ctx->opt.pp_tol) pp_mode = false;
                } else if (pp_distance(r, false) < ctx->opt.pp_tol) {
                    pp_init(r);
                    pp_mode = true;
                    ++pp_refs;
                }
            } else if (pp_mode) {
                ++pp_sweeps;
            }
            done = k;
            if (tol > 0.0) {
                TK_HIP(hipMemcpyAsync(hf.data(), p.fits + k - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
                TK_HIP(hipStreamSynchronize(s));
                if (std::fabs(hf[1] - hf[0]) < tol) break;
            }
        }
        // FP32 refinement sweeps after reduced-precision ones, warm-started from their factors; each
        // large-mode update iterates to the leading subspace of its FP32 Gram (kRefineInner steps),
        // since the warm start carries the reduced-precision error
        r.inner_override = kRefineInner;
        r.orth_tol = kOrthTol;
        for (int k = 1; k <= p.refine; ++k) {
            sweep_tree(r);
            core_norm_and_fit(r, p.fits + done + k);
        }
        r.inner_override = 0;
        if (last_pp) core_from_x(r);     // the returned core is exact, not the first-order one
        ctx->stats.pp_sweeps = pp_sweeps;
        ctx->stats.pp_refs = pp_refs;
        TK_HIP(hipEventRecord(ctx->ev[2], s));
        expand_chain(r, p.G, p.U32, nullptr, tensor);
        TK_HIP(fit_from_resid(p.scal + 0, p.scal + 2, p.scal + 3, s));
        TK_HIP(hipMemcpyAsync(core, p.G, prod(p.R, 0, p.N) * sizeof(float), hipMemcpyDeviceToDevice, s));
        for (int n = 0; n < p.N; ++n)
            TK_HIP(hipMemcpyAsync(factors[n], p.U32[n], p.s[n] * p.R[n] * sizeof(float), hipMemcpyDeviceToDevice, s));
        TK_HIP(hipEventRecord(ctx->ev[3], s));
        const int total = done + p.refine;
        std::vector<double> fits(total + 1);
        double fexact = 0.0;
        TK_HIP(hipMemcpyAsync(fits.data(), p.fits, (total + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        TK_HIP(hipMemcpyAsync(&fexact, p.scal + 3, sizeof(double), hipMemcpyDeviceToHost, s));
        int shifts2[8] = {}, shifts3[8] = {};
        TK_HIP(hipMemcpyAsync(shifts2, p.shifts, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        if (p.has_alt) TK_HIP(hipMemcpyAsync(shifts3, p.shiftsb, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        ctx->stats.wait_timeouts = shifts2[kWaitTimeoutSlot] + shifts3[kWaitTimeoutSlot];
        if (ctx->stats.wait_timeouts)
            throw Fail{TUCKER_ERR_DEVICE, "Cholesky task graph: a wait gave up in " +
                                              std::to_string(ctx->stats.wait_timeouts) +
                                              " call(s) (wait_spin_limit reached); the factors are invalid"};
        *fit = fexact;
        if (fit_history)
            for (int k = 0; k <= done; ++k) fit_history[k] = fits[k];
        if (sweeps_done) *sweeps_done = done;
        for (int i = 0; i < TUCKER_NUM_STAGES; ++i) {
            ctx->stats.stage_ms[i] = 0.0;
            ctx->stats.stage_calls[i] = 0;
        }
        for (const auto& m : r.marks) {
            ctx->stats.stage_ms[m.stage] += elapsed(ctx->pool[m.b], ctx->pool[m.e]);
            ctx->stats.stage_calls[m.stage] += 1;
        }
        ctx->stats.init_ms = elapsed(ctx->ev[0], ctx->ev[1]);
        ctx->stats.sweeps_ms = elapsed(ctx->ev[1], ctx->ev[2]);
        ctx->stats.final_fit_ms = elapsed(ctx->ev[2], ctx->ev[3]);
        ctx->stats.fit_gram = fits[total];
        ctx->stats.sweeps = done;
        ctx->stats.refine_sweeps = p.refine;
        ctx->stats.chol_shifts = shifts2[0] + shifts3[0];
        ctx->stats.orth_second_passes = shifts2[1] + shifts3[1];
        ctx->stats.oi_steps_init = r.oi_steps_init;
        ctx->stats.oi_steps_sweeps = r.oi_steps_sweeps;
        ctx->stats.oi_residual_max = r.oi_resid_max;
        ctx->stats.rr_sweeps = r.rr_sweeps;
        ctx->stats.workspace_bytes = ctx->ws_bytes;
        if (!std::isfinite(fexact)) throw Fail{TUCKER_ERR_NUMERICAL, "non-finite fit"};
    });
}

tucker_status tucker_decompose(tucker_ctx* ctx, const float* tensor, int ndim, const int64_t* dims,
                               const int64_t* ranks, int max_iters, double tol, float* core, float* const* factors,
                               double* fit, int* sweeps_done) {
    return tucker_decompose_ex(ctx, tensor, ndim, dims, ranks, max_iters, tol, nullptr, core, factors, fit, nullptr,
                               sweeps_done);
}

tucker_status tucker_reconstruct(tucker_ctx* ctx, const float* core, const float* const* factors, int ndim,
                                 const int64_t* dims, const int64_t* ranks, float* out) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    ctx->err.clear();
    std::string why;
    tucker_status st = validate_args(ndim, dims, ranks, 0, 0.0, why);
    if (st != TUCKER_OK) {
        ctx->err = why;
        return st;
    }
    if (!core || !factors || !out) return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (!factors[n]) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        TuneScope tune(ctx->opt.autotune != 0);
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        make_plan(r.p, ndim, dims, ranks, 0);
        bind(ctx, r.p);
        float* U[TUCKER_MAX_ORDER];
        for (int n = 0; n < ndim; ++n) U[n] = const_cast<float*>(factors[n]);
        expand_chain(r, core, U, out, nullptr);
    });
}

tucker_status tucker_order_core(tucker_ctx* ctx, const float* core, const float* const* factors, int ndim,
                                const int64_t* dims, const int64_t* ranks, float* core_out, float* const* factors_out,
                                double* sigma) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    ctx->err.clear();
    std::string why;
    tucker_status st = validate_args(ndim, dims, ranks, 0, 0.0, why);
    if (st != TUCKER_OK) {
        ctx->err = why;
        return st;
    }
    if (!core || !factors || !core_out || !factors_out) return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n) {
        if (!factors[n] || !factors_out[n]) return TUCKER_ERR_INVALID_ARG;
        if (ranks[n] > 1024) {
            ctx->err = "tucker_order_core: ranks above 1024 are not supported";
            return TUCKER_ERR_UNSUPPORTED;
        }
    }
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        Plan& p = r.p;
        const int N = ndim;
        const int64_t G = prod(ranks, 0, N);
        int64_t rmax = 1, rsum = 0, work = 1, pmax = 1;
        for (int n = 0; n < N; ++n) {
            rmax = std::max(rmax, ranks[n]);
            rsum += ranks[n];
            if (ranks[n] > kSmallMode) {
                work = std::max<int64_t>(work, sym_eig_work_doubles((int)ranks[n]));
                pmax = std::max<int64_t>(pmax, (int64_t)gram_splits(ranks[n], G / ranks[n]) * ranks[n] * ranks[n]);
            }
        }
        double *V64 = nullptr, *lam = nullptr, *ework = nullptr;
        float *V32 = nullptr, *buf0 = nullptr, *buf1 = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            p.Fpart = a.take<double>(64 * 64 * 64);
            p.S64_elems = rmax * rmax;
            p.S64 = a.take<double>(p.S64_elems);
            p.P_elems = pmax;
            p.P = a.take<double>(pmax);
            V64 = a.take<double>(rmax * rmax * N);
            V32 = a.take<float>(rmax * rmax * N);
            lam = a.take<double>(rsum);
            ework = a.take<double>(work);
            buf0 = a.take<float>(G);
            buf1 = a.take<float>(G);
        });
        // the rotation of every mode comes from the original core: rotating mode m leaves the Gram of
        // every other mode unchanged (it multiplies that unfolding by an orthogonal matrix on the right)
        int64_t loff = 0;
        for (int n = 0; n < N; ++n) {
            const int64_t R = ranks[n];
            gram(r, core, ranks, N, n);
            double* Vn = V64 + rmax * rmax * n;
            float* Vn32 = V32 + rmax * rmax * n;
            if (R <= kSmallMode) {
                TK_HIP(jacobi_eig(p.S64, (int)R, (int)R, Vn, Vn32, lam + loff, r.st));
            } else {
                TK_HIP(sym_eig_blocked(p.S64, (int)R, (int)R, lam + loff, Vn, Vn32, ework, r.st));
            }
            // U_n V_n: FP32 factor times the FP64 rotation, FP64 accumulation, rounded once
            GemmArgs g{};
            g.alpha = 1.0;
            g.M = dims[n];
            g.N = R;
            g.K = R;
            g.a = plain(factors[n], R);     // A(m, k) = U[m][k]
            g.b = plain(Vn, R);             // B(k, n) = V[k][n]
            g.c = plain(factors_out[n], R);
            g.c_f32 = 1;
            TK_HIP(gemm_f64(g, MK, KM, EPI_STORE, true, false, r.st));
            loff += R;
        }
        if (sigma) TK_HIP(sqrt_clamp(lam, rsum, sigma, r.st));
        // G <- G x_1 V_1^T ... x_N V_N^T
        int64_t d[TUCKER_MAX_ORDER];
        for (int n = 0; n < N; ++n) d[n] = ranks[n];
        const float* cur = core;
        float* bufs[2] = {buf0, buf1};
        for (int n = 0; n < N; ++n) {
            float* dst = (n == N - 1) ? core_out : bufs[n & 1];
            ttm(r, cur, d, N, n, V32 + rmax * rmax * n, ranks[n], false, dst);
            cur = dst;
        }
    });
}

tucker_status tucker_quantize_core(tucker_ctx* ctx, const float* core, int ndim, const int64_t* ranks,
                                   const int64_t* keep, int bits, int32_t* codes, float* dequantized, float* step) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!core || !ranks || !keep || !codes || !dequantized || !step || ndim < 1 || ndim > TUCKER_MAX_ORDER ||
        bits < 2 || bits > 24)
        return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (ranks[n] < 1 || keep[n] < 1 || keep[n] > ranks[n]) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        const int64_t total = prod(keep, 0, ndim);
        float *blk = nullptr, *scal = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            blk = a.take<float>(total);
            scal = a.take<float>(2);
        });
        TK_HIP(gather_block(core, ndim, ranks, keep, blk, ctx->stream));
        TK_HIP(quantize_uniform(blk, total, bits, scal, codes, dequantized, scal + 1, ctx->stream));
        TK_HIP(hipMemcpyAsync(step, scal + 1, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        TK_HIP(hipStreamSynchronize(ctx->stream));
    });
}

tucker_status tucker_ttm(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims, int mode, const float* U,
                         int64_t rnew, float* out) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!in || !dims || !U || !out || ndim < 1 || ndim > TUCKER_MAX_ORDER || mode < 0 || mode >= ndim || rnew < 1)
        return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (dims[n] < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        ttm(r, in, dims, ndim, mode, U, rnew, false, out);
    });
}

tucker_status tucker_gram(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims, int mode, float* out) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!in || !dims || !out || ndim < 1 || ndim > TUCKER_MAX_ORDER || mode < 0 || mode >= ndim)
        return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (dims[n] < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        Plan& p = r.p;
        const int64_t sdim = dims[mode];
        const int64_t K = prod(dims, 0, ndim) / sdim;
        with_scratch(ctx, [&](Arena& a) {
            p.Fpart = a.take<double>(64 * 64 * 64);
            p.S64 = a.take<double>(sdim * sdim);
            p.S64_elems = sdim * sdim;
            p.P_elems = (int64_t)gram_splits(sdim, K) * sdim * sdim;
            p.P = a.take<double>(sdim > kSmallMode ? p.P_elems : 1);
        });
        gram(r, in, dims, ndim, mode);
        TK_HIP(f64_to_f32(p.S64, out, sdim * sdim, r.st));
    });
}

tucker_status tucker_quantize(tucker_ctx* ctx, const float* x, int64_t rows, int64_t L, tucker_precision precision,
                              float* out, float* scales) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!x || !out || rows < 0 || L < 1 || L > 256 || precision < TUCKER_BF16 || precision > TUCKER_FP8_E4M3 ||
        (precision == TUCKER_FP8_E4M3 && !scales))
        return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        const int64_t n = rows * L;
        void* q = nullptr;
        float* part = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            q = a.take<uint16_t>(n);
            part = a.take<float>(kLpScaleBlocks * L);
        });
        const float* sc = nullptr;
        if (precision == TUCKER_FP8_E4M3) {
            TK_HIP(slice_scales(x, rows, (int)L, part, kLpScaleBlocks, scales, r.st));
            sc = scales;
        }
        TK_HIP(to_lowp(x, n, (int)precision, (int)L, sc, q, r.st));
        TK_HIP(from_lowp(q, n, (int)precision, (int)L, sc, out, r.st));
    });
}

tucker_status tucker_ttm_lowp(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims, int mode,
                              const float* U, int64_t rnew, tucker_precision precision, float* out) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!in || !dims || !U || !out || ndim < 1 || ndim > TUCKER_MAX_ORDER || mode < 0 || mode >= ndim || rnew < 1 ||
        precision < TUCKER_BF16 || precision > TUCKER_FP8_E4M3)
        return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (dims[n] < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        const int64_t A = prod(dims, 0, mode), K = dims[mode], B = prod(dims, mode + 1, ndim);
        const int64_t Last = dims[ndim - 1], n = A * K * B, Kp = (K + 7) / 8 * 8;
        void *xq = nullptr, *ut = nullptr;
        float *xs = nullptr, *us = nullptr, *part = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            xq = a.take<uint16_t>(n);
            ut = a.take<uint16_t>(rnew * Kp);
            xs = a.take<float>(Last);
            us = a.take<float>(rnew);
            part = a.take<float>(kLpScaleBlocks * Last);
        });
        const bool f8 = precision == TUCKER_FP8_E4M3;
        if (f8 && Last > 256) throw Fail{TUCKER_ERR_UNSUPPORTED, "FP8 slice scales need a last mode <= 256"};
        if (f8) TK_HIP(slice_scales(in, n / Last, (int)Last, part, kLpScaleBlocks, xs, r.st));
        TK_HIP(to_lowp(in, n, (int)precision, (int)Last, f8 ? xs : nullptr, xq, r.st));
        TK_HIP(factor_lowp(U, K, rnew, Kp, (int)precision, f8 ? us : nullptr, ut, r.st));
        // out[a][r][b] = sum_k Ut[r][k] X[a][k][b]: M = r, N = (a, b), B operand rows k
        LpGemmArgs g{};
        g.a = plain(ut, Kp);
        g.b = (B == 1) ? folded(xq, 1, 1, K) : folded(xq, B, B, K * B);
        g.c = (B == 1) ? folded(out, 1, 1, rnew) : folded(out, B, B, rnew * B);
        g.M = rnew;
        g.N = A * B;
        g.K = K;
        g.alpha = 1.0;
        g.sa = f8 ? us : nullptr;
        g.sb = f8 ? xs : nullptr;
        g.sb_mod = Last;
        if (f8 && B % Last != 0 && B != 1)
            throw Fail{TUCKER_ERR_UNSUPPORTED, "FP8 product needs the scaled mode among the kept columns"};
        if (f8 && B == 1) throw Fail{TUCKER_ERR_UNSUPPORTED, "FP8 product over the scaled (last) mode"};
        TK_HIP(gemm_lp(g, (int)precision, KM, LP_F32OUT, r.st));
    });
}

tucker_status tucker_gram_lowp(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims, int mode,
                               tucker_precision precision, float* out) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!in || !dims || !out || ndim < 1 || ndim > TUCKER_MAX_ORDER || mode < 0 || mode >= ndim ||
        (precision != TUCKER_BF16 && precision != TUCKER_FP16))
        return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < ndim; ++n)
        if (dims[n] < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        Plan& p = r.p;
        const int64_t A = prod(dims, 0, mode), sd = dims[mode], B = prod(dims, mode + 1, ndim);
        const int64_t n = A * sd * B, K = A * B;
        void* xq = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            xq = a.take<uint16_t>(n);
            p.S64 = a.take<double>(sd * sd);
            p.Pf_elems = lp_gram_partials(sd, K);
            p.Pf = a.take<float>(p.Pf_elems);
        });
        p.ip = (int)precision;
        TK_HIP(to_lowp(in, n, (int)precision, 1, nullptr, xq, r.st));
        // rows i of the mode, columns (a, b) with b contiguous
        const Desc y = (B == 1) ? folded(xq, 1, 1, sd) : folded(xq, B, B, sd * B);
        lp_gram(r, y, sd, K, -1);
        TK_HIP(f64_to_f32(p.S64, out, sd * sd, r.st));
    });
}

tucker_status tucker_orthonormalize(tucker_ctx* ctx, const float* Z, int64_t rows, int64_t cols, float* Q) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!Z || !Q || cols < 1 || rows < cols) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        Plan& p = r.p;
        double* U64 = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            p.W = a.take<double>(cols * cols);
            p.Wpart_elems = 16 * cols * cols;
            p.Wpart = a.take<double>(p.Wpart_elems);
            p.Tm = a.take<double>(cols * cols);
            p.chol_ws = a.take<int>(chol_counter_ints(cols));
            p.chol_dsc = a.take<double>(cols);
            p.chol_cap = cols;
            p.Q1 = a.take<double>(rows * cols);
            p.shifts = a.take<int>(8);
            p.red = a.take<double>(kSumsqBlocks);
            U64 = a.take<double>(rows * cols);
        });
        reset_counters(r);
        orthonormalize(r, Z, true, rows, cols, U64, Q, true);
        check_chol_calls(ctx, p.shifts, r.st);
    });
}

tucker_status tucker_gram_tn64(tucker_ctx* ctx, const float* Z, int64_t rows, int64_t cols, double* W) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!Z || !W || cols < 1 || rows < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        Run r{ctx, Plan{}, ctx->stream, nullptr};
        Plan& p = r.p;
        with_scratch(ctx, [&](Arena& a) {
            p.Wpart_elems = 16 * cols * cols;
            p.Wpart = a.take<double>(p.Wpart_elems);
        });
        gram_tn64(r, Z, true, rows, cols, W);
    });
}

tucker_status tucker_chol_inv(tucker_ctx* ctx, const double* W, int64_t n, double* T) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!W || !T || n < 1) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        double* Wc = nullptr;
        double* dsc = nullptr;
        int* cw = nullptr;
        int* shifts = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            Wc = a.take<double>(n * n);
            cw = a.take<int>(chol_counter_ints(n));
            dsc = a.take<double>(n);
            shifts = a.take<int>(8);
        });
        TK_HIP(fill_zero(shifts, 8 * sizeof(int), ctx->stream));
        TK_HIP(fill_zero(cw, chol_counter_ints(n) * (int64_t)sizeof(int), ctx->stream));
        TK_HIP(hipMemcpyAsync(Wc, W, n * n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        TK_HIP(chol_inv_scaled(Wc, n, true, 0.0, T, cw, dsc, shifts, ctx->stream, nullptr,
                               (long long)ctx->opt.wait_spin_limit));
        check_chol_calls(ctx, shifts, ctx->stream);
    });
}

tucker_status tucker_chol_inv_noalloc(tucker_ctx* ctx, const double* W, int64_t n, double* T) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!W || !T || n < 1) return TUCKER_ERR_INVALID_ARG;
    if (n > kNoAllocMaxN) {
        ctx->err = "tucker_chol_inv_noalloc: n = " + std::to_string(n) + " exceeds the scratch limit of " +
                   std::to_string(kNoAllocMaxN);
        return TUCKER_ERR_INVALID_ARG;
    }
    return guarded(ctx, [&]() {
        char* base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch[ctx->device] : nullptr;
        if (!base) throw Fail{TUCKER_ERR_DEVICE, "scratch of this device was not set up"};
        double* Wc = reinterpret_cast<double*>(base + kNoAllocW);
        int* cw = reinterpret_cast<int*>(base + kNoAllocCtr);
        double* dsc = reinterpret_cast<double*>(base + kNoAllocDsc);
        int* shifts = reinterpret_cast<int*>(base + kNoAllocShifts);
        // the counters of the task graph and the shift counters start at zero (a fill kernel, so that
        // the enqueued work stays free of memset nodes)
        TK_HIP(fill_zero(shifts, 8 * sizeof(int), ctx->stream));
        TK_HIP(fill_zero(cw, chol_counter_ints(n) * (int64_t)sizeof(int), ctx->stream));
        TK_HIP(hipMemcpyAsync(Wc, W, n * n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        TK_HIP(chol_inv_scaled(Wc, n, true, 0.0, T, cw, dsc, shifts, ctx->stream, nullptr,
                               (long long)ctx->opt.wait_spin_limit));
        check_chol_calls(ctx, shifts, ctx->stream);
    });
}

tucker_status tucker_sym_eig(tucker_ctx* ctx, const float* S, int64_t n, int64_t rr, float* U, double* lam) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!S || !U || n < 1 || n > 1024 || rr < 1 || rr > n) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        double *S64 = nullptr, *U64 = nullptr, *work = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            S64 = a.take<double>(n * n);
            U64 = a.take<double>(n * rr);
            if (n > kSmallMode) work = a.take<double>(sym_eig_work_doubles((int)n));
        });
        TK_HIP(f32_to_f64(S, S64, n * n, ctx->stream));
        if (n <= kSmallMode) {
            TK_HIP(jacobi_eig(S64, (int)n, (int)rr, U64, U, lam, ctx->stream));
        } else {
            int sweeps = 0;
            TK_HIP(sym_eig_blocked(S64, (int)n, (int)rr, lam, nullptr, U, work, ctx->stream, &sweeps));
        }
    });
}

tucker_status tucker_sumsq(tucker_ctx* ctx, const float* x, int64_t n, double* result) {
    if (!ctx) return TUCKER_ERR_INVALID_ARG;
    if (!x || !result || n < 0) return TUCKER_ERR_INVALID_ARG;
    return guarded(ctx, [&]() {
        double *red = nullptr, *out = nullptr;
        with_scratch(ctx, [&](Arena& a) {
            red = a.take<double>(kSumsqBlocks);
            out = a.take<double>(1);
        });
        TK_HIP(sumsq_f32(x, n, red, kSumsqBlocks, out, ctx->stream));
        TK_HIP(hipMemcpyAsync(result, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        TK_HIP(hipStreamSynchronize(ctx->stream));
    });
}

tucker_status tucker_autotune_dump(char* buf, size_t len, size_t* needed) {
    const std::string t = tune_dump();
    if (needed) *needed = t.size() + 1;
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, t.size());
        std::memcpy(buf, t.data(), n);
        buf[n] = '\0';
    }
    return TUCKER_OK;
}

tucker_status tucker_autotune_clear(void) {
    tune_clear();
    return TUCKER_OK;
}

tucker_status tucker_autotune_force(int op, int choice) {
    return tune_force(op, choice) ? TUCKER_OK : TUCKER_ERR_INVALID_ARG;
}

const char* tucker_status_string(tucker_status s) {
    switch (s) {
        case TUCKER_OK: return "ok";
        case TUCKER_ERR_INVALID_ARG: return "invalid argument";
        case TUCKER_ERR_OUT_OF_MEMORY: return "out of device memory";
        case TUCKER_ERR_DEVICE: return "device error";
        case TUCKER_ERR_NUMERICAL: return "numerical error";
        case TUCKER_ERR_UNSUPPORTED: return "unsupported";
        case TUCKER_ERR_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

const char* tucker_last_error(const tucker_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

tucker_status tucker_get_stats(const tucker_ctx* ctx, tucker_stats* out) {
    if (!ctx || !out) return TUCKER_ERR_INVALID_ARG;
    *out = ctx->stats;
    return TUCKER_OK;
}

tucker_status tucker_set_timing(tucker_ctx* ctx, int timing, uint32_t stages) {
    if (!ctx || (timing != 0 && timing != 1)) return TUCKER_ERR_INVALID_ARG;
    ctx->opt.timing = timing;
    ctx->opt.timing_stages = stages;
    return TUCKER_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- hooks for the request server
// (C++ linkage; not part of the public C ABI)
void tk_ctx_set_async_alloc(tucker_ctx* ctx, bool on) { ctx->async_alloc = on; }

void tk_ctx_release_workspace(tucker_ctx* ctx) {
    if (!ctx->ws) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->async_alloc) {
        (void)hipFreeAsync(ctx->ws, ctx->stream);
    } else {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws);
    }
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
}

void tk_ctx_set_graphs(tucker_ctx* ctx, bool on) { ctx->opt.use_graphs = on ? 1 : 0; }

void tk_ctx_set_run_options(tucker_ctx* ctx, tucker_precision precision, int refine_sweeps) {
    ctx->opt.precision = precision;
    ctx->opt.refine_sweeps = refine_sweeps;
}
