// Reduced-precision (BF16 / FP16 / FP8-e4m3) contraction kernels of the HOOI sweep.
#pragma once
#include <condition_variable>
#include <mutex>
#include <vector>

#include "tk_common.h"

namespace tk {

// storage types (numbered as tucker_precision); LP_F32OUT selects a float output
enum { LP_F32OUT = 0, LP_BF16 = 1, LP_F16 = 2, LP_FP8 = 3 };

struct LpGemmArgs {
    Desc a, b, c;
    int64_t M, N, K;
    double alpha;
    int64_t k_split;      // multiple of 64 (or == K)
    int64_t c_zstride;    // element offset between split outputs
    int lower_only;
    const float* sa;      // per-row output scale (nullable)
    const float* sb;      // per-column output scale, index n % sb_mod (nullable)
    int64_t sb_mod;
    int64_t c_valid;      // > 0: columns n with n % c.seg >= c_valid are padding and not written
};

// C = alpha diag(sa) (A B) diag(sb): A k-contiguous (desc rows m, columns k); B n-contiguous
// (ob == KM: desc rows k, columns n) or k-contiguous (ob == MK: desc rows n, columns k).
// Operands in the storage type prec; output float (outp == LP_F32OUT) or BF16/FP16.
// FP8 is provided for ob == KM with a BF16 output (the full-tensor product).
// A group of products of one kind (storage type, B orientation, output type), launched as one
// persistent grid over their work items (tiles x k splits); ctr: two device counters that are zero on
// entry and zero again when the launch has finished (one pair per stream that launches groups).
constexpr int kLpGroupMax = 12;
struct LpGroupArgs {
    LpGemmArgs p[kLpGroupMax];
    int64_t start[kLpGroupMax + 1];   // prefix sums of the products' work items
    int n;
    unsigned* ctr;
};
// work items of one product in a grouped launch: 128 x 128 output tiles (lower-triangle tiles of a
// Gram) times k splits
inline int64_t lp_work_items(const LpGemmArgs& g) {
    const int64_t tilesM = (g.M + 127) / 128;
    const int64_t tilesN = (g.N + 127) / 128;
    const int64_t tiles = g.lower_only ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
    return tiles * ((g.K + g.k_split - 1) / g.k_split);
}
// C_i = A_i B_i for the n (<= kLpGroupMax) products g[0..n-1], all of the given kind; each C_i is bit
// for bit the result gemm_lp gives for g[i] alone.
hipError_t gemm_lp_grouped(const LpGemmArgs* g, int n, int prec, Orient ob, int outp, unsigned* ctr,
                           hipStream_t s);

// Lock-step grouping of the reduced-precision products of several decompositions of one shape
// (served requests admitted together), each running on its own host thread and stream.  A member's
// product call waits until every active member has made its call of the round; the last to arrive
// launches the round's products as grouped persistent grids on the group's stream, after that
// stream has waited for each member's stream, and every member's stream then waits for the grids.
// Each product's result is bit for bit the one it gets alone.  A member that stops calling (done, or
// failed) leaves, so that the others never wait for it.  Thread-local: lp_group_set(g) makes the
// calling thread's products go through g (nullptr: ordinary launches).
class LpGrouper {
  public:
    LpGrouper(int members, int device);
    ~LpGrouper();
    bool ok() const { return ok_; }
    hipError_t gemm(const LpGemmArgs& g, int prec, Orient ob, int outp, hipStream_t member_stream);
    void leave();
    int64_t launches() const { return launches_; }
    int64_t products() const { return products_; }

  private:
    struct Item {
        LpGemmArgs g;
        int prec, outp;
        Orient ob;
    };
    void launch_locked();
    std::mutex mu_;
    std::condition_variable cv_;
    int members_, arrived_ = 0;
    uint64_t gen_ = 0;
    std::vector<Item> items_;
    std::vector<hipEvent_t> in_ev_;
    hipEvent_t done_ev_ = nullptr;
    hipStream_t gs_ = nullptr;
    unsigned* ctr_ = nullptr;
    hipError_t result_ = hipSuccess;
    bool ok_ = false;
    int64_t launches_ = 0, products_ = 0;
};
void lp_group_set(LpGrouper* g);
LpGrouper* lp_group_current();

// Outputs: float, or the 16-bit type of the sweep's intermediates (BF16 for BF16 and FP8 operands,
// FP16 for FP16 operands); other combinations return hipErrorInvalidValue.
hipError_t gemm_lp(const LpGemmArgs& g, int prec, Orient ob, int outp, hipStream_t s);

// k step of the GEMM's tiles (k_split must be a multiple of it or cover all of K)
constexpr int kLpGemmK = 64;
// the per-type instantiations behind gemm_lp (vec: 8-element vector loads are legal)
hipError_t gemm_lp_bf16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_f16(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_fp8(const LpGemmArgs& g, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_grouped_bf16(const LpGroupArgs& a, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_grouped_f16(const LpGroupArgs& a, Orient ob, int outp, bool vec, hipStream_t s);
hipError_t gemm_lp_grouped_fp8(const LpGroupArgs& a, Orient ob, int outp, bool vec, hipStream_t s);

// out[i] = enc(x[i] / scale[i % L]) (scale nullable)
hipError_t to_lowp(const float* x, int64_t n, int prec, int L, const float* scale, void* out, hipStream_t s);
// rows of L floats -> rows of Lp (>= L) BF16/FP16 values, the tail of each row zero
hipError_t to_lowp_padded(const float* x, int64_t rows, int L, int Lp, int prec, void* out, hipStream_t s);
// out[i] = dec(in[i]) * scale[i % L] (scale nullable)
hipError_t from_lowp(const void* in, int64_t n, int prec, int L, const float* scale, float* out, hipStream_t s);
// scale[l] = max_a |x[a][l]| / 448 (1 where the slice is zero); partial: nblocks * L floats
hipError_t slice_scales(const float* x, int64_t A, int L, float* partial, int nblocks, float* scale, hipStream_t s);
// Ut[r][k] = enc(U[k][r] / scale[r]) for k < rows, 0 up to ldk; scale (FP8 only) = amax of column r / 448
hipError_t factor_lowp(const float* U, int64_t rows, int64_t R, int64_t ldk, int prec, float* scale, void* Ut,
                       hipStream_t s);
// out[a][r R4 + t] = sum_{c,i} U3[c][r] U4[i][t] dec(in[a][c q + i]) scale[c q + i], rows of ldo
// 16-bit outp elements, the tail of each row zero.  u3_identity: U3 is the p x p identity (a mode
// kept at full rank), which lets the fixed-shape kernels skip its product.
hipError_t pair_lowp(const void* in, int64_t A, int p, int q, const float* U3, int R3, const float* U4, int R4,
                     int prec, const float* scale, int outp, int ldo, void* out, hipStream_t s,
                     bool u3_identity = false);

}  // namespace tk
