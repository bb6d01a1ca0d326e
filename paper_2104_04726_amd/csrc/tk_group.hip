// Lock-step grouping of reduced-precision products across decompositions (served requests of one
// shape admitted together): the host rendezvous, and the launch of a round's products as grouped
// persistent grids (gemm_lp_grouped) on the group's own stream.
#include <algorithm>

#include "tk_lowp.h"

namespace tk {
namespace {
thread_local LpGrouper* t_group = nullptr;
}  // namespace

void lp_group_set(LpGrouper* g) { t_group = g; }
LpGrouper* lp_group_current() { return t_group; }

LpGrouper::LpGrouper(int members, int device) : members_(members) {
    if (members < 1 || hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    bool good = hipStreamCreateWithFlags(&gs_, hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&done_ev_, hipEventDisableTiming) == hipSuccess &&
                hipMalloc((void**)&ctr_, 2 * sizeof(unsigned)) == hipSuccess &&
                hipMemsetAsync(ctr_, 0, 2 * sizeof(unsigned), gs_) == hipSuccess &&
                hipStreamSynchronize(gs_) == hipSuccess;
    for (int i = 0; good && i < members; ++i) {
        hipEvent_t e = nullptr;
        good = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (good) in_ev_.push_back(e);
    }
    if (!good) (void)hipGetLastError();
    ok_ = good;
}

LpGrouper::~LpGrouper() {
    if (gs_) (void)hipStreamSynchronize(gs_);
    for (hipEvent_t e : in_ev_) (void)hipEventDestroy(e);
    if (done_ev_) (void)hipEventDestroy(done_ev_);
    if (ctr_) (void)hipFree(ctr_);
    if (gs_) (void)hipStreamDestroy(gs_);
    (void)hipGetLastError();
}

// the round's products, grouped by kind in arrival order, at most kLpGroupMax per grid
void LpGrouper::launch_locked() {
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < items_.size() && e == hipSuccess; ++i) e = hipStreamWaitEvent(gs_, in_ev_[i], 0);
    std::vector<bool> used(items_.size(), false);
    for (size_t i = 0; i < items_.size() && e == hipSuccess; ++i) {
        if (used[i]) continue;
        std::vector<LpGemmArgs> batch;
        for (size_t j = i; j < items_.size(); ++j) {
            if (used[j] || items_[j].prec != items_[i].prec || items_[j].ob != items_[i].ob ||
                items_[j].outp != items_[i].outp)
                continue;
            used[j] = true;
            batch.push_back(items_[j].g);
            if ((int)batch.size() == kLpGroupMax) {
                e = gemm_lp_grouped(batch.data(), (int)batch.size(), items_[i].prec, items_[i].ob, items_[i].outp,
                                    ctr_, gs_);
                ++launches_;
                batch.clear();
                if (e != hipSuccess) break;
            }
        }
        if (e == hipSuccess && !batch.empty()) {
            e = gemm_lp_grouped(batch.data(), (int)batch.size(), items_[i].prec, items_[i].ob, items_[i].outp, ctr_,
                                gs_);
            ++launches_;
        }
    }
    products_ += (int64_t)items_.size();
    if (e == hipSuccess) e = hipEventRecord(done_ev_, gs_);
    result_ = e;
    items_.clear();
    arrived_ = 0;
    ++gen_;
    cv_.notify_all();
}

hipError_t LpGrouper::gemm(const LpGemmArgs& g, int prec, Orient ob, int outp, hipStream_t member_stream) {
    if (!ok_) return hipErrorNotReady;
    std::unique_lock<std::mutex> lk(mu_);
    const uint64_t my = gen_;
    hipError_t e = hipEventRecord(in_ev_[arrived_], member_stream);
    if (e != hipSuccess) return e;
    items_.push_back(Item{g, prec, outp, ob});
    ++arrived_;
    if (arrived_ >= members_) launch_locked();
    else cv_.wait(lk, [&] { return gen_ != my; });
    if (result_ != hipSuccess) return result_;
    return hipStreamWaitEvent(member_stream, done_ev_, 0);
}

void LpGrouper::leave() {
    std::lock_guard<std::mutex> lk(mu_);
    if (members_ > 0) --members_;
    if (arrived_ > 0 && arrived_ >= members_) launch_locked();
}

}  // namespace tk
