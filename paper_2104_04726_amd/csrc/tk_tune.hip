// The library's autotuner: launch choices measured on the device on first use and cached.
//
// A choice is keyed by the operation and the shape that determines it (and the device).  The first
// call of a key in the process fixes its choice for the rest of the process: when tuning is on for the
// calling thread (tucker_options.autotune) and the stream is not being captured into a graph, every
// candidate is launched three times on the caller's stream, the last two timed with HIP events (the
// shorter counts), and the fastest is kept unless the heuristic choice is within the operation's tie
// margin of it (near ties, whose order the timing noise decides, then give the same choice in every
// process; the margin is wider where the candidates round differently, so that a process's results
// change only for a clear gain); otherwise the heuristic choice is kept.  Every later call with the
// same key reuses
// it, so within a process a shape's results do not depend on which calls ran before or beside it.
// Candidates of one key must leave identical results or results of one fixed reduction order each,
// and their outputs must be idempotent (stores, not accumulations).  tune_force overrides the choice
// of one operation process-wide (for comparing candidates) without touching the table.
#include <atomic>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "tk_common.h"

namespace tk {
namespace {

using Key = std::tuple<int, int, int64_t, int64_t, int64_t, int64_t, int64_t>;   // op, device, shape...

struct Entry {
    int choice;
    std::vector<double> ms;     // measured time of every candidate (ms)
};

std::mutex g_mu;
std::map<Key, Entry> g_table;
thread_local bool t_enabled = false;
constexpr int kMaxOp = 4;
// the heuristic choice stands unless another is this much faster: 3% for the FP32 tile shape; 10% for
// the Gram split count, whose candidates sum the k ranges in different groupings; 10% for the
// reduced-precision LDS staging, whose isolated timing (the operand still in the last-level cache from
// the warm-up launch) favours the two-stage variant by a few percent, while inside a sweep, with the
// operand coming from HBM, the one-stage variant with more resident workgroups is faster (BF16 pass
// C1 at 1080p: 132 against 151 us)
double tie_margin(int op) { return op == kTuneGramSplit || op == kTuneLpTile ? 0.10 : 0.03; }
std::atomic<int> g_force[kMaxOp] = {-1, -1, -1, -1};

}  // namespace

void tune_set_enabled(bool on) { t_enabled = on; }
bool tune_enabled() { return t_enabled; }

int tune_choose(int op, const int64_t shape[5], int ncand, int heuristic, hipStream_t s,
                const std::function<hipError_t(int)>& launch, hipError_t* err) {
    *err = hipSuccess;
    if (op > 0 && op < kMaxOp) {
        const int f = g_force[op].load(std::memory_order_relaxed);
        if (f >= 0) return f < ncand ? f : ncand - 1;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    const Key key{op, dev, shape[0], shape[1], shape[2], shape[3], shape[4]};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(key);
        if (it != g_table.end()) return it->second.choice;
    }
    auto keep = [&](const Entry& en) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(key);                      // another thread may have fixed it meanwhile
        if (it != g_table.end()) return it->second.choice;
        g_table.emplace(key, en);
        return en.choice;
    };
    bool timed = t_enabled && ncand > 1;
    if (timed) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            timed = false;
        }
    }
    if (!timed) return keep(Entry{heuristic, {}});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return keep(Entry{heuristic, {}});
    }
    Entry en{heuristic, std::vector<double>(ncand, -1.0)};
    double best = 0.0;
    for (int c = 0; c < ncand && *err == hipSuccess; ++c) {
        *err = launch(c);                                   // warm-up (code objects, caches)
        double ms = -1.0;
        for (int rep = 0; rep < 2 && *err == hipSuccess; ++rep) {
            *err = hipEventRecord(e0, s);
            if (*err == hipSuccess) *err = launch(c);
            if (*err == hipSuccess) *err = hipEventRecord(e1, s);
            if (*err == hipSuccess) *err = hipEventSynchronize(e1);
            float t = 0.f;
            if (*err == hipSuccess) *err = hipEventElapsedTime(&t, e0, e1);
            if (*err == hipSuccess && (ms < 0.0 || t < ms)) ms = t;
        }
        if (*err != hipSuccess) break;
        en.ms[c] = ms;
        if (c == 0 || ms < best) {
            best = ms;
            en.choice = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (*err != hipSuccess) return heuristic;
    if (heuristic >= 0 && heuristic < ncand && en.ms[heuristic] >= 0.0 && en.ms[heuristic] <= best * (1.0 + tie_margin(op)))
        en.choice = heuristic;
    return keep(en);
}

std::string tune_dump() {
    std::lock_guard<std::mutex> lk(g_mu);
    std::ostringstream os;
    for (const auto& kv : g_table) {
        const Key& k = kv.first;
        os << "op " << std::get<0>(k) << " dev " << std::get<1>(k) << " shape " << std::get<2>(k) << ' '
           << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << std::get<6>(k)
           << " choice " << kv.second.choice << " ms";
        for (double m : kv.second.ms) os << ' ' << m;
        if (kv.second.ms.empty()) os << " (heuristic)";
        os << '\n';
    }
    return os.str();
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

bool tune_force(int op, int choice) {
    if (op <= 0 || op >= kMaxOp) return false;
    g_force[op].store(choice < 0 ? -1 : choice, std::memory_order_relaxed);
    return true;
}

size_t tune_size() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table.size();
}

}  // namespace tk
