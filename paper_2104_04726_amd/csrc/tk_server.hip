// Served execution of many decompositions on one GPU (the request loop of the image-stack
// pipeline): first-come-first-served admission by HBM budget, `slots` requests in flight, each on
// its own stream and workspace so that their kernels overlap on the device.
//
// Threads: one worker per slot.  A worker takes the head of the queue when its footprint fits in
// the unused budget, copies the tensor in, runs tucker_decompose_ex on its own context (stream-
// ordered allocations, so no device-wide synchronisation from allocation), copies the outputs
// out, frees its device memory and returns the footprint to the budget.  Requests queue strictly
// in arrival order: a large request at the head is not overtaken by smaller ones behind it.
//
// Groups: when the head may be grouped (reduced-precision sweeps, no tolerance), the worker also
// admits the requests right behind it that have the same shape class and fit in the budget (up to
// group_requests in all).  It runs the first itself and each other member in a thread of its own on
// a pooled helper context; the members' sweep products are launched in lock step as grouped
// persistent grids over all their tiles (LpGrouper), and their sweeps are not replayed as graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tucker.h"
#include "tk_lowp.h"

void tk_ctx_set_async_alloc(tucker_ctx* ctx, bool on);
void tk_ctx_release_workspace(tucker_ctx* ctx);
void tk_ctx_set_run_options(tucker_ctx* ctx, tucker_precision precision, int refine_sweeps);
void tk_ctx_set_graphs(tucker_ctx* ctx, bool on);

namespace {

using Clock = std::chrono::steady_clock;

// requests admitted together that share grouped launches of their reduced-precision products
struct Group {
    tk::LpGrouper lp;
    Group(int members, int device) : lp(members, device) {}
};

struct Job {
    uint64_t id = 0;
    tucker_request req{};
    size_t footprint = 0;
    bool done = false;
    tucker_result res{};
    std::shared_ptr<Group> grp;
};

// requests that may run as one group: same shape and schedule, reduced-precision sweeps, no
// data-dependent stopping (every member makes the same sequence of products)
bool groupable(const tucker_request& q) {
    return q.precision != TUCKER_FP32 && !(q.tol > 0.0) && q.max_iters > 0;
}
bool same_class(const tucker_request& a, const tucker_request& b) {
    if (a.ndim != b.ndim || a.precision != b.precision || a.max_iters != b.max_iters ||
        a.refine_sweeps != b.refine_sweeps || a.tol != b.tol)
        return false;
    for (int n = 0; n < a.ndim; ++n)
        if (a.dims[n] != b.dims[n] || a.ranks[n] != b.ranks[n]) return false;
    return true;
}

int64_t prod(const int64_t* d, int n) {
    int64_t p = 1;
    for (int i = 0; i < n; ++i) p *= d[i];
    return p;
}

void set_error(tucker_result& r, tucker_status st, const std::string& msg) {
    r.status = st;
    std::snprintf(r.error, sizeof(r.error), "%s", msg.c_str());
}

}  // namespace

struct tucker_server {
    tucker_server_options opt{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;   // workers: queue or budget changed
    std::condition_variable cv_done;   // waiters: a job finished
    std::deque<Job*> queue;
    std::mutex helper_mu;              // contexts (each with its own stream) for group members
    std::vector<std::pair<tucker_ctx*, hipStream_t>> helpers_free, helpers_all;
    std::map<uint64_t, Job*> jobs;
    uint64_t next_id = 1;
    size_t budget = 0, admitted = 0;
    int running = 0;
    bool stop = false;
    tucker_server_stats stats{};
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<tucker_ctx*> ctxs;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void run_job(int slot, Job* j) { run_job_on(ctxs[slot], streams[slot], j); }

    void run_job_on(tucker_ctx* ctx, hipStream_t s, Job* j) {
        const tucker_request& q = j->req;
        tucker_result& r = j->res;
        r.t_start = now();
        const int N = q.ndim;
        const int64_t xn = prod(q.dims, N), gn = prod(q.ranks, N);
        if (j->grp) {
            tk::lp_group_set(&j->grp->lp);
            tk_ctx_set_graphs(ctx, false);
        }
        float* dx = nullptr;
        float* dg = nullptr;
        std::vector<float*> df(N, nullptr);
        auto fail = [&](tucker_status st, const std::string& m) { set_error(r, st, m); };
        auto halloc = [&](float** p, int64_t n) {
            return hipMallocAsync((void**)p, (size_t)std::max<int64_t>(n, 1) * sizeof(float), s) == hipSuccess;
        };
        bool ok = halloc(&dx, xn) && halloc(&dg, gn);
        for (int n = 0; ok && n < N; ++n) ok = halloc(&df[n], q.dims[n] * q.ranks[n]);
        if (!ok) {
            (void)hipGetLastError();
            fail(TUCKER_ERR_OUT_OF_MEMORY, "device allocation for the request failed");
        } else if (hipMemcpyAsync(dx, q.host_tensor, xn * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess) {
            fail(TUCKER_ERR_DEVICE, "host to device copy failed");
        } else {
            tk_ctx_set_run_options(ctx, q.precision, q.refine_sweeps);
            double fit = 0.0;
            int sweeps = 0;
            tucker_status st = tucker_decompose_ex(ctx, dx, N, q.dims, q.ranks, q.max_iters, q.tol, nullptr, dg,
                                                   df.data(), &fit, nullptr, &sweeps);
            if (st != TUCKER_OK) {
                fail(st, tucker_last_error(ctx));
            } else {
                bool cp = hipMemcpyAsync(q.host_core, dg, gn * sizeof(float), hipMemcpyDeviceToHost, s) == hipSuccess;
                for (int n = 0; cp && n < N; ++n)
                    cp = hipMemcpyAsync(q.host_factors[n], df[n], q.dims[n] * q.ranks[n] * sizeof(float),
                                        hipMemcpyDeviceToHost, s) == hipSuccess;
                cp = cp && hipStreamSynchronize(s) == hipSuccess;
                if (!cp) {
                    fail(TUCKER_ERR_DEVICE, "device to host copy failed");
                } else {
                    r.status = TUCKER_OK;
                    r.fit = fit;
                    r.sweeps = sweeps;
                }
            }
        }
        if (dx) (void)hipFreeAsync(dx, s);
        if (dg) (void)hipFreeAsync(dg, s);
        for (float* p : df)
            if (p) (void)hipFreeAsync(p, s);
        if (j->grp) {
            j->grp->lp.leave();
            tk::lp_group_set(nullptr);
            tk_ctx_set_graphs(ctx, opt.use_graphs != 0);
        }
        tk_ctx_release_workspace(ctx);
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        r.t_finish = now();
    }

    // a context and stream for one more group member: from the pool, or created (nullptr on failure)
    bool acquire_helper(std::pair<tucker_ctx*, hipStream_t>& out) {
        {
            std::lock_guard<std::mutex> lk(helper_mu);
            if (!helpers_free.empty()) {
                out = helpers_free.back();
                helpers_free.pop_back();
                return true;
            }
        }
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        tucker_options co;
        tucker_default_options(&co);
        co.device = opt.device;
        co.inner_iters = opt.inner_iters;
        co.init_iters = opt.init_iters;
        co.seed = opt.seed;
        co.use_graphs = opt.use_graphs;
        co.autotune = opt.autotune;
        co.stream = st;
        tucker_ctx* c = nullptr;
        if (tucker_create(&co, &c) != TUCKER_OK) {
            (void)hipStreamDestroy(st);
            return false;
        }
        tk_ctx_set_async_alloc(c, true);
        out = {c, st};
        std::lock_guard<std::mutex> lk(helper_mu);
        helpers_all.push_back(out);
        return true;
    }
    void release_helper(const std::pair<tucker_ctx*, hipStream_t>& h) {
        std::lock_guard<std::mutex> lk(helper_mu);
        helpers_free.push_back(h);
    }

    // admit j (the queue head, already popped) and, when it may be grouped, the consecutive queued
    // requests of its class that fit in the budget, up to opt.group_requests in all; mu held
    std::vector<Job*> admit_locked(Job* j, int slot) {
        std::vector<Job*> members{j};
        auto take = [&](Job* x) {
            admitted += x->footprint;
            ++running;
            x->res.t_admit = now();
            x->res.slot = slot;
        };
        take(j);
        if (opt.group_requests > 1 && groupable(j->req)) {
            while (!queue.empty() && (int)members.size() < opt.group_requests &&
                   same_class(queue.front()->req, j->req) && admitted + queue.front()->footprint <= budget) {
                Job* x = queue.front();
                queue.pop_front();
                take(x);
                members.push_back(x);
            }
        }
        stats.peak_admitted_bytes = std::max(stats.peak_admitted_bytes, admitted);
        stats.peak_running = std::max(stats.peak_running, running);
        return members;
    }

    void finish_locked(Job* j) {
        admitted -= j->footprint;
        --running;
        j->done = true;
        stats.completed += 1;
        if (j->res.status != TUCKER_OK) stats.failed += 1;
    }

    // members[0] runs on the worker's own context; the others on helper contexts in threads of their
    // own, all in lock step through one LpGrouper (a member that cannot get a context fails alone)
    void run_group(int slot, const std::vector<Job*>& members) {
        const int g = (int)members.size();
        auto grp = std::make_shared<Group>(g, opt.device);
        if (!grp->lp.ok()) {
            for (Job* x : members) run_job(slot, x);   // one after another, ungrouped
            return;
        }
        for (Job* x : members) x->grp = grp;
        std::vector<std::thread> th;
        std::vector<std::pair<tucker_ctx*, hipStream_t>> hs(g);
        for (int k = 1; k < g; ++k) {
            if (!acquire_helper(hs[k])) {
                hs[k] = {nullptr, nullptr};
                set_error(members[k]->res, TUCKER_ERR_DEVICE, "no context for a group member");
                grp->lp.leave();
                continue;
            }
            th.emplace_back([this, k, &hs, &members] {
                (void)hipSetDevice(opt.device);
                run_job_on(hs[k].first, hs[k].second, members[k]);
            });
        }
        run_job(slot, members[0]);
        for (auto& t : th) t.join();
        for (int k = 1; k < g; ++k)
            if (hs[k].first) release_helper(hs[k]);
        std::lock_guard<std::mutex> lk(mu);
        stats.grouped_requests += g;
        stats.group_launches += grp->lp.launches();
        stats.grouped_products += grp->lp.products();
    }

    void worker(int slot) {
        (void)hipSetDevice(opt.device);
        for (;;) {
            std::vector<Job*> members;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return stop || (!queue.empty() && admitted + queue.front()->footprint <= budget);
                });
                if (stop) return;
                Job* j = queue.front();
                queue.pop_front();
                members = admit_locked(j, slot);
            }
            if (members.size() == 1) run_job(slot, members[0]);
            else run_group(slot, members);
            {
                std::lock_guard<std::mutex> lk(mu);
                for (Job* x : members) {
                    finish_locked(x);
                    x->grp.reset();
                }
            }
            cv_work.notify_all();
            cv_done.notify_all();
        }
    }
};

extern "C" {

void tucker_default_server_options(tucker_server_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->slots = 4;
    o->hbm_budget_bytes = 0;
    o->inner_iters = 1;
    o->init_iters = 20;
    o->seed = 0x5eedull;
    o->use_graphs = 1;
    o->autotune = 1;
    o->group_requests = 0;
}

tucker_status tucker_server_create(const tucker_server_options* opts, tucker_server** out) {
    if (!out) return TUCKER_ERR_INVALID_ARG;
    *out = nullptr;
    tucker_server_options o;
    tucker_default_server_options(&o);
    if (opts) o = *opts;
    if (o.slots < 1 || o.slots > 64 || o.inner_iters < 1 || o.init_iters < 1 || o.device < 0 ||
        o.group_requests < 0 || o.group_requests > tk::kLpGroupMax)
        return TUCKER_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= o.device) {
        (void)hipGetLastError();
        return TUCKER_ERR_DEVICE;
    }
    if (hipSetDevice(o.device) != hipSuccess) return TUCKER_ERR_DEVICE;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return TUCKER_ERR_DEVICE;
    // keep freed request memory in the device's pool for the next request
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, o.device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    tucker_server* srv = new tucker_server();
    srv->opt = o;
    srv->t0 = Clock::now();
    srv->budget = o.hbm_budget_bytes ? o.hbm_budget_bytes : (size_t)(0.9 * (double)freeb);
    srv->stats.budget_bytes = srv->budget;
    for (int k = 0; k < o.slots; ++k) {
        hipStream_t s = nullptr;
        tucker_options co;
        tucker_default_options(&co);
        co.device = o.device;
        co.inner_iters = o.inner_iters;
        co.init_iters = o.init_iters;
        co.seed = o.seed;
        co.use_graphs = o.use_graphs;
        co.autotune = o.autotune;
        tucker_ctx* c = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            tucker_server_destroy(srv);
            return TUCKER_ERR_DEVICE;
        }
        srv->streams.push_back(s);
        co.stream = s;
        if (tucker_create(&co, &c) != TUCKER_OK) {
            tucker_server_destroy(srv);
            return TUCKER_ERR_DEVICE;
        }
        tk_ctx_set_async_alloc(c, true);
        srv->ctxs.push_back(c);
    }
    for (int k = 0; k < o.slots; ++k) srv->workers.emplace_back([srv, k] { srv->worker(k); });
    *out = srv;
    return TUCKER_OK;
}

tucker_status tucker_server_submit(tucker_server* srv, const tucker_request* req, uint64_t* id) {
    if (!srv || !req || !id) return TUCKER_ERR_INVALID_ARG;
    const tucker_request& q = *req;
    if (!q.host_tensor || !q.host_core || q.ndim < 2 || q.ndim > TUCKER_MAX_ORDER) return TUCKER_ERR_INVALID_ARG;
    for (int n = 0; n < q.ndim; ++n)
        if (!q.host_factors[n]) return TUCKER_ERR_INVALID_ARG;
    if (q.refine_sweeps < 0 || q.precision < TUCKER_FP32 || q.precision > TUCKER_FP8_E4M3)
        return TUCKER_ERR_INVALID_ARG;
    tucker_status st = tucker_validate(q.ndim, q.dims, q.ranks, q.max_iters, q.tol);
    if (st != TUCKER_OK) return st;
    size_t ws = 0;
    st = tucker_workspace_size(q.ndim, q.dims, q.ranks, q.precision, &ws);
    if (st != TUCKER_OK) return st;
    size_t io = (size_t)prod(q.dims, q.ndim) + (size_t)prod(q.ranks, q.ndim);
    for (int n = 0; n < q.ndim; ++n) io += (size_t)(q.dims[n] * q.ranks[n]);
    const size_t footprint = ws + io * sizeof(float) + (size_t)(q.ndim + 2) * 256;
    if (footprint > srv->budget) return TUCKER_ERR_OUT_OF_MEMORY;
    Job* j = new Job();
    j->req = q;
    j->footprint = footprint;
    j->res.tag = q.tag;
    j->res.footprint_bytes = footprint;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            delete j;
            return TUCKER_ERR_INVALID_ARG;
        }
        j->id = srv->next_id++;
        j->res.t_submit = srv->now();
        srv->jobs[j->id] = j;
        srv->queue.push_back(j);
        srv->stats.submitted += 1;
        *id = j->id;
    }
    srv->cv_work.notify_all();
    return TUCKER_OK;
}

tucker_status tucker_server_wait(tucker_server* srv, uint64_t id, double timeout_s, tucker_result* out) {
    if (!srv || !out) return TUCKER_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(id);
    if (it == srv->jobs.end()) return TUCKER_ERR_INVALID_ARG;
    Job* j = it->second;
    auto ready = [&] { return j->done; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return TUCKER_ERR_TIMEOUT;
    }
    *out = j->res;
    srv->jobs.erase(it);
    delete j;
    return TUCKER_OK;
}

tucker_status tucker_server_get_stats(tucker_server* srv, tucker_server_stats* out) {
    if (!srv || !out) return TUCKER_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    return TUCKER_OK;
}

tucker_status tucker_server_destroy(tucker_server* srv) {
    if (!srv) return TUCKER_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // queued (not admitted) requests fail; running ones finish inside their worker
        for (Job* j : srv->queue) {
            set_error(j->res, TUCKER_ERR_DEVICE, "server destroyed before the request ran");
            j->done = true;
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (auto& t : srv->workers)
        if (t.joinable()) t.join();
    for (tucker_ctx* c : srv->ctxs) tucker_destroy(c);
    for (auto& h : srv->helpers_all) {
        tucker_destroy(h.first);
        (void)hipStreamDestroy(h.second);
    }
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    for (auto& kv : srv->jobs) delete kv.second;
    delete srv;
    return TUCKER_OK;
}

}  // extern "C"
