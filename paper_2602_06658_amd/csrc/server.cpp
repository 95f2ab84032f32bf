// Serving loop: continuous batching of independent CNT-GW solves (Algorithm 1)
// on one GPU.
//
// A host thread owns every GPU-side step of the requests it has admitted.
// Requests wait in a FIFO queue and are admitted while a slot is free and
// their planned device footprint fits the HBM budget; admission happens
// between Sinkhorn iterations, so a request that arrives while others run
// joins them at the next round.  Each round advances every active request by
// one Sinkhorn iteration: symmetric MFMA-path requests go through one
// batched launch per kernel (pass, safe pass, combine, retry pass, retry
// combine) over a table of up to 16 requests, whose work-groups share the
// GPU; other requests launch their own kernels.  A request's prologue and
// covariance run at its own outer-step boundaries.  Finished requests are
// checked in FP64 (Appendix A.1's Err), their results recorded, and their
// device memory released.
//
// Each request has its own context (workspace, penalties, landmarks) and
// runs the same kernels as gw_solve with the same per-problem arguments, so
// its result does not depend on what else is in the batch.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include <rocblas/rocblas.h>

#include "runtime.h"

using gwr::hip_fail;
using gwr::Status;
using namespace gwl;

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { RQ_QUEUED, RQ_ACTIVE, RQ_DONE, RQ_CANCELLED, RQ_FAILED };

struct Request {
    uint64_t ticket = 0;
    gw_request r{};
    ReqState state = RQ_QUEUED;
    gw_status status = GW_OK;
    std::string msg;
    Clock::time_point t_submit;
    double latency = 0.0;
    gw_result res{};
    size_t footprint = 0;
    bool cancel = false;
    // GPU-side state, touched by the server thread only
    std::unique_ptr<gwr::Ctx> ctx;
    std::unique_ptr<gwr::Solve> solve;
    int k = 0;
    bool in_outer = false;
};

}  // namespace

struct gw_server {
    gwr::Ctx* base = nullptr;
    int max_slots = 1;
    size_t budget = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    gw_server_stats stats{};
    size_t resident = 0;
    void* rocblas = nullptr;  // shared by the requests' landmark eigensolves
    std::vector<Request*> active;  // server thread only
};

namespace {

void configure_sides(gwr::Ctx& c, const gw_request& r) {
    for (int s = 0; s < 2; ++s) {
        gwr::SideCfg& sc = c.side[s];
        sc.kind = r.penalty;
        sc.p = r.p;
        sc.lifted_dim = r.lifted_dim;
        sc.n_landmarks = r.n_landmarks;
        sc.seed = r.seed + (uint64_t)s;
    }
}

std::unique_ptr<gwr::Ctx> make_ctx(gw_server* s, const gw_request& r) {
    auto c = std::make_unique<gwr::Ctx>();
    c->device = s->base->device;
    c->stream = s->base->stream;
    configure_sides(*c, r);
    return c;
}

// Free a request's device memory (the stream must be idle for it).
void release(gw_server* s, Request* q) {
    if (q->ctx) {
        if (q->ctx->rocblas == s->rocblas) q->ctx->rocblas = nullptr;  // shared handle stays
        gwr::release_landmarks(*q->ctx);
        q->ctx->ws.release_all();
    }
    q->solve.reset();
    q->ctx.reset();
}

void complete(gw_server* s, Request* q, ReqState st, gw_status code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    q->state = st;
    q->status = code;
    q->msg = msg;
    q->latency = std::chrono::duration<double>(Clock::now() - q->t_submit).count();
    s->resident -= q->footprint;
    if (st == RQ_DONE) s->stats.completed++;
    if (st == RQ_CANCELLED) s->stats.cancelled++;
    if (st == RQ_FAILED) s->stats.completed++;
    s->cv_done.notify_all();
}

gwr::Status start(gw_server* s, Request* q) {
    q->ctx = make_ctx(s, q->r);
    if (q->r.penalty == GW_PEN_POWER) {
        if (!s->rocblas) {
            rocblas_handle h;
            if (rocblas_create_handle(&h) != rocblas_status_success)
                return gwr::fail(GW_EDEVICE, "rocblas_create_handle");
            s->rocblas = h;
        }
        q->ctx->rocblas = s->rocblas;
    }
    q->solve = std::make_unique<gwr::Solve>(*q->ctx, "q.");
    const gw_request& r = q->r;
    GW_TRY(gwr::validate_inputs(*q->ctx, r.x, r.n, r.dx, r.a, r.y, r.m, r.dy, r.b, &r.params, "q."));
    GW_TRY(q->solve->setup(r.x, r.n, r.dx, r.a, r.y, r.m, r.dy, r.b, r.params, nullptr, nullptr, nullptr, r.penalty,
                           r.penalty, q->ctx->stream));
    q->k = 0;
    q->in_outer = false;
    return gwr::Status::ok();
}

// One round: every active request advances by one Sinkhorn iteration.
gwr::Status round(gw_server* s, std::vector<Request*>& finished) {
    std::vector<gwk::PassItem> items;
    std::vector<gwk::CombineArgs> mains, retries;
    std::vector<int*> ctls;
    std::vector<Request*> batched;
    hipStream_t st = s->base->stream;
    for (Request* q : s->active) {
        if (!q->in_outer) {
            GW_TRY(q->solve->begin_outer());
            q->in_outer = true;
            q->k = 0;
        }
        if (q->solve->batchable()) {
            gwk::PassItem it;
            gwk::CombineArgs ma, ra;
            int* ctl = nullptr;
            q->solve->iteration_items(it, ma, ra, &ctl);
            items.push_back(it);
            mains.push_back(ma);
            retries.push_back(ra);
            ctls.push_back(ctl);
            batched.push_back(q);
        } else {
            GW_TRY(q->solve->inner_iteration(q->k));
        }
    }
    if (!items.empty()) {
        const int nb = (int)items.size();
        GW_HIP(gwk::launch_pass_batch(items.data(), nb, RUN_STAB, 0, st));
        GW_HIP(gwk::launch_pass_batch(items.data(), nb, RUN_SAFE, 1, st));
        GW_HIP(gwk::launch_combine_batch(mains.data(), ctls.data(), nb, RUN_ALWAYS, st));
        GW_HIP(gwk::launch_pass_batch(items.data(), nb, RUN_RETRY, 1, st));
        GW_HIP(gwk::launch_combine_batch(retries.data(), ctls.data(), nb, RUN_RETRY, st));
        for (Request* q : batched) q->solve->advance_parity();
    }
    for (Request* q : s->active) {
        if (++q->k == q->solve->n_inner()) {
            GW_TRY(q->solve->end_outer());
            q->in_outer = false;
            if (q->solve->done()) finished.push_back(q);
        }
    }
    return gwr::Status::ok();
}

void fail_all_active(gw_server* s, const gwr::Status& st) {
    (void)hipStreamSynchronize(s->base->stream);
    for (Request* q : s->active) {
        release(s, q);
        complete(s, q, RQ_FAILED, st.code, st.msg);
    }
    s->active.clear();
}

void server_main(gw_server* s) {
    (void)hipSetDevice(s->base->device);
    hipEvent_t ev[2] = {nullptr, nullptr};
    (void)hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
    int evi = 0;
    bool ev_used[2] = {false, false};
    Clock::time_point busy_from;
    for (;;) {
        std::vector<Request*> admit, cancelled;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->active.empty()) {
                if (s->stats.active == 0 && s->queue.empty() && !s->stop) {
                    s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                }
            }
            if (s->stop) break;
            for (Request* q : s->active)
                if (q->cancel) cancelled.push_back(q);
            // FIFO admission by slot and footprint
            while (!s->queue.empty() && (int)(s->active.size() + admit.size()) < s->max_slots) {
                Request* q = s->reqs[s->queue.front()].get();
                if (s->budget && s->resident + q->footprint > s->budget) break;
                s->queue.pop_front();
                q->state = RQ_ACTIVE;
                s->resident += q->footprint;
                admit.push_back(q);
            }
            s->stats.queued = (int32_t)s->queue.size();
        }
        if (!cancelled.empty()) {
            (void)hipStreamSynchronize(s->base->stream);
            for (Request* q : cancelled) {
                s->active.erase(std::find(s->active.begin(), s->active.end(), q));
                release(s, q);
                complete(s, q, RQ_CANCELLED, GW_ECANCELLED, "cancelled");
            }
        }
        const bool was_idle = s->active.empty();
        for (Request* q : admit) {
            gwr::Status st = start(s, q);
            if (!st.good()) {
                (void)hipStreamSynchronize(s->base->stream);
                release(s, q);
                complete(s, q, RQ_FAILED, st.code, st.msg);
                continue;
            }
            s->active.push_back(q);
        }
        if (s->active.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.active = 0;
            continue;
        }
        if (was_idle) busy_from = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.active = (int32_t)s->active.size();
        }
        std::vector<Request*> finished;
        gwr::Status st = round(s, finished);
        if (!st.good()) {
            fail_all_active(s, st);
            continue;
        }
        for (Request* q : finished) {
            q->res = gw_result{};
            q->res.f = q->r.f;
            q->res.g = q->r.g;
            q->res.gamma = q->r.gamma;
            gwr::Status fs = q->solve->finish(&q->res);  // FP64 check; waits for the stream
            s->active.erase(std::find(s->active.begin(), s->active.end(), q));
            release(s, q);
            if (fs.good()) complete(s, q, RQ_DONE, GW_OK, "");
            else complete(s, q, RQ_FAILED, fs.code, fs.msg);
        }
        if (s->active.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.busy_seconds += std::chrono::duration<double>(Clock::now() - busy_from).count();
            s->stats.active = 0;
        }
        // keep at most two rounds in flight so admissions stay prompt
        (void)hipEventRecord(ev[evi], s->base->stream);
        ev_used[evi] = true;
        evi ^= 1;
        if (ev_used[evi]) (void)hipEventSynchronize(ev[evi]);
    }
    // shutdown: cancel whatever is left
    (void)hipStreamSynchronize(s->base->stream);
    for (Request* q : s->active) {
        release(s, q);
        complete(s, q, RQ_CANCELLED, GW_ECANCELLED, "server stopped");
    }
    s->active.clear();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t t : s->queue) {
            Request* q = s->reqs[t].get();
            q->state = RQ_CANCELLED;
            q->status = GW_ECANCELLED;
            s->stats.cancelled++;
        }
        s->queue.clear();
        s->cv_done.notify_all();
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
}

}  // namespace

extern "C" {

gw_status gw_server_create(gw_ctx* ctx, int max_slots, size_t hbm_budget_bytes, gw_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 64) return GW_EINVAL;
    *out = nullptr;
    gw_server* s = new (std::nothrow) gw_server();
    if (!s) return GW_ENOMEM;
    s->base = &ctx->c;
    s->max_slots = max_slots;
    s->budget = hbm_budget_bytes;
    s->th = std::thread(server_main, s);
    *out = s;
    return GW_OK;
}

gw_status gw_server_submit(gw_server* s, const gw_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return GW_EINVAL;
    if (!req->x || !req->a || !req->y || !req->b || req->n < 1 || req->m < 1) return GW_EINVAL;
    auto q = std::make_unique<Request>();
    q->r = *req;
    q->t_submit = Clock::now();
    {
        // footprint of the solve's buffers for admission (landmark data of
        // the |x - x'|^p penalty comes on top: n_l^2 doubles per side)
        gwr::Ctx probe;
        configure_sides(probe, *req);
        q->footprint = gwr::Solve::plan_bytes(probe, req->n, req->dx, req->m, req->dy, req->params);
        if (req->penalty == GW_PEN_POWER) q->footprint += 2 * (size_t)req->n_landmarks * req->n_landmarks * 8;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.submitted++;
    if (q->footprint == 0 || (s->budget && q->footprint > s->budget)) {
        s->stats.rejected++;
        return q->footprint == 0 ? GW_EINVAL : GW_ENOMEM;
    }
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->queue.push_back(q->ticket);
    s->reqs.emplace(q->ticket, std::move(q));
    s->stats.queued = (int32_t)s->queue.size();
    s->cv_work.notify_one();
    return GW_OK;
}

static gw_status report(Request* q, gw_result* out, double* latency_s) {
    if (q->state == RQ_QUEUED || q->state == RQ_ACTIVE) return GW_EBUSY;
    if (latency_s) *latency_s = q->latency;
    if (q->state == RQ_CANCELLED) return GW_ECANCELLED;
    if (q->state == RQ_FAILED) return q->status;
    if (out) *out = q->res;
    return GW_OK;
}

gw_status gw_server_poll(gw_server* s, uint64_t ticket, gw_result* out, double* latency_s) {
    if (!s) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GW_EINVAL;
    return report(it->second.get(), out, latency_s);
}

gw_status gw_server_wait(gw_server* s, uint64_t ticket, gw_result* out, double* latency_s) {
    if (!s) return GW_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GW_EINVAL;
    Request* q = it->second.get();
    s->cv_done.wait(lk, [&] { return q->state != RQ_QUEUED && q->state != RQ_ACTIVE; });
    return report(q, out, latency_s);
}

gw_status gw_server_cancel(gw_server* s, uint64_t ticket) {
    if (!s) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GW_EINVAL;
    Request* q = it->second.get();
    if (q->state == RQ_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
        q->state = RQ_CANCELLED;
        q->status = GW_ECANCELLED;
        q->latency = std::chrono::duration<double>(Clock::now() - q->t_submit).count();
        s->stats.cancelled++;
        s->stats.queued = (int32_t)s->queue.size();
        s->cv_done.notify_all();
    } else if (q->state == RQ_ACTIVE) {
        q->cancel = true;
    }
    return GW_OK;
}

gw_status gw_server_get_stats(gw_server* s, gw_server_stats* out) {
    if (!s || !out) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return GW_OK;
}

void gw_server_destroy(gw_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    if (s->rocblas) rocblas_destroy_handle((rocblas_handle)s->rocblas);
    delete s;
}

}  // extern "C"
