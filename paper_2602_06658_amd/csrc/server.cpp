// Serving loop: continuous batching of independent CNT-GW solves (Algorithm 1)
// on one GPU.
//
// Host threads share the work of the requests a server has admitted:
//
// * setup workers (SETUP_WORKERS of them) take admitted requests in FIFO
//   order and each runs a request's setup (validation, lifting with its
//   landmark eigensolve, initial state) on a stream and rocBLAS handle of its
//   own, then records an event and hands the request over;
// * the round thread issues rounds on the context's stream: every active
//   request advances by one Sinkhorn iteration.  Symmetric MFMA-path requests
//   go through one batched launch per kernel (stabilised pass, its combine,
//   safe or retry pass, its combine) over a table of up to 16 requests whose work-groups
//   share the GPU; other requests launch their own kernels.  A request's
//   prologue and covariance run at its own outer-step boundaries.  A finished
//   request's FP64 check (Appendix A.1's Err) and result readback are queued
//   behind its last round and collected when an event says they are done.
//
// No thread waits for another's GPU work: a request joins the rounds
// once the round stream has been made to wait on its setup event, so setups
// and their host-side synchronisations overlap the rounds of others.
// Requests are admitted while a slot is free and their planned device
// footprint fits the HBM budget.  Request contexts (workspace, pinned
// staging, event) are pooled and reused, so the rounds never wait for a
// device free; with a budget, a returned slot frees its workspace so that
// idle slots hold no memory the budget does not see.
//
// Each request runs the same kernels as gw_solve with the same per-problem
// arguments, so its result does not depend on what else is in the batch.
#include <algorithm>
#include <atomic>
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

enum ReqState { RQ_QUEUED, RQ_SETUP, RQ_ACTIVE, RQ_DONE, RQ_CANCELLED, RQ_FAILED };

// A pooled request context: workspace, penalties, pinned staging, event.
struct Slot {
    std::unique_ptr<gwr::Ctx> ctx;
    hipEvent_t ev = nullptr;
};

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
    std::atomic<bool> cancel{false};
    // GPU-side state, owned by one thread at a time (setup, then rounds)
    Slot* slot = nullptr;
    std::unique_ptr<gwr::Solve> solve;
    int k = 0;
    bool in_outer = false;
};

}  // namespace

// Setup workers: each runs whole request setups (validation, lifting with
// its landmark eigensolve, initial state) on a stream and a rocBLAS handle of
// its own.  The landmark eigensolve is a long chain of small launches, so
// several setups in flight keep the rounds fed with new requests.
constexpr int SETUP_WORKERS = 3;

struct gw_server {
    gwr::Ctx* base = nullptr;
    int max_slots = 1;
    size_t budget = 0;
    hipStream_t setup_stream[SETUP_WORKERS] = {};
    std::thread th, worker[SETUP_WORKERS];
    std::mutex mu;
    std::condition_variable cv_work, cv_setup, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> queue;           // submitted, not admitted
    std::deque<Request*> to_setup;        // admitted, waiting for a setup worker
    std::vector<Request*> ready;          // set up, waiting to join the rounds
    std::vector<std::unique_ptr<Slot>> free_slots;
    std::vector<std::unique_ptr<Slot>> used_slots;
    int in_flight = 0;                    // admitted and not yet completed
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    gw_server_stats stats{};
    size_t resident = 0;                  // planned footprints of admitted requests
    void* rocblas[SETUP_WORKERS] = {};    // one per setup worker
    // round thread only
    std::vector<Request*> active, finishing;
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
        sc.explicit_idx.clear();
        sc.lm.fitted = false;
    }
}

// Device bytes a slot holds: its workspace and landmark data.
size_t slot_bytes(const Slot& sl) {
    size_t b = sl.ctx->ws.total();
    for (int k = 0; k < 2; ++k) {
        const gwr::Landmarks& lm = sl.ctx->side[k].lm;
        if (lm.fitted) b += 4 * ((size_t)lm.n_l * (lm.d_in + lm.dim + 1) + lm.dim);
    }
    return b;
}

// Update the held-memory statistics by delta (under s->mu).
void account(gw_server* s, int64_t delta) {
    s->stats.device_bytes = (uint64_t)((int64_t)s->stats.device_bytes + delta);
    s->stats.peak_device_bytes = std::max(s->stats.peak_device_bytes, s->stats.device_bytes);
}

// Planned device footprint of a request: every buffer of its solve
// (including the FP64 check's sums) and, for the |x - x'|^p penalty, the
// lifting's buffers: the landmark kernel (n_l^2 doubles), eigen-workspace
// (3 n_l doubles), the Nystrom features before centring (n_pad x D floats),
// the centring partials and the landmark data, per side.
size_t request_footprint(const gw_request& r) {
    gwr::Ctx probe;
    configure_sides(probe, r);
    size_t b = gwr::Solve::plan_bytes(probe, r.n, r.dx, r.m, r.dy, r.params);
    if (b == 0) return 0;
    const int64_t np[2] = {(r.n + 31) / 32 * 32, (r.m + 31) / 32 * 32};
    const int64_t nn[2] = {r.n, r.m};
    const int din[2] = {r.dx, r.dy};
    for (int k = 0; k < 2; ++k) {
        const int D = r.penalty == GW_PEN_POWER ? r.lifted_dim : din[k];
        b += 8 * (gwk::centre_part_doubles(nn[k], D) + D) + 2 * (16 + 64 * 8);
        if (r.penalty == GW_PEN_POWER) {
            const size_t nl = (size_t)std::max(0, r.n_landmarks);
            b += 8 * (nl * nl + 3 * nl + 1) + 8 * nl + 4 * (size_t)np[k] * D;
            b += 4 * (nl * (din[k] + D + 1) + D);
        }
    }
    return b + 64 * 256;  // alignment slack
}

Slot* acquire_slot(gw_server* s) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->free_slots.empty()) {
        std::unique_ptr<Slot> sl = std::move(s->free_slots.back());
        s->free_slots.pop_back();
        Slot* p = sl.get();
        s->used_slots.push_back(std::move(sl));
        return p;
    }
    auto sl = std::make_unique<Slot>();
    sl->ctx = std::make_unique<gwr::Ctx>();
    sl->ctx->device = s->base->device;
    (void)hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming);
    Slot* p = sl.get();
    s->used_slots.push_back(std::move(sl));
    return p;
}

// Return a slot whose GPU work has completed.  Its landmark data is freed
// (only read while lifting); the workspace stays for the next request unless
// the server has a budget, which idle memory would escape.
void release_slot(gw_server* s, Request* q) {
    q->solve.reset();
    Slot* sl = q->slot;
    q->slot = nullptr;
    if (!sl) return;
    for (void* h : s->rocblas)
        if (sl->ctx->rocblas == h) sl->ctx->rocblas = nullptr;  // the worker's handle stays
    const size_t before = slot_bytes(*sl);
    gwr::release_landmarks(*sl->ctx);
    if (s->budget) sl->ctx->ws.release_all();
    const size_t after = slot_bytes(*sl);
    std::lock_guard<std::mutex> lk(s->mu);
    account(s, (int64_t)after - (int64_t)before);
    for (auto it = s->used_slots.begin(); it != s->used_slots.end(); ++it)
        if (it->get() == sl) {
            s->free_slots.push_back(std::move(*it));
            s->used_slots.erase(it);
            break;
        }
}

void complete(gw_server* s, Request* q, ReqState st, gw_status code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    q->state = st;
    q->status = code;
    q->msg = msg;
    q->latency = std::chrono::duration<double>(Clock::now() - q->t_submit).count();
    s->resident -= q->footprint;
    s->in_flight--;
    if (st == RQ_DONE || st == RQ_FAILED) s->stats.completed++;
    if (st == RQ_CANCELLED) s->stats.cancelled++;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

// Setup of one request on setup worker w's stream (validation, lifting,
// initial state); the host-side waits in it block only that worker.
gwr::Status start(gw_server* s, Request* q, int w) {
    q->slot = acquire_slot(s);
    gwr::Ctx& c = *q->slot->ctx;
    const size_t before = slot_bytes(*q->slot);
    struct Account {  // record the slot's growth on every exit path
        gw_server* s;
        Slot* sl;
        size_t before;
        ~Account() {
            const size_t after = slot_bytes(*sl);
            std::lock_guard<std::mutex> lk(s->mu);
            account(s, (int64_t)after - (int64_t)before);
        }
    } acct{s, q->slot, before};
    c.stream = s->setup_stream[w];
    configure_sides(c, q->r);
    if (q->r.penalty == GW_PEN_POWER) {
        if (!s->rocblas[w]) {
            rocblas_handle h;
            if (rocblas_create_handle(&h) != rocblas_status_success)
                return gwr::fail(GW_EDEVICE, "rocblas_create_handle");
            s->rocblas[w] = h;
        }
        c.rocblas = s->rocblas[w];
    }
    q->solve = std::make_unique<gwr::Solve>(c, "q.");
    const gw_request& r = q->r;
    GW_TRY(gwr::validate_inputs(c, r.x, r.n, r.dx, r.a, r.y, r.m, r.dy, r.b, &r.params, "q."));
    if (r.params.adaptive_inner) return gwr::fail(GW_EUNSUPPORTED, "adaptive_inner is not served");
    GW_TRY(q->solve->setup(r.x, r.n, r.dx, r.a, r.y, r.m, r.dy, r.b, r.params, r.gamma0, nullptr, nullptr, r.penalty,
                           r.penalty, c.stream));
    GW_HIP(hipEventRecord(q->slot->ev, c.stream));
    q->k = 0;
    q->in_outer = false;
    return gwr::Status::ok();
}

void setup_main(gw_server* s, int w) {
    (void)hipSetDevice(s->base->device);
    for (;;) {
        Request* q = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_setup.wait(lk, [&] { return s->stop || !s->to_setup.empty(); });
            if (s->stop) return;
            q = s->to_setup.front();
            s->to_setup.pop_front();
        }
        if (q->cancel) {
            complete(s, q, RQ_CANCELLED, GW_ECANCELLED, "cancelled");
            continue;
        }
        gwr::Status st = start(s, q, w);
        if (!st.good()) {
            (void)hipStreamSynchronize(s->setup_stream[w]);
            release_slot(s, q);
            complete(s, q, RQ_FAILED, st.code, st.msg);
            continue;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->ready.push_back(q);
        s->cv_work.notify_all();
    }
}

// One round on the main stream: every active request advances by one
// Sinkhorn iteration.
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
        GW_TRY(q->solve->before_inner(q->k));
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
        GW_HIP(gwk::launch_combine_batch(mains.data(), ctls.data(), nb, RUN_STAB, st));
        GW_HIP(gwk::launch_pass_batch(items.data(), nb, RUN_SAFE_OR_RETRY, 1, st));
        GW_HIP(gwk::launch_combine_batch(retries.data(), ctls.data(), nb, RUN_SAFE_OR_RETRY, st));
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

void drop_all_active(gw_server* s, ReqState st, gw_status code, const std::string& msg) {
    (void)hipStreamSynchronize(s->base->stream);
    for (Request* q : s->active) {
        release_slot(s, q);
        complete(s, q, st, code, msg);
    }
    s->active.clear();
}

void round_main(gw_server* s) {
    (void)hipSetDevice(s->base->device);
    hipStream_t main = s->base->stream;
    // rounds in flight: deep enough that small rounds (few, small requests)
    // do not leave the GPU waiting for launches, shallow enough that new
    // arrivals join within a few rounds
    constexpr int PACE = 3;
    hipEvent_t pace[PACE];
    bool pace_used[PACE];
    for (int k = 0; k < PACE; ++k) {
        (void)hipEventCreateWithFlags(&pace[k], hipEventDisableTiming);
        pace_used[k] = false;
    }
    int pi = 0;
    bool busy = false;
    Clock::time_point busy_from;
    for (;;) {
        std::vector<Request*> joining, cancelled;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->active.empty() && s->finishing.empty() && s->ready.empty() && !s->stop) {
                if (busy) {
                    s->stats.busy_seconds += std::chrono::duration<double>(Clock::now() - busy_from).count();
                    busy = false;
                }
                s->cv_work.wait_for(lk, std::chrono::milliseconds(50),
                                    [&] { return s->stop || !s->ready.empty() || !s->queue.empty(); });
            }
            if (s->stop) break;
            // FIFO admission by slot and footprint; setup happens elsewhere
            while (!s->queue.empty() && s->in_flight < s->max_slots) {
                Request* q = s->reqs[s->queue.front()].get();
                if (s->budget && s->resident + q->footprint > s->budget) break;
                s->queue.pop_front();
                q->state = RQ_SETUP;
                s->resident += q->footprint;
                s->in_flight++;
                s->to_setup.push_back(q);
                s->cv_setup.notify_one();
            }
            joining.swap(s->ready);
            for (Request* q : joining) q->state = RQ_ACTIVE;
            for (Request* q : s->active)
                if (q->cancel) cancelled.push_back(q);
            s->stats.queued = (int32_t)s->queue.size();
            s->stats.active = (int32_t)(s->active.size() + joining.size());
        }
        if (!busy && (!joining.empty() || !s->active.empty())) {
            busy = true;
            busy_from = Clock::now();
        }
        for (Request* q : joining) {
            (void)hipStreamWaitEvent(main, q->slot->ev, 0);
            q->slot->ctx->stream = main;
            q->solve->set_stream(main);
            s->active.push_back(q);
        }
        if (!cancelled.empty()) {
            (void)hipStreamSynchronize(main);
            for (Request* q : cancelled) {
                s->active.erase(std::find(s->active.begin(), s->active.end(), q));
                release_slot(s, q);
                complete(s, q, RQ_CANCELLED, GW_ECANCELLED, "cancelled");
            }
        }
        if (!s->active.empty()) {
            std::vector<Request*> finished;
            gwr::Status st = round(s, finished);
            if (!st.good()) {
                drop_all_active(s, RQ_FAILED, st.code, st.msg);
                continue;
            }
            for (Request* q : finished) {
                q->res = gw_result{};
                q->res.f = q->r.f;
                q->res.g = q->r.g;
                q->res.gamma = q->r.gamma;
                s->active.erase(std::find(s->active.begin(), s->active.end(), q));
                gwr::Status fs = q->solve->finish_enqueue(&q->res);
                if (fs.good() && hipEventRecord(q->slot->ev, main) == hipSuccess) {
                    s->finishing.push_back(q);
                } else {
                    (void)hipStreamSynchronize(main);
                    release_slot(s, q);
                    complete(s, q, RQ_FAILED, fs.good() ? GW_EDEVICE : fs.code, fs.good() ? "event" : fs.msg);
                }
            }
            (void)hipEventRecord(pace[pi], main);
            pace_used[pi] = true;
            pi = (pi + 1) % PACE;
            if (pace_used[pi]) (void)hipEventSynchronize(pace[pi]);
        } else if (!s->finishing.empty()) {
            (void)hipEventSynchronize(s->finishing.front()->slot->ev);
        }
        // collect finished checks whose events have completed
        for (size_t i = 0; i < s->finishing.size();) {
            Request* q = s->finishing[i];
            if (hipEventQuery(q->slot->ev) != hipSuccess) {
                ++i;
                continue;
            }
            gwr::Status cs = q->solve->finish_collect(&q->res);
            s->finishing.erase(s->finishing.begin() + i);
            release_slot(s, q);
            if (cs.good()) complete(s, q, RQ_DONE, GW_OK, "");
            else complete(s, q, RQ_FAILED, cs.code, cs.msg);
        }
    }
    // shutdown: everything still resident is cancelled
    (void)hipStreamSynchronize(main);
    for (Request* q : s->finishing) {
        release_slot(s, q);
        complete(s, q, RQ_CANCELLED, GW_ECANCELLED, "server stopped");
    }
    s->finishing.clear();
    drop_all_active(s, RQ_CANCELLED, GW_ECANCELLED, "server stopped");
    for (int k = 0; k < PACE; ++k) (void)hipEventDestroy(pace[k]);
}

void cancel_unstarted(gw_server* s, Request* q) {
    q->state = RQ_CANCELLED;
    q->status = GW_ECANCELLED;
    s->stats.cancelled++;
}

void destroy_slot(gw_server* s, Slot& sl) {
    for (void* h : s->rocblas)
        if (sl.ctx->rocblas == h) sl.ctx->rocblas = nullptr;
    gwr::release_landmarks(*sl.ctx);
    (void)hipEventDestroy(sl.ev);
}

}  // namespace

extern "C" {

gw_status gw_server_create(gw_ctx* ctx, int max_slots, size_t hbm_budget_bytes, gw_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 64) return GW_EINVAL;
    *out = nullptr;
    if (hipSetDevice(ctx->c.device) != hipSuccess) return GW_EDEVICE;
    gw_server* s = new (std::nothrow) gw_server();
    if (!s) return GW_ENOMEM;
    s->base = &ctx->c;
    s->max_slots = max_slots;
    s->budget = hbm_budget_bytes;
    for (int w = 0; w < SETUP_WORKERS; ++w)
        if (hipStreamCreateWithFlags(&s->setup_stream[w], hipStreamNonBlocking) != hipSuccess) {
            for (int k = 0; k < w; ++k) (void)hipStreamDestroy(s->setup_stream[k]);
            delete s;
            return GW_EDEVICE;
        }
    for (int w = 0; w < SETUP_WORKERS; ++w) s->worker[w] = std::thread(setup_main, s, w);
    s->th = std::thread(round_main, s);
    *out = s;
    return GW_OK;
}

gw_status gw_server_submit(gw_server* s, const gw_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return GW_EINVAL;
    if (!req->x || !req->a || !req->y || !req->b || req->n < 1 || req->m < 1) return GW_EINVAL;
    auto q = std::make_unique<Request>();
    q->r = *req;
    q->t_submit = Clock::now();
    q->footprint = request_footprint(*req);
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
    s->cv_work.notify_all();
    return GW_OK;
}

static gw_status report(Request* q, gw_result* out, double* latency_s) {
    if (q->state == RQ_QUEUED || q->state == RQ_SETUP || q->state == RQ_ACTIVE) return GW_EBUSY;
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
    s->cv_done.wait(lk, [&] { return q->state != RQ_QUEUED && q->state != RQ_SETUP && q->state != RQ_ACTIVE; });
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
        cancel_unstarted(s, q);
        q->latency = std::chrono::duration<double>(Clock::now() - q->t_submit).count();
        s->stats.queued = (int32_t)s->queue.size();
        s->cv_done.notify_all();
    } else if (q->state == RQ_SETUP || q->state == RQ_ACTIVE) {
        q->cancel = true;  // taken by a setup worker or the next round
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
        s->cv_setup.notify_all();
    }
    for (auto& t : s->worker)
        if (t.joinable()) t.join();
    if (s->th.joinable()) s->th.join();
    for (hipStream_t st : s->setup_stream) (void)hipStreamSynchronize(st);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Request* q : s->to_setup) cancel_unstarted(s, q);
        s->to_setup.clear();
        for (uint64_t t : s->queue) cancel_unstarted(s, s->reqs[t].get());
        s->queue.clear();
    }
    for (Request* q : s->ready) {
        release_slot(s, q);
        std::lock_guard<std::mutex> lk(s->mu);
        cancel_unstarted(s, q);
    }
    s->ready.clear();
    s->cv_done.notify_all();
    for (auto& sl : s->free_slots) destroy_slot(s, *sl);
    for (auto& sl : s->used_slots) destroy_slot(s, *sl);
    s->free_slots.clear();
    s->used_slots.clear();
    for (void* h : s->rocblas)
        if (h) rocblas_destroy_handle((rocblas_handle)h);
    for (hipStream_t st : s->setup_stream) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
