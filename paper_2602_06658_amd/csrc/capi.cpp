// extern "C" entry points of libgwmi.so (declared in include/gw.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "gw_grad.h"
#include "gw_lift.h"
#include "gw_scratch.h"
#include "runtime.h"

using gwr::Ctx;
using gwr::hip_fail;
using gwr::Status;


namespace {
// Readback staging of gw_solve_noalloc: 16 scalars, the moments of both
// sides (2 + D^2 + D doubles each, D <= 256) and the control words.
constexpr size_t NOALLOC_STAGE_DOUBLES = 16 + 2 * (2 + 256 * 256 + 256) + 8;
double g_noalloc_stage[NOALLOC_STAGE_DOUBLES];
// gw_solve_noalloc calls of this process share the scratch array and the
// staging above, so they run one at a time.
std::mutex g_noalloc_mu;
}  // namespace

static gw_status ret(gw_ctx* ctx, const Status& s) {
    if (ctx) ctx->c.err = s.good() ? std::string() : s.msg;
    return s.code;
}

// Independent solves of one call (the three problems of a divergence or of
// a barycentre step), set up in order on the context's stream, then run
// with their outer steps interleaved, each on a stream of its own, so that
// the GPU overlaps the kernels of problems too small to fill it alone.
// Each solve issues the launches it issues alone, on buffers of its own
// (its tag), so its result is the same bit for bit; finish() and
// gradients() wait on each solve's own stream.
static Status outer_steps_side_by_side(Ctx& c, gwr::Solve* const* solves, int k) {
    hipStream_t st[Ctx::SIDE_STREAMS];
    GW_TRY(c.side_streams(k, st));
    hipEvent_t ready = nullptr;
    GW_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ready, c.stream);
    for (int i = 0; e == hipSuccess && i < k; ++i) e = hipStreamWaitEvent(st[i], ready, 0);
    (void)hipEventDestroy(ready);
    if (e != hipSuccess) return hip_fail(e, "side-by-side solves");
    for (int i = 0; i < k; ++i) solves[i]->set_stream(st[i]);
    Status s;
    for (bool more = true; more && s.good();) {
        more = false;
        for (int i = 0; i < k && s.good(); ++i)
            if (!solves[i]->done()) {
                s = solves[i]->outer_step();
                more = more || !solves[i]->done();
            }
    }
    if (!s.good())
        for (int i = 0; i < k; ++i) (void)hipStreamSynchronize(st[i]);
    return s;
}

// Problems of at most this many entries run side by side; a larger one
// fills the GPU alone, and the solves then run one after another on one set
// of buffers (side by side, each holds its own).
constexpr double SIDE_BY_SIDE_MAX_ENTRIES = 1.0e9;

// cnt (at most 3) independent solves: setup(i, solve) sets solve i up on the
// context's stream, done(i, solve) collects its result once it has finished.
template <class Setup, class Done>
static Status run_independent(Ctx& c, int cnt, bool side_by_side, Setup setup, Done done) {
    if (!side_by_side) {
        for (int i = 0; i < cnt; ++i) {
            gwr::Solve s(c, "s.");
            GW_TRY(setup(i, s));
            while (!s.done()) GW_TRY(s.outer_step());
            GW_TRY(done(i, s));
        }
        return Status::ok();
    }
    gwr::Solve s0(c, "s0."), s1(c, "s1."), s2(c, "s2.");
    gwr::Solve* const all[3] = {&s0, &s1, &s2};
    for (int i = 0; i < cnt; ++i) GW_TRY(setup(i, *all[i]));
    GW_TRY(outer_steps_side_by_side(c, all, cnt));
    Status st;
    for (int i = 0; st.good() && i < cnt; ++i) st = done(i, *all[i]);
    if (!st.good()) {  // the others' work must end before their buffers are reused
        hipStream_t ss[Ctx::SIDE_STREAMS];
        if (c.side_streams(cnt, ss).good())
            for (int i = 0; i < cnt; ++i) (void)hipStreamSynchronize(ss[i]);
    }
    return st;
}

extern "C" {

gw_status gw_create(gw_ctx** out, int device, void* hip_stream, size_t workspace_limit_bytes) {
    if (!out) return GW_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GW_EDEVICE;
    if (device < 0 || device >= ndev) return GW_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return GW_EDEVICE;
    gw_ctx* ctx = new (std::nothrow) gw_ctx();
    if (!ctx) return GW_ENOMEM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    ctx->c.ws.set_limit(workspace_limit_bytes);
    *out = ctx;
    return GW_OK;
}

gw_status gw_set_penalty(gw_ctx* ctx, int side, int kind, double p, int lifted_dim, int n_landmarks, uint64_t seed) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (side < 0 || side > 2) return ret(ctx, gwr::fail(GW_EINVAL, "side must be 0, 1 or 2"));
    if (kind < GW_PEN_SQEUCLID || kind > GW_PEN_FEATURES) return ret(ctx, gwr::fail(GW_EINVAL, "unknown penalty"));
    if (kind == GW_PEN_POWER) {
        if (!(p > 0.0 && p < 2.0)) return ret(ctx, gwr::fail(GW_EINVAL, "power penalty needs 0 < p < 2"));
        if (lifted_dim < 1 || lifted_dim > gwl::MAX_DIM)
            return ret(ctx, gwr::fail(GW_EINVAL, "lifted_dim must be in [1, 256]"));
        if (n_landmarks < lifted_dim + 1) return ret(ctx, gwr::fail(GW_EINVAL, "need n_landmarks > lifted_dim"));
    }
    for (int s = 0; s < 2; ++s) {
        if (side != 2 && side != s) continue;
        gwr::SideCfg& c = ctx->c.side[s];
        c.kind = kind;
        c.p = kind == GW_PEN_POWER ? p : 2.0;
        c.lifted_dim = kind == GW_PEN_POWER ? lifted_dim : 0;
        c.n_landmarks = n_landmarks;
        c.seed = seed;
        c.explicit_idx.clear();
        c.lm.fitted = false;
    }
    return ret(ctx, Status::ok());
}

gw_status gw_seeded_landmarks(int64_t n, int n_landmarks, uint64_t seed, int64_t* idx_host) {
    if (n < 1 || n_landmarks < 1 || !idx_host) return GW_EINVAL;
    const std::vector<int64_t> idx = gwr::seeded_landmarks(n, n_landmarks, seed);
    std::copy(idx.begin(), idx.end(), idx_host);
    return GW_OK;
}

gw_status gw_set_landmarks(gw_ctx* ctx, int side, const int64_t* idx_host, int n_landmarks) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (side < 0 || side > 2 || !idx_host || n_landmarks < 2) return ret(ctx, gwr::fail(GW_EINVAL, "bad landmarks"));
    for (int s = 0; s < 2; ++s) {
        if (side != 2 && side != s) continue;
        gwr::SideCfg& c = ctx->c.side[s];
        if (c.kind != GW_PEN_POWER) return ret(ctx, gwr::fail(GW_ESTATE, "landmarks need GW_PEN_POWER"));
        if (n_landmarks < c.lifted_dim + 1) return ret(ctx, gwr::fail(GW_EINVAL, "need n_landmarks > lifted_dim"));
        c.explicit_idx.assign(idx_host, idx_host + n_landmarks);
        c.n_landmarks = n_landmarks;
        c.lm.fitted = false;
    }
    return ret(ctx, Status::ok());
}

int gw_feature_dim(const gw_ctx* ctx, int side, int d) {
    if (!ctx || side < 0 || side > 1) return -1;
    return gwr::feature_dim(ctx->c.side[side], d);
}

gw_status gw_lift(gw_ctx* ctx, int side, const float* x, int64_t n, int d, const float* w, float* features) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (side < 0 || side > 1 || !x || !w || !features || n < 1 || d < 1 || d > gwl::MAX_DIM)
        return ret(ctx, gwr::fail(GW_EINVAL, "bad lift arguments"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    const int D = gwr::feature_dim(ctx->c.side[side], d);
    const int64_t n_pad = (n + 31) / 32 * 32;
    Status st;
    float* X = ctx->c.ws.get_t<float>("lift.X", (size_t)n_pad * D, &st);
    if (!st.good()) return ret(ctx, st);
    st = gwr::lift_side(ctx->c, side, x, n, d, w, X, n_pad, "lift.");
    if (!st.good()) return ret(ctx, st);
    if (hipMemcpyAsync(features, X, (size_t)n * D * sizeof(float), hipMemcpyDeviceToDevice, ctx->c.stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->c.stream) != hipSuccess)
        return ret(ctx, gwr::fail(GW_EDEVICE, "copy of lifted features"));
    return ret(ctx, Status::ok());
}

static gw_status solve_impl(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m,
                            int dy, const float* b, const gw_params* params, const float* gamma0, gw_result* out,
                            float* grad_x, float* grad_a, float* grad_y, float* grad_b, bool want_grad) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!out) return ret(ctx, gwr::fail(GW_EINVAL, "result is NULL"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, dx, a, y, m, dy, b, params, "s.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials && (!out->f || !out->g))
        return ret(ctx, gwr::fail(GW_EINVAL, "warm start needs result->f and result->g"));
    gwr::Solve solve(ctx->c, "s.");
    const float* f0 = params->use_init_potentials ? out->f : nullptr;
    const float* g0 = params->use_init_potentials ? out->g : nullptr;
    st = solve.setup(x, n, dx, a, y, m, dy, b, *params, gamma0, f0, g0, ctx->c.side[0].kind, ctx->c.side[1].kind,
                     ctx->c.stream);
    if (!st.good()) return ret(ctx, st);
    while (!solve.done()) {
        st = solve.outer_step();
        if (!st.good()) return ret(ctx, st);
    }
    st = solve.finish(out);
    if (!st.good()) return ret(ctx, st);
    if (want_grad) {
        st = solve.gradients(grad_x, grad_a, grad_y, grad_b);
        if (!st.good()) return ret(ctx, st);
    }
    return ret(ctx, Status::ok());
}

gw_status gw_solve(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                   const float* b, const gw_params* params, const float* gamma0, gw_result* out) {
    return solve_impl(ctx, x, n, dx, a, y, m, dy, b, params, gamma0, out, nullptr, nullptr, nullptr, nullptr, false);
}

gw_status gw_solve_noalloc(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m,
                           int dy, const float* b, const gw_params* params, const float* gamma0, gw_result* out) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!out) return ret(ctx, gwr::fail(GW_EINVAL, "result is NULL"));
    for (int s = 0; s < 2; ++s)
        if (ctx->c.side[s].kind == GW_PEN_POWER)
            return ret(ctx, gwr::fail(GW_EUNSUPPORTED,
                                      "gw_solve_noalloc takes squared-norm or feature penalties (lifting allocates)"));
    if (params && params->adaptive_inner)
        return ret(ctx, gwr::fail(GW_EUNSUPPORTED, "gw_solve_noalloc does not run adaptive counts"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, dx, a, y, m, dy, b, params, "n.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials && (!out->f || !out->g))
        return ret(ctx, gwr::fail(GW_EINVAL, "warm start needs result->f and result->g"));
    // this device's copy of the fixed scratch array: its address is looked
    // up once per device, here rather than in gw_create so that a failure
    // can only affect this entry point
    if (gwr::scratch_init(ctx->c.device) != hipSuccess)
        return ret(ctx, gwr::fail(GW_EDEVICE, "scratch array address unavailable on this device"));
    void* scratch = gwr::scratch_ptr(ctx->c.device);
    if (!scratch) return ret(ctx, gwr::fail(GW_EDEVICE, "scratch array address unavailable on this device"));
    // every buffer the solve takes: its planned footprint, the validation
    // and centring partials, the FP64 check's per-row sums, and alignment
    const size_t plan = gwr::Solve::plan_bytes(ctx->c, n, dx, m, dy, *params);
    if (plan == 0) return ret(ctx, gwr::fail(GW_EINVAL, "sizes rejected"));
    const size_t need = plan + 8 * (gwk::centre_part_doubles(n, dx) + gwk::centre_part_doubles(m, dy) + dx + dy) +
                        2 * (16 + 64 * 8) + 96 * 256;
    if (need > gwr::SCRATCH_BYTES)
        return ret(ctx, gwr::fail(GW_ENOMEM, "problem needs about " + std::to_string(need) +
                                                 " bytes of scratch; gw_solve_noalloc holds " +
                                                 std::to_string(gwr::SCRATCH_BYTES)));
    std::lock_guard<std::mutex> glk(g_noalloc_mu);
    gwr::Ctx local;
    local.device = ctx->c.device;
    local.stream = ctx->c.stream;
    for (int s = 0; s < 2; ++s) local.side[s].kind = ctx->c.side[s].kind;
    local.ws.use_arena(scratch, gwr::SCRATCH_BYTES);
    local.set_host_stage(g_noalloc_stage, sizeof(g_noalloc_stage));
    gwr::Solve solve(local, "n.");
    const float* f0 = params->use_init_potentials ? out->f : nullptr;
    const float* g0 = params->use_init_potentials ? out->g : nullptr;
    st = solve.setup(x, n, dx, a, y, m, dy, b, *params, gamma0, f0, g0, local.side[0].kind, local.side[1].kind,
                     local.stream);
    while (st.good() && !solve.done()) st = solve.outer_step();
    if (st.good()) st = solve.finish(out);
    // finish waits for the stream; on an error path wait too, so that no
    // kernel still reads the scratch array when the next call starts
    (void)hipStreamSynchronize(local.stream);
    return ret(ctx, st);
}

gw_status gw_solve_begin(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m,
                         int dy, const float* b, const gw_params* params, const float* gamma0, const gw_result* warm) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    ctx->c.stepped.reset();
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, dx, a, y, m, dy, b, params, "p.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials && (!warm || !warm->f || !warm->g))
        return ret(ctx, gwr::fail(GW_EINVAL, "warm start needs warm->f and warm->g"));
    std::unique_ptr<gwr::Solve> solve(new (std::nothrow) gwr::Solve(ctx->c, "p."));
    if (!solve) return ret(ctx, gwr::fail(GW_ENOMEM, "stepwise solve"));
    const float* f0 = params->use_init_potentials ? warm->f : nullptr;
    const float* g0 = params->use_init_potentials ? warm->g : nullptr;
    st = solve->setup(x, n, dx, a, y, m, dy, b, *params, gamma0, f0, g0, ctx->c.side[0].kind, ctx->c.side[1].kind,
                      ctx->c.stream);
    if (!st.good()) return ret(ctx, st);
    ctx->c.stepped = std::move(solve);
    return ret(ctx, Status::ok());
}

gw_status gw_solve_advance(gw_ctx* ctx, int n_steps, int32_t* outer_done) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (n_steps < 0) return ret(ctx, gwr::fail(GW_EINVAL, "n_steps must be >= 0"));
    gwr::Solve* solve = ctx->c.stepped.get();
    if (!solve) return ret(ctx, gwr::fail(GW_ESTATE, "no stepwise solve: call gw_solve_begin first"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st;
    for (int k = 0; k < n_steps && !solve->done() && st.good(); ++k) st = solve->outer_step();
    if (outer_done) *outer_done = solve->outer_done();
    if (!st.good()) ctx->c.stepped.reset();
    return ret(ctx, st);
}

gw_status gw_solve_end(gw_ctx* ctx, gw_result* out) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!out) return ret(ctx, gwr::fail(GW_EINVAL, "result is NULL"));
    gwr::Solve* solve = ctx->c.stepped.get();
    if (!solve) return ret(ctx, gwr::fail(GW_ESTATE, "no stepwise solve: call gw_solve_begin first"));
    if (solve->outer_done() < 1) return ret(ctx, gwr::fail(GW_ESTATE, "no outer step has run yet"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = solve->finish(out);
    ctx->c.stepped.reset();
    return ret(ctx, st);
}

gw_status gw_loss_and_grad(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m,
                           int dy, const float* b, const gw_params* params, const float* gamma0, gw_result* out,
                           float* grad_x, float* grad_a, float* grad_y, float* grad_b) {
    return solve_impl(ctx, x, n, dx, a, y, m, dy, b, params, gamma0, out, grad_x, grad_a, grad_y, grad_b, true);
}

gw_status gw_sgw(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                 const float* b, const gw_params* params, gw_sgw_result* out) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!out) return ret(ctx, gwr::fail(GW_EINVAL, "result is NULL"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, dx, a, y, m, dy, b, params, "sgw.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials) return ret(ctx, gwr::fail(GW_EINVAL, "the divergence starts from zero potentials"));
    gwr::Ctx& c = ctx->c;
    const int D = gwr::feature_dim(c.side[0], dx), E = gwr::feature_dim(c.side[1], dy);
    const int64_t n_pad = (n + 31) / 32 * 32, m_pad = (m + 31) / 32 * 32;
    float* X = c.ws.get_t<float>("sgw.X", (size_t)n_pad * D, &st);
    float* Y = c.ws.get_t<float>("sgw.Y", (size_t)m_pad * E, &st);
    if (!st.good()) return ret(ctx, st);
    st = gwr::lift_side(c, 0, x, n, dx, a, X, n_pad, "sgw.");
    if (st.good()) st = gwr::lift_side(c, 1, y, m, dy, b, Y, m_pad, "sgw.");
    if (!st.good()) return ret(ctx, st);
    gwr::FeatureSides guard(c);
    // (alpha, beta), (alpha, alpha), (beta, beta)
    const float* P[3] = {X, X, Y};
    const float* Q[3] = {Y, X, Y};
    const float* wp[3] = {a, a, b};
    const float* wq[3] = {b, a, b};
    const int64_t np[3] = {n, n, m}, nq[3] = {m, n, m};
    const int dp[3] = {D, D, E}, dq[3] = {E, D, E};
    gw_result r[3] = {};
    const double most = std::max({(double)n * m, (double)n * n, (double)m * m});
    st = run_independent(
        c, 3, most <= SIDE_BY_SIDE_MAX_ENTRIES,
        [&](int i, gwr::Solve& s) {
            return s.setup(P[i], np[i], dp[i], wp[i], Q[i], nq[i], dq[i], wq[i], *params, nullptr, nullptr, nullptr,
                           GW_PEN_FEATURES, GW_PEN_FEATURES, c.stream);
        },
        [&](int i, gwr::Solve& s) { return s.finish(&r[i]); });
    if (!st.good()) return ret(ctx, st);
    const gw_result &rxy = r[0], &rxx = r[1], &ryy = r[2];
    out->gw_xy = rxy.egw_objective;
    out->gw_xx = rxx.egw_objective;
    out->gw_yy = ryy.egw_objective;
    out->sgw = rxy.egw_objective - 0.5 * (rxx.egw_objective + ryy.egw_objective);
    out->marginal_err = std::max(rxy.marginal_err, std::max(rxx.marginal_err, ryy.marginal_err));
    out->dim_x = D;
    out->dim_y = E;
    return ret(ctx, Status::ok());
}

gw_status gw_sgw_grad(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m,
                      int dy, const float* b, const gw_params* params, gw_sgw_result* out, float* grad_x,
                      float* grad_y, float* grad_a, float* grad_b) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!out || !grad_x || !grad_y) return ret(ctx, gwr::fail(GW_EINVAL, "result or gradient is NULL"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, dx, a, y, m, dy, b, params, "sgw.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials) return ret(ctx, gwr::fail(GW_EINVAL, "the divergence starts from zero potentials"));
    gwr::Ctx& c = ctx->c;
    float* gxs = c.ws.get_t<float>("sgw.gxs", (size_t)n * dx, &st);
    float* gxt = c.ws.get_t<float>("sgw.gxt", (size_t)n * dx, &st);
    float* gys = c.ws.get_t<float>("sgw.gys", (size_t)m * dy, &st);
    float* gyt = c.ws.get_t<float>("sgw.gyt", (size_t)m * dy, &st);
    // weight gradients of the self terms (source and target sides)
    float* was = grad_a ? c.ws.get_t<float>("sgw.was", (size_t)n, &st) : nullptr;
    float* wat = grad_a ? c.ws.get_t<float>("sgw.wat", (size_t)n, &st) : nullptr;
    float* wbs = grad_b ? c.ws.get_t<float>("sgw.wbs", (size_t)m, &st) : nullptr;
    float* wbt = grad_b ? c.ws.get_t<float>("sgw.wbt", (size_t)m, &st) : nullptr;
    if (!st.good()) return ret(ctx, st);
    // each measure keeps its own side's penalty in every term: the pair
    // solve fits the landmark maps of |x - x'|^p (source on x, target on y),
    // and the self terms use that one map on both of their sides (in their
    // setups, which lift, and in their gradients, which chain through it)
    const float* P[3] = {x, x, y};
    const float* Q[3] = {y, x, y};
    const float* wp[3] = {a, a, b};
    const float* wq[3] = {b, a, b};
    const int64_t np[3] = {n, n, m}, nq[3] = {m, n, m};
    const int dp[3] = {dx, dx, dy}, dq[3] = {dy, dx, dy};
    float* gP[3] = {grad_x, gxs, gys};
    float* gQ[3] = {grad_y, gxt, gyt};
    float* gwP[3] = {grad_a, was, wbs};
    float* gwQ[3] = {grad_b, wat, wbt};
    auto share = [&](int i) {
        std::unique_ptr<gwr::SideShare> sh;
        if (i == 1) sh.reset(new gwr::SideShare(c, 0, 1));
        if (i == 2) sh.reset(new gwr::SideShare(c, 1, 0));
        return sh;
    };
    gw_result r[3] = {};
    const double most = std::max({(double)n * m, (double)n * n, (double)m * m});
    st = run_independent(
        c, 3, most <= SIDE_BY_SIDE_MAX_ENTRIES,
        [&](int i, gwr::Solve& s) {
            auto sh = share(i);
            return s.setup(P[i], np[i], dp[i], wp[i], Q[i], nq[i], dq[i], wq[i], *params, nullptr, nullptr, nullptr,
                           c.side[0].kind, c.side[1].kind, c.stream);
        },
        [&](int i, gwr::Solve& s) -> Status {
            auto sh = share(i);
            GW_TRY(s.finish(&r[i]));
            return s.gradients(gP[i], gwP[i], gQ[i], gwQ[i]);
        });
    if (!st.good()) return ret(ctx, st);
    const gw_result &rxy = r[0], &rxx = r[1], &ryy = r[2];
    // a self term carries its measure's weights in both marginals: its weight
    // gradient is the sum of its source and target gradients
    if (gwk::launch_sub_half_sum(grad_x, gxs, gxt, n * dx, c.stream) != hipSuccess ||
        gwk::launch_sub_half_sum(grad_y, gys, gyt, m * dy, c.stream) != hipSuccess ||
        (grad_a && gwk::launch_sub_half_sum(grad_a, was, wat, n, c.stream) != hipSuccess) ||
        (grad_b && gwk::launch_sub_half_sum(grad_b, wbs, wbt, m, c.stream) != hipSuccess) ||
        hipStreamSynchronize(c.stream) != hipSuccess)
        return ret(ctx, gwr::fail(GW_EDEVICE, "divergence gradient"));
    out->gw_xy = rxy.egw_objective;
    out->gw_xx = rxx.egw_objective;
    out->gw_yy = ryy.egw_objective;
    out->sgw = rxy.egw_objective - 0.5 * (rxx.egw_objective + ryy.egw_objective);
    out->marginal_err = std::max(rxy.marginal_err, std::max(rxx.marginal_err, ryy.marginal_err));
    out->dim_x = rxy.dim_x;
    out->dim_y = rxy.dim_y;
    return ret(ctx, Status::ok());
}

// Barycentre flow for |x - x'|^p lifted by frozen landmark maps: z is
// embedded by a map with side 0's settings fitted on z as given (its
// landmark points stay there while z moves), alpha and beta by maps with
// side 1's settings fitted on x and on y (seeds s and s + 1 unless side 1
// has explicit indices, which then index both).  Every solve runs on the
// embedded features; z's feature gradients chain through its map's
// Jacobian (Algorithm 12 with Algorithm 13).
static Status bary_lifted(gwr::Ctx& c, const float* x, int64_t n, const float* a, const float* y, int64_t m,
                          const float* b, int d, float* z, int64_t k, const float* w, double lambda, double step,
                          int n_steps, const gw_params* params, double* objective) {
    gwr::SideCfg cz = c.side[0], ca = c.side[1], cb = c.side[1];
    cz.lm = gwr::Landmarks();
    ca.lm = gwr::Landmarks();
    cb.lm = gwr::Landmarks();
    if (cb.explicit_idx.empty()) cb.seed = ca.seed + 1;
    struct FreeMaps {
        gwr::SideCfg* s[3];
        ~FreeMaps() {
            for (gwr::SideCfg* p : s) gwr::free_landmarks(p->lm);
        }
    } maps{{&cz, &ca, &cb}};
    const int Dz = cz.lifted_dim, Da = ca.lifted_dim;
    auto pad = [](int64_t v) { return (v + 31) / 32 * 32; };
    Status st;
    float* Zf = c.ws.get_t<float>("bc.Zf", (size_t)pad(k) * Dz, &st);
    float* Xa = c.ws.get_t<float>("bc.Xa", (size_t)pad(n) * Da, &st);
    float* Xb = c.ws.get_t<float>("bc.Xb", (size_t)pad(m) * Da, &st);
    float* gf[4];
    float* gp[4];
    for (int q = 0; q < 4; ++q) {
        gf[q] = c.ws.get_t<float>("bc.gf" + std::to_string(q), (size_t)k * Dz, &st);
        gp[q] = c.ws.get_t<float>("bc.gp" + std::to_string(q), (size_t)k * d, &st);
    }
    if (!st.good()) return st;
    // lift with a given side configuration in slot 0; the map fitted on the
    // first lift stays in cfg
    auto lift_with = [&](gwr::SideCfg& cfg, const float* P, int64_t np, const float* wp, float* out) -> Status {
        gwr::SideCfg saved = std::move(c.side[0]);
        c.side[0] = std::move(cfg);
        Status s = gwr::lift_side(c, 0, P, np, d, wp, out, pad(np), "bc.");
        cfg = std::move(c.side[0]);
        c.side[0] = std::move(saved);
        return s;
    };
    GW_TRY(lift_with(ca, x, n, a, Xa));
    GW_TRY(lift_with(cb, y, m, b, Xb));
    // problems on the lifted features: P (dimension dp) against Q (dq), and
    // where to write the feature gradients of P and Q (null: not wanted)
    struct Problem {
        const float *P, *wp, *Q, *wq;
        int64_t np, nq;
        int dp, dq;
        float *gP, *gQ;
    };
    const double most = std::max({(double)k * n, (double)k * m, (double)k * k, (double)n * n, (double)m * m});
    auto run = [&](const Problem* pr, int cnt, double* egw) -> Status {
        gwr::FeatureSides fs(c);
        return run_independent(
            c, cnt, most <= SIDE_BY_SIDE_MAX_ENTRIES,
            [&](int i, gwr::Solve& s) {
                return s.setup(pr[i].P, pr[i].np, pr[i].dp, pr[i].wp, pr[i].Q, pr[i].nq, pr[i].dq, pr[i].wq, *params,
                               nullptr, nullptr, nullptr, GW_PEN_FEATURES, GW_PEN_FEATURES, c.stream);
            },
            [&](int i, gwr::Solve& s) -> Status {
                gw_result r{};
                GW_TRY(s.finish(&r));
                egw[i] = r.egw_objective;
                if (pr[i].gP || pr[i].gQ) GW_TRY(s.gradients(pr[i].gP, nullptr, pr[i].gQ, nullptr));
                return Status::ok();
            });
    };
    double eself[2] = {0.0, 0.0};
    const Problem selfs[2] = {{Xa, a, Xa, a, n, n, Da, Da, nullptr, nullptr},
                              {Xb, b, Xb, b, m, m, Da, Da, nullptr, nullptr}};
    GW_TRY(run(selfs, 2, eself));
    const double eaa = eself[0], ebb = eself[1];
    for (int s = 0; s <= n_steps; ++s) {
        const bool last = s == n_steps;
        GW_TRY(lift_with(cz, z, k, w, Zf));
        double ez[3] = {0.0, 0.0, 0.0};
        const Problem probs[3] = {{Zf, w, Xa, a, k, n, Dz, Da, last ? nullptr : gf[0], nullptr},
                                  {Zf, w, Xb, b, k, m, Dz, Da, last ? nullptr : gf[1], nullptr},
                                  {Zf, w, Zf, w, k, k, Dz, Dz, last ? nullptr : gf[2], last ? nullptr : gf[3]}};
        GW_TRY(run(probs, 3, ez));
        const double ezx = ez[0], ezy = ez[1], ezz = ez[2];
        if (objective)
            objective[s] = (1.0 - lambda) * (ezx - 0.5 * (ezz + eaa)) + lambda * (ezy - 0.5 * (ezz + ebb));
        if (last) break;
        const gwr::Landmarks& lm = cz.lm;
        for (int q = 0; q < 4; ++q)
            GW_HIP(gwk::launch_nystrom_jt(z, k, lm.d_in, lm.pts, lm.n_l, lm.W, lm.dim, (float)cz.p, gf[q], gp[q],
                                          c.stream));
        GW_HIP(gwk::launch_bary_step(z, k, d, w, gp[0], gp[1], gp[2], gp[3], (float)lambda, (float)step, c.stream));
    }
    GW_HIP(hipStreamSynchronize(c.stream));
    return Status::ok();
}

gw_status gw_sgw_barycenter(gw_ctx* ctx, const float* x, int64_t n, const float* a, const float* y, int64_t m,
                            const float* b, int d, float* z, int64_t k, const float* w, double lambda, double step,
                            int n_steps, const gw_params* params, double* objective) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!z || !w) return ret(ctx, gwr::fail(GW_EINVAL, "z or w is NULL"));
    if (k < 1 || k > ((int64_t)1 << 30)) return ret(ctx, gwr::fail(GW_EINVAL, "k out of range"));
    if (!(lambda >= 0.0 && lambda <= 1.0)) return ret(ctx, gwr::fail(GW_EINVAL, "lambda must be in [0, 1]"));
    if (!(step >= 0.0) || !std::isfinite(step)) return ret(ctx, gwr::fail(GW_EINVAL, "step must be finite and >= 0"));
    if (n_steps < 0 || n_steps > 100000) return ret(ctx, gwr::fail(GW_EINVAL, "n_steps must be in [0, 100000]"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(ctx->c, x, n, d, a, y, m, d, b, params, "bc.");
    if (st.good()) st = gwr::validate_inputs(ctx->c, z, k, d, w, x, n, d, a, params, "bc.");
    if (!st.good()) return ret(ctx, st);
    if (params->use_init_potentials) return ret(ctx, gwr::fail(GW_EINVAL, "the divergence starts from zero potentials"));
    gwr::Ctx& c = ctx->c;
    const int kind = c.side[0].kind;
    if (kind == GW_PEN_POWER && c.side[1].kind == GW_PEN_POWER)
        return ret(ctx, bary_lifted(c, x, n, a, y, m, b, d, z, k, w, lambda, step, n_steps, params, objective));
    if (c.side[1].kind != kind || (kind != GW_PEN_SQEUCLID && kind != GW_PEN_FEATURES))
        return ret(ctx, gwr::fail(GW_EUNSUPPORTED,
                                  "the barycentre flow needs the same penalty kind on both sides"));
    float* g1 = c.ws.get_t<float>("bc.g1", (size_t)k * d, &st);
    float* g2 = c.ws.get_t<float>("bc.g2", (size_t)k * d, &st);
    float* gs = c.ws.get_t<float>("bc.gs", (size_t)k * d, &st);
    float* gt = c.ws.get_t<float>("bc.gt", (size_t)k * d, &st);
    if (!st.good()) return ret(ctx, st);
    // one problem: P against Q with weights wp and wq, and where to write
    // the gradients of P and Q (null: not wanted)
    struct Problem {
        const float *P, *wp, *Q, *wq;
        int64_t np, nq;
        float *gP, *gQ;
    };
    const double most = std::max({(double)k * n, (double)k * m, (double)k * k, (double)n * n, (double)m * m});
    auto run = [&](const Problem* pr, int cnt, double* egw) -> Status {
        return run_independent(
            c, cnt, most <= SIDE_BY_SIDE_MAX_ENTRIES,
            [&](int i, gwr::Solve& s) {
                return s.setup(pr[i].P, pr[i].np, d, pr[i].wp, pr[i].Q, pr[i].nq, d, pr[i].wq, *params, nullptr,
                               nullptr, nullptr, kind, kind, c.stream);
            },
            [&](int i, gwr::Solve& s) -> Status {
                gw_result r{};
                GW_TRY(s.finish(&r));
                egw[i] = r.egw_objective;
                if (pr[i].gP || pr[i].gQ) GW_TRY(s.gradients(pr[i].gP, nullptr, pr[i].gQ, nullptr));
                return Status::ok();
            });
    };
    // GW(alpha, alpha) and GW(beta, beta) do not move with z
    double eself[2] = {0.0, 0.0};
    const Problem selfs[2] = {{x, a, x, a, n, n, nullptr, nullptr}, {y, b, y, b, m, m, nullptr, nullptr}};
    st = run(selfs, 2, eself);
    const double eaa = eself[0], ebb = eself[1];
    for (int s = 0; st.good() && s <= n_steps; ++s) {
        const bool last = s == n_steps;
        double ez[3] = {0.0, 0.0, 0.0};
        const Problem probs[3] = {{z, w, x, a, k, n, last ? nullptr : g1, nullptr},
                                  {z, w, y, b, k, m, last ? nullptr : g2, nullptr},
                                  {z, w, z, w, k, k, last ? nullptr : gs, last ? nullptr : gt}};
        st = run(probs, 3, ez);
        if (!st.good()) break;
        const double ezx = ez[0], ezy = ez[1], ezz = ez[2];
        if (objective)
            objective[s] = (1.0 - lambda) * (ezx - 0.5 * (ezz + eaa)) + lambda * (ezy - 0.5 * (ezz + ebb));
        if (!last && gwk::launch_bary_step(z, k, d, w, g1, g2, gs, gt, (float)lambda, (float)step, c.stream) !=
                         hipSuccess)
            st = gwr::fail(GW_EDEVICE, "barycentre step");
    }
    if (st.good() && hipStreamSynchronize(c.stream) != hipSuccess) st = gwr::fail(GW_EDEVICE, "barycentre flow");
    return ret(ctx, st);
}

gw_status gw_set_profiling(gw_ctx* ctx, int enable) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx->c.prof.reset();
    ctx->c.prof.on = enable != 0;
    return ret(ctx, Status::ok());
}

gw_status gw_get_profile(gw_ctx* ctx, gw_profile* out) {
    if (!ctx || !out) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    (void)hipSetDevice(ctx->c.device);
    Status st = ctx->c.prof.collect(ctx->c.stream);
    if (!st.good()) return ret(ctx, st);
    for (int k = 0; k < GW_PROF_CLASSES; ++k) {
        out->launches[k] = ctx->c.prof.launches[k];
        out->milliseconds[k] = ctx->c.prof.ms[k];
        out->idle_launches[k] = ctx->c.prof.idle_launches[k];
        out->idle_milliseconds[k] = ctx->c.prof.idle_ms[k];
    }
    out->entries_per_pass = ctx->c.prof.entries;
    return ret(ctx, Status::ok());
}

void gw_destroy(gw_ctx* ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->c.mu);
        (void)hipSetDevice(ctx->c.device);
        (void)hipStreamSynchronize(ctx->c.stream);
        gwr::release_landmarks(ctx->c);
        ctx->c.ws.release_all();
    }
    delete ctx;
}

const char* gw_last_error(const gw_ctx* ctx) {
    if (!ctx) return "NULL context";
    return ctx->c.err.c_str();
}

}  // extern "C"
