// Multiscale-GW (Appendix B, "Implementation of Multiscale-GW"): the K-Means
// coarsening, Algorithm 8 (Interpolate), Algorithm 7, and their extern "C"
// entry points (declared in include/gw.h).
#include <chrono>
#include <cmath>
#include <cstring>

#include "gw_msgw.h"
#include "runtime.h"

namespace gwr {

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Weighted K-Means of the first n rows of X (row stride ldx, D columns):
// starts at the seeded rows, n_lloyd Lloyd iterations, non-empty clusters
// compacted into Xc / wc (dense, D columns); assign (device, nullable).
static Status kmeans(Ctx& c, const float* X, int64_t n, int ldx, int D, const float* w, int64_t k, int n_lloyd,
                     uint64_t seed, float* Xc, float* wc, int* assign, int64_t* kc, const std::string& tag) {
    Status st;
    const std::vector<int64_t> idx = seeded_landmarks(n, (int)k, seed);
    if ((int64_t)idx.size() != k) return fail(GW_EINVAL, "k-means start rows");
    int64_t* d_idx = c.ws.get_t<int64_t>(tag + "km.idx", k, &st);
    float* C = c.ws.get_t<float>(tag + "km.C", (size_t)k * D, &st);
    unsigned long long* sums = c.ws.get_t<unsigned long long>(tag + "km.S", (size_t)k * D + k, &st);
    int* asg = assign ? assign : c.ws.get_t<int>(tag + "km.assign", n, &st);
    int* kept = c.ws.get_t<int>(tag + "km.kept", k, &st);
    int* dkc = c.ws.get_t<int>(tag + "km.kc", 1, &st);
    unsigned int* dmax = c.ws.get_t<unsigned int>(tag + "km.max", 1, &st);
    if (!st.good()) return st;
    GW_HIP(hipMemcpyAsync(d_idx, idx.data(), k * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    GW_HIP(gwk::launch_km_maxabs(X, n, ldx, D, dmax, c.stream));
    unsigned int mbits = 0;
    GW_HIP(hipMemcpyAsync(&mbits, dmax, sizeof(mbits), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    float mx = 0.f;
    std::memcpy(&mx, &mbits, sizeof(mx));
    if (!std::isfinite(mx)) return fail(GW_EINVAL, "non-finite feature in k-means input");
    // grid 2^-S of the cluster sums: max|X| 2^S <= 2^61
    int S = gwk::KM_WEIGHT_EXP;
    if (mx > 0.f) {
        int e = 0;
        std::frexp((double)mx, &e);
        S = gwk::KM_WEIGHT_EXP - e;
    }
    GW_HIP(gwk::launch_km_gather(X, ldx, D, d_idx, (int)k, C, D, c.stream));
    for (int it = 0; it < n_lloyd; ++it)
        GW_HIP(gwk::launch_km_iteration(X, n, ldx, D, w, C, (int)k, D, S, asg, sums, sums + (size_t)k * D,
                                        c.stream));
    GW_HIP(gwk::launch_km_compact(sums + (size_t)k * D, C, (int)k, D, D, Xc, wc, kept, dkc, c.stream));
    int hk = 0;
    GW_HIP(hipMemcpyAsync(&hk, dkc, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    if (hk < 1 || hk > k) return fail(GW_EDEVICE, "k-means compaction");
    *kc = hk;
    return Status::ok();
}

// Algorithm 8 for one side (see gw_interpolate); P, Q with row strides ldp, ldq.
static Status interpolate(Ctx& c, int side, const float* h, const float* P, int64_t nq, int ldp, const float* Q,
                          int64_t nr, int ldq, const float* w, const float* gamma, int D, int E, double eps,
                          float* out, const std::string& tag) {
    Status st;
    const int ld = (D + 3) / 4 * 4;
    float* Pb = c.ws.get_t<float>(tag + "ip.P", (size_t)nq * ld, &st);
    float* Qb = c.ws.get_t<float>(tag + "ip.Q", (size_t)nr * ld, &st);
    float* ph = c.ws.get_t<float>(tag + "ip.ph", nq, &st);
    float* qh = c.ws.get_t<float>(tag + "ip.qh", nr, &st);
    float* hb = c.ws.get_t<float>(tag + "ip.hb", nr, &st);
    if (!st.good()) return st;
    if (side == 0) {
        GW_HIP(gwk::launch_lift_bar(P, nq, ldp, D, nullptr, D, Pb, ld, ph, c.stream));
        GW_HIP(gwk::launch_lift_bar(Q, nr, ldq, E, gamma, D, Qb, ld, qh, c.stream));
    } else {
        GW_HIP(gwk::launch_lift_bar(P, nq, ldp, E, gamma, D, Pb, ld, ph, c.stream));
        GW_HIP(gwk::launch_lift_bar(Q, nr, ldq, D, nullptr, D, Qb, ld, qh, c.stream));
    }
    GW_HIP(gwk::launch_interp(Pb, nq, ld, Qb, (int)nr, ld, D, ph, qh, w, h, eps / 8.0, hb, out, c.stream));
    return Status::ok();
}

}  // namespace gwr

using gwr::Ctx;
using gwr::Status;

static gw_status ret(gw_ctx* ctx, const Status& s) {
    if (ctx) ctx->c.err = s.good() ? std::string() : s.msg;
    return s.code;
}

extern "C" {

gw_status gw_kmeans(gw_ctx* ctx, const float* X, int64_t n, int D, const float* w, int64_t k, int n_lloyd,
                    uint64_t seed, float* Xc, float* wc, int32_t* assign, int64_t* kc) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!X || !w || !Xc || !wc || !kc) return ret(ctx, gwr::fail(GW_EINVAL, "NULL pointer"));
    if (n < 1 || n > ((int64_t)1 << 30)) return ret(ctx, gwr::fail(GW_EINVAL, "n out of range"));
    if (D < 1 || D > 256) return ret(ctx, gwr::fail(GW_EINVAL, "D must be in [1, 256]"));
    if (k < 1 || k > n) return ret(ctx, gwr::fail(GW_EINVAL, "k must be in [1, n]"));
    if (n_lloyd < 1 || n_lloyd > 10000) return ret(ctx, gwr::fail(GW_EINVAL, "n_lloyd must be in [1, 10000]"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::check_points(ctx->c, X, n * D, w, n, "km.", "k-means input");
    if (st.good()) st = gwr::kmeans(ctx->c, X, n, D, D, w, k, n_lloyd, seed, Xc, wc, assign, kc, "km.");
    return ret(ctx, st);
}

gw_status gw_interpolate(gw_ctx* ctx, int side, const float* h, const float* P, int64_t nq, const float* Q,
                         int64_t nr, const float* w, const float* gamma, int D, int E, double eps, float* out) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!h || !P || !Q || !w || !gamma || !out) return ret(ctx, gwr::fail(GW_EINVAL, "NULL pointer"));
    if (side != 0 && side != 1) return ret(ctx, gwr::fail(GW_EINVAL, "side must be 0 or 1"));
    if (nq < 1 || nr < 1 || nq > ((int64_t)1 << 30) || nr > ((int64_t)1 << 30))
        return ret(ctx, gwr::fail(GW_EINVAL, "sizes out of range"));
    if (D < 1 || D > 256 || E < 1 || E > 256) return ret(ctx, gwr::fail(GW_EINVAL, "D and E must be in [1, 256]"));
    if (!(eps > 0.0) || !std::isfinite(eps)) return ret(ctx, gwr::fail(GW_EINVAL, "eps must be finite and > 0"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    const int dp = side == 0 ? D : E, dr = side == 0 ? E : D;
    Status st = gwr::interpolate(ctx->c, side, h, P, nq, dp, Q, nr, dr, w, gamma, D, E, eps, out, "ip.");
    if (st.good() && hipStreamSynchronize(ctx->c.stream) != hipSuccess)
        st = gwr::fail(GW_EDEVICE, "interpolation");
    return ret(ctx, st);
}

gw_status gw_msgw(gw_ctx* ctx, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                  const float* b, const gw_params* coarse, const gw_params* fine, const gw_msgw_opts* opts,
                  const float* gamma0, gw_result* out, gw_msgw_info* info) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    Ctx& c = ctx->c;
    if (!out || !opts) return ret(ctx, gwr::fail(GW_EINVAL, "result or options is NULL"));
    if (!out->f || !out->g) return ret(ctx, gwr::fail(GW_EINVAL, "result->f and result->g are required"));
    if (hipSetDevice(c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::validate_inputs(c, x, n, dx, a, y, m, dy, b, coarse, "ms.");
    if (st.good()) st = gwr::validate_inputs(c, x, n, dx, a, y, m, dy, b, fine, "ms.");
    if (!st.good()) return ret(ctx, st);
    if (coarse->use_init_potentials || fine->use_init_potentials)
        return ret(ctx, gwr::fail(GW_EINVAL, "use_init_potentials must be 0"));
    if (!(opts->rho > 0.0 && opts->rho <= 1.0)) return ret(ctx, gwr::fail(GW_EINVAL, "rho must be in (0, 1]"));
    if (opts->n_lloyd < 1 || opts->n_lloyd > 10000)
        return ret(ctx, gwr::fail(GW_EINVAL, "n_lloyd must be in [1, 10000]"));
    if (opts->reserved != 0) return ret(ctx, gwr::fail(GW_EINVAL, "reserved must be 0"));
    st = gwr::check_points(c, x, n * dx, a, n, "ms.", "source");
    if (st.good()) st = gwr::check_points(c, y, m * dy, b, m, "ms.", "target");
    if (!st.good()) return ret(ctx, st);

    const double t0 = gwr::now_ms();
    const int D = gwr::feature_dim(c.side[0], dx), E = gwr::feature_dim(c.side[1], dy);
    if (D < 1 || E < 1 || D > 256 || E > 256) return ret(ctx, gwr::fail(GW_EINVAL, "lifted dimension out of range"));
    const int64_t n_pad = (n + 31) / 32 * 32, m_pad = (m + 31) / 32 * 32;
    auto clusters = [&](int64_t count) {
        int64_t k = (int64_t)std::ceil(opts->rho * (double)count);
        return k < 1 ? (int64_t)1 : (k > count ? count : k);
    };
    const int64_t kx = clusters(n), ky = clusters(m);
    const int64_t kx_pad = (kx + 31) / 32 * 32, ky_pad = (ky + 31) / 32 * 32;
    float* X = c.ws.get_t<float>("ms.X", (size_t)n_pad * D, &st);
    float* Y = c.ws.get_t<float>("ms.Y", (size_t)m_pad * E, &st);
    float* Xc = c.ws.get_t<float>("ms.Xc", (size_t)kx * D, &st);
    float* Yc = c.ws.get_t<float>("ms.Yc", (size_t)ky * E, &st);
    float* ac = c.ws.get_t<float>("ms.ac", kx, &st);
    float* bc = c.ws.get_t<float>("ms.bc", ky, &st);
    float* Xcc = c.ws.get_t<float>("ms.Xcc", (size_t)kx_pad * D, &st);
    float* Ycc = c.ws.get_t<float>("ms.Ycc", (size_t)ky_pad * E, &st);
    double* cpart = c.ws.get_t<double>("ms.cpart", gwk::centre_part_doubles(kx > ky ? kx : ky, D > E ? D : E), &st);
    double* cmean = c.ws.get_t<double>("ms.cmean", D > E ? D : E, &st);
    float* fc = c.ws.get_t<float>("ms.fc", kx, &st);
    float* gc = c.ws.get_t<float>("ms.gc", ky, &st);
    float* Gc = c.ws.get_t<float>("ms.G", (size_t)D * E, &st);
    if (!st.good()) return ret(ctx, st);
    st = gwr::lift_side(c, 0, x, n, dx, a, X, n_pad, "ms.");
    if (st.good()) st = gwr::lift_side(c, 1, y, m, dy, b, Y, m_pad, "ms.");
    if (!st.good()) return ret(ctx, st);

    // Coarsen both sides, then re-centre the coarse features with their weights
    int64_t kcx = 0, kcy = 0;
    st = gwr::kmeans(c, X, n, D, D, a, kx, opts->n_lloyd, opts->seed, Xc, ac, nullptr, &kcx, "ms.x.");
    if (st.good())
        st = gwr::kmeans(c, Y, m, E, E, b, ky, opts->n_lloyd, opts->seed + 1, Yc, bc, nullptr, &kcy, "ms.y.");
    if (!st.good()) return ret(ctx, st);
    const int64_t kcx_pad = (kcx + 31) / 32 * 32, kcy_pad = (kcy + 31) / 32 * 32;
    if (gwk::launch_centre(Xc, kcx, kcx_pad, D, D, ac, cpart, cmean, Xcc, c.stream) != hipSuccess ||
        gwk::launch_centre(Yc, kcy, kcy_pad, E, E, bc, cpart, cmean, Ycc, c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
        return ret(ctx, gwr::fail(GW_EDEVICE, "centring of the coarse features"));
    const double t1 = gwr::now_ms();

    gwr::FeatureSides guard(c);
    gw_result rc{};
    rc.f = fc;
    rc.g = gc;
    rc.gamma = Gc;
    {
        gwr::Solve s1(c, "s.");
        st = s1.setup(Xcc, kcx, D, ac, Ycc, kcy, E, bc, *coarse, gamma0, nullptr, nullptr, GW_PEN_FEATURES,
                      GW_PEN_FEATURES, c.stream);
        while (st.good() && !s1.done()) st = s1.outer_step();
        if (st.good()) st = s1.finish(&rc);
        if (!st.good()) return ret(ctx, st);
    }
    const double t2 = gwr::now_ms();

    st = gwr::interpolate(c, 0, gc, X, n, D, Ycc, kcy, E, bc, Gc, D, E, fine->eps_start, out->f, "ms.");
    if (st.good()) st = gwr::interpolate(c, 1, fc, Y, m, E, Xcc, kcx, D, ac, Gc, D, E, fine->eps_start, out->g, "ms.");
    if (!st.good()) return ret(ctx, st);
    if (hipStreamSynchronize(c.stream) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "interpolation"));
    const double t3 = gwr::now_ms();

    gw_params pf = *fine;
    pf.use_init_potentials = 1;
    {
        gwr::Solve s2(c, "s.");
        st = s2.setup(X, n, D, a, Y, m, E, b, pf, Gc, out->f, out->g, GW_PEN_FEATURES, GW_PEN_FEATURES, c.stream);
        while (st.good() && !s2.done()) st = s2.outer_step();
        if (st.good()) st = s2.finish(out);
        if (!st.good()) return ret(ctx, st);
    }
    const double t4 = gwr::now_ms();
    if (info) {
        info->n_coarse = kcx;
        info->m_coarse = kcy;
        info->coarse_loss_lift = rc.loss_lift;
        info->coarse_egw_objective = rc.egw_objective;
        info->coarse_marginal_err = rc.marginal_err;
        info->ms_coarsen = t1 - t0;
        info->ms_coarse_solve = t2 - t1;
        info->ms_interpolate = t3 - t2;
        info->ms_fine_solve = t4 - t3;
    }
    return ret(ctx, Status::ok());
}

}  // extern "C"
