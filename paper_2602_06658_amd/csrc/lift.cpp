// Landmark kernel PCA for GW_PEN_POWER (Section 5, "CNT Embeddings";
// Algorithm 4, the Kernel PCA paragraph of Appendix B.2, Algorithm 13).
// The landmark eigensolve runs once per side in FP64 (rocSOLVER dsyevd) and
// is frozen in the context until the penalty is set again.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <iterator>
#include <numeric>

#include "gw_lift.h"
#include "runtime.h"

namespace gwr {

static void free_lm(Landmarks& lm) {
    if (lm.pts) (void)hipFree(lm.pts);
    if (lm.W) (void)hipFree(lm.W);
    if (lm.chat) (void)hipFree(lm.chat);
    if (lm.sumW) (void)hipFree(lm.sumW);
    lm = Landmarks();
}

void free_landmarks(Landmarks& lm) { free_lm(lm); }

void release_landmarks(Ctx& c) {
    for (int s = 0; s < 2; ++s) free_lm(c.side[s].lm);
    if (c.rocblas) {
        rocblas_destroy_handle((rocblas_handle)c.rocblas);
        c.rocblas = nullptr;
    }
}

// SplitMix64 (Steele, Lea, Flood 2014) driving a Fisher-Yates shuffle; the
// landmark set is the first n_l entries of the permutation.
static uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::vector<int64_t> seeded_landmarks(int64_t n, int nl, uint64_t seed) {
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    uint64_t st = seed;
    for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(splitmix64(st) % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
    }
    perm.resize(std::min<int64_t>(nl, n));
    std::sort(perm.begin(), perm.end());
    return perm;
}

static Status fit_landmarks(Ctx& c, int side, const float* x, int64_t n, int d, const std::string& tag) {
    SideCfg& s = c.side[side];
    Landmarks& lm = s.lm;
    free_lm(lm);
    std::vector<int64_t> idx = s.explicit_idx.empty() ? seeded_landmarks(n, s.n_landmarks, s.seed) : s.explicit_idx;
    for (int64_t v : idx)
        if (v < 0 || v >= n) return fail(GW_EINVAL, "landmark index out of range");
    const int nl = (int)idx.size();
    const int D = s.lifted_dim;
    if (nl < D + 1) return fail(GW_EINVAL, "fewer landmarks than lifted_dim + 1");
    if (d > 32) return fail(GW_EUNSUPPORTED, "power penalty lifting supports input dimension <= 32");
    Status st;
    auto& ws = c.ws;
    int64_t* didx = (int64_t*)ws.get(tag + "lmidx", nl * sizeof(int64_t), &st);
    double* K = ws.get_t<double>(tag + "lmK", (size_t)nl * nl, &st);
    double* rmean = ws.get_t<double>(tag + "lmr", nl, &st);
    double* g = ws.get_t<double>(tag + "lmg", 1, &st);
    double* eval = ws.get_t<double>(tag + "lmev", nl, &st);
    double* ework = ws.get_t<double>(tag + "lmew", nl, &st);
    int* info = ws.get_t<int>(tag + "lminfo", 1, &st);
    if (!st.good()) return st;
    GW_HIP(hipMalloc(&lm.pts, (size_t)nl * d * sizeof(float)));
    GW_HIP(hipMalloc(&lm.W, (size_t)nl * D * sizeof(float)));
    GW_HIP(hipMalloc(&lm.chat, (size_t)nl * sizeof(float)));
    GW_HIP(hipMalloc(&lm.sumW, (size_t)D * sizeof(float)));
    GW_HIP(hipMemcpyAsync(didx, idx.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    GW_HIP(gwk::launch_gather(x, d, didx, nl, lm.pts, c.stream));
    GW_HIP(gwk::launch_landmark_kernel(lm.pts, nl, d, s.p, K, rmean, g, c.stream));
    if (!c.rocblas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) return fail(GW_EDEVICE, "rocblas_create_handle");
        c.rocblas = h;
    }
    rocblas_handle h = (rocblas_handle)c.rocblas;
    if (rocblas_set_stream(h, c.stream) != rocblas_status_success) return fail(GW_EDEVICE, "rocblas_set_stream");
    if (rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nl, K, nl, eval, ework, info) !=
        rocblas_status_success)
        return fail(GW_EDEVICE, "rocsolver_dsyevd");
    GW_HIP(gwk::launch_nystrom_weights(K, eval, nl, D, 1e-12, rmean, lm.W, lm.chat, lm.sumW, c.stream));
    int hinfo = 0;
    double hg = 0.0;
    std::vector<double> hev(nl);
    GW_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipMemcpyAsync(&hg, g, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipMemcpyAsync(hev.data(), eval, nl * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    if (hinfo != 0) return fail(GW_ENUMERIC, "landmark eigensolve did not converge");
    lm.cbarbar = hg;
    lm.lambda.assign(hev.rbegin(), hev.rbegin() + std::min(D, nl));
    lm.n_l = nl;
    lm.d_in = d;
    lm.dim = D;
    lm.fitted = true;
    return Status::ok();
}

// Both sides' landmark maps with one batched eigensolve.  A 512 x 512 dsyevd
// is a chain of some 2,800 small launches, and the batched routine issues
// the same chain for both matrices.  Fits only when both sides use the power
// penalty, neither is fitted and both have the same landmark count and
// valid settings; otherwise it leaves the sides to the per-side fit (which
// also reports any error).  The per-matrix arithmetic is that of the
// single-matrix routine.
Status fit_landmarks_pair(Ctx& c, const float* x, int64_t n, int dx, const float* y, int64_t m, int dy,
                          const std::string& tag) {
    SideCfg* sc[2] = {&c.side[0], &c.side[1]};
    const float* pts_in[2] = {x, y};
    const int64_t cnt[2] = {n, m};
    const int din[2] = {dx, dy};
    std::vector<int64_t> idx[2];
    for (int k = 0; k < 2; ++k) {
        const SideCfg& s = *sc[k];
        if (s.kind != GW_PEN_POWER || s.lm.fitted) return Status::ok();
        idx[k] = s.explicit_idx.empty() ? seeded_landmarks(cnt[k], s.n_landmarks, s.seed) : s.explicit_idx;
        for (int64_t v : idx[k])
            if (v < 0 || v >= cnt[k]) return Status::ok();
        if ((int)idx[k].size() < s.lifted_dim + 1 || din[k] > 32) return Status::ok();
    }
    if (idx[0].size() != idx[1].size()) return Status::ok();
    const int nl = (int)idx[0].size();
    Status st;
    auto& ws = c.ws;
    double* K = ws.get_t<double>(tag + "pairK", 2 * (size_t)nl * nl, &st);
    double* eval = ws.get_t<double>(tag + "pairev", 2 * (size_t)nl, &st);
    double* ework = ws.get_t<double>(tag + "pairew", 2 * (size_t)nl, &st);
    int* info = ws.get_t<int>(tag + "pairinfo", 2, &st);
    int64_t* didx[2];
    double* rmean[2];
    double* g[2];
    for (int k = 0; k < 2; ++k) {
        const std::string t = tag + "pair" + std::to_string(k);
        didx[k] = (int64_t*)ws.get(t + "idx", nl * sizeof(int64_t), &st);
        rmean[k] = ws.get_t<double>(t + "r", nl, &st);
        g[k] = ws.get_t<double>(t + "g", 1, &st);
    }
    if (!st.good()) return st;
    for (int k = 0; k < 2; ++k) {
        Landmarks& lm = sc[k]->lm;
        free_lm(lm);
        const int D = sc[k]->lifted_dim, d = din[k];
        GW_HIP(hipMalloc(&lm.pts, (size_t)nl * d * sizeof(float)));
        GW_HIP(hipMalloc(&lm.W, (size_t)nl * D * sizeof(float)));
        GW_HIP(hipMalloc(&lm.chat, (size_t)nl * sizeof(float)));
        GW_HIP(hipMalloc(&lm.sumW, (size_t)D * sizeof(float)));
        GW_HIP(hipMemcpyAsync(didx[k], idx[k].data(), nl * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
        GW_HIP(gwk::launch_gather(pts_in[k], d, didx[k], nl, lm.pts, c.stream));
        GW_HIP(gwk::launch_landmark_kernel(lm.pts, nl, d, sc[k]->p, K + (size_t)k * nl * nl, rmean[k], g[k],
                                           c.stream));
    }
    if (!c.rocblas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) return fail(GW_EDEVICE, "rocblas_create_handle");
        c.rocblas = h;
    }
    rocblas_handle h = (rocblas_handle)c.rocblas;
    if (rocblas_set_stream(h, c.stream) != rocblas_status_success) return fail(GW_EDEVICE, "rocblas_set_stream");
    if (rocsolver_dsyevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, nl, K, nl,
                                         (rocblas_stride)nl * nl, eval, nl, ework, nl, info, 2) != rocblas_status_success)
        return fail(GW_EDEVICE, "rocsolver_dsyevd_strided_batched");
    for (int k = 0; k < 2; ++k) {
        Landmarks& lm = sc[k]->lm;
        GW_HIP(gwk::launch_nystrom_weights(K + (size_t)k * nl * nl, eval + (size_t)k * nl, nl, sc[k]->lifted_dim,
                                           1e-12, rmean[k], lm.W, lm.chat, lm.sumW, c.stream));
    }
    int hinfo[2] = {0, 0};
    double hg[2] = {0.0, 0.0};
    std::vector<double> hev(2 * (size_t)nl);
    GW_HIP(hipMemcpyAsync(hinfo, info, 2 * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    for (int k = 0; k < 2; ++k) GW_HIP(hipMemcpyAsync(&hg[k], g[k], sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipMemcpyAsync(hev.data(), eval, 2 * (size_t)nl * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    for (int k = 0; k < 2; ++k) {
        Landmarks& lm = sc[k]->lm;
        if (hinfo[k] != 0) {
            free_lm(sc[0]->lm);
            free_lm(sc[1]->lm);
            return fail(GW_ENUMERIC, "landmark eigensolve did not converge");
        }
        const int D = sc[k]->lifted_dim;
        const double* ev = hev.data() + (size_t)k * nl;
        lm.cbarbar = hg[k];
        lm.lambda.assign(std::reverse_iterator<const double*>(ev + nl),
                         std::reverse_iterator<const double*>(ev + nl) + std::min(D, nl));
        lm.n_l = nl;
        lm.d_in = din[k];
        lm.dim = D;
        lm.fitted = true;
    }
    return Status::ok();
}

Status lift_nystrom(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                    const std::string& tag) {
    SideCfg& s = c.side[side];
    if (!s.lm.fitted) GW_TRY(fit_landmarks(c, side, x, n, d, tag + "fit" + std::to_string(side)));
    Landmarks& lm = s.lm;
    if (lm.d_in != d) return fail(GW_ESTATE, "landmarks were fitted for another input dimension");
    const int D = lm.dim;
    Status st;
    float* P = c.ws.get_t<float>(tag + "nysP" + std::to_string(side), (size_t)n_pad * D, &st);
    double* part = c.ws.get_t<double>(tag + "cpart" + std::to_string(side), gwk::centre_part_doubles(n, D), &st);
    double* mean = c.ws.get_t<double>(tag + "cmean" + std::to_string(side), D, &st);
    if (!st.good()) return st;
    GW_HIP(gwk::launch_nystrom(x, n, n_pad, d, lm.pts, lm.n_l, lm.W, lm.chat, lm.sumW, D, (float)s.p,
                               (float)lm.cbarbar, P, c.stream));
    // re-centre with the weights (Section 5 requires sum_i a_i X_i = 0)
    GW_HIP(gwk::launch_centre(P, n, n_pad, D, D, w, part, mean, X, c.stream));
    return Status::ok();
}

}  // namespace gwr
