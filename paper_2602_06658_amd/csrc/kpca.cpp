// Full-N kernel PCA (Appendix B, "Kernel PCA": the top-D eigenpairs of the
// centred kernel of Algorithm 4 on all n points, X_i = V_i sqrt(Lambda)),
// matrix-free by randomized subspace iteration (Halko, Martinsson, Tropp
// 2011, Algorithm 4.4 with Rayleigh-Ritz): the n x n kernel is never stored.
//
// With rho_i = sum_k a_k c_ik and tau = sum_i a_i rho_i, Algorithm 4's kernel
// is K = -(C - rho 1^T - 1 rho^T + tau 1 1^T) / 2, so for a block M,
//   K M = -(C M)/2 + rho s^T / 2 + 1 (u - tau s)^T / 2,  s = M^T 1, u = M^T rho;
// C M runs in k_kpca_cm, the tall-skinny Gram matrices and products in
// k_kpca_gram / k_kpca_rowmul, the rank-one terms and the l x l problems
// (SVQB orthonormalisation, twice; the Ritz eigensolve) in rocBLAS /
// rocSOLVER, all in FP64.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

#include "gw_kpca.h"
#include "runtime.h"

namespace gwr {

#define GW_RB(call)                                                                  \
    do {                                                                             \
        if ((call) != rocblas_status_success) return fail(GW_EDEVICE, #call);        \
    } while (0)

struct KpcaPlan {
    const float* x;
    int64_t n;
    int d;
    double p;
    int l;
    double* ones;
    double* rho;
    double tau;
    double* s;
    double* u;
};

// Yout = K M (M != Yout), column-major n x l.
static Status apply_kernel(Ctx& c, rocblas_handle h, const KpcaPlan& k, const double* M, double* Yout) {
    const int n = (int)k.n, l = k.l;
    const double one = 1.0, zero = 0.0, mhalf = -0.5, half = 0.5, mtau = -k.tau;
    GW_HIP(gwk::launch_kpca_cm(k.x, k.n, k.d, k.p, M, k.n, l, Yout, k.n, c.stream));
    GW_RB(rocblas_dgemv(h, rocblas_operation_transpose, n, l, &one, M, n, k.ones, 1, &zero, k.s, 1));
    GW_RB(rocblas_dgemv(h, rocblas_operation_transpose, n, l, &one, M, n, k.rho, 1, &zero, k.u, 1));
    GW_RB(rocblas_dscal(h, n * l, &mhalf, Yout, 1));
    GW_RB(rocblas_dger(h, n, l, &half, k.rho, 1, k.s, 1, Yout, n));
    GW_RB(rocblas_daxpy(h, l, &mtau, k.s, 1, k.u, 1));
    GW_RB(rocblas_dger(h, n, l, &half, k.ones, 1, k.u, 1, Yout, n));
    return Status::ok();
}

// Orthonormal basis of the block (SVQB, Stathopoulos and Wu 2002, twice):
// Y^T Y = W Sigma W^T, Y <- Y W Sigma^-1/2.  Directions whose Sigma is at or
// below 1e-24 of the largest (a block wider than the kernel's rank) get zero
// columns, which later give zero Ritz values.  The result lands in Y (T is
// scratch of the same size; the two pointers are swapped).
static Status orthonormalise(Ctx& c, rocblas_handle h, int64_t n64, int l, double*& Y, double*& T, double* G,
                             double* W, double* sig, double* ework, double* scale, int* info, double* gpart) {
    std::vector<double> hs(l), hscale(l);
    for (int pass = 0; pass < 2; ++pass) {
        GW_HIP(gwk::launch_kpca_gram(Y, Y, n64, l, gpart, G, c.stream));
        GW_RB(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, l, G, l, sig, ework, info));
        int hinfo = 0;
        GW_HIP(hipMemcpyAsync(hs.data(), sig, l * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        GW_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        GW_HIP(hipStreamSynchronize(c.stream));
        if (hinfo != 0) return fail(GW_ENUMERIC, "kernel PCA: Gram eigensolve did not converge");
        const double smax = std::max(hs[l - 1], 0.0);
        if (!(smax > 0.0) || !std::isfinite(smax)) return fail(GW_ENUMERIC, "kernel PCA: the block vanished");
        for (int q = 0; q < l; ++q) hscale[q] = hs[q] > 1e-24 * smax ? 1.0 / std::sqrt(hs[q]) : 0.0;
        GW_HIP(hipMemcpyAsync(scale, hscale.data(), l * sizeof(double), hipMemcpyHostToDevice, c.stream));
        GW_RB(rocblas_ddgmm(h, rocblas_side_right, l, l, G, l, scale, 1, W, l));
        GW_HIP(gwk::launch_kpca_rowmul(Y, n64, l, W, T, c.stream));
        std::swap(Y, T);
        GW_HIP(hipStreamSynchronize(c.stream));  // hscale is read by the copy above
    }
    return Status::ok();
}

Status kpca_full(Ctx& c, const float* x, int64_t n, int d, const float* w, double p, int D, int n_iter, uint64_t seed,
                 float* X, int ldx, std::vector<double>* lambda, const std::string& tag) {
    Status st;
    const int l = (int)std::min<int64_t>(D + 32, n);
    double* wd = c.ws.get_t<double>(tag + "kp.w", n, &st);
    double* ones = c.ws.get_t<double>(tag + "kp.1", n, &st);
    double* rho = c.ws.get_t<double>(tag + "kp.rho", n, &st);
    double* Y = c.ws.get_t<double>(tag + "kp.Y", (size_t)n * l, &st);
    double* Z = c.ws.get_t<double>(tag + "kp.Z", (size_t)n * l, &st);
    double* G = c.ws.get_t<double>(tag + "kp.G", (size_t)l * l, &st);
    double* B = c.ws.get_t<double>(tag + "kp.B", (size_t)l * l, &st);
    double* theta = c.ws.get_t<double>(tag + "kp.th", l, &st);
    double* ework = c.ws.get_t<double>(tag + "kp.ew", l, &st);
    double* su = c.ws.get_t<double>(tag + "kp.su", 2 * (size_t)l, &st);
    double* sig = c.ws.get_t<double>(tag + "kp.sig", l, &st);
    double* scale = c.ws.get_t<double>(tag + "kp.sc", l, &st);
    int* info = c.ws.get_t<int>(tag + "kp.info", 1, &st);
    double* gpart = c.ws.get_t<double>(tag + "kp.gp", gwk::kpca_gram_part_doubles(n, l), &st);
    if (!st.good()) return st;
    if (!c.rocblas) {
        rocblas_handle hh;
        if (rocblas_create_handle(&hh) != rocblas_status_success) return fail(GW_EDEVICE, "rocblas_create_handle");
        c.rocblas = hh;
    }
    rocblas_handle h = (rocblas_handle)c.rocblas;
    GW_RB(rocblas_set_stream(h, c.stream));
    GW_RB(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));

    KpcaPlan k{x, n, d, p, l, ones, rho, 0.0, su, su + l};
    GW_HIP(gwk::launch_kpca_widen(w, n, wd, c.stream));
    GW_HIP(gwk::launch_kpca_fill(ones, n, 1.0, c.stream));
    // rho = C a, tau = a^T rho
    GW_HIP(gwk::launch_kpca_cm(x, n, d, p, wd, n, 1, rho, n, c.stream));
    double tau = 0.0;
    GW_RB(rocblas_ddot(h, (int)n, wd, 1, rho, 1, &tau));
    k.tau = tau;

    // Y = K Omega, then n_iter rounds of orthonormalise + apply
    GW_HIP(gwk::launch_kpca_start(n, l, seed, Z, c.stream));
    GW_TRY(apply_kernel(c, h, k, Z, Y));
    for (int it = 0; it < n_iter; ++it) {
        GW_TRY(orthonormalise(c, h, n, l, Y, Z, G, B, sig, ework, scale, info, gpart));
        GW_TRY(apply_kernel(c, h, k, Y, Z));
        std::swap(Y, Z);
    }
    // Rayleigh-Ritz on the final basis Q (= Y after orthonormalisation)
    GW_TRY(orthonormalise(c, h, n, l, Y, Z, G, B, sig, ework, scale, info, gpart));
    GW_TRY(apply_kernel(c, h, k, Y, Z));
    const double half = 0.5;
    GW_HIP(gwk::launch_kpca_gram(Y, Z, n, l, gpart, G, c.stream));
    GW_RB(rocblas_dgeam(h, rocblas_operation_none, rocblas_operation_transpose, l, l, &half, G, l, &half, G, l, B, l));
    GW_RB(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, l, B, l, theta, ework, info));
    GW_HIP(gwk::launch_kpca_rowmul(Y, n, l, B, Z, c.stream));
    std::vector<double> hth(l);
    int hinfo = 0;
    GW_HIP(hipMemcpyAsync(hth.data(), theta, l * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    if (hinfo != 0) return fail(GW_ENUMERIC, "kernel PCA: Ritz eigensolve did not converge");
    const double floor = 1e-12 * std::max(hth[l - 1], 0.0);
    GW_HIP(gwk::launch_kpca_features(Z, n, n, l, D, theta, floor, X, ldx, c.stream));
    if (lambda) {
        lambda->assign(D, 0.0);
        for (int q = 0; q < D; ++q) (*lambda)[q] = hth[l - 1 - q] > floor ? hth[l - 1 - q] : 0.0;
    }
    GW_HIP(hipStreamSynchronize(c.stream));
    return Status::ok();
}

}  // namespace gwr

using gwr::Ctx;
using gwr::Status;

static gw_status ret(gw_ctx* ctx, const Status& s) {
    if (ctx) ctx->c.err = s.good() ? std::string() : s.msg;
    return s.code;
}

extern "C" gw_status gw_kpca_full(gw_ctx* ctx, const float* x, int64_t n, int d, const float* w, double p, int D,
                                  int n_iter, uint64_t seed, float* X, double* lambda) {
    if (!ctx) return GW_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    if (!x || !w || !X) return ret(ctx, gwr::fail(GW_EINVAL, "NULL pointer"));
    if (n < 2 || n > ((int64_t)1 << 30)) return ret(ctx, gwr::fail(GW_EINVAL, "n must be in [2, 2^30]"));
    if (d < 1 || d > gwk::KPCA_MAX_IN_DIM) return ret(ctx, gwr::fail(GW_EUNSUPPORTED, "input dimension must be in [1, 8]"));
    if (!(p > 0.0 && p <= 2.0)) return ret(ctx, gwr::fail(GW_EINVAL, "p must be in (0, 2]"));
    if (D < 1 || D > 256 || D > n - 1) return ret(ctx, gwr::fail(GW_EINVAL, "D must be in [1, min(256, n - 1)]"));
    if (n_iter < 0 || n_iter > 100) return ret(ctx, gwr::fail(GW_EINVAL, "n_iter must be in [0, 100]"));
    if (n * (int64_t)std::min<int64_t>(D + 32, n) > (int64_t)INT32_MAX)
        return ret(ctx, gwr::fail(GW_EUNSUPPORTED, "n * (D + 32) must fit a 32-bit BLAS size"));
    if (hipSetDevice(ctx->c.device) != hipSuccess) return ret(ctx, gwr::fail(GW_EDEVICE, "hipSetDevice"));
    Status st = gwr::check_points(ctx->c, x, n * d, w, n, "kp.", "kernel PCA input");
    std::vector<double> lam;
    if (st.good()) st = gwr::kpca_full(ctx->c, x, n, d, w, p, D, n_iter, seed, X, D, &lam, "kp.");
    if (st.good() && lambda) std::copy(lam.begin(), lam.end(), lambda);
    return ret(ctx, st);
}
