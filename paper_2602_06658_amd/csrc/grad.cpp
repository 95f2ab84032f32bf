// Envelope gradients of GW_eps (Appendix B.6) from the final state of a
// solve: the coupling of (f_T, g_T, Gamma_{T-1}) and Gamma_T = X^T pi Y.
// Positions chain through the centring of the features and, for the
// |x - x'|^p penalty, through the frozen Nystrom map (Algorithm 12 with
// Algorithm 13); weights use the potential of the linearised problem.
#include "gw_grad.h"
#include "gw_lift.h"
#include "runtime.h"

namespace gwr {

Status Solve::side_gradient(int side, float* grad_pos, float* grad_w) {
    Status st;
    auto& ws = c_.ws;
    const bool src = side == 0;
    const int64_t rows = src ? n_ : m_;
    const int d = src ? D_ : E_;
    const int e = src ? E_ : D_;
    const std::string t = tag_ + (src ? "gs." : "gt.");
    float* T = ws.get_t<float>(t + "T", (size_t)rows * e, &st);
    float* r = ws.get_t<float>(t + "r", rows, &st);
    float* rm = ws.get_t<float>(t + "rm", rows, &st);
    double* G = ws.get_t<double>(t + "G", (size_t)rows * d, &st);
    double* gw = ws.get_t<double>(t + "gw", rows, &st);
    double* part = ws.get_t<double>(t + "part", gwk::grad_part_doubles(rows, d), &st);
    double* wpart = ws.get_t<double>(t + "wpart", (size_t)((rows + 511) / 512) * d, &st);
    double* vec = ws.get_t<double>(t + "vec", 2 * (size_t)(d + 1), &st);
    if (!st.good()) return st;
    double* wvec = vec;
    double* sums = vec + d + 1;

    // T_i = sum_j pi_ij W_j and rm_i = sum_j pi_ij |W_j|^2 for this side's rows
    GW_TRY(covariance(side, T, r, rm));
    const float* Xs = src ? X_ : Y_;
    GW_HIP(gwk::launch_wsum(Xs, rows, d, rm, wpart, wvec, st_));

    gwk::GradSide gs{};
    gs.X = Xs;
    gs.rows = rows;
    gs.d = d;
    gs.w = src ? a_ : b_;
    gs.wscale = 1.0 / (src ? asum_ : bsum_);
    gs.T = T;
    gs.e = e;
    gs.rm = rm;
    gs.gam = gam64_;            // Gamma_T, D x E
    gs.ldc = src ? E_ : 1;      // source: (Gamma T_i)_c = sum_k Gamma[c][k] T_ik
    gs.ldk = src ? 1 : E_;      // target: (Gamma^T T'_j)_c = sum_k Gamma[k][c] T'_jk
    gs.mom = src ? momx_ : momy_;
    double s_other = 0.0;
    GW_HIP(hipMemcpyAsync(&s_other, src ? momy_ : momx_, sizeof(double), hipMemcpyDeviceToHost, st_));
    GW_HIP(hipStreamSynchronize(st_));
    gs.s_other = s_other;
    gs.wvec = wvec;
    gs.P = src ? U_[pa_] : V_[pb_];
    gs.Pl = src ? Ul_[pa_] : Vl_[pb_];
    gs.lw2 = src ? la2_ : lb2_;
    gs.kappa = kappa_;
    // the MFMA path keeps the potentials shifted by alpha / beta already;
    // the direct form keeps Algorithm 1's potentials
    gs.shift_kind = geo_.path == 0 ? 0 : (src ? 1 : 2);
    gs.Z = Zs_;
    gs.dz = D_;
    GW_HIP(gwk::launch_grad_rows(gs, G, gw, part, sums, st_));

    const SideCfg& cfg = c_.side[side];
    float* gfeat = nullptr;
    if (grad_pos) {
        if (cfg.kind == GW_PEN_POWER) {
            gfeat = ws.get_t<float>(t + "gfeat", (size_t)rows * d, &st);
            if (!st.good()) return st;
        } else {
            gfeat = grad_pos;  // features are the centred inputs: same shape
        }
    }
    GW_HIP(gwk::launch_grad_apply(G, gw, rows, d, gs.w, gs.wscale, sums, gfeat, grad_w, st_));
    if (grad_pos && cfg.kind == GW_PEN_POWER) {
        const Landmarks& lm = cfg.lm;
        const float* xin = src ? x_ : y_;
        GW_HIP(gwk::launch_nystrom_jt(xin, rows, lm.d_in, lm.pts, lm.n_l, lm.W, lm.dim, (float)cfg.p, gfeat, grad_pos,
                                      st_));
    }
    return Status::ok();
}

Status Solve::gradients(float* grad_x, float* grad_a, float* grad_y, float* grad_b) {
    c_.prof.begin(GW_PROF_GRAD, st_);
    if (grad_x || grad_a) GW_TRY(side_gradient(0, grad_x, grad_a));
    if (grad_y || grad_b) GW_TRY(side_gradient(1, grad_y, grad_b));
    c_.prof.end(st_);
    GW_HIP(hipStreamSynchronize(st_));
    return Status::ok();
}

}  // namespace gwr
