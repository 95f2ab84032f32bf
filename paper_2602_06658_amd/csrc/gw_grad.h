// Launchers of the envelope-gradient kernels (Appendix B.6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwk {

// One side of the problem, seen from its own rows i, with W the other
// side's features:
//   T_i  = sum_j pi_ij W_j,   rm_i = sum_j pi_ij |W_j|^2
// (the covariance pass with this side as the row operand).
struct GradSide {
    const float* X;       // rows x d centred features (row stride d)
    int64_t rows;
    int d;
    const float* w;       // weights (rows), as passed by the caller
    double wscale;        // 1 / sum(w)
    const float* T;       // rows x e
    int e;
    const float* rm;      // rows
    const double* gam;    // Gamma (D x E, FP64); operator element (c, k) = gam[c * ldc + k * ldk]
    int ldc, ldk;
    const double* mom;    // [s, m4, Sigma (d x d), m3 (d)] of this side
    double s_other;       // s = sum w |W|^2 of the other side
    const double* wvec;   // sum_k X_k rm_k (d)
    // final potential of this side, log2 units, (hi, lo) FP32 pair:
    //   P = log2(w / sum w) + kappa * (pot - shift)
    const float* P;
    const float* Pl;
    const float* lw2;
    double kappa;
    int shift_kind;       // 0: P already holds the shifted potential;
                          // 1: subtract alpha = |X|^2 + |X|^4 / 4;
                          // 2: subtract beta = |Z|^2 + |X|^4 / 4, Z rows below
    const float* Z;       // rows x dz (shift_kind 2)
    int dz;
};

// FP64 partial / final buffers
size_t grad_part_doubles(int64_t rows, int d);
// out[c] = sum_k coef_k X_k[c] in FP64, fixed order
hipError_t launch_wsum(const float* X, int64_t rows, int d, const float* coef, double* part, double* out,
                       hipStream_t stream);
// Per row: G_i (rows x d, FP64) of the feature gradient before the centring
// chain, gw_i (rows, FP64) of the weight gradient before centring, and
// sums = [sum_i G_i (d), sum_i w_i gw_i / sum w].
hipError_t launch_grad_rows(const GradSide& s, double* G, double* gw, double* part, double* sums,
                            hipStream_t stream);
// gfeat_i = G_i - (w_i / sum w) sum_k G_k; gweight_i = gw_i - sum_k (w_k / sum w) gw_k.
// Either output may be NULL.
hipError_t launch_grad_apply(const double* G, const double* gw, int64_t rows, int d, const float* w, double wscale,
                             const double* sums, float* gfeat, float* gweight, hipStream_t stream);

// out_i -= (p_i + q_i) / 2, count floats.
hipError_t launch_sub_half_sum(float* out, const float* p, const float* q, int64_t count, hipStream_t stream);

// z_i -= step / w_i ((1 - lam) g1_i + lam g2_i - (gs_i + gt_i) / 2), k x d floats.
hipError_t launch_bary_step(float* z, int64_t k, int d, const float* w, const float* g1, const float* g2,
                            const float* gs, const float* gt, float lam, float step, hipStream_t stream);

}  // namespace gwk
