// Launchers of the setup, prologue, covariance, check, lifting and gradient
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwk {

hipError_t launch_validate(const float* x, int64_t nx, const float* w, int64_t nw, int* flags, double* wsum_part,
                           int blocks, hipStream_t stream);
size_t centre_part_doubles(int64_t n, int d);
hipError_t launch_centre(const float* x, int64_t n, int64_t n_pad, int d, int ldx, const float* w, double* part,
                         double* mean, float* X, hipStream_t stream);
// |X_i|^2 and log2(w_i / wsum) (-inf on padded rows).
hipError_t launch_norms_logw(const float* X, int64_t n, int64_t n_pad, int d, const float* w, double wsum, float* nrm,
                             float* lw2, hipStream_t stream);
hipError_t launch_pack(const float* F, int64_t rows, int64_t rows_pad, int d, float scale, int prec, int side,
                       const float* ph, const float* pl, const float* aux, void* pack, hipStream_t stream);
hipError_t launch_pack_pot(const float* ph, const float* pl, int64_t rows_pad, int d, int prec, int side, void* pack,
                           hipStream_t stream);
// Prologue of one outer step.  expanded = 1 for the MFMA packs (Zout = 2 k
// Gamma Y, ms = k m / 2), 0 for the VALU direct form (Zout = Gamma Y,
// ms = m).  first = 1 initialises from f0 / g0 (NULL = 0).
hipError_t launch_prologue_cols(const float* Y, int64_t m, int64_t m_pad, int dE, int dD, const float* gamma,
                                const float* ynorm, const float* lb2, const float* g0, int first, int expanded,
                                double kappa, double kappa_old, float* Zout, double* beta, float* Vh, float* Vl,
                                float* ms, hipStream_t stream);
hipError_t launch_prologue_rows(int64_t n, int64_t n_pad, const float* xnorm, const float* la2, const float* f0,
                                int first, int expanded, double kappa, double kappa_old, float* Uh, float* Ul,
                                hipStream_t stream);
// kind: 0 direct form, 1 expanded rows (alpha from xnorm), 2 expanded
// columns (beta).
hipError_t launch_epilogue(int64_t n, const float* Uh, const float* Ul, const float* lw2, const float* xnorm,
                           const double* beta, int kind, double kappa, float* f, hipStream_t stream);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t stream);
size_t moments_part_doubles(int64_t n, int d);
hipError_t launch_moments(const float* X, int64_t n, int d, const float* w, double* part, double* out,
                          hipStream_t stream);

// Covariance pass over the final coupling: per row i, T_i = sum_j pi_ij W_j
// (W: column-side features of width dw), r_i = sum_j pi_ij and
// rm_i = sum_j pi_ij mw_j, as partials per column macro tile.
struct CovOut {
    float* Tp;     // [n_mt_c][n_pad][tw]
    float* rp;     // [n_mt_c][n_pad]
    float* rmp;    // [n_mt_c][n_pad]
    int tw;        // width of a T row in the partials
};
int cov_tw(int path, int dw);
int cov_rows_per_group(int path, int prec, int d, int dw);
// VALU path (path 1): direct form with X/xn/U rows, Zs = Z/ms = |Y|^2/V
// columns and kappa; mw is ignored there (the column norm is the weight).
// PW: payload pack (launch_pack_payload of W) when cov_bf16_form holds, else
// unused.
hipError_t launch_cov(int path, int prec, int d, const void* A, const void* B, const void* PW, const float* X,
                      const float* xn, const float* U, const float* Ul, const float* Zs, const float* ms,
                      const float* V, const float* Vl, float kappa, const float* W, const float* mw, int dw,
                      int64_t n_pad, int64_t m_pad, int rg, int bc_chunks, int n_mt_r, int n_mt_c,
                      const CovOut& out, hipStream_t stream);
// The BF16 precision form's covariance (pi and payload split into BF16
// hi/lo pairs) applies to these shapes; its payload pack is built once per
// solve from the row-major payload W (m x dw).
bool cov_bf16_form(int path, int prec, int d, int dw);
size_t payload_pack_bytes(int64_t rows_pad, int dw);
hipError_t launch_pack_payload(const float* W, int64_t m, int64_t m_pad, int dw, void* out, hipStream_t stream);

// Reduce the covariance partials: T (n x dw, optional), r, rm (optional),
// Gamma partials Xs^T T in FP64 and scalar partials [sum r, sum xs_norm rm].
size_t cov_reduce_part_doubles(int64_t n, int dx, int dw);
hipError_t launch_cov_reduce(const CovOut& in, int n_mt_c, int64_t n, int64_t n_pad, const float* Xs, int dx,
                             const float* xs_norm, int dw, float* T, float* r, float* rm, double* part,
                             hipStream_t stream);
// Final sum of Gamma partials: gamma64 (dx x dw), gamma32, scal[0..3] =
// [sum r, sum pi n m, |Gamma|^2, |Gamma - gamma_old|^2].
hipError_t launch_gamma_final(const double* part, int64_t n, int dx, int dw, const float* gamma_old, double* gamma64,
                              float* gamma32, double* scal, hipStream_t stream);

// FP64 evaluation of the coupling defined by the packed operands, one sweep:
// r64_i = sum_j pi_ij, kl_i = ln2 sum_j pi_ij (s_ij - log2 a_i - log2 b_j),
// c64_j = sum_i pi_ij.  `part` holds check64_part_doubles(n, m) doubles.
size_t check64_part_doubles(int64_t n, int64_t m);
hipError_t launch_check64(int prec, int d, const void* Arows, const void* Bcols, int64_t n, int64_t m,
                          const float* la2, const float* lb2, double* part, double* r64, double* kl, double* c64,
                          hipStream_t stream);
hipError_t launch_check64_direct(int d, const float* X, const float* xn, const float* U, const float* Ul,
                                 const float* Z, const float* zm, const float* V, const float* Vl, float kappa,
                                 int64_t n, int64_t m, const float* la2, const float* lb2, double* rsum, double* kl,
                                 hipStream_t stream);
// scal[4] = Err against the normalised weights, scal[5] = KL, scal[6] = mass.
hipError_t launch_check_final(const double* r64, const double* kl, int64_t n, const float* a, const double* c64,
                              int64_t m, const float* b, double asum, double bsum, double* scal, hipStream_t stream);

}  // namespace gwk
