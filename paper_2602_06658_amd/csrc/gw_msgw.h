// Launchers of the Multiscale-GW kernels (Appendix B): K-Means coarsening
// and Algorithm 8 (Interpolate).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwk {

// Fixed-point exponent of the cluster weights: W = sum rint(w_i 2^61).
constexpr int KM_WEIGHT_EXP = 61;

// *out = bits of max |X_id| over n rows of D (row stride ldx).
hipError_t launch_km_maxabs(const float* X, int64_t n, int ldx, int D, unsigned int* out, hipStream_t stream);
// C_j = X_{idx[j]}, j < k.
hipError_t launch_km_gather(const float* X, int ldx, int D, const int64_t* idx, int k, float* C, int ldc,
                            hipStream_t stream);
// One Lloyd iteration: assignment, fixed-point sums at grid 2^-S (sums: k*D
// words followed by the k weight words, one allocation), centroid update.
hipError_t launch_km_iteration(const float* X, int64_t n, int ldx, int D, const float* w, float* C, int k, int ldc,
                               int S, int* assign, unsigned long long* sums, unsigned long long* wsum,
                               hipStream_t stream);
// Non-empty clusters in index order: Xc (dense, D columns), wc, kept, *kc.
hipError_t launch_km_compact(const unsigned long long* wsum, const float* C, int k, int D, int ldc, float* Xc,
                             float* wc, int* kept, int* kc, hipStream_t stream);
// out_i = G V_i (G: D x dv row-major) or V_i when G is NULL, zero-padded to
// ldo; half_i = |V_i|^2 / 2.
hipError_t launch_lift_bar(const float* V, int64_t n, int ldv, int dv, const float* G, int D, float* out, int ldo,
                           float* half, hipStream_t stream);
// out_q = -eps' ln sum_r w_r exp((h_r - |Pbar_q - Qbar_r|^2) / eps'), Pbar_q =
// [P_q (dl coordinates), ph_q], Qbar_r = [Q_r, qh_r]; hb: nr floats of scratch.
hipError_t launch_interp(const float* P, int64_t nq, int ldp, const float* Q, int nr, int ldq, int dl,
                         const float* ph, const float* qh, const float* w, const float* h, double eps_prime, float* hb,
                         float* out, hipStream_t stream);

}  // namespace gwk
