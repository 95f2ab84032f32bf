// Launchers of the full-N kernel PCA kernels (Appendix B, "Kernel PCA").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwk {

constexpr int KPCA_MAX_IN_DIM = 8;

// R[:, 0:l] = C M, C_ij = |x_i - x_j|^p (x: n x d row-major, d <= 8; M, R:
// column-major n x l with leading dimensions ldm, ldr), FP64 accumulation.
hipError_t launch_kpca_cm(const float* x, int64_t n, int d, double p, const double* M, int64_t ldm, int l, double* R,
                          int64_t ldr, hipStream_t stream);
// Om (column-major n x l): uniform numbers in [-1, 1) from SplitMix64 of (seed, index).
hipError_t launch_kpca_start(int64_t n, int l, uint64_t seed, double* Om, hipStream_t stream);
hipError_t launch_kpca_widen(const float* a, int64_t n, double* out, hipStream_t stream);
// X (row-major n x D, row stride ldx) from Ritz vectors V (column-major
// n x l) and ascending Ritz values theta: the D largest, sqrt-scaled.
hipError_t launch_kpca_features(const double* V, int64_t ldv, int64_t n, int l, int D, const double* theta,
                                double floor, float* X, int ldx, hipStream_t stream);
hipError_t launch_kpca_fill(double* p, int64_t n, double v, hipStream_t stream);
// G (column-major l x l) = A^T B for column-major n x l blocks A, B (l <= 288),
// summed per chunk of rows into part (kpca_gram_part_doubles) and reduced in
// chunk order.
size_t kpca_gram_part_doubles(int64_t n, int l);
hipError_t launch_kpca_gram(const double* A, const double* B, int64_t n, int l, double* part, double* G,
                            hipStream_t stream);
// T = Y W for a column-major n x l block Y and l x l matrix W (l <= 288).
hipError_t launch_kpca_rowmul(const double* Y, int64_t n, int l, const double* W, double* T, hipStream_t stream);

}  // namespace gwk
