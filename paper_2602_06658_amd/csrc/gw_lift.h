// Launchers of the landmark kernel-PCA lifting kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwk {

hipError_t launch_gather(const float* x, int d, const int64_t* idx, int nl, float* out, hipStream_t stream);
// K = -1/2 J C J of the landmark cost (FP64, nl x nl), with the row means
// of C and their grand mean.
hipError_t launch_landmark_kernel(const float* L, int nl, int d, double p, double* K, double* rmean, double* g,
                                  hipStream_t stream);
hipError_t launch_nystrom_weights(const double* evec, const double* eval, int nl, int D, double rel_floor,
                                  const double* rmean, float* W, float* chat, float* sW, hipStream_t stream);
hipError_t launch_nystrom(const float* x, int64_t n, int64_t n_pad, int d, const float* L, int nl, const float* W,
                          const float* chat, const float* sW, int D, float p, float cbarbar, float* out,
                          hipStream_t stream);
hipError_t launch_nystrom_jt(const float* x, int64_t n, int d, const float* L, int nl, const float* W, int D, float p,
                             const float* G, float* gx, hipStream_t stream);

}  // namespace gwk
