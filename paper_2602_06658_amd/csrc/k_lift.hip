// Lifting of |x - x'|^p penalties (0 < p < 2, conditionally of negative type,
// Section 2) into centred features by landmark kernel PCA:
//   - the landmark cost matrix and its double centring K = -1/2 J C J
//     (Algorithm 4 with uniform landmark weights; base-point free form),
//   - the Nystrom map of Algorithm 13 for every point,
//       Pi(x)_d = lambda_d^{-1/2} sum_l k~(x, x_l) V_ld,
//       k~(x, x_l) = -1/2 [c(x, x_l) - cbar(x) - chat_l + cbarbar],
//     written as Pi(x)_d = sum_l (c(x, x_l) - chat_l) W_ld - (cbar(x) - cbarbar) sW_d
//     with W_ld = -V_ld / (2 sqrt(lambda_d)), sW_d = sum_l W_ld,
//   - and its Jacobian contracted with feature gradients (Algorithm 12's
//     chain rule through the frozen map).
#include "gw_device.h"
#include "gw_lift.h"

namespace gwk {

__device__ __forceinline__ double pow_cost(double r2, double p) {
    if (p == 2.0) return r2;
    if (p == 1.0) return sqrt(r2);
    return r2 > 0.0 ? pow(r2, 0.5 * p) : 0.0;
}
__device__ __forceinline__ float pow_cost_f(float r2, float p) {
    if (p == 2.0f) return r2;
    if (p == 1.0f) return sqrtf(r2);
    return r2 > 0.f ? powf(r2, 0.5f * p) : 0.f;
}

// Gather landmark points.
__global__ void k_gather(const float* x, int d, const int64_t* idx, int nl, float* out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nl * d) return;
    const int l = t / d, k = t - l * d;
    out[t] = x[idx[l] * d + k];
}

hipError_t launch_gather(const float* x, int d, const int64_t* idx, int nl, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_gather, dim3((nl * d + 255) / 256), dim3(256), 0, stream, x, d, idx, nl, out);
    return hipGetLastError();
}

// Landmark cost matrix (FP64, symmetric, column-major = row-major).
__global__ void k_landmark_cost(const float* L, int nl, int d, double p, double* C) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nl * nl) return;
    const int i = t / nl, j = t - i * nl;
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double df = (double)L[i * d + k] - (double)L[j * d + k];
        r2 += df * df;
    }
    C[t] = pow_cost(r2, p);
}

// Row means of C (deterministic: one thread per row), then the double
// centring in place: K = -1/2 (C - r_i - r_j + g).
__global__ void k_rowmean(const double* C, int nl, double* rmean) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    double s = 0.0;
    for (int j = 0; j < nl; ++j) s += C[(size_t)i * nl + j];
    rmean[i] = s / nl;
}
__global__ void k_grandmean(const double* rmean, int nl, double* g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nl; ++i) s += rmean[i];
        g[0] = s / nl;
    }
}
__global__ void k_centre_kernel(double* C, int nl, const double* rmean, const double* g) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nl * nl) return;
    const int i = t / nl, j = t - i * nl;
    C[t] = -0.5 * (C[t] - rmean[i] - rmean[j] + g[0]);
}

hipError_t launch_landmark_kernel(const float* L, int nl, int d, double p, double* K, double* rmean, double* g,
                                  hipStream_t stream) {
    const int tot = nl * nl;
    hipLaunchKernelGGL(k_landmark_cost, dim3((tot + 255) / 256), dim3(256), 0, stream, L, nl, d, p, K);
    hipLaunchKernelGGL(k_rowmean, dim3((nl + 255) / 256), dim3(256), 0, stream, K, nl, rmean);
    hipLaunchKernelGGL(k_grandmean, dim3(1), dim3(64), 0, stream, rmean, nl, g);
    hipLaunchKernelGGL(k_centre_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, K, nl, rmean, g);
    return hipGetLastError();
}

// Top-D eigenpairs (eigenvalues ascending from the solver) -> W, chat, sW.
// keep: lambda_d > rel_floor * lambda_max.
__global__ void k_nystrom_weights(const double* evec, const double* eval, int nl, int D, double rel_floor,
                                  const double* rmean, float* W, float* chat, float* sW) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const double lmax = eval[nl - 1];
    if (l < nl) {
        for (int dd = 0; dd < D; ++dd) {
            const int col = nl - 1 - dd;  // descending
            const double lam = col >= 0 ? eval[col] : 0.0;
            double w = 0.0;
            if (col >= 0 && lam > rel_floor * lmax && lam > 0.0) w = -0.5 * evec[(size_t)col * nl + l] / sqrt(lam);
            W[(size_t)l * D + dd] = (float)w;
        }
        chat[l] = (float)rmean[l];
    }
    if (l < D) {
        const int col = nl - 1 - l;
        const double lam = col >= 0 ? eval[col] : 0.0;
        double s = 0.0;
        if (col >= 0 && lam > rel_floor * lmax && lam > 0.0)
            for (int m = 0; m < nl; ++m) s += -0.5 * evec[(size_t)col * nl + m] / sqrt(lam);
        sW[l] = (float)s;
    }
}

hipError_t launch_nystrom_weights(const double* evec, const double* eval, int nl, int D, double rel_floor,
                                  const double* rmean, float* W, float* chat, float* sW, hipStream_t stream) {
    const int n = nl > D ? nl : D;
    hipLaunchKernelGGL(k_nystrom_weights, dim3((n + 255) / 256), dim3(256), 0, stream, evec, eval, nl, D, rel_floor,
                       rmean, W, chat, sW);
    return hipGetLastError();
}

// Nystrom map of every point.  One thread per point; landmarks and W staged
// through LDS in chunks; D processed in blocks of 32 accumulators.
constexpr int LCH = 64;     // landmarks per LDS chunk
constexpr int DB = 32;      // feature block per pass
constexpr int MAXD_IN = 32; // input dimension held in registers

__global__ void __launch_bounds__(256) k_nystrom(const float* x, int64_t n, int64_t n_pad, int d, const float* L,
                                                 int nl, const float* W, const float* chat, const float* sW, int D,
                                                 float p, float cbarbar, float* out) {
    __shared__ float ls[LCH * MAXD_IN];
    __shared__ float ws[LCH * DB];
    __shared__ float cs[LCH];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < n;
    float xr[MAXD_IN];
#pragma unroll
    for (int k = 0; k < MAXD_IN; ++k) xr[k] = (act && k < d) ? x[i * d + k] : 0.f;
    for (int d0 = 0; d0 < D; d0 += DB) {
        float acc[DB];
#pragma unroll
        for (int k = 0; k < DB; ++k) acc[k] = 0.f;
        float csum = 0.f;
        for (int l0 = 0; l0 < nl; l0 += LCH) {
            const int nch = min(LCH, nl - l0);
            __syncthreads();
            for (int u = threadIdx.x; u < nch * d; u += blockDim.x) ls[u] = L[(size_t)l0 * d + u];
            for (int u = threadIdx.x; u < nch * DB; u += blockDim.x) {
                const int l = u / DB, k = u - l * DB;
                ws[u] = (d0 + k < D) ? W[(size_t)(l0 + l) * D + d0 + k] : 0.f;
            }
            for (int u = threadIdx.x; u < nch; u += blockDim.x) cs[u] = chat[l0 + u];
            __syncthreads();
            for (int l = 0; l < nch; ++l) {
                float r2 = 0.f;
                for (int k = 0; k < d; ++k) {
                    const float df = xr[k] - ls[l * d + k];
                    r2 = fmaf(df, df, r2);
                }
                const float c = pow_cost_f(r2, p);
                csum += c;
                const float cc = c - cs[l];
#pragma unroll
                for (int k = 0; k < DB; ++k) acc[k] = fmaf(cc, ws[l * DB + k], acc[k]);
            }
        }
        if (i < n_pad) {
            const float cbar = csum / (float)nl;
            for (int k = 0; k < DB && d0 + k < D; ++k)
                out[i * D + d0 + k] = act ? acc[k] - (cbar - cbarbar) * sW[d0 + k] : 0.f;
        }
    }
}

hipError_t launch_nystrom(const float* x, int64_t n, int64_t n_pad, int d, const float* L, int nl, const float* W,
                          const float* chat, const float* sW, int D, float p, float cbarbar, float* out,
                          hipStream_t stream) {
    if (d > MAXD_IN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nystrom, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, stream, x, n, n_pad, d, L, nl,
                       W, chat, sW, D, p, cbarbar, out);
    return hipGetLastError();
}

// Chain rule through the frozen map: given feature gradients G (n x D),
//   grad_x_i = sum_d G_id dPi_d/dx (x_i)
//            = sum_l h_il grad_x c(x_i, x_l) - (sum_l h_il) (1/nl) sum_l grad_x c(x_i, x_l)
// with h_il = sum_d G_id W_ld, grad_x c = p |x - x_l|^{p-2} (x - x_l)
// (0 at x = x_l, the subgradient central differences return for p = 1).
__global__ void __launch_bounds__(256) k_nystrom_jt(const float* x, int64_t n, int d, const float* L, int nl,
                                                    const float* W, int D, float p, const float* G, float* gx) {
    __shared__ float ls[LCH * MAXD_IN];
    __shared__ float ws[LCH * 64];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < n;
    float xr[MAXD_IN], acc[MAXD_IN], mg[MAXD_IN];
#pragma unroll
    for (int k = 0; k < MAXD_IN; ++k) {
        xr[k] = (act && k < d) ? x[i * d + k] : 0.f;
        acc[k] = 0.f;
        mg[k] = 0.f;
    }
    float hsum = 0.f;
    for (int l0 = 0; l0 < nl; l0 += LCH) {
        const int nch = min(LCH, nl - l0);
        // h_il for this chunk needs G_i . W_l over all D: accumulate in parts
        float h[LCH];
#pragma unroll
        for (int l = 0; l < LCH; ++l) h[l] = 0.f;
        for (int d0 = 0; d0 < D; d0 += 64) {
            __syncthreads();
            for (int u = threadIdx.x; u < nch * 64; u += blockDim.x) {
                const int l = u / 64, k = u - l * 64;
                ws[u] = (d0 + k < D) ? W[(size_t)(l0 + l) * D + d0 + k] : 0.f;
            }
            __syncthreads();
            if (act) {
                for (int k = 0; k < 64 && d0 + k < D; ++k) {
                    const float gk = G[i * D + d0 + k];
                    for (int l = 0; l < nch; ++l) h[l] = fmaf(gk, ws[l * 64 + k], h[l]);
                }
            }
        }
        __syncthreads();
        for (int u = threadIdx.x; u < nch * d; u += blockDim.x) ls[u] = L[(size_t)l0 * d + u];
        __syncthreads();
        if (act) {
            for (int l = 0; l < nch; ++l) {
                float r2 = 0.f;
                for (int k = 0; k < d; ++k) {
                    const float df = xr[k] - ls[l * d + k];
                    r2 = fmaf(df, df, r2);
                }
                float coef;
                if (p == 2.0f) coef = 2.f;
                else coef = r2 > 0.f ? p * powf(r2, 0.5f * p - 1.f) : 0.f;
                hsum += h[l];
                for (int k = 0; k < d; ++k) {
                    const float gc = coef * (xr[k] - ls[l * d + k]);
                    acc[k] = fmaf(h[l], gc, acc[k]);
                    mg[k] += gc;
                }
            }
        }
    }
    if (act)
        for (int k = 0; k < d; ++k) gx[i * d + k] = acc[k] - hsum * mg[k] / (float)nl;
}

hipError_t launch_nystrom_jt(const float* x, int64_t n, int d, const float* L, int nl, const float* W, int D, float p,
                             const float* G, float* gx, hipStream_t stream) {
    if (d > MAXD_IN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nystrom_jt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, n, d, L, nl, W, D, p,
                       G, gx);
    return hipGetLastError();
}

}  // namespace gwk
