// Envelope gradient of GW_eps (Appendix B.6, "EGW Gradient Computations").
//
// At the optimum (Gamma, pi) the loss of Lemma C.1 is differentiated with pi
// and Gamma held fixed.  For the source side, with centred features X,
// n_i = |X_i|^2, s = sum_k a_k n_k, Sigma = sum_k a_k X_k X_k^T,
// m3 = sum_k a_k n_k X_k and s' the other side's s:
//   d C / d X_i          = 8 a_i [ (n_i + s - s') X_i - m3 + 2 Sigma X_i ]
//   d <pi, c_Gamma> / dX_i = -16 Gamma T_i - 8 rm_i X_i
// with T_i = sum_j pi_ij Y_j, rm_i = sum_j pi_ij |Y_j|^2 (Remark C.2's
// bilinear cost c_Gamma = -16 X^T Gamma Y - 4 |X|^2 |Y|^2).  Centring
// X = x - sum_k a_k x_k chains as G_i - a_i sum_k G_k.
//
// Weights: the derivative of GW_eps along the simplex is the EOT potential of
// the full linearised cost 2 sum_kl (c_X(i,k) - c_Y(j,l))^2 pi_kl at eps.
// For centred features that cost is c_Gamma plus terms of i alone,
//   2 sum_k a_k |X_i - X_k|^4 - 4 (n_i s' - 2 X_i . w),  w = sum_k X_k rm_k,
//   sum_k a_k |X_i - X_k|^4 = n_i^2 + m4 + 2 n_i s - 4 X_i . m3 + 4 X_i^T Sigma X_i,
// plus terms of j alone, so its potential is 8 fhat_i plus those terms, where
// fhat is Algorithm 1's potential at eps / 8 with the separable part
// alpha_i = n_i + n_i^2 / 4 removed (the factor 8 undoes the temperature).
// The result is centred, sum_i a_i g_i = 0: constants do not move along the
// simplex.  The target side is the same with the roles swapped.
#include "gw_device.h"
#include "gw_grad.h"

using namespace gwl;

namespace gwk {

constexpr int WS_ROWS = 512;  // rows per block of the weighted sums

__global__ void __launch_bounds__(256) k_wsum_part(const float* X, int64_t rows, int d, const float* coef,
                                                   double* part) {
    const int64_t r0 = (int64_t)blockIdx.x * WS_ROWS;
    const int64_t r1 = min(rows, r0 + WS_ROWS);
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += (double)coef[r] * (double)X[r * d + c];
        part[(size_t)blockIdx.x * d + c] = acc;
    }
}

__global__ void __launch_bounds__(256) k_sum_parts(const double* part, int nblk, int width, double* out) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < width; c += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * width + c];
        out[c] = s;
    }
}

hipError_t launch_wsum(const float* X, int64_t rows, int d, const float* coef, double* part, double* out,
                       hipStream_t stream) {
    const int nblk = (int)((rows + WS_ROWS - 1) / WS_ROWS);
    hipLaunchKernelGGL(k_wsum_part, dim3(nblk), dim3(256), 0, stream, X, rows, d, coef, part);
    hipLaunchKernelGGL(k_sum_parts, dim3((d + 255) / 256), dim3(256), 0, stream, part, nblk, d, out);
    return hipGetLastError();
}

// Block = floor(256 / d) rows, d threads per row (thread c owns component c).
__global__ void __launch_bounds__(256) k_grad_rows(GradSide s, double* G, double* gw, double* part) {
    __shared__ double red[4][256];
    const int d = s.d;
    const int RB = 256 / d;
    const int tid = threadIdx.x, r = tid / d, c = tid - r * d;
    const int64_t i = (int64_t)blockIdx.x * RB + r;
    const bool act = r < RB && i < s.rows;
    double gc = 0.0, p_sig = 0.0, p_m3 = 0.0, p_w = 0.0, n = 0.0, ai = 0.0;
    if (act) {
        const float* xi = s.X + i * d;
        const double* sig_row = s.mom + 2 + (size_t)c * d;
        double sig = 0.0;
        for (int k = 0; k < d; ++k) {
            const double xk = (double)xi[k];
            n += xk * xk;
            sig += sig_row[k] * xk;
        }
        const float* ti = s.T + i * s.e;
        double gt = 0.0;
        for (int k = 0; k < s.e; ++k) gt += s.gam[(size_t)c * s.ldc + (size_t)k * s.ldk] * (double)ti[k];
        const double xc = (double)xi[c];
        const double m3c = s.mom[2 + (size_t)d * d + c];
        ai = (double)s.w[i] * s.wscale;
        gc = 8.0 * ai * ((n + s.mom[0] - s.s_other) * xc - m3c + 2.0 * sig) - 16.0 * gt - 8.0 * xc * (double)s.rm[i];
        G[i * d + c] = gc;
        p_sig = xc * sig;
        p_m3 = xc * m3c;
        p_w = xc * s.wvec[c];
    }
    red[0][tid] = p_sig;
    red[1][tid] = p_m3;
    red[2][tid] = p_w;
    red[3][tid] = gc;
    __syncthreads();
    double gwi = 0.0;
    if (act && c == 0) {
        double xsx = 0.0, xm3 = 0.0, xw = 0.0;
        for (int k = 0; k < d; ++k) {
            xsx += red[0][r * d + k];
            xm3 += red[1][r * d + k];
            xw += red[2][r * d + k];
        }
        const double quart = n * n + s.mom[1] + 2.0 * n * s.mom[0] - 4.0 * xm3 + 4.0 * xsx;
        const double sep = 2.0 * quart - 4.0 * (n * s.s_other - 2.0 * xw);
        double fh = (join_df(s.P[i], s.Pl[i]) - (double)s.lw2[i]) / s.kappa;
        if (s.shift_kind == 1) {
            fh -= n + 0.25 * n * n;
        } else if (s.shift_kind == 2) {
            const float* zi = s.Z + i * s.dz;
            double z2 = 0.0;
            for (int k = 0; k < s.dz; ++k) z2 += (double)zi[k] * (double)zi[k];
            fh -= z2 + 0.25 * n * n;
        }
        gwi = 8.0 * fh + sep;
        gw[i] = gwi;
    }
    __syncthreads();
    // per-block partials in a fixed order: sum_i G_i, sum_i a_i gw_i
    red[0][tid] = (act && c == 0) ? ai * gwi : 0.0;
    __syncthreads();
    const int width = d + 1;
    double* out = part + (size_t)blockIdx.x * width;
    if (tid < d) {
        double acc = 0.0;
        for (int rr = 0; rr < RB; ++rr) acc += red[3][rr * d + tid];
        out[tid] = acc;
    }
    if (tid == 0) {
        double acc = 0.0;
        for (int rr = 0; rr < RB; ++rr) acc += red[0][rr * d];
        out[d] = acc;
    }
}

size_t grad_part_doubles(int64_t rows, int d) {
    const int RB = 256 / d;
    return (size_t)((rows + RB - 1) / RB) * (d + 1) + (size_t)(d + 1);
}

hipError_t launch_grad_rows(const GradSide& s, double* G, double* gw, double* part, double* sums,
                            hipStream_t stream) {
    if (s.d < 1 || s.d > 256) return hipErrorInvalidValue;
    const int RB = 256 / s.d;
    const int nblk = (int)((s.rows + RB - 1) / RB);
    hipLaunchKernelGGL(k_grad_rows, dim3(nblk), dim3(256), 0, stream, s, G, gw, part);
    hipLaunchKernelGGL(k_sum_parts, dim3((s.d + 1 + 255) / 256), dim3(256), 0, stream, part, nblk, s.d + 1, sums);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_grad_apply(const double* G, const double* gw, int64_t rows, int d,
                                                    const float* w, double wscale, const double* sums, float* gfeat,
                                                    float* gweight) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * d) return;
    const int64_t i = t / d;
    const int c = (int)(t - i * d);
    const double ai = (double)w[i] * wscale;
    if (gfeat) gfeat[t] = (float)(G[t] - ai * sums[c]);
    if (gweight && c == 0) gweight[i] = (float)(gw[i] - sums[d]);
}

hipError_t launch_grad_apply(const double* G, const double* gw, int64_t rows, int d, const float* w, double wscale,
                             const double* sums, float* gfeat, float* gweight, hipStream_t stream) {
    const int64_t total = rows * d;
    hipLaunchKernelGGL(k_grad_apply, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, G, gw, rows, d, w,
                       wscale, sums, gfeat, gweight);
    return hipGetLastError();
}

// out_i -= (p_i + q_i) / 2 (the divergence's self terms, Section 4).
__global__ void k_sub_half_sum(float* out, const float* __restrict__ p, const float* __restrict__ q, int64_t count) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) out[i] -= 0.5f * (p[i] + q[i]);
}

hipError_t launch_sub_half_sum(float* out, const float* p, const float* q, int64_t count, hipStream_t stream) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_sub_half_sum, dim3((int)((count + 255) / 256)), dim3(256), 0, stream, out, p, q, count);
    return hipGetLastError();
}

// One descent step of the barycentre flow: z_i -= step / w_i * ((1 - lam) g1_i
// + lam g2_i - (gs_i + gt_i) / 2), the gradient of (1 - lam) SGW(z, alpha) +
// lam SGW(z, beta) scaled by the inverse point weights.
__global__ void k_bary_step(float* z, int64_t k, int d, const float* __restrict__ w, const float* __restrict__ g1,
                            const float* __restrict__ g2, const float* __restrict__ gs, const float* __restrict__ gt,
                            float lam, float step) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= k * d) return;
    const float g = (1.f - lam) * g1[e] + lam * g2[e] - 0.5f * (gs[e] + gt[e]);
    z[e] -= step / w[e / d] * g;
}

hipError_t launch_bary_step(float* z, int64_t k, int d, const float* w, const float* g1, const float* g2,
                            const float* gs, const float* gt, float lam, float step, hipStream_t stream) {
    const int64_t count = k * d;
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_bary_step, dim3((int)((count + 255) / 256)), dim3(256), 0, stream, z, k, d, w, g1, g2, gs,
                       gt, lam, step);
    return hipGetLastError();
}

}  // namespace gwk
