// Setup and per-outer-step kernels of Algorithm 1:
//   - input validation (finite values, positive weights, weight sums in FP64)
//   - centring of features with the weights (Section 5 requires
//     sum_i a_i X_i = 0; Section 3's squared-norm example centres the points)
//   - squared norms, log2 weights
//   - packing of the row operand X into the MFMA layout
//   - the per-outer-step prologue: Z = Gamma_t Y, |Z_j|^2, conversion of the
//     potentials from Algorithm 1's convention (cost units) to the log2
//     exponent terms, packing of the column operand
//   - the epilogue converting back
//   - FP64 moments for the constant C(alpha, beta) of Lemma C.1
#include "gw_device.h"
#include "gw_prep.h"

using namespace gwl;

namespace gwk {

constexpr double LOG2E = 1.4426950408889634;

// ---------------------------------------------------------------------------
// Validation: flags[0] |= 1 non-finite value, 2 non-positive weight;
// sums[blk] = partial FP64 sum of weights.
// ---------------------------------------------------------------------------

__global__ void k_validate(const float* x, int64_t nx, const float* w, int64_t nw, int* flags, double* wsum_part) {
    __shared__ double red[256];
    double acc = 0.0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nx; i += stride)
        if (!isfinite(x[i])) bad |= 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nw; i += stride) {
        const float v = w[i];
        if (!isfinite(v)) bad |= 1;
        else if (!(v > 0.f)) bad |= 2;
        acc += (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum_part[blockIdx.x] = red[0];
    if (bad) atomicOr(flags, bad);
}

hipError_t launch_validate(const float* x, int64_t nx, const float* w, int64_t nw, int* flags, double* wsum_part,
                           int blocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, stream, x, nx, w, nw, flags, wsum_part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weighted column means in FP64 (deterministic: fixed block partition, fixed
// order of the final sum), then centring.
// ---------------------------------------------------------------------------

__global__ void k_colmean_part(const float* x, int64_t n, int d, int ld, const float* w, double* part, int rows_per_blk) {
    // one block per row range; thread t accumulates columns t, t+256, ...
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(n, r0 + rows_per_blk);
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)w[r] * (double)x[r * ld + c];
        part[(size_t)blockIdx.x * d + c] = s;
    }
}

__global__ void k_colmean_final(const double* part, int nblk, int d, double* mean) {
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * d + c];
        mean[c] = s;
    }
}

// X (n_pad x d, row-major) = x - mean for rows < n, 0 for padded rows.
__global__ void k_centre(const float* x, int64_t n, int64_t n_pad, int d, int ldx, const double* mean, float* X) {
    const int64_t total = n_pad * d;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t r = t / d;
        const int c = (int)(t - r * d);
        X[t] = r < n ? (float)((double)x[r * ldx + c] - mean[c]) : 0.f;
    }
}

hipError_t launch_centre(const float* x, int64_t n, int64_t n_pad, int d, int ldx, const float* w, double* part,
                         double* mean, float* X, hipStream_t stream) {
    const int rows_per_blk = 256;
    const int nblk = (int)((n + rows_per_blk - 1) / rows_per_blk);
    hipLaunchKernelGGL(k_colmean_part, dim3(nblk), dim3(64), 0, stream, x, n, d, ldx, w, part, rows_per_blk);
    hipLaunchKernelGGL(k_colmean_final, dim3(1), dim3(256), 0, stream, part, nblk, d, mean);
    const int64_t total = n_pad * d;
    const int64_t nb = (total + 255) / 256;
    const int grid = (int)(nb < 65536 ? nb : 65536);
    hipLaunchKernelGGL(k_centre, dim3(grid), dim3(256), 0, stream, x, n, n_pad, d, ldx, mean, X);
    return hipGetLastError();
}

size_t centre_part_doubles(int64_t n, int d) { return (size_t)((n + 255) / 256) * d; }

// ---------------------------------------------------------------------------
// Norms and log2 weights
// ---------------------------------------------------------------------------

__global__ void k_norms_logw(const float* X, int64_t n, int64_t n_pad, int d, const float* w, double wsum, float* nrm,
                             float* lw2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i < n) {
        float s = 0.f;
        for (int c = 0; c < d; ++c) {
            const float v = X[i * d + c];
            s = fmaf(v, v, s);
        }
        nrm[i] = s;
        lw2[i] = (float)log2((double)w[i] / wsum);
    } else {
        nrm[i] = 0.f;
        lw2[i] = -INFINITY;
    }
}

hipError_t launch_norms_logw(const float* X, int64_t n, int64_t n_pad, int d, const float* w, double wsum, float* nrm,
                             float* lw2, hipStream_t stream) {
    hipLaunchKernelGGL(k_norms_logw, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, stream, X, n, n_pad, d, w,
                       wsum, nrm, lw2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing a feature matrix F (rows x d, row-major) into the MFMA layout with
// bias slots.  side 0: row operand A (potential (Ph, Pl), aux = |X|^2);
// side 1: column operand B (potential (Ph, Pl), aux = ms).  Split BF16:
// A = [Fh, Fh, Fl], B = [Fh, Fl, Fh].
// ---------------------------------------------------------------------------

__global__ void k_pack(const float* F, int64_t rows, int64_t rows_pad, int d, float scale, int prec, int side,
                       const float* ph, const float* pl, const float* aux, void* pack) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= rows_pad) return;
    const int dp = feat_pad_dev(d);
    const bool real = r < rows;
    const float Ph = real ? ph[r] : -INFINITY;
    const float Pl = real ? pl[r] : 0.f;
    const float Q = real ? aux[r] : 0.f;
    if (prec == PREC_F32) {
        const int groups = (dp + BIAS_F32) / 8;
        float* pk = (float*)pack;
        for (int k = 0; k < dp; ++k) {
            const float v = (real && k < d) ? F[r * d + k] * scale : 0.f;
            pk[f32_pack_off((int)r, k, groups)] = v;
        }
        if (side == 0) write_bias_a_f32(pk, (int)r, dp, groups, Ph, Pl, Q);
        else write_bias_b_f32(pk, (int)r, dp, groups, Ph, Pl, Q);
        return;
    }
    uint16_t* pk = (uint16_t*)pack;
    const int slabs = prec == PREC_BF16 ? (dp + BIAS_BF16) / 16 : (3 * dp + BIAS_BF16) / 16;
    const int kb = prec == PREC_BF16 ? dp : 3 * dp;
    for (int k = 0; k < dp; ++k) {
        const float v = (real && k < d) ? F[r * d + k] * scale : 0.f;
        uint16_t h, l;
        split2_bf16(v, h, l);
        if (prec == PREC_BF16) {
            pk[bf16_pack_off((int)r, k, slabs)] = h;
        } else {
            pk[bf16_pack_off((int)r, k, slabs)] = h;
            pk[bf16_pack_off((int)r, dp + k, slabs)] = side == 0 ? h : l;
            pk[bf16_pack_off((int)r, 2 * dp + k, slabs)] = side == 0 ? l : h;
        }
    }
    if (side == 0) write_bias_a_bf16(pk, (int)r, kb, slabs, Ph, Pl, Q);
    else write_bias_b_bf16(pk, (int)r, kb, slabs, Ph, Pl, Q);
}

hipError_t launch_pack(const float* F, int64_t rows, int64_t rows_pad, int d, float scale, int prec, int side,
                       const float* ph, const float* pl, const float* aux, void* pack, hipStream_t stream) {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((rows_pad + 127) / 128)), dim3(128), 0, stream, F, rows, rows_pad, d,
                       scale, prec, side, ph, pl, aux, pack);
    return hipGetLastError();
}

// Refresh only the potential slots of a pack.
__global__ void k_pack_pot(const float* ph, const float* pl, int64_t rows_pad, int d, int prec, int side, void* pack) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= rows_pad) return;
    const int dp = feat_pad_dev(d);
    if (prec == PREC_F32) {
        const int groups = (dp + BIAS_F32) / 8;
        if (side == 0) write_pot_a_f32((float*)pack, (int)r, dp, groups, ph[r], pl[r]);
        else write_pot_b_f32((float*)pack, (int)r, dp, groups, ph[r], pl[r]);
        return;
    }
    const int slabs = prec == PREC_BF16 ? (dp + BIAS_BF16) / 16 : (3 * dp + BIAS_BF16) / 16;
    const int kb = prec == PREC_BF16 ? dp : 3 * dp;
    if (side == 0) write_pot_a_bf16((uint16_t*)pack, (int)r, kb, slabs, ph[r], pl[r]);
    else write_pot_b_bf16((uint16_t*)pack, (int)r, kb, slabs, ph[r], pl[r]);
}

hipError_t launch_pack_pot(const float* ph, const float* pl, int64_t rows_pad, int d, int prec, int side, void* pack,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_pack_pot, dim3((unsigned)((rows_pad + 255) / 256)), dim3(256), 0, stream, ph, pl, rows_pad,
                       d, prec, side, pack);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-outer-step prologue (Algorithm 1: Zbar_j = [Gamma_t Y_j, |Y_j|^2 / 2]).
// Potentials live in log2 units as FP32 (hi, lo) pairs and are rebased in
// FP64 when the temperature or Gamma changes, keeping f and g (Algorithm 1's
// convention, cost units) fixed across the outer step boundary:
//   expanded form: U = log2 a + k (f - alpha),  V = log2 b + k (g - beta)
//   direct form:   U = log2 a + k f,            V = log2 b + k g
// with alpha_i = n_i + n_i^2/4, beta_j = |Z_j|^2 + m_j^2/4 (FP64).
// first != 0: start from f0/g0 (NULL = 0) instead of the previous state.
// ---------------------------------------------------------------------------

// One work-group takes 256 / dD columns; thread (column, c) computes
// (Gamma Y_j)_c with the products added in e order, and one thread per column
// adds |Z_j|^2 in c order and rebases V_j, so every value is the one a
// thread-per-column loop gives.  Gamma sits in LDS with rows padded by one
// float (no bank conflicts between the c threads).
constexpr int PRO_THREADS = 256;
__global__ void __launch_bounds__(PRO_THREADS) k_prologue_cols(const float* Y, int64_t m, int64_t m_pad, int dE,
                                                               int dD, const float* gamma, const float* ynorm,
                                                               const float* lb2, const float* g0, int first,
                                                               int expanded, double kappa, double kappa_old,
                                                               float* Zout, double* beta, float* Vh, float* Vl,
                                                               float* ms) {
    extern __shared__ float gsh_dyn[];
    __shared__ float sbuf[PRO_THREADS];
    const int gs = dE + 1;  // padded row stride of Gamma in LDS
    const bool in_lds = dD * gs <= 16128;  // with sbuf, at most 64 KiB of LDS
    if (in_lds) {
        for (int t = threadIdx.x; t < dD * dE; t += blockDim.x) gsh_dyn[(t / dE) * gs + t % dE] = gamma[t];
        __syncthreads();
    }
    const int cpb = PRO_THREADS / dD;  // columns per work-group (dD <= 256)
    const int jl = threadIdx.x / dD, c = threadIdx.x - jl * dD;
    const int64_t j = blockIdx.x * (int64_t)cpb + jl;
    const bool act = jl < cpb && j < m_pad;
    const float sc = expanded ? (float)(2.0 * kappa) : 1.f;
    if (act) {
        if (j < m) {
            float s = 0.f;
            if (in_lds) {
                for (int e = 0; e < dE; ++e) s = fmaf(gsh_dyn[c * gs + e], Y[j * dE + e], s);
            } else {
                for (int e = 0; e < dE; ++e) s = fmaf(gamma[c * dE + e], Y[j * dE + e], s);
            }
            Zout[j * dD + c] = sc * s;
            sbuf[jl * dD + c] = s;
        } else {
            Zout[j * dD + c] = 0.f;
        }
    }
    __syncthreads();
    if (!act || c != 0) return;
    if (j >= m) {
        Vh[j] = -INFINITY;
        Vl[j] = 0.f;
        ms[j] = 0.f;
        if (expanded) beta[j] = 0.0;
        return;
    }
    double z2 = 0.0;
    for (int k = 0; k < dD; ++k) {
        const double v = (double)sbuf[jl * dD + k];
        z2 += v * v;
    }
    const double mj = (double)ynorm[j];
    const double lb = (double)lb2[j];
    double V;
    if (expanded) {
        const double bnew = z2 + 0.25 * mj * mj;
        if (first) {
            V = lb + kappa * ((g0 ? (double)g0[j] : 0.0) - bnew);
        } else {
            const double ghat = (join_df(Vh[j], Vl[j]) - lb) / kappa_old;
            V = lb + kappa * (ghat + beta[j] - bnew);
        }
        beta[j] = bnew;
        ms[j] = (float)(0.5 * kappa * mj);
    } else {
        V = first ? lb + kappa * (g0 ? (double)g0[j] : 0.0) : lb + (kappa / kappa_old) * (join_df(Vh[j], Vl[j]) - lb);
        ms[j] = (float)mj;
    }
    float h, l;
    split_df(V, h, l);
    Vh[j] = h;
    Vl[j] = l;
}

hipError_t launch_prologue_cols(const float* Y, int64_t m, int64_t m_pad, int dE, int dD, const float* gamma,
                                const float* ynorm, const float* lb2, const float* g0, int first, int expanded,
                                double kappa, double kappa_old, float* Zout, double* beta, float* Vh, float* Vl,
                                float* ms, hipStream_t stream) {
    if (dD < 1 || dD > PRO_THREADS) return hipErrorInvalidValue;
    const size_t sh = dD * (dE + 1) <= 16128 ? (size_t)dD * (dE + 1) * sizeof(float) : 0;
    const int cpb = PRO_THREADS / dD;
    hipLaunchKernelGGL(k_prologue_cols, dim3((unsigned)((m_pad + cpb - 1) / cpb)), dim3(PRO_THREADS), sh, stream, Y,
                       m, m_pad, dE, dD, gamma, ynorm, lb2, g0, first, expanded, kappa, kappa_old, Zout, beta, Vh, Vl,
                       ms);
    return hipGetLastError();
}

__global__ void k_prologue_rows(int64_t n, int64_t n_pad, const float* xnorm, const float* la2, const float* f0,
                                int first, int expanded, double kappa, double kappa_old, float* Uh, float* Ul) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i >= n) {
        Uh[i] = -INFINITY;
        Ul[i] = 0.f;
        return;
    }
    const double la = (double)la2[i];
    double U;
    if (first) {
        const double ni = (double)xnorm[i];
        const double alpha = expanded ? ni + 0.25 * ni * ni : 0.0;
        U = la + kappa * ((f0 ? (double)f0[i] : 0.0) - alpha);
    } else {
        U = la + (kappa / kappa_old) * (join_df(Uh[i], Ul[i]) - la);
    }
    float h, l;
    split_df(U, h, l);
    Uh[i] = h;
    Ul[i] = l;
}

hipError_t launch_prologue_rows(int64_t n, int64_t n_pad, const float* xnorm, const float* la2, const float* f0,
                                int first, int expanded, double kappa, double kappa_old, float* Uh, float* Ul,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_prologue_rows, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, stream, n, n_pad, xnorm,
                       la2, f0, first, expanded, kappa, kappa_old, Uh, Ul);
    return hipGetLastError();
}

// Back to Algorithm 1's convention: f = (U - log2 a) / kappa + shift, with
// shift = alpha_i (kind 1: rows, expanded), beta_j (kind 2: columns,
// expanded) or 0 (kind 0: direct form).
__global__ void k_epilogue(int64_t n, const float* Uh, const float* Ul, const float* lw2, const float* xnorm,
                           const double* beta, int kind, double kappa, float* f) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sh = 0.0;
    if (kind == 1) {
        const double ni = (double)xnorm[i];
        sh = ni + 0.25 * ni * ni;
    } else if (kind == 2) {
        sh = beta[i];
    }
    f[i] = (float)((join_df(Uh[i], Ul[i]) - (double)lw2[i]) / kappa + sh);
}

hipError_t launch_epilogue(int64_t n, const float* Uh, const float* Ul, const float* lw2, const float* xnorm,
                           const double* beta, int kind, double kappa, float* f, hipStream_t stream) {
    hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, Uh, Ul, lw2, xnorm,
                       beta, kind, kappa, f);
    return hipGetLastError();
}

// Fill a float array (used to give padded potentials -inf in both parities).
__global__ void k_fill(float* p, int64_t n, float v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 moments of centred features with weights w:
//   s = sum w |X|^2, m4 = sum w |X|^4, Sigma = sum w X X^T (d x d),
//   m3 = sum w |X|^2 X (d).
// part layout per block: [s, m4, Sigma (d*d), m3 (d)].
// ---------------------------------------------------------------------------

// Rows are staged 32 at a time in LDS with their FP64 norms and weights;
// block (x, y) covers rows of block x and outputs [2048 y, 2048 (y + 1)),
// eight per thread, accumulated over the staged rows in order.
constexpr int MOM_CHUNK = 32, MOM_PER_THREAD = 8, MOM_OUT_BLK = 256 * MOM_PER_THREAD;

__global__ void __launch_bounds__(256) k_moments_part(const float* X, int64_t n, int d, const float* w, double* part,
                                                      int rows_per_blk) {
    extern __shared__ float xs[];  // MOM_CHUNK x d
    __shared__ double nr[MOM_CHUNK], wr[MOM_CHUNK];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(n, r0 + rows_per_blk);
    const int width = 2 + d * d + d;
    const int t0 = blockIdx.y * MOM_OUT_BLK + threadIdx.x;
    double acc[MOM_PER_THREAD];
#pragma unroll
    for (int k = 0; k < MOM_PER_THREAD; ++k) acc[k] = 0.0;
    for (int64_t c0 = r0; c0 < r1; c0 += MOM_CHUNK) {
        const int nc = (int)min((int64_t)MOM_CHUNK, r1 - c0);
        __syncthreads();
        for (int u = threadIdx.x; u < nc * d; u += blockDim.x) xs[u] = X[c0 * d + u];
        __syncthreads();
        if (threadIdx.x < nc) {
            double q = 0.0;
            for (int c = 0; c < d; ++c) {
                const double v = (double)xs[threadIdx.x * d + c];
                q += v * v;
            }
            nr[threadIdx.x] = q;
            wr[threadIdx.x] = (double)w[c0 + threadIdx.x];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MOM_PER_THREAD; ++k) {
            const int t = t0 + k * 256;
            if (t >= width) break;
            double a = acc[k];
            if (t == 0) {
                for (int r = 0; r < nc; ++r) a += wr[r] * nr[r];
            } else if (t == 1) {
                for (int r = 0; r < nc; ++r) a += wr[r] * nr[r] * nr[r];
            } else if (t < 2 + d * d) {
                const int u = (t - 2) / d, v = (t - 2) - u * d;
                for (int r = 0; r < nc; ++r) a += wr[r] * (double)xs[r * d + u] * (double)xs[r * d + v];
            } else {
                const int c = t - 2 - d * d;
                for (int r = 0; r < nc; ++r) a += wr[r] * nr[r] * (double)xs[r * d + c];
            }
            acc[k] = a;
        }
    }
    double* out = part + (size_t)blockIdx.x * width;
#pragma unroll
    for (int k = 0; k < MOM_PER_THREAD; ++k) {
        const int t = t0 + k * 256;
        if (t < width) out[t] = acc[k];
    }
}

__global__ void k_moments_final(const double* part, int nblk, int width, double* out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= width) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * width + t];
    out[t] = s;
}

size_t moments_part_doubles(int64_t n, int d) { return (size_t)((n + 511) / 512) * (2 + d * d + d); }

hipError_t launch_moments(const float* X, int64_t n, int d, const float* w, double* part, double* out,
                          hipStream_t stream) {
    const int rows_per_blk = 512;
    const int nblk = (int)((n + rows_per_blk - 1) / rows_per_blk);
    const int width = 2 + d * d + d;
    const int oblk = (width + MOM_OUT_BLK - 1) / MOM_OUT_BLK;
    hipLaunchKernelGGL(k_moments_part, dim3(nblk, oblk), dim3(256), (size_t)MOM_CHUNK * d * sizeof(float), stream, X,
                       n, d, w, part, rows_per_blk);
    hipLaunchKernelGGL(k_moments_final, dim3((width + 255) / 256), dim3(256), 0, stream, part, nblk, width, out);
    return hipGetLastError();
}

}  // namespace gwk
