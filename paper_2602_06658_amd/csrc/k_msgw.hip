// Kernels of Multiscale-GW (Appendix B, "Implementation of Multiscale-GW"):
//   - Coarsen: weighted K-Means.  Assignment of every point to its nearest
//     centroid, cluster sums in exact fixed-point integers, centroid update,
//     compaction of the non-empty clusters.
//   - Algorithm 8 (Interpolate): one Sinkhorn operator of fine points
//     against a coarse measure, f_q = -eps' ln sum_r w_r exp((h_r - |P_q - Q_r|^2) / eps'),
//     over lifted features P = [X, |X|^2/2] and Q = [Gamma Y, |Y|^2/2] (the
//     last coordinate passed apart, so that D = 64 fills one 64-wide chunk).
//
// Both scans are one thread per point against tiles of MS_TJ reference rows
// staged in LDS (every lane reads the same LDS word: a broadcast), with the
// point's coordinates in registers, CH at a time.  Work per pair is
// O(D); these run once per multiscale solve, next to the O(N M) Sinkhorn
// passes, so they are plain VALU code.
#include <hip/hip_runtime.h>

#include "gw_msgw.h"

namespace gwk {

constexpr int MS_THREADS = 256;
constexpr int MS_TJ = 16;
constexpr int MS_MAXDP = 256;  // coordinates of an LDS row: up to 256, in chunks of 64

// ---------------------------------------------------------------------------
// K-Means assignment: assign[i] = argmin_j |X_i - C_j|^2, ties to the lowest
// j.  The distance is summed over the coordinates in order in single
// precision with every subtraction, square and addition rounded on its own
// (no fused multiply-add), so that the integer it decides is reproducible.
// Zero padding beyond D adds (0 - 0)^2 = +0 and leaves every partial sum
// unchanged.
// ---------------------------------------------------------------------------

template <int CH>
__global__ void __launch_bounds__(MS_THREADS) k_km_assign(const float* __restrict__ X, int64_t n, int ldx, int D,
                                                          const float* __restrict__ C, int k, int ldc,
                                                          int* __restrict__ assign) {
#pragma clang fp contract(off)
    const int NCH = (D + CH - 1) / CH;
    const int DP = CH * NCH;
    __shared__ float tile[MS_TJ * MS_MAXDP];
    const int64_t i = blockIdx.x * (int64_t)MS_THREADS + threadIdx.x;
    const bool live = i < n;
    const float* xi = X + (live ? i : 0) * (int64_t)ldx;
    float r[CH];
    if (NCH == 1) {
#pragma unroll
        for (int d = 0; d < CH; ++d) r[d] = (live && d < D) ? xi[d] : 0.f;
    }
    float best = INFINITY;
    int arg = 0;
    for (int j0 = 0; j0 < k; j0 += MS_TJ) {
        const int nj = min(MS_TJ, k - j0);
        __syncthreads();
        for (int e = threadIdx.x; e < MS_TJ * DP; e += MS_THREADS) {
            const int jj = e / DP, d = e - jj * DP;
            tile[e] = (jj < nj && d < D) ? C[(int64_t)(j0 + jj) * ldc + d] : 0.f;
        }
        __syncthreads();
        float dist[MS_TJ];
#pragma unroll
        for (int jj = 0; jj < MS_TJ; ++jj) dist[jj] = 0.f;
#pragma unroll 1
        for (int c = 0; c < NCH; ++c) {
            if (NCH > 1) {
#pragma unroll
                for (int d = 0; d < CH; ++d) r[d] = (live && c * CH + d < D) ? xi[c * CH + d] : 0.f;
            }
#pragma unroll
            for (int jj = 0; jj < MS_TJ; ++jj) {
#pragma unroll
                for (int d = 0; d < CH; ++d) {
                    const float t = r[d] - tile[jj * DP + c * CH + d];
                    const float sq = t * t;
                    dist[jj] = dist[jj] + sq;
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < MS_TJ; ++jj)
            if (jj < nj && dist[jj] < best) {
                best = dist[jj];
                arg = j0 + jj;
            }
    }
    if (live) assign[i] = arg;
}

// ---------------------------------------------------------------------------
// Cluster sums: S[c][d] += rint(w_i X_id 2^S), W[c] += rint(w_i 2^61).  The
// product of two single-precision numbers is exact in double precision and
// the scaling by a power of two is exact, so each term is rounded once; the
// integer sums do not depend on the order of the atomics.
// ---------------------------------------------------------------------------

__global__ void k_km_zero(unsigned long long* s, int64_t count) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < count) s[e] = 0ull;
}

__global__ void k_km_zero32(unsigned int* p) {
    if (threadIdx.x == 0) p[0] = 0u;
}

__global__ void k_km_accum(const float* __restrict__ X, int64_t n, int ldx, int D, const float* __restrict__ w,
                           const int* __restrict__ assign, int S, unsigned long long* sums, unsigned long long* wsum) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)(D + 1)) return;
    const int64_t i = e / (D + 1);
    const int d = (int)(e - i * (D + 1));
    const int c = assign[i];
    const double wi = (double)w[i];
    if (d < D) {
        const double v = rint(ldexp(wi * (double)X[i * ldx + d], S));
        atomicAdd(&sums[(int64_t)c * D + d], (unsigned long long)(long long)v);
    } else {
        const double v = rint(ldexp(wi, KM_WEIGHT_EXP));
        atomicAdd(&wsum[c], (unsigned long long)(long long)v);
    }
}

// C_j = (S_j 2^-S) / (W_j 2^-61) rounded to single precision; empty
// clusters keep their centroid.
__global__ void k_km_update(const unsigned long long* __restrict__ sums, const unsigned long long* __restrict__ wsum,
                            int k, int D, int S, float* C, int ldc) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * D) return;
    const int j = (int)(e / D), d = (int)(e - (int64_t)j * D);
    const long long wj = (long long)wsum[j];
    if (wj == 0) return;
    const double num = ldexp((double)(long long)sums[e], -S);
    const double den = ldexp((double)wj, -KM_WEIGHT_EXP);
    C[(int64_t)j * ldc + d] = (float)(num / den);
}

__global__ void k_km_gather(const float* __restrict__ X, int ldx, int D, const int64_t* __restrict__ idx, int k,
                            float* C, int ldc) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * D) return;
    const int j = (int)(e / D), d = (int)(e - (int64_t)j * D);
    C[(int64_t)j * ldc + d] = X[idx[j] * ldx + d];
}

// Largest |X_id| as the bits of a non-negative float (ordered like the
// values, so an unsigned max finds it).
__global__ void k_km_maxabs(const float* __restrict__ X, int64_t n, int ldx, int D, unsigned int* out) {
    unsigned int m = 0u;
    const int64_t total = n * (int64_t)D;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / D;
        const int d = (int)(e - i * D);
        m = max(m, __float_as_uint(fabsf(X[i * ldx + d])));
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned int)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Compaction of the non-empty clusters in index order (one block): Xc, wc
// (the cluster weight W 2^-61 rounded to single precision), kept[p] = j,
// *kc = count.
__global__ void __launch_bounds__(1024) k_km_compact(const unsigned long long* __restrict__ wsum,
                                                     const float* __restrict__ C, int k, int D, int ldc, float* Xc,
                                                     float* wc, int* kept, int* kc) {
    __shared__ int wave_tot[16];
    __shared__ int base_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base_s = 0;
    __syncthreads();
    for (int j0 = 0; j0 < k; j0 += 1024) {
        const int j = j0 + tid;
        const bool on = j < k && wsum[j] != 0ull;
        const unsigned long long mask = __ballot(on);
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wave] = __popcll(mask);
        __syncthreads();
        int off = base_s;
        for (int v = 0; v < wave; ++v) off += wave_tot[v];
        if (on) {
            const int p = off + below;
            kept[p] = j;
            wc[p] = (float)ldexp((double)(long long)wsum[j], -KM_WEIGHT_EXP);
            for (int d = 0; d < D; ++d) Xc[(int64_t)p * D + d] = C[(int64_t)j * ldc + d];
        }
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int v = 0; v < 16; ++v) t += wave_tot[v];
            base_s += t;
        }
        __syncthreads();
    }
    if (tid == 0) *kc = base_s;
}

// ---------------------------------------------------------------------------
// Lifted features for Algorithm 8: out_i = G V_i (or V_i), zero-padded to
// ldo, and half_i = |V_i|^2 / 2, the last lifted coordinate.
// ---------------------------------------------------------------------------

__global__ void k_lift_bar(const float* __restrict__ V, int64_t n, int ldv, int dv, const float* __restrict__ G,
                           int D, float* out, int ldo, float* half) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* v = V + i * ldv;
    float* o = out + i * ldo;
    float nv = 0.f;
    for (int e = 0; e < dv; ++e) nv = fmaf(v[e], v[e], nv);
    const int dl = G ? D : dv;
    if (G) {
        for (int d = 0; d < D; ++d) {
            float s = 0.f;
            for (int e = 0; e < dv; ++e) s = fmaf(G[d * dv + e], v[e], s);
            o[d] = s;
        }
    } else {
        for (int d = 0; d < dv; ++d) o[d] = v[d];
    }
    for (int d = dl; d < ldo; ++d) o[d] = 0.f;
    half[i] = 0.5f * nv;
}

// hb_r = log2 w_r + kappa h_r, kappa = log2(e) / eps'.
__global__ void k_interp_bias(const float* __restrict__ w, const float* __restrict__ h, int64_t nr, float kappa,
                              float* hb) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < nr) hb[r] = log2f(w[r]) + kappa * h[r];
}

// out_q = -eps' ln2 log2 sum_r 2^(hb_r - kappa |P_q - Q_r|^2), an online
// max-shifted sum per thread, one rescale per tile.
template <int CH>
__global__ void __launch_bounds__(MS_THREADS) k_interp(const float* __restrict__ P, int64_t nq, int ldp,
                                                       const float* __restrict__ Q, int nr, int ldq, int dl,
                                                       const float* __restrict__ ph, const float* __restrict__ qh,
                                                       const float* __restrict__ hb, float kappa, float scale_out,
                                                       float* __restrict__ out) {
    const int NCH = (dl + CH - 1) / CH;
    const int DP = CH * NCH;
    __shared__ float tile[MS_TJ * MS_MAXDP];
    __shared__ float htile[MS_TJ];
    __shared__ float qtile[MS_TJ];
    const int64_t i = blockIdx.x * (int64_t)MS_THREADS + threadIdx.x;
    const bool live = i < nq;
    const float* pi = P + (live ? i : 0) * (int64_t)ldp;
    const float phi = live ? ph[i] : 0.f;
    float r[CH];
    if (NCH == 1) {
#pragma unroll
        for (int d = 0; d < CH; ++d) r[d] = (live && d < dl) ? pi[d] : 0.f;
    }
    float mx = -INFINITY, sum = 0.f;
    for (int j0 = 0; j0 < nr; j0 += MS_TJ) {
        const int nj = min(MS_TJ, nr - j0);
        __syncthreads();
        for (int e = threadIdx.x; e < MS_TJ * DP; e += MS_THREADS) {
            const int jj = e / DP, d = e - jj * DP;
            tile[e] = (jj < nj && d < dl) ? Q[(int64_t)(j0 + jj) * ldq + d] : 0.f;
        }
        if (threadIdx.x < MS_TJ) {
            htile[threadIdx.x] = threadIdx.x < nj ? hb[j0 + threadIdx.x] : -INFINITY;
            qtile[threadIdx.x] = threadIdx.x < nj ? qh[j0 + threadIdx.x] : 0.f;
        }
        __syncthreads();
        float dist[MS_TJ];
#pragma unroll
        for (int jj = 0; jj < MS_TJ; ++jj) {
            const float t = phi - qtile[jj];
            dist[jj] = t * t;
        }
#pragma unroll 1
        for (int c = 0; c < NCH; ++c) {
            if (NCH > 1) {
#pragma unroll
                for (int d = 0; d < CH; ++d) r[d] = (live && c * CH + d < dl) ? pi[c * CH + d] : 0.f;
            }
#pragma unroll
            for (int jj = 0; jj < MS_TJ; ++jj) {
#pragma unroll
                for (int d = 0; d < CH; ++d) {
                    const float t = r[d] - tile[jj * DP + c * CH + d];
                    dist[jj] = fmaf(t, t, dist[jj]);
                }
            }
        }
        float s[MS_TJ];
        float tmax = -INFINITY;
#pragma unroll
        for (int jj = 0; jj < MS_TJ; ++jj) {
            s[jj] = htile[jj] - kappa * dist[jj];
            tmax = fmaxf(tmax, s[jj]);
        }
        if (tmax > mx) {
            sum *= exp2f(mx - tmax);
            mx = tmax;
        }
#pragma unroll
        for (int jj = 0; jj < MS_TJ; ++jj) sum += exp2f(s[jj] - mx);
    }
    if (live) out[i] = scale_out * (mx + log2f(sum));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int blocks_for(int64_t count, int threads) { return (int)((count + threads - 1) / threads); }

// Chunk width 16, 32 or 64 (rows longer than 64 run in chunks of 64).
#define MS_DISPATCH(KERNEL, dims, grid, stream, ...)                                                    \
    do {                                                                                               \
        if ((dims) <= 16)                                                                              \
            hipLaunchKernelGGL((KERNEL<16>), dim3(grid), dim3(MS_THREADS), 0, stream, __VA_ARGS__);    \
        else if ((dims) <= 32)                                                                         \
            hipLaunchKernelGGL((KERNEL<32>), dim3(grid), dim3(MS_THREADS), 0, stream, __VA_ARGS__);    \
        else                                                                                           \
            hipLaunchKernelGGL((KERNEL<64>), dim3(grid), dim3(MS_THREADS), 0, stream, __VA_ARGS__);    \
    } while (0)

hipError_t launch_km_maxabs(const float* X, int64_t n, int ldx, int D, unsigned int* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_km_zero32, dim3(1), dim3(64), 0, stream, out);
    const int64_t total = n * (int64_t)D;
    int grid = blocks_for(total, 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_km_maxabs, dim3(grid), dim3(256), 0, stream, X, n, ldx, D, out);
    return hipGetLastError();
}

hipError_t launch_km_gather(const float* X, int ldx, int D, const int64_t* idx, int k, float* C, int ldc,
                            hipStream_t stream) {
    hipLaunchKernelGGL(k_km_gather, dim3(blocks_for((int64_t)k * D, 256)), dim3(256), 0, stream, X, ldx, D, idx, k, C,
                       ldc);
    return hipGetLastError();
}

hipError_t launch_km_iteration(const float* X, int64_t n, int ldx, int D, const float* w, float* C, int k, int ldc,
                               int S, int* assign, unsigned long long* sums, unsigned long long* wsum,
                               hipStream_t stream) {
    if (D < 1 || D > MS_MAXDP || k < 1 || n < 1) return hipErrorInvalidValue;
    const int64_t zc = (int64_t)k * D + k;  // sums and wsum are one allocation
    hipLaunchKernelGGL(k_km_zero, dim3(blocks_for(zc, 256)), dim3(256), 0, stream, sums, zc);
    MS_DISPATCH(k_km_assign, D, blocks_for(n, MS_THREADS), stream, X, n, ldx, D, (const float*)C, k, ldc, assign);
    hipLaunchKernelGGL(k_km_accum, dim3(blocks_for(n * (int64_t)(D + 1), 256)), dim3(256), 0, stream, X, n, ldx, D, w,
                       (const int*)assign, S, sums, wsum);
    hipLaunchKernelGGL(k_km_update, dim3(blocks_for((int64_t)k * D, 256)), dim3(256), 0, stream,
                       (const unsigned long long*)sums, (const unsigned long long*)wsum, k, D, S, C, ldc);
    return hipGetLastError();
}

hipError_t launch_km_compact(const unsigned long long* wsum, const float* C, int k, int D, int ldc, float* Xc,
                             float* wc, int* kept, int* kc, hipStream_t stream) {
    hipLaunchKernelGGL(k_km_compact, dim3(1), dim3(1024), 0, stream, wsum, C, k, D, ldc, Xc, wc, kept, kc);
    return hipGetLastError();
}

hipError_t launch_lift_bar(const float* V, int64_t n, int ldv, int dv, const float* G, int D, float* out, int ldo,
                           float* half, hipStream_t stream) {
    hipLaunchKernelGGL(k_lift_bar, dim3(blocks_for(n, 256)), dim3(256), 0, stream, V, n, ldv, dv, G, D, out, ldo,
                       half);
    return hipGetLastError();
}

hipError_t launch_interp(const float* P, int64_t nq, int ldp, const float* Q, int nr, int ldq, int dl,
                         const float* ph, const float* qh, const float* w, const float* h, double eps_prime, float* hb,
                         float* out, hipStream_t stream) {
    if (dl < 1 || dl > MS_MAXDP || nr < 1 || nq < 1) return hipErrorInvalidValue;
    const double kappa = 1.4426950408889634 / eps_prime;
    hipLaunchKernelGGL(k_interp_bias, dim3(blocks_for(nr, 256)), dim3(256), 0, stream, w, h, (int64_t)nr,
                       (float)kappa, hb);
    const float scale_out = (float)(-eps_prime * 0.6931471805599453);
    MS_DISPATCH(k_interp, dl, blocks_for(nq, MS_THREADS), stream, P, nq, ldp, Q, nr, ldq, dl, ph, qh,
                (const float*)hb, (float)kappa, scale_out, out);
    return hipGetLastError();
}

}  // namespace gwk
