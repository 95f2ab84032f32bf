// Kernels of the full-N kernel PCA (Appendix B, "Kernel PCA" with
// Algorithm 4's kernel from a CNT cost), run matrix-free by randomized
// subspace iteration (blocks of up to 16 columns in k_kpca_cm, wider ones in
// k_kpca_cm_wide):
//   - R = C M for C_ij = |x_i - x_j|^p generated on the fly (never stored),
//     M an n x l block of vectors (column-major FP64), accumulated in FP64;
//   - the start block: counter-based uniform numbers in [-1, 1);
//   - the features X_i = V_i sqrt(Lambda) from the Ritz vectors.
// The double centring of Algorithm 4 is applied outside the product as
// rank-one corrections, so this kernel only sees the raw cost.
#include <hip/hip_runtime.h>

#include "gw_kpca.h"

namespace gwk {

constexpr int KP_THREADS = 256;
constexpr int KP_ROWS = 4;    // rows of C per thread
constexpr int KP_COLS = 16;   // columns of M per block (gridDim.y covers l)
constexpr int KP_TJ = 64;     // points j per LDS tile

// pmode: 0 p = 2 (squared distance), 1 p = 1 (distance), 2 general p.
template <int MAXD>
__global__ void __launch_bounds__(KP_THREADS) k_kpca_cm(const float* __restrict__ x, int64_t n, int d, int pmode,
                                                        float half_p, const double* __restrict__ M, int64_t ldm,
                                                        int l, double* __restrict__ R, int64_t ldr) {
    __shared__ float xs[KP_TJ * MAXD];
    __shared__ double ms[KP_TJ * KP_COLS];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.y * KP_COLS;
    const int64_t i0 = ((int64_t)blockIdx.x * KP_THREADS + tid) * KP_ROWS;
    float xi[KP_ROWS][MAXD];
#pragma unroll
    for (int r = 0; r < KP_ROWS; ++r)
#pragma unroll
        for (int dd = 0; dd < MAXD; ++dd) xi[r][dd] = (i0 + r < n && dd < d) ? x[(i0 + r) * d + dd] : 0.f;
    double acc[KP_ROWS][KP_COLS];
#pragma unroll
    for (int r = 0; r < KP_ROWS; ++r)
#pragma unroll
        for (int cc = 0; cc < KP_COLS; ++cc) acc[r][cc] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += KP_TJ) {
        __syncthreads();
        for (int e = tid; e < KP_TJ * MAXD; e += KP_THREADS) {
            const int jj = e / MAXD, dd = e - jj * MAXD;
            xs[e] = (j0 + jj < n && dd < d) ? x[(j0 + jj) * d + dd] : 0.f;
        }
        for (int e = tid; e < KP_TJ * KP_COLS; e += KP_THREADS) {
            const int cc = e / KP_TJ, jj = e - cc * KP_TJ;
            ms[jj * KP_COLS + cc] = (j0 + jj < n && c0 + cc < l) ? M[(int64_t)(c0 + cc) * ldm + j0 + jj] : 0.0;
        }
        __syncthreads();
        const int nj = (int)(n - j0 < KP_TJ ? n - j0 : KP_TJ);
        for (int jj = 0; jj < nj; ++jj) {
            double cij[KP_ROWS];
#pragma unroll
            for (int r = 0; r < KP_ROWS; ++r) {
                float s = 0.f;
#pragma unroll
                for (int dd = 0; dd < MAXD; ++dd) {
                    const float t = xi[r][dd] - xs[jj * MAXD + dd];
                    s = fmaf(t, t, s);
                }
                float c;
                if (pmode == 0) c = s;
                else if (pmode == 1) c = sqrtf(s);
                else c = s > 0.f ? exp2f(half_p * log2f(s)) : 0.f;
                cij[r] = (double)c;
            }
#pragma unroll
            for (int cc = 0; cc < KP_COLS; ++cc) {
                const double mv = ms[jj * KP_COLS + cc];
#pragma unroll
                for (int r = 0; r < KP_ROWS; ++r) acc[r][cc] = fma(cij[r], mv, acc[r][cc]);
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < KP_COLS; ++cc)
#pragma unroll
        for (int r = 0; r < KP_ROWS; ++r)
            if (i0 + r < n && c0 + cc < l) R[(int64_t)(c0 + cc) * ldr + i0 + r] = acc[r][cc];
}

// Wide form for blocks of more than 16 columns: a workgroup of 6 waves covers
// 256 rows x 96 columns.  The costs of a 256 x 32 tile are computed once into
// LDS (instead of once per column group); wave w owns columns 8 w..8 w+7 of
// the workgroup's 96 and thread t of the wave rows 4 t..4 t+3, so the four
// costs of a point are one 16-byte LDS read and the M values are broadcasts.
constexpr int KW_ROWS = 256, KW_COLS = 96, KW_TJ = 32, KW_CPW = 6, KW_THREADS = 64 * (KW_COLS / KW_CPW);

template <int MAXD>
__global__ void __launch_bounds__(KW_THREADS) k_kpca_cm_wide(const float* __restrict__ x, int64_t n, int d,
                                                             int pmode, float half_p, const double* __restrict__ M,
                                                             int64_t ldm, int l, double* __restrict__ R,
                                                             int64_t ldr) {
    __shared__ float xr[KW_ROWS * MAXD];
    __shared__ float xs[KW_TJ * MAXD];
    __shared__ __attribute__((aligned(16))) float cs[KW_TJ * KW_ROWS];
    __shared__ __attribute__((aligned(16))) double ms[KW_TJ * KW_COLS];
    const int tid = threadIdx.x;
    const int lane = tid & 63, grp = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * KW_ROWS;
    const int col0 = blockIdx.y * KW_COLS;
    for (int e = tid; e < KW_ROWS * MAXD; e += KW_THREADS) {
        const int r = e / MAXD, dd = e - r * MAXD;
        xr[e] = (row0 + r < n && dd < d) ? x[(row0 + r) * d + dd] : 0.f;
    }
    double acc[4][KW_CPW];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int cc = 0; cc < KW_CPW; ++cc) acc[r][cc] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += KW_TJ) {
        __syncthreads();
        for (int e = tid; e < KW_TJ * MAXD; e += KW_THREADS) {
            const int jj = e / MAXD, dd = e - jj * MAXD;
            xs[e] = (j0 + jj < n && dd < d) ? x[(j0 + jj) * d + dd] : 0.f;
        }
        for (int e = tid; e < KW_TJ * KW_COLS; e += KW_THREADS) {
            const int cc = e / KW_TJ, jj = e - cc * KW_TJ;
            ms[jj * KW_COLS + cc] = (j0 + jj < n && col0 + cc < l) ? M[(int64_t)(col0 + cc) * ldm + j0 + jj] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < KW_TJ * KW_ROWS; e += KW_THREADS) {
            const int jj = e / KW_ROWS, r = e - jj * KW_ROWS;
            float s = 0.f;
#pragma unroll
            for (int dd = 0; dd < MAXD; ++dd) {
                const float t = xr[r * MAXD + dd] - xs[jj * MAXD + dd];
                s = fmaf(t, t, s);
            }
            float c;
            if (pmode == 0) c = s;
            else if (pmode == 1) c = sqrtf(s);
            else c = s > 0.f ? exp2f(half_p * log2f(s)) : 0.f;
            cs[jj * KW_ROWS + r] = c;
        }
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < KW_TJ; ++jj) {
            const float4 c4 = *(const float4*)&cs[jj * KW_ROWS + lane * 4];
            const double cr[4] = {(double)c4.x, (double)c4.y, (double)c4.z, (double)c4.w};
            const double* mrow = &ms[jj * KW_COLS + grp * KW_CPW];
#pragma unroll
            for (int cc = 0; cc < KW_CPW; ++cc) {
                const double mv = mrow[cc];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r][cc] = fma(cr[r], mv, acc[r][cc]);
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < KW_CPW; ++cc) {
        const int col = col0 + grp * KW_CPW + cc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = row0 + lane * 4 + r;
            if (i < n && col < l) R[(int64_t)col * ldr + i] = acc[r][cc];
        }
    }
}

// Omega_ij uniform in [-1, 1) from SplitMix64 of (seed, j * n + i).
__global__ void k_kpca_start(int64_t n, int l, uint64_t seed, double* Om) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)l) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    Om[e] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

__global__ void k_kpca_widen(const float* __restrict__ a, int64_t n, double* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)a[i];
}

// X[i][k] = V[i][l-1-k] sqrt(theta_{l-1-k}), k < D: the D largest Ritz values
// (V = Q U, column-major n x l, theta ascending); 0 where theta <= floor.
__global__ void k_kpca_features(const double* __restrict__ V, int64_t ldv, int64_t n, int l, int D,
                                const double* __restrict__ theta, double floor, float* X, int ldx) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)D) return;
    const int64_t i = e / D;
    const int k = (int)(e - i * D);
    const int col = l - 1 - k;
    const double th = theta[col];
    X[i * ldx + k] = th > floor ? (float)(V[(int64_t)col * ldv + i] * sqrt(th)) : 0.f;
}

static int blocks_for(int64_t count, int threads) { return (int)((count + threads - 1) / threads); }

hipError_t launch_kpca_cm(const float* x, int64_t n, int d, double p, const double* M, int64_t ldm, int l, double* R,
                          int64_t ldr, hipStream_t stream) {
    if (n < 1 || l < 1 || d < 1 || d > KPCA_MAX_IN_DIM) return hipErrorInvalidValue;
    const int pmode = p == 2.0 ? 0 : (p == 1.0 ? 1 : 2);
    if (l > KP_COLS) {
        const dim3 gw(blocks_for(n, KW_ROWS), (l + KW_COLS - 1) / KW_COLS);
        if (d <= 4)
            hipLaunchKernelGGL(k_kpca_cm_wide<4>, gw, dim3(KW_THREADS), 0, stream, x, n, d, pmode, (float)(0.5 * p),
                               M, ldm, l, R, ldr);
        else
            hipLaunchKernelGGL(k_kpca_cm_wide<8>, gw, dim3(KW_THREADS), 0, stream, x, n, d, pmode, (float)(0.5 * p),
                               M, ldm, l, R, ldr);
        return hipGetLastError();
    }
    const dim3 grid(blocks_for(n, KP_THREADS * KP_ROWS), (l + KP_COLS - 1) / KP_COLS);
    if (d <= 4)
        hipLaunchKernelGGL(k_kpca_cm<4>, grid, dim3(KP_THREADS), 0, stream, x, n, d, pmode, (float)(0.5 * p), M, ldm,
                           l, R, ldr);
    else
        hipLaunchKernelGGL(k_kpca_cm<8>, grid, dim3(KP_THREADS), 0, stream, x, n, d, pmode, (float)(0.5 * p), M, ldm,
                           l, R, ldr);
    return hipGetLastError();
}

hipError_t launch_kpca_start(int64_t n, int l, uint64_t seed, double* Om, hipStream_t stream) {
    hipLaunchKernelGGL(k_kpca_start, dim3(blocks_for(n * (int64_t)l, 256)), dim3(256), 0, stream, n, l, seed, Om);
    return hipGetLastError();
}

hipError_t launch_kpca_widen(const float* a, int64_t n, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_kpca_widen, dim3(blocks_for(n, 256)), dim3(256), 0, stream, a, n, out);
    return hipGetLastError();
}

hipError_t launch_kpca_features(const double* V, int64_t ldv, int64_t n, int l, int D, const double* theta,
                                double floor, float* X, int ldx, hipStream_t stream) {
    hipLaunchKernelGGL(k_kpca_features, dim3(blocks_for(n * (int64_t)D, 256)), dim3(256), 0, stream, V, ldv, n, l, D,
                       theta, floor, X, ldx);
    return hipGetLastError();
}

}  // namespace gwk

namespace gwk {

__global__ void k_kpca_fill(double* p, int64_t n, double v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_kpca_fill(double* p, int64_t n, double v, hipStream_t stream) {
    hipLaunchKernelGGL(k_kpca_fill, dim3((int)((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace gwk

namespace gwk {

// ---------------------------------------------------------------------------
// Tall-skinny products of the subspace iteration (n x l blocks, column-major,
// l small): G = A^T B and T = Y W.  Both are bound by reading the n x l
// blocks once; the Gram matrix is summed per chunk of rows and the chunks are
// reduced in a fixed order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------

constexpr int KG_ROWS = 2048;   // rows per chunk
constexpr int KG_SUB = 32;      // rows per LDS stage
constexpr int KG_B = 96;        // output block edge (16 x 16 threads, 6 x 6 each)

// part[chunk][bp][bq] 96 x 96 block (row-major, padded) of A^T B over the chunk.
__global__ void __launch_bounds__(256) k_kpca_gram_part(const double* __restrict__ A, const double* __restrict__ B,
                                                        int64_t n, int l, double* part, int nb) {
    __shared__ double as[KG_SUB * KG_B];
    __shared__ double bs[KG_SUB * KG_B];
    const int tid = threadIdx.x, tp = tid >> 4, tq = tid & 15;
    const int bp = blockIdx.y, bq = blockIdx.z;
    const int64_t r0 = (int64_t)blockIdx.x * KG_ROWS;
    double acc[6][6];
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
        for (int v = 0; v < 6; ++v) acc[u][v] = 0.0;
    for (int s0 = 0; s0 < KG_ROWS; s0 += KG_SUB) {
        __syncthreads();
        for (int e = tid; e < KG_SUB * KG_B; e += 256) {
            const int c = e / KG_SUB, r = e - c * KG_SUB;
            const int64_t i = r0 + s0 + r;
            const int ca = bp * KG_B + c, cb = bq * KG_B + c;
            as[r * KG_B + c] = (i < n && ca < l) ? A[(int64_t)ca * n + i] : 0.0;
            bs[r * KG_B + c] = (i < n && cb < l) ? B[(int64_t)cb * n + i] : 0.0;
        }
        __syncthreads();
        for (int r = 0; r < KG_SUB; ++r) {
            double av[6], bv[6];
#pragma unroll
            for (int u = 0; u < 6; ++u) av[u] = as[r * KG_B + tp * 6 + u];
#pragma unroll
            for (int v = 0; v < 6; ++v) bv[v] = bs[r * KG_B + tq * 6 + v];
#pragma unroll
            for (int u = 0; u < 6; ++u)
#pragma unroll
                for (int v = 0; v < 6; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
    }
    double* out = part + (((int64_t)blockIdx.x * nb + bp) * nb + bq) * (KG_B * KG_B);
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
        for (int v = 0; v < 6; ++v) out[(tp * 6 + u) * KG_B + tq * 6 + v] = acc[u][v];
}

// G (column-major l x l) = sum over chunks, in chunk order.
__global__ void k_kpca_gram_reduce(const double* __restrict__ part, int nchunks, int l, int nb, double* G) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)l * l) return;
    const int q = (int)(e / l), p = (int)(e - (int64_t)q * l);
    const int bp = p / KG_B, bq = q / KG_B, pp = p - bp * KG_B, qq = q - bq * KG_B;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(((int64_t)c * nb + bp) * nb + bq) * (KG_B * KG_B) + pp * KG_B + qq];
    G[e] = s;
}

// T[:, c0:c0+16] = Y W[:, c0:c0+16] (W column-major l x l, l <= 288).
__global__ void __launch_bounds__(256) k_kpca_rowmul(const double* __restrict__ Y, int64_t n, int l,
                                                     const double* __restrict__ W, double* __restrict__ T) {
    __shared__ double ws[288 * 16];
    const int c0 = blockIdx.y * 16;
    for (int e = threadIdx.x; e < l * 16; e += 256) {
        const int k = e / 16, c = e - k * 16;
        ws[e] = c0 + c < l ? W[(int64_t)(c0 + c) * l + k] : 0.0;
    }
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    for (int k = 0; k < l; ++k) {
        const double y = Y[(int64_t)k * n + i];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = fma(y, ws[k * 16 + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (c0 + c < l) T[(int64_t)(c0 + c) * n + i] = acc[c];
}

size_t kpca_gram_part_doubles(int64_t n, int l) {
    const int64_t nchunks = (n + KG_ROWS - 1) / KG_ROWS;
    const int nb = (l + KG_B - 1) / KG_B;
    return (size_t)nchunks * nb * nb * KG_B * KG_B;
}

hipError_t launch_kpca_gram(const double* A, const double* B, int64_t n, int l, double* part, double* G,
                            hipStream_t stream) {
    if (l < 1 || l > 288 || n < 1) return hipErrorInvalidValue;
    const int nchunks = (int)((n + KG_ROWS - 1) / KG_ROWS);
    const int nb = (l + KG_B - 1) / KG_B;
    hipLaunchKernelGGL(k_kpca_gram_part, dim3(nchunks, nb, nb), dim3(256), 0, stream, A, B, n, l, part, nb);
    hipLaunchKernelGGL(k_kpca_gram_reduce, dim3((int)(((int64_t)l * l + 255) / 256)), dim3(256), 0, stream,
                       (const double*)part, nchunks, l, nb, G);
    return hipGetLastError();
}

hipError_t launch_kpca_rowmul(const double* Y, int64_t n, int l, const double* W, double* T, hipStream_t stream) {
    if (l < 1 || l > 288 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kpca_rowmul, dim3((int)((n + 255) / 256), (l + 15) / 16), dim3(256), 0, stream, Y, n, l, W,
                       T);
    return hipGetLastError();
}

}  // namespace gwk
