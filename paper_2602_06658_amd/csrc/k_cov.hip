// Covariance pass of Algorithm 1 (X~_j and Gamma_{t+1} = sum_j b_j X~_j Y_j^T,
// i.e. Gamma_{t+1} = sum_ij pi_ij X_i Y_j^T), computed row-wise as
// T_i = sum_j pi_ij Y_j, then Gamma = sum_i X_i T_i^T in FP64; the same pass
// gives r_i = sum_j pi_ij and rm_i = sum_j pi_ij |Y_j|^2 for the lifted loss
// of Lemma C.1 (sum pi |x|^2 |y|^2 = sum_i |X_i|^2 rm_i).  With the operands
// swapped it gives the column-side sums the target gradient needs.
//
// Also: the FP64 evaluation of the final coupling for Err(pi) (Appendix A.1)
// and KL(pi | a x b).
#include "gw_cores.h"
#include "gw_prep.h"

using namespace gwl;

namespace gwk {

struct CovArgs {
    const uint4* A;     // row-side pack
    const uint4* B;     // column-side pack
    const uint4* PW;    // BF16 form: payload pack (see k_pack_payload), else unused
    const float* W;     // column-side features, m_pad x dw
    const float* mw;    // column-side norms
    int dw;
    float* Tp;
    float* rp;
    float* rmp;
    int tw;
    int n_chunks_r, n_chunks_c, rg, bc_chunks, n_mt_r, n_mt_c, n_pad, m_pad;
};

// lane = row (within a 32-row tile); tileT gives s^T so that lane l holds
// pi[i = l%32][j = acc_row(q, l)].  T accumulates with v_mfma_f32_32x32x2f32:
// D[e][i] += sum_{k=h} W[j(q,h)][e] pi[i][j(q,h)].
template <class C, int RW, int ES>
__global__ void __launch_bounds__(THREADS) k_cov_mfma(CovArgs p) {
    constexpr int NU = C::UNITS * 64;
    constexpr int WS = ES * 32 + 1;  // LDS row stride of the W chunk
    __shared__ uint4 zbuf[2][NU];
    __shared__ float wbuf[2][32 * WS];
    __shared__ float mbuf[2][32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int rb, cb;
    tile_coords(blockIdx.x, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);

    auto load_w = [&](int buf, int c) {
        for (int u = tid; u < 32 * ES * 32; u += THREADS) {
            const int j = u / (ES * 32), e = u - j * (ES * 32);
            const int col = c * 32 + j;
            wbuf[buf][j * WS + e] = e < p.dw ? p.W[(size_t)col * p.dw + e] : 0.f;
        }
        if (tid < 32) mbuf[buf][tid] = p.mw[c * 32 + tid];
    };
    ChunkStage<NU> st;
    st.load(p.B + (size_t)c0 * NU, tid);
    st.store(zbuf[0], tid);
    load_w(0, c0);
    __syncthreads();

    typename C::A a[RW];
    f32x16_t tacc[RW][ES];
    float r[RW], rm[RW];
    bool act[RW];
    int rchunk0 = 0;
    const int total = p.rg * nch;
    for (int it = 0; it < total; ++it) {
        const int g = it / nch, cc = it - g * nch;
        if (cc == 0) {
            rchunk0 = (rb * p.rg + g) * (WAVES * RW) + wave * RW;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                act[t] = rchunk0 + t < p.n_chunks_r;
                if (act[t]) C::load(a[t], p.A, rchunk0 + t, lane);
#pragma unroll
                for (int es = 0; es < ES; ++es) tacc[t][es] = (f32x16_t)0.0f;
                r[t] = 0.f;
                rm[t] = 0.f;
            }
        }
        const bool has_next = it + 1 < total;
        const int cn = c0 + (it + 1) % nch;
        if (has_next) st.load(p.B + (size_t)cn * NU, tid);
        const uint4* zb = zbuf[it & 1];
        const float* wb = wbuf[it & 1];
        const float* mb = mbuf[it & 1];
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            if (act[t]) {
                f32x16_t s = C::tileT(a[t], zb, lane);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const float pq = fast_exp2(s[q]);
                    const int jr = acc_row(q, lane);
                    r[t] += pq;
                    rm[t] = fmaf(pq, mb[jr], rm[t]);
#pragma unroll
                    for (int es = 0; es < ES; ++es)
                        tacc[t][es] = __builtin_amdgcn_mfma_f32_32x32x2f32(wb[jr * WS + es * 32 + (lane & 31)], pq,
                                                                           tacc[t][es], 0, 0, 0);
                }
            }
        }
        if (cc == nch - 1) {
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (act[t]) {
                    const float rt = r[t] + shfl_xor_f(r[t], 32);
                    const float rmt = rm[t] + shfl_xor_f(rm[t], 32);
                    const int row = (rchunk0 + t) * 32 + (lane & 31);
                    if (lane < 32) {
                        p.rp[(size_t)cb * p.n_pad + row] = rt;
                        p.rmp[(size_t)cb * p.n_pad + row] = rmt;
                    }
                    float* dst = p.Tp + ((size_t)cb * p.n_pad + row) * p.tw;
#pragma unroll
                    for (int es = 0; es < ES; ++es)
#pragma unroll
                        for (int q = 0; q < 16; ++q) dst[es * 32 + acc_row(q, lane)] = tacc[t][es][q];
                }
            }
        }
        if (has_next) {
            st.store(zbuf[(it + 1) & 1], tid);
            load_w((it + 1) & 1, cn);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Covariance of the BF16 precision form: pi and the payload W split into BF16
// (hi, lo) pairs, T accumulated from hi*hi + hi*lo + lo*hi on BF16 MFMA with
// FP32 accumulators (relative error of each product ~2^-17 instead of the
// 2^-9 of plain BF16; the lo*lo term, ~2^-18, is dropped).
//
// The exponent tile in transposed form leaves lane l with pi[i = l%32][j]
// for j = acc_row(q, l), q = 0..15.  Taking q = 8 kb + e (e = 0..7) as the
// k slots of block kb makes those eight values the lane's A fragment as they
// are, provided the payload is packed with the same j order:
//   slot (kb, h = l/32, e) <-> j = 16 kb + (e < 4 ? 4h + e : 4 + 4h + e).
// Payload pack: [chunk of 32 j][es][kb][hi, lo][lane 64][8 bf16], lane l
// holding W[32 chunk + j(kb, l/32, e)][32 es + l%32] (zero outside).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int pw_j(int kb, int h, int e) { return 16 * kb + (e < 4 ? 4 * h + e : 4 + 4 * h + e); }

__global__ void __launch_bounds__(256) k_pack_payload(const float* W, int64_t m, int dw, int es_n, int64_t n_chunks,
                                                     uint16_t* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_chunks * es_n * 2 * 64) return;
    const int lane = (int)(t & 63);
    int64_t r = t >> 6;
    const int kb = (int)(r & 1);
    r >>= 1;
    const int es = (int)(r % es_n);
    const int64_t c = r / es_n;
    const int h = lane >> 5, col = es * 32 + (lane & 31);
    uint16_t* base = out + ((((size_t)c * es_n + es) * 2 + kb) * 2) * 64 * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t j = c * 32 + pw_j(kb, h, e);
        const float v = (j < m && col < dw) ? W[j * dw + col] : 0.f;
        const uint16_t hi = f32_to_bf16_bits(v);
        base[lane * 8 + e] = hi;
        base[64 * 8 + lane * 8 + e] = f32_to_bf16_bits(v - bf16_bits_to_f32(hi));
    }
}

size_t payload_pack_bytes(int64_t rows_pad, int dw) {
    const int es_n = cov_tw(0, dw) / 32;
    return (size_t)(rows_pad / 32) * es_n * 2 * 2 * 64 * 16;
}

hipError_t launch_pack_payload(const float* W, int64_t m, int64_t m_pad, int dw, void* out, hipStream_t stream) {
    const int es_n = cov_tw(0, dw) / 32;
    const int64_t n_chunks = m_pad / 32;
    const int64_t total = n_chunks * es_n * 2 * 64;
    hipLaunchKernelGGL(k_pack_payload, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, W, m, dw, es_n,
                       n_chunks, (uint16_t*)out);
    return hipGetLastError();
}

template <int KS, int RW, int ES>
__global__ void __launch_bounds__(THREADS) k_cov_bf16(CovArgs p) {
    using C = CoreBF16<KS>;
    constexpr int NU = KS * 64;
    constexpr int NW = ES * 2 * 2 * 64;
    __shared__ uint4 zbuf[2][NU];
    __shared__ uint4 wbuf[2][NW];
    __shared__ float mbuf[2][32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int rb, cb;
    tile_coords(blockIdx.x, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);

    ChunkStage<NU> st;
    ChunkStage<NW> sw;
    float mnext = 0.f;
    st.load(p.B + (size_t)c0 * NU, tid);
    sw.load(p.PW + (size_t)c0 * NW, tid);
    if (tid < 32) mnext = p.mw[c0 * 32 + tid];
    st.store(zbuf[0], tid);
    sw.store(wbuf[0], tid);
    if (tid < 32) mbuf[0][tid] = mnext;
    __syncthreads();

    typename C::A a[RW];
    f32x16_t tacc[RW][ES];
    float r[RW], rm[RW];
    bool act[RW];
    int rchunk0 = 0;
    const int total = p.rg * nch;
    for (int it = 0; it < total; ++it) {
        const int g = it / nch, cc = it - g * nch;
        if (cc == 0) {
            rchunk0 = (rb * p.rg + g) * (WAVES * RW) + wave * RW;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                act[t] = rchunk0 + t < p.n_chunks_r;
                if (act[t]) C::load(a[t], p.A, rchunk0 + t, lane);
#pragma unroll
                for (int es = 0; es < ES; ++es) tacc[t][es] = (f32x16_t)0.0f;
                r[t] = 0.f;
                rm[t] = 0.f;
            }
            wait_vmem_all();
        }
        const bool has_next = it + 1 < total;
        const int cn = c0 + (it + 1) % nch;
        if (has_next) {
            st.load(p.B + (size_t)cn * NU, tid);
            sw.load(p.PW + (size_t)cn * NW, tid);
            if (tid < 32) mnext = p.mw[cn * 32 + tid];
        }
        const uint4* zb = zbuf[it & 1];
        const uint4* wb = wbuf[it & 1];
        const float* mb = mbuf[it & 1];
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            if (act[t]) {
                const f32x16_t s = C::tileT(a[t], zb, lane);
                bf16x8_t ah[2], al[2];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const float pq = fast_exp2(s[q]);
                    r[t] += pq;
                    rm[t] = fmaf(pq, mb[acc_row(q, lane)], rm[t]);
                    const __bf16 h = (__bf16)pq;
                    ah[q >> 3][q & 7] = h;
                    al[q >> 3][q & 7] = (__bf16)(pq - (float)h);
                }
#pragma unroll
                for (int es = 0; es < ES; ++es)
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb) {
                        const bf16x8_t bh = __builtin_bit_cast(bf16x8_t, wb[((es * 2 + kb) * 2 + 0) * 64 + lane]);
                        const bf16x8_t bl = __builtin_bit_cast(bf16x8_t, wb[((es * 2 + kb) * 2 + 1) * 64 + lane]);
                        tacc[t][es] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kb], bh, tacc[t][es], 0, 0, 0);
                        tacc[t][es] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kb], bl, tacc[t][es], 0, 0, 0);
                        tacc[t][es] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[kb], bh, tacc[t][es], 0, 0, 0);
                    }
            }
        }
        if (cc == nch - 1) {
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (act[t]) {
                    const float rt = r[t] + shfl_xor_f(r[t], 32);
                    const float rmt = rm[t] + shfl_xor_f(rm[t], 32);
                    const int row = (rchunk0 + t) * 32 + (lane & 31);
                    if (lane < 32) {
                        p.rp[(size_t)cb * p.n_pad + row] = rt;
                        p.rmp[(size_t)cb * p.n_pad + row] = rmt;
                    }
                    // lane = payload column, q = row acc_row(q, lane)
#pragma unroll
                    for (int es = 0; es < ES; ++es)
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const size_t rr = (size_t)cb * p.n_pad + (size_t)(rchunk0 + t) * 32 + acc_row(q, lane);
                            p.Tp[rr * p.tw + es * 32 + (lane & 31)] = tacc[t][es][q];
                        }
                }
            }
        }
        if (has_next) {
            st.store(zbuf[(it + 1) & 1], tid);
            sw.store(wbuf[(it + 1) & 1], tid);
            if (tid < 32) mbuf[(it + 1) & 1][tid] = mnext;
        }
        __syncthreads();
    }
}

// VALU covariance for D < 16 in the direct exponent form of the VALU pass:
// lane = row, column records [Z (D), Vh, m/2, Vl, W (dw)] in LDS; the column
// norm m_j doubles as the weight of rm_i.
constexpr int CRV = 2;                      // rows per lane
constexpr int COV_VALU_ROWS = WAVES * 64 * CRV;
constexpr int MAX_VALU_W = 16;

struct CovValuArgs {
    const float* X;
    const float* xn;
    const float* U;
    const float* Ul;
    const float* Z;
    const float* mm;
    const float* V;
    const float* Vl;
    const float* W;
    float kappa;
    int dw;
    float* Tp;
    float* rp;
    float* rmp;
    int tw;
    int n_pad, m_pad, n_chunks_c, rg, bc_chunks, n_mt_r, n_mt_c;
};

template <int D>
__global__ void __launch_bounds__(THREADS) k_cov_valu(CovValuArgs p) {
    const int R = D + 3 + p.dw;
    extern __shared__ float zc[];  // [2][32 * R]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int rb, cb;
    tile_coords(blockIdx.x, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);
    auto load = [&](int buf, int c) {
        float* dst = zc + buf * 32 * R;
        for (int u = tid; u < 32 * R; u += THREADS) {
            const int j = u / R, k = u - j * R;
            const int col = c * 32 + j;
            float v;
            if (k < D) v = p.Z[(size_t)col * D + k];
            else if (k == D) v = p.V[col];
            else if (k == D + 1) v = 0.5f * p.mm[col];
            else if (k == D + 2) v = p.Vl[col];
            else v = p.W[(size_t)col * p.dw + (k - D - 3)];
            dst[u] = v;
        }
    };
    load(0, c0);
    __syncthreads();
    float xr[CRV][D], ur[CRV], ulr[CRV], nr[CRV], r[CRV], rm[CRV], T[CRV][MAX_VALU_W];
    int row0 = 0;
    const int total = p.rg * nch;
    for (int it = 0; it < total; ++it) {
        const int g = it / nch, cc = it - g * nch;
        if (cc == 0) {
            row0 = (rb * p.rg + g) * COV_VALU_ROWS + wave * 64 * CRV;
#pragma unroll
            for (int k = 0; k < CRV; ++k) {
                const int row = row0 + k * 64 + lane;
                const bool ok = row < p.n_pad;
#pragma unroll
                for (int d = 0; d < D; ++d) xr[k][d] = ok ? p.X[(size_t)row * D + d] : 0.f;
                ur[k] = ok ? p.U[row] : -INFINITY;
                ulr[k] = ok ? p.Ul[row] : 0.f;
                nr[k] = ok ? 0.5f * p.xn[row] : 0.f;
                r[k] = 0.f;
                rm[k] = 0.f;
#pragma unroll
                for (int e = 0; e < MAX_VALU_W; ++e) T[k][e] = 0.f;
            }
        }
        const float* zb = zc + (it & 1) * 32 * R;
        for (int j = 0; j < 32; ++j) {
            const float* zr = zb + j * R;
#pragma unroll
            for (int k = 0; k < CRV; ++k) {
                const float dl = nr[k] - zr[D + 1];
                float dist = dl * dl;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const float df = xr[k][d] - zr[d];
                    dist = fmaf(df, df, dist);
                }
                const float e = fast_exp2(assemble_exponent(ur[k], ulr[k], zr[D], zr[D + 2], p.kappa * dist));
                r[k] += e;
                rm[k] = fmaf(e, 2.f * zr[D + 1], rm[k]);
#pragma unroll
                for (int w = 0; w < MAX_VALU_W; ++w)
                    if (w < p.dw) T[k][w] = fmaf(e, zr[D + 3 + w], T[k][w]);
            }
        }
        if (cc == nch - 1) {
#pragma unroll
            for (int k = 0; k < CRV; ++k) {
                const int row = row0 + k * 64 + lane;
                if (row < p.n_pad) {
                    p.rp[(size_t)cb * p.n_pad + row] = r[k];
                    p.rmp[(size_t)cb * p.n_pad + row] = rm[k];
                    float* dst = p.Tp + ((size_t)cb * p.n_pad + row) * p.tw;
                    for (int w = 0; w < p.dw; ++w) dst[w] = T[k][w];
                }
            }
        }
        if (it + 1 < total) load((it + 1) & 1, c0 + (it + 1) % nch);
        __syncthreads();
    }
}

// payload width of the MFMA covariance, in 32-column groups the kernel is
// instantiated for (1, 2, 3, 4, 6, 8); padded columns carry zeros
int cov_tw(int path, int dw) {
    if (path == 1) return dw;
    int es = (dw + 31) / 32;
    if (es == 5) es = 6;
    if (es == 7) es = 8;
    return es * 32;
}

bool cov_bf16_form(int path, int prec, int d, int dw) {
    return path == 0 && prec == PREC_BF16 && pack_units(prec, d) <= 9 && cov_tw(0, dw) / 32 <= 4;
}

// row tiles per wave of the covariance kernels (register budget)
static int cov_rw(int path, int prec, int d, int dw) {
    const int units = pack_units(prec, d), es = cov_tw(path, dw) / 32;
    if (cov_bf16_form(path, prec, d, dw)) return (units <= 5 && es <= 2) ? 2 : 1;
    return (units <= 9 && es <= 4) ? 2 : 1;
}

int cov_rows_per_group(int path, int prec, int d, int dw) {
    if (path == 1) return COV_VALU_ROWS;
    return WAVES * cov_rw(path, prec, d, dw) * 32;
}

template <int KS, int RW, int ES>
static hipError_t launch_bf16_cov(const CovArgs& a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((k_cov_bf16<KS, RW, ES>), dim3(grid), dim3(THREADS), 0, stream, a);
    return hipGetLastError();
}

template <int KS>
static hipError_t launch_bf16_cov_es(const CovArgs& a, int es, int rw, int grid, hipStream_t stream) {
    if constexpr (KS <= 5) {
        if (rw == 2) {
            if (es == 1) return launch_bf16_cov<KS, 2, 1>(a, grid, stream);
            if (es == 2) return launch_bf16_cov<KS, 2, 2>(a, grid, stream);
            return hipErrorInvalidValue;
        }
    }
    switch (es) {
        case 1: return launch_bf16_cov<KS, 1, 1>(a, grid, stream);
        case 2: return launch_bf16_cov<KS, 1, 2>(a, grid, stream);
        case 3: return launch_bf16_cov<KS, 1, 3>(a, grid, stream);
        case 4: return launch_bf16_cov<KS, 1, 4>(a, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

template <class C, int RW>
static hipError_t launch_cov_mfma_es(const CovArgs& a, int es, int grid, hipStream_t stream) {
    switch (es) {
        case 1: hipLaunchKernelGGL((k_cov_mfma<C, RW, 1>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        case 2: hipLaunchKernelGGL((k_cov_mfma<C, RW, 2>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        case 3: hipLaunchKernelGGL((k_cov_mfma<C, RW, 3>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        case 4: hipLaunchKernelGGL((k_cov_mfma<C, RW, 4>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        case 6: hipLaunchKernelGGL((k_cov_mfma<C, 1, 6>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        case 8: hipLaunchKernelGGL((k_cov_mfma<C, 1, 8>), dim3(grid), dim3(THREADS), 0, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cov(int path, int prec, int d, const void* A, const void* B, const void* PW, const float* X,
                      const float* xn, const float* U, const float* Ul, const float* Zs, const float* ms,
                      const float* V, const float* Vl, float kappa, const float* W, const float* mw, int dw,
                      int64_t n_pad, int64_t m_pad, int rg, int bc_chunks, int n_mt_r, int n_mt_c,
                      const CovOut& out, hipStream_t stream) {
    const int grid = n_mt_r * n_mt_c;
    if (path == 1) {
        if (dw > MAX_VALU_W) return hipErrorInvalidValue;
        CovValuArgs a;
        a.X = X;
        a.xn = xn;
        a.U = U;
        a.Ul = Ul;
        a.Z = Zs;
        a.mm = ms;
        a.V = V;
        a.Vl = Vl;
        a.W = W;
        a.kappa = kappa;
        a.dw = dw;
        a.Tp = out.Tp;
        a.rp = out.rp;
        a.rmp = out.rmp;
        a.tw = out.tw;
        a.n_pad = (int)n_pad;
        a.m_pad = (int)m_pad;
        a.n_chunks_c = (int)(m_pad / 32);
        a.rg = rg;
        a.bc_chunks = bc_chunks;
        a.n_mt_r = n_mt_r;
        a.n_mt_c = n_mt_c;
        const size_t lds = 2 * 32 * (size_t)(d + 3 + dw) * sizeof(float);
        switch (d) {
#define GW_COV_CASE(DD)                                                                             \
    case DD:                                                                                        \
        hipLaunchKernelGGL((k_cov_valu<DD>), dim3(grid), dim3(THREADS), lds, stream, a); \
        break;
            GW_COV_CASE(1) GW_COV_CASE(2) GW_COV_CASE(3) GW_COV_CASE(4) GW_COV_CASE(5)
            GW_COV_CASE(6) GW_COV_CASE(7) GW_COV_CASE(8) GW_COV_CASE(9) GW_COV_CASE(10)
            GW_COV_CASE(11) GW_COV_CASE(12) GW_COV_CASE(13) GW_COV_CASE(14) GW_COV_CASE(15)
#undef GW_COV_CASE
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    CovArgs a;
    a.A = (const uint4*)A;
    a.B = (const uint4*)B;
    a.PW = (const uint4*)PW;
    a.W = W;
    a.mw = mw;
    a.dw = dw;
    a.Tp = out.Tp;
    a.rp = out.rp;
    a.rmp = out.rmp;
    a.tw = out.tw;
    a.n_chunks_r = (int)(n_pad / 32);
    a.n_chunks_c = (int)(m_pad / 32);
    a.rg = rg;
    a.bc_chunks = bc_chunks;
    a.n_mt_r = n_mt_r;
    a.n_mt_c = n_mt_c;
    a.n_pad = (int)n_pad;
    a.m_pad = (int)m_pad;
    const int es = out.tw / 32;
    const int units = pack_units(prec, d);
    if (cov_bf16_form(path, prec, d, dw)) {
        if (!PW) return hipErrorInvalidValue;
        const int rw = cov_rw(path, prec, d, dw);
        switch (units) {
            case 2: return launch_bf16_cov_es<2>(a, es, rw, grid, stream);
            case 3: return launch_bf16_cov_es<3>(a, es, rw, grid, stream);
            case 4: return launch_bf16_cov_es<4>(a, es, rw, grid, stream);
            case 5: return launch_bf16_cov_es<5>(a, es, rw, grid, stream);
            case 7: return launch_bf16_cov_es<7>(a, es, rw, grid, stream);
            case 9: return launch_bf16_cov_es<9>(a, es, rw, grid, stream);
            default: return hipErrorInvalidValue;
        }
    }
    if (prec == PREC_F32) {
        switch (units) {
            case 3: return launch_cov_mfma_es<CoreF32<3>, 2>(a, es, grid, stream);
            case 5: return launch_cov_mfma_es<CoreF32<5>, 2>(a, es, grid, stream);
            case 7: return launch_cov_mfma_es<CoreF32<7>, 2>(a, es, grid, stream);
            case 9: return launch_cov_mfma_es<CoreF32<9>, 2>(a, es, grid, stream);
            case 13: return launch_cov_mfma_es<CoreF32<13>, 1>(a, es, grid, stream);
            case 17: return launch_cov_mfma_es<CoreF32<17>, 1>(a, es, grid, stream);
            case 25: return launch_cov_mfma_es<CoreF32<25>, 1>(a, es, grid, stream);
            case 33: return launch_cov_mfma_es<CoreF32<33>, 1>(a, es, grid, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (units) {
        case 2: return launch_cov_mfma_es<CoreBF16<2>, 2>(a, es, grid, stream);
        case 3: return launch_cov_mfma_es<CoreBF16<3>, 2>(a, es, grid, stream);
        case 4: return launch_cov_mfma_es<CoreBF16<4>, 2>(a, es, grid, stream);
        case 5: return launch_cov_mfma_es<CoreBF16<5>, 2>(a, es, grid, stream);
        case 7: return launch_cov_mfma_es<CoreBF16<7>, 2>(a, es, grid, stream);
        case 9: return launch_cov_mfma_es<CoreBF16<9>, 2>(a, es, grid, stream);
        case 10: return launch_cov_mfma_es<CoreBF16<10>, 1>(a, es, grid, stream);
        case 13: return launch_cov_mfma_es<CoreBF16<13>, 1>(a, es, grid, stream);
        case 17: return launch_cov_mfma_es<CoreBF16<17>, 1>(a, es, grid, stream);
        case 19: return launch_cov_mfma_es<CoreBF16<19>, 1>(a, es, grid, stream);
        case 25: return launch_cov_mfma_es<CoreBF16<25>, 1>(a, es, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Reduction of the covariance partials (fixed order) and Gamma in FP64.
// ---------------------------------------------------------------------------

// Rows per reduction block: the block keeps its rows' T_i in LDS as FP64,
// 64 rows up to 64 columns (33 KB), fewer for wider payloads.
__host__ __device__ inline int red_rows(int dw) { return dw <= 64 ? 64 : (dw <= 128 ? 32 : 16); }

// Partials of every column tile summed in FP64 (T_i, r_i, rm_i), then the
// block's share of Gamma = sum_i X_i T_i^T in FP64 from those FP64 sums.
__global__ void __launch_bounds__(256) k_cov_reduce(const float* Tp, const float* rp, const float* rmp, int n_mt_c,
                                                    int tw, int64_t n, int64_t n_pad, const float* Xs, int dx,
                                                    const float* xs_norm, int dw, float* T, float* r, float* rm,
                                                    double* part) {
    extern __shared__ double tsh[];  // rows x (dw + 1)
    __shared__ double sred[256];
    const int rows = red_rows(dw);
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    double acc_r = 0.0, acc_nm = 0.0;
    for (int u = threadIdx.x; u < rows * dw; u += blockDim.x) {
        const int li = u / dw, e = u - li * dw;
        const int64_t i = r0 + li;
        double s = 0.0;
        if (i < n)
            for (int c = 0; c < n_mt_c; ++c) s += (double)Tp[((size_t)c * n_pad + i) * tw + e];
        tsh[li * (dw + 1) + e] = s;
        if (T && i < n) T[i * dw + e] = (float)s;
    }
    if (threadIdx.x < rows) {
        const int64_t i = r0 + threadIdx.x;
        if (i < n) {
            double sr = 0.0, sm = 0.0;
            for (int c = 0; c < n_mt_c; ++c) {
                sr += (double)rp[(size_t)c * n_pad + i];
                sm += (double)rmp[(size_t)c * n_pad + i];
            }
            if (r) r[i] = (float)sr;
            if (rm) rm[i] = (float)sm;
            acc_r = sr;
            acc_nm = sm * (double)xs_norm[i];
        }
    }
    __syncthreads();
    const int width = dx * dw;
    double* out = part + (size_t)blockIdx.x * (width + 2);
    for (int pidx = threadIdx.x; pidx < width; pidx += blockDim.x) {
        const int dd = pidx / dw, e = pidx - dd * dw;
        double s = 0.0;
        for (int li = 0; li < rows; ++li) {
            const int64_t i = r0 + li;
            if (i >= n) break;
            s += (double)Xs[i * dx + dd] * tsh[li * (dw + 1) + e];
        }
        out[pidx] = s;
    }
    // fixed-order block sums of the two scalars
    sred[threadIdx.x] = acc_r;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sred[threadIdx.x] += sred[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[width] = sred[0];
    __syncthreads();
    sred[threadIdx.x] = acc_nm;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sred[threadIdx.x] += sred[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[width + 1] = sred[0];
}

size_t cov_reduce_part_doubles(int64_t n, int dx, int dw) {
    const int rows = red_rows(dw);
    return (size_t)((n + rows - 1) / rows) * (dx * dw + 2);
}

hipError_t launch_cov_reduce(const CovOut& in, int n_mt_c, int64_t n, int64_t n_pad, const float* Xs, int dx,
                             const float* xs_norm, int dw, float* T, float* r, float* rm, double* part,
                             hipStream_t stream) {
    const int rows = red_rows(dw);
    const int nblk = (int)((n + rows - 1) / rows);
    const size_t lds = (size_t)rows * (dw + 1) * sizeof(double);
    hipLaunchKernelGGL(k_cov_reduce, dim3(nblk), dim3(256), lds, stream, in.Tp, in.rp, in.rmp, n_mt_c, in.tw, n,
                       n_pad, Xs, dx, xs_norm, dw, T, r, rm, part);
    return hipGetLastError();
}

// Sum of the per-block FP64 partials: one thread per output column of the
// partial table, four strided lanes per column combined in a fixed order.
__global__ void __launch_bounds__(256) k_gamma_sum(const double* part, int nblk, int width, double* gamma64,
                                                   float* gamma32, double* scal) {
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, s = threadIdx.x >> 6;
    const int pidx = blockIdx.x * 64 + c;
    double acc = 0.0;
    if (pidx < width + 2)
        for (int b = s; b < nblk; b += 4) acc += part[(size_t)b * (width + 2) + pidx];
    red[s][c] = acc;
    __syncthreads();
    if (s == 0 && pidx < width + 2) {
        const double v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
        if (pidx < width) {
            gamma64[pidx] = v;
            gamma32[pidx] = (float)v;
        } else {
            scal[pidx - width] = v;
        }
    }
}

// ||Gamma||^2 and ||Gamma - Gamma_old||^2 in one block, fixed order.
__global__ void __launch_bounds__(256) k_gamma_norms(const double* gamma64, const float* gamma_old, int width,
                                                     double* scal) {
    __shared__ double s1[256], s2[256];
    double a1 = 0.0, a2 = 0.0;
    for (int p = threadIdx.x; p < width; p += blockDim.x) {
        const double v = gamma64[p], d = v - (double)gamma_old[p];
        a1 += v * v;
        a2 += d * d;
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s1[threadIdx.x] += s1[threadIdx.x + st];
            s2[threadIdx.x] += s2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[2] = s1[0];
        scal[3] = s2[0];
    }
}

hipError_t launch_gamma_final(const double* part, int64_t n, int dx, int dw, const float* gamma_old, double* gamma64,
                              float* gamma32, double* scal, hipStream_t stream) {
    const int rows = red_rows(dw);
    const int nblk = (int)((n + rows - 1) / rows);
    const int width = dx * dw;
    hipLaunchKernelGGL(k_gamma_sum, dim3((width + 2 + 63) / 64), dim3(256), 0, stream, part, nblk, width, gamma64,
                       gamma32, scal);
    // gamma_old must not alias gamma32 (the caller double-buffers Gamma)
    hipLaunchKernelGGL(k_gamma_norms, dim3(1), dim3(256), 0, stream, gamma64, gamma_old, width, scal);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 check: s_ij = sum_k A_ik B_jk evaluated exactly in FP64 from the
// packed operands (the coupling the passes iterate), pi = 2^s.  One sweep
// over the entries gives the row sums, the row KL terms and the column sums:
// each work-group takes a span x span macro tile and writes per-tile
// partials, which a second kernel adds up in tile order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float pack_elem(const void* pack, int prec, int units, int row, int k) {
    if (prec == PREC_F32) return ((const float*)pack)[f32_pack_off(row, k, units)];
    return bf16_bits_to_f32(((const uint16_t*)pack)[bf16_pack_off(row, k, units)]);
}

// 64 x 64 sub-tiles of (row, column) entries; K consumed in blocks of 40
// (K = 80 at D = 64 in two) decoded to float in LDS; each thread owns a
// 4 x 4 block of entries (rows 4 ty + u, columns 4 tx + v).  The reduction
// scratch reuses the operand tiles' LDS.
constexpr int CK_T = 64, CK_KB = 40, CKM = 2048;
static_assert(CK_KB % 8 == 0, "K blocks hold whole 8-k groups");

// Eight consecutive k (k0 a multiple of 8) of one packed row as floats, the
// values pack_elem gives: one 16-byte unit of a BF16 pack, or the two units
// (lanes r and r + 32) of an FP32 pack that hold the even and odd k.  Every
// pack's K is a multiple of 8, so a group is either whole or past K.
__device__ __forceinline__ void pack_group8(const void* pack, int prec, int units, int row, int k0, float* v) {
    if (prec == PREC_F32) {
        const float4 ev = *reinterpret_cast<const float4*>((const float*)pack + f32_pack_off(row, k0, units));
        const float4 od = *reinterpret_cast<const float4*>((const float*)pack + f32_pack_off(row, k0 + 1, units));
        v[0] = ev.x; v[1] = od.x; v[2] = ev.y; v[3] = od.y;
        v[4] = ev.z; v[5] = od.z; v[6] = ev.w; v[7] = od.w;
        return;
    }
    const uint4 u = *reinterpret_cast<const uint4*>((const uint16_t*)pack + bf16_pack_off(row, k0, units));
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v[2 * t] = bf16_bits_to_f32((uint16_t)(w[t] & 0xffffu));
        v[2 * t + 1] = bf16_bits_to_f32((uint16_t)(w[t] >> 16));
    }
}

// The macro tile's side: CKM, halved (down to one 64 x 64 sub-tile) while the
// grid would have fewer than 512 work-groups, so that problems of a few
// thousand points still spread over the CUs (the partials grow as the tile
// shrinks, so large problems keep the full tile).
int check_span(int64_t n, int64_t m) {
    int s = CKM;
    while (s > CK_T && ((n + s - 1) / s) * ((m + s - 1) / s) < 512) s >>= 1;
    return s;
}

__global__ void __launch_bounds__(256) k_check64_tiles(int prec, int units, int K, const void* A, const void* B,
                                                       int64_t n, int64_t m, int span, const float* la2,
                                                       const float* lb2, double* rpart, double* klpart,
                                                       double* cpart) {
    constexpr int TILE_FLOATS = CK_T * (CK_KB + 1);
    static_assert(2 * TILE_FLOATS * sizeof(float) >= 2 * 16 * CK_T * sizeof(double), "row scratch fits");
    static_assert(TILE_FLOATS * sizeof(float) >= 16 * CK_T * sizeof(double), "column scratch fits");
    __shared__ double tiles_mem[(2 * TILE_FLOATS + 1) / 2];
    __shared__ float lbs[CK_T];
    __shared__ double colacc[CKM];
    float(*As)[CK_KB + 1] = reinterpret_cast<float(*)[CK_KB + 1]>(tiles_mem);
    float(*Bs)[CK_KB + 1] = reinterpret_cast<float(*)[CK_KB + 1]>(reinterpret_cast<float*>(tiles_mem) + TILE_FLOATS);
    // reduction scratch over the operand tiles (used only between K loops)
    double(*redc)[CK_T] = reinterpret_cast<double(*)[CK_T]>(tiles_mem);
    double(*redr)[16][CK_T] = reinterpret_cast<double(*)[16][CK_T]>(tiles_mem);
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int rt = blockIdx.y, ct = blockIdx.x;
    const int64_t R0 = (int64_t)rt * span, C0 = (int64_t)ct * span;
    const int n_sub = span / CK_T;
    for (int j = tid; j < span; j += 256) colacc[j] = 0.0;
    for (int rs = 0; rs < n_sub && R0 + rs * CK_T < n; ++rs) {
        const int64_t r0 = R0 + rs * CK_T;
        double rsum[4] = {0, 0, 0, 0}, rkl[4] = {0, 0, 0, 0}, la[4];
        bool rin[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = r0 + ty * 4 + u;
            rin[u] = i < n;
            la[u] = rin[u] ? (double)la2[i] : 0.0;
        }
        for (int cs = 0; cs < n_sub && C0 + cs * CK_T < m; ++cs) {
            const int64_t c0 = C0 + cs * CK_T;
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
            for (int k0 = 0; k0 < K; k0 += CK_KB) {
                __syncthreads();
                // one thread per (row, 8-k group) of each operand
                for (int e = tid; e < 2 * CK_T * (CK_KB / 8); e += 256) {
                    const int op = e / (CK_T * (CK_KB / 8)), f = e - op * (CK_T * (CK_KB / 8));
                    const int rr = f / (CK_KB / 8), q = f - rr * (CK_KB / 8);
                    const int64_t row = (op ? c0 : r0) + rr;
                    const int k = k0 + 8 * q;
                    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (row < (op ? m : n) && k < K) pack_group8(op ? B : A, prec, units, (int)row, k, v);
                    float* dst = op ? &Bs[rr][8 * q] : &As[rr][8 * q];
#pragma unroll
                    for (int t = 0; t < 8; ++t) dst[t] = v[t];
                }
                if (tid < CK_T) lbs[tid] = c0 + tid < m ? lb2[c0 + tid] : 0.f;
                __syncthreads();
#pragma unroll 4
                for (int kk = 0; kk < CK_KB; ++kk) {
                    double av[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        av[u] = (double)As[ty * 4 + u][kk];
                        bv[u] = (double)Bs[tx * 4 + u][kk];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
                }
            }
            double csum[4] = {0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (c0 + tx * 4 + v >= m) continue;
                const double lbj = (double)lbs[tx * 4 + v];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!rin[u]) continue;
                    const double pv = exp2(acc[u][v]);
                    rsum[u] += pv;
                    if (pv > 0.0) rkl[u] += pv * (acc[u][v] - la[u] - lbj);
                    csum[v] += pv;
                }
            }
            // column sums of the sub-tile over its 16 row groups, fixed order
            __syncthreads();  // every thread is done reading the operand tiles
#pragma unroll
            for (int v = 0; v < 4; ++v) redc[ty][tx * 4 + v] = csum[v];
            __syncthreads();
            if (tid < CK_T) {
                double q = 0.0;
                for (int t = 0; t < 16; ++t) q += redc[t][tid];
                colacc[cs * CK_T + tid] += q;
            }
        }
        // row sums of the macro tile's columns over the 16 column groups
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            redr[0][tx][ty * 4 + u] = rsum[u];
            redr[1][tx][ty * 4 + u] = rkl[u];
        }
        __syncthreads();
        if (tid < CK_T && r0 + tid < n) {
            double q = 0.0, w = 0.0;
            for (int t = 0; t < 16; ++t) {
                q += redr[0][t][tid];
                w += redr[1][t][tid];
            }
            rpart[(size_t)ct * n + r0 + tid] = q;
            klpart[(size_t)ct * n + r0 + tid] = w;
        }
    }
    __syncthreads();
    for (int j = tid; j < span && C0 + j < m; j += 256) cpart[(size_t)rt * m + C0 + j] = colacc[j];
}

// r64_i = sum over column tiles of the row partials (and kl), c64_j over row
// tiles, in tile order.
__global__ void __launch_bounds__(256) k_check64_reduce(const double* rpart, const double* klpart, const double* cpart,
                                                        int n_ct, int n_rt, int64_t n, int64_t m, double* r64,
                                                        double* kl, double* c64) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        double q = 0.0, w = 0.0;
        for (int c = 0; c < n_ct; ++c) {
            q += rpart[(size_t)c * n + t];
            w += klpart[(size_t)c * n + t];
        }
        r64[t] = q;
        kl[t] = w * 0.6931471805599453;
    } else if (t < n + m) {
        const int64_t j = t - n;
        double q = 0.0;
        for (int r = 0; r < n_rt; ++r) q += cpart[(size_t)r * m + j];
        c64[j] = q;
    }
}

size_t check64_part_doubles(int64_t n, int64_t m) {
    const int64_t s = check_span(n, m);
    return 2 * (size_t)((m + s - 1) / s) * n + (size_t)((n + s - 1) / s) * m;
}

hipError_t launch_check64(int prec, int d, const void* Arows, const void* Bcols, int64_t n, int64_t m,
                          const float* la2, const float* lb2, double* part, double* r64, double* kl, double* c64,
                          hipStream_t stream) {
    const int K = pack_k(prec, d);
    const int units = pack_units(prec, d);
    if (K % 8 != 0) return hipErrorInvalidValue;  // the tiles load whole 8-k groups
    const int span = check_span(n, m);
    const int n_rt = (int)((n + span - 1) / span), n_ct = (int)((m + span - 1) / span);
    double* rpart = part;
    double* klpart = part + (size_t)n_ct * n;
    double* cpart = part + 2 * (size_t)n_ct * n;
    hipLaunchKernelGGL(k_check64_tiles, dim3((unsigned)n_ct, (unsigned)n_rt), dim3(256), 0, stream, prec, units, K,
                       Arows, Bcols, n, m, span, la2, lb2, rpart, klpart, cpart);
    hipLaunchKernelGGL(k_check64_reduce, dim3((unsigned)((n + m + 255) / 256)), dim3(256), 0, stream, rpart, klpart,
                       cpart, n_ct, n_rt, n, m, r64, kl, c64);
    return hipGetLastError();
}

// FP64 check in the direct form of the VALU path.
__global__ void __launch_bounds__(256) k_check64_direct(int d, const float* X, const float* xn, const float* U,
                                                        const float* Ul, const float* Z, const float* zm,
                                                        const float* V, const float* Vl, float kappa, int64_t n,
                                                        int64_t m, const float* la2, const float* lb2, double* rsum,
                                                        double* kl) {
    extern __shared__ float rec[];  // 32 x (d + 4): Z, Vh, m, lb2, Vl
    const int R = d + 4;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < n;
    double xi[16];
    for (int k = 0; k < 16; ++k) xi[k] = (act && k < d) ? (double)X[i * d + k] : 0.0;
    const double ni = act ? (double)xn[i] : 0.0;
    const double ui = act ? join_df(U[i], Ul[i]) : 0.0;
    const double lai = act ? (double)la2[i] : 0.0;
    const double kap = (double)kappa;
    double rs = 0.0, klr = 0.0;
    const int64_t nchunks = (m + 31) / 32;
    for (int64_t c = 0; c < nchunks; ++c) {
        __syncthreads();
        for (int u = threadIdx.x; u < 32 * R; u += blockDim.x) {
            const int j = u / R, k = u - j * R;
            const int64_t col = c * 32 + j;
            float v = 0.f;
            if (col < m) {
                if (k < d) v = Z[col * d + k];
                else if (k == d) v = V[col];
                else if (k == d + 1) v = zm[col];
                else if (k == d + 2) v = lb2 ? lb2[col] : 0.f;
                else v = Vl[col];
            }
            rec[u] = v;
        }
        __syncthreads();
        if (!act) continue;
        for (int j = 0; j < 32 && c * 32 + j < m; ++j) {
            const float* zr = rec + j * R;
            double dist = 0.0;
            for (int k = 0; k < d; ++k) {
                const double df = xi[k] - (double)zr[k];
                dist += df * df;
            }
            const double dl = 0.5 * (ni - (double)zr[d + 1]);
            dist += dl * dl;
            const double s = ui + join_df(zr[d], zr[d + 3]) - kap * dist;
            const double p = exp2(s);
            rs += p;
            if (kl && p > 0.0) klr += p * (s - lai - (double)zr[d + 2]);
        }
    }
    if (act) {
        rsum[i] = rs;
        if (kl) kl[i] = klr * 0.6931471805599453;
    }
}

hipError_t launch_check64_direct(int d, const float* X, const float* xn, const float* U, const float* Ul,
                                 const float* Z, const float* zm, const float* V, const float* Vl, float kappa,
                                 int64_t n, int64_t m, const float* la2, const float* lb2, double* rsum, double* kl,
                                 hipStream_t stream) {
    const size_t lds = (size_t)32 * (d + 4) * sizeof(float);
    hipLaunchKernelGGL(k_check64_direct, dim3((unsigned)((n + 255) / 256)), dim3(256), lds, stream, d, X, xn, U, Ul,
                       Z, zm, V, Vl, kappa, n, m, la2, lb2, rsum, kl);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_check_final(const double* r64, const double* kl, int64_t n, const float* a,
                                                     const double* c64, int64_t m, const float* b, double asum,
                                                     double bsum, double* scal) {
    __shared__ double s1[256], s2[256], s3[256];
    double e = 0.0, k = 0.0, t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        e += fabs(r64[i] - (double)a[i] / asum);
        k += kl[i];
        t += r64[i];
    }
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) e += fabs(c64[j] - (double)b[j] / bsum);
    s1[threadIdx.x] = e;
    s2[threadIdx.x] = k;
    s3[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s1[threadIdx.x] += s1[threadIdx.x + st];
            s2[threadIdx.x] += s2[threadIdx.x + st];
            s3[threadIdx.x] += s3[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[4] = s1[0];
        scal[5] = s2[0];
        scal[6] = s3[0];
    }
}

hipError_t launch_check_final(const double* r64, const double* kl, int64_t n, const float* a, const double* c64,
                              int64_t m, const float* b, double asum, double bsum, double* scal, hipStream_t stream) {
    hipLaunchKernelGGL(k_check_final, dim3(1), dim3(256), 0, stream, r64, kl, n, a, c64, m, b, asum, bsum, scal);
    return hipGetLastError();
}

}  // namespace gwk
