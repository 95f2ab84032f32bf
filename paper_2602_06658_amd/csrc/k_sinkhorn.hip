// Log-domain Sinkhorn pass over the implicit N x M coupling of Algorithm 1
// (Section 5) and the deterministic combine of its partial sums.
//
// Exponent of one entry, in log2 units (the bilinear form of Remark C.2 at
// temperature eps/8, Alg. 1's squared-norm cost expanded):
//   s_ij = U_i + V_j + X_i . Zs_j + n_i ms_j,      pi_ij = 2^{s_ij}
// with U_i = log2 a_i + k (f_i - alpha_i), V_j = log2 b_j + k (g_j - beta_j),
// Zs_j = 2 k Gamma Y_j, ms_j = k |Y_j|^2 / 2, n_i = |X_i|^2, k = log2(e) 8/eps.
// One pass produces per-macro-tile partial row sums r_i = sum_j pi_ij and
// column sums c_j = sum_i pi_ij from the same s_ij, which is what one
// symmetric iteration (Algorithm 3) needs: f <- f - (eps/16) ln(r_i / a_i),
// g <- g - (eps/16) ln(c_j / b_j).
//
// Two forms: stabilised (one 2^x per entry feeds both sums; valid while the
// marginals stay within 2^+-40 of the weights) and safe (two phases over the
// macro tile: maxima, then max-shifted sums; (max, sum) partials).
#include "gw_device.h"
#include "gw_kernels.h"
#include "gw_cores.h"

using namespace gwl;

namespace gwk {

// ---------------------------------------------------------------------------
// Pass arguments
// ---------------------------------------------------------------------------

struct PassArgs {
    const uint4* A;
    const uint4* B;
    float* rp;
    float* rp2;
    float* cp;
    float* cp2;
    const int* ctl;
    int run_if;
    int token;
    int n_chunks_r, n_chunks_c;
    int rg, bc_chunks;
    int n_mt_r, n_mt_c;
    int n_pad, m_pad;
};


// ---------------------------------------------------------------------------
// Stabilised MFMA pass
// ---------------------------------------------------------------------------

// Column partials (the per-wave accumulators summed in wave order) and the
// macro tile's row partials from LDS to the partial buffers.
template <int RW>
__device__ __forceinline__ void pass_stab_store(const PassArgs& p, const float* dyn, int rb, int cb, int c0,
                                                int nch) {
    const int tid = threadIdx.x, bcw = p.bc_chunks * 32;
    const float* rowacc = dyn + WAVES * bcw;
    for (int i = tid; i < nch * 32; i += THREADS) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) s += dyn[w * bcw + i];
        p.cp[(size_t)rb * p.m_pad + c0 * 32 + i] = s;
    }
    const int rows = p.rg * WAVES * RW * 32;
    const int row0 = rb * rows;
    const int nrows = min(rows, p.n_chunks_r * 32 - row0);
    for (int i = tid; i < nrows; i += THREADS) p.rp[(size_t)cb * p.n_pad + row0 + i] = rowacc[i];
}

// One exponent tile set of a stabilised step: 2^s for the wave's RW row
// tiles against one column chunk, accumulated into the row sums (racc) and
// returned summed over the chunk's rows (lanes l and l + 32 hold column l).
template <class C, int RW>
__device__ __forceinline__ float stab_exp_sums(const f32x16_t (&s)[RW], float (&racc)[RW][16], int nact) {
    float cs = -0.0f;  // exact identity for the first add
#pragma unroll
    for (int t = 0; t < RW; ++t)
        if (t < nact) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float e = fast_exp2(s[t][q]);
                racc[t][q] += e;
                cs += e;
            }
        }
    return cs + shfl_xor_f(cs, 32);
}

// Column chunks of a full macro tile (every row tile in range, even chunk
// count) stream through a 4-slot LDS ring filled by LDS-direct loads: one L2
// read per chunk per work-group, nothing staged in registers.  Chunks go in
// pairs with one barrier per pair, the next pair in flight.  Wave w moves
// slabs w, w + WAVES, ... of each chunk.
constexpr int RING_MAX_UNITS = 9;
template <class C, int RW>
__device__ __forceinline__ void stab_ring_tile(const PassArgs& p, int rb, int c0, int nch, int wave, int lane,
                                               float* colacc, float* rowacc) {
    constexpr int NU = C::UNITS * 64, RING = 4;
    __shared__ uint4 ring[RING * NU];
    auto issue = [&](int k) {
        const uint4* src = p.B + (size_t)(c0 + k % nch) * NU;
        uint4* dst = ring + (k % RING) * NU;
        for (int sl = wave; sl < C::UNITS; sl += WAVES)
            __builtin_amdgcn_global_load_lds(src + sl * 64 + lane,
                                             (__attribute__((address_space(3))) void*)(dst + sl * 64), 16, 0, 0);
    };
    issue(0);
    issue(1);
    typename C::A a[RW];
    float racc[RW][16];
    for (int g = 0; g < p.rg; ++g) {
        const int rchunk0 = (rb * p.rg + g) * (WAVES * RW) + wave * RW;
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            C::load(a[t], p.A, rchunk0 + t, lane);
#pragma unroll
            for (int q = 0; q < 16; ++q) racc[t][q] = 0.f;
        }
        const int k0 = g * nch;
        auto step = [&](int cc) {
            typename C::B b;
            C::load_b(b, ring + ((k0 + cc) % RING) * NU, lane);
            f32x16_t s[RW];
#pragma unroll
            for (int t = 0; t < RW; ++t) s[t] = C::tile_ab(a[t], b);
            const float cs = stab_exp_sums<C, RW>(s, racc, RW);
            if (lane < 32) colacc[cc * 32 + lane] += cs;
        };
        for (int cc = 0; cc < nch; cc += 2) {
            // this wave's loads of the pair (and at a row group's start the
            // row operand) have landed; after the barrier every wave's have,
            // and every wave is done with the pair before, whose slots the
            // next loads reuse.  Positions past the tile's end reload chunks
            // that are never read.
            wait_vmem_all();
            barrier_only();
            issue(k0 + cc + 2);
            issue(k0 + cc + 3);
            step(cc);
            step(cc + 1);
        }
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            const float tot = half_transpose_sum16(racc[t], lane);
            if (!(lane & 16)) rowacc[((g * WAVES + wave) * RW + t) * 32 + acc_row(lane & 15, lane)] = tot;
        }
    }
}

// Stabilised pass over one macro tile.  Full macro tiles of cores up to
// RING_MAX_UNITS units take the LDS ring above.  Other tiles (the last row
// of macro tiles, a last column tile with an odd chunk count, wide cores)
// read each wave's column fragments straight from the pack, one chunk ahead
// in registers (loaded once this chunk's MFMAs have read them), with
// per-tile bounds.  Row partials go to LDS and are stored with the column
// partials after the loop.
template <class C, int RW>
__device__ __forceinline__ void pass_stab_body(const PassArgs& p, int wg) {
    if (!should_run(p.ctl, p.run_if, p.token)) return;
    constexpr int NU = C::UNITS * 64;
    extern __shared__ float dyn[];
    // the wave index through readfirstlane: row-tile bounds derived from it
    // are known to be wave-uniform and branch with scalar branches
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int rb, cb;
    tile_coords(wg, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);
    const int bcw = p.bc_chunks * 32;
    float* colacc = dyn + wave * bcw;
    float* rowacc = dyn + WAVES * bcw;
    for (int i = lane; i < nch * 32; i += 64) colacc[i] = 0.f;

    // full macro tiles: every row tile in range, even chunk count
    const bool full = (rb + 1) * p.rg * WAVES * RW <= p.n_chunks_r && (nch & 1) == 0;
    bool done = false;
    if constexpr (C::UNITS <= RING_MAX_UNITS) {
        if (full) {
            stab_ring_tile<C, RW>(p, rb, c0, nch, wave, lane, colacc, rowacc);
            done = true;
        }
    }
    if (!done) {
        auto chunk_ptr = [&](int k) { return p.B + (size_t)(c0 + k % nch) * NU; };
        typename C::A a[RW];
        float racc[RW][16];
        typename C::B b;
        C::load_b(b, chunk_ptr(0), lane);
        for (int g = 0; g < p.rg; ++g) {
            const int rchunk0 = (rb * p.rg + g) * (WAVES * RW) + wave * RW;
            const int nact = min(RW, p.n_chunks_r - rchunk0);  // wave-uniform
            if (nact <= 0) break;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (t < nact) C::load(a[t], p.A, rchunk0 + t, lane);
#pragma unroll
                for (int q = 0; q < 16; ++q) racc[t][q] = 0.f;
            }
            wait_vmem_all();
            for (int cc = 0; cc < nch; ++cc) {
                f32x16_t s[RW];
#pragma unroll
                for (int t = 0; t < RW; ++t)
                    if (t < nact) s[t] = C::tile_ab(a[t], b);
                C::load_b(b, chunk_ptr(g * nch + cc + 1), lane);
                const float cs = stab_exp_sums<C, RW>(s, racc, nact);
                if (lane < 32) colacc[cc * 32 + lane] += cs;
            }
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (t < nact) {
                    const float tot = half_transpose_sum16(racc[t], lane);
                    if (!(lane & 16)) rowacc[((g * WAVES + wave) * RW + t) * 32 + acc_row(lane & 15, lane)] = tot;
                }
            }
        }
    }
    __syncthreads();
    pass_stab_store<RW>(p, dyn, rb, cb, c0, nch);
}


// Several independent problems in one launch (the serving loop): each
// work-group finds its problem in the prefix table of work-group counts.
constexpr int BATCH_MAX = 16;
struct PassBatch {
    int n;
    int start[BATCH_MAX + 1];
    PassArgs req[BATCH_MAX];
};

__device__ __forceinline__ int batch_slot(const int* start, int n, int wg) {
    int r = 0;
    while (r + 1 < n && wg >= start[r + 1]) ++r;
    return r;
}

template <class C, int RW>
__global__ void __launch_bounds__(THREADS) k_pass_stab(PassArgs p) {
    pass_stab_body<C, RW>(p, blockIdx.x);
}

template <class C, int RW>
__global__ void __launch_bounds__(THREADS) k_pass_stab_batch(PassBatch b) {
    const int r = batch_slot(b.start, b.n, blockIdx.x);
    pass_stab_body<C, RW>(b.req[r], blockIdx.x - b.start[r]);
}

// ---------------------------------------------------------------------------
// Safe (max-shifted) MFMA pass: per row group, phase 0 finds lane-local row
// maxima and wave-local column maxima, phase 1 sums 2^{s - max}.
// ---------------------------------------------------------------------------

template <class C, int RW>
__device__ __forceinline__ void pass_safe_body(const PassArgs& p, int wg) {
    if (!should_run(p.ctl, p.run_if, p.token)) return;
    constexpr int NU = C::UNITS * 64;
    __shared__ uint4 zbuf[2][NU];
    extern __shared__ float dyn[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int rb, cb;
    tile_coords(wg, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);
    const int bcw = p.bc_chunks * 32;
    float* cmg = dyn + (0 * WAVES + wave) * bcw;
    float* cM = dyn + (1 * WAVES + wave) * bcw;
    float* cS = dyn + (2 * WAVES + wave) * bcw;
    for (int i = lane; i < nch * 32; i += 64) {
        cM[i] = -3.0e38f;
        cS[i] = 0.f;
    }

    ChunkStage<NU> st;
    st.load(p.B + (size_t)c0 * NU, tid);
    st.store(zbuf[0], tid);
    __syncthreads();

    typename C::A a[RW];
    float rmax[RW][16], rsum[RW][16];
    bool act[RW];
    int rchunk0 = 0;
    const int per_g = 2 * nch;
    const int total = p.rg * per_g;
    for (int it = 0; it < total; ++it) {
        const int g = it / per_g, rem = it - g * per_g;
        const int phase = rem >= nch ? 1 : 0;
        const int cc = rem - phase * nch;
        if (rem == 0) {
            rchunk0 = (rb * p.rg + g) * (WAVES * RW) + wave * RW;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                act[t] = rchunk0 + t < p.n_chunks_r;
                if (act[t]) C::load(a[t], p.A, rchunk0 + t, lane);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    rmax[t][q] = -3.0e38f;
                    rsum[t][q] = 0.f;
                }
            }
        }
        const bool has_next = it + 1 < total;
        if (has_next) {
            const int nrem = (it + 1) % per_g;
            st.load(p.B + (size_t)(c0 + nrem % nch) * NU, tid);
        }
        const uint4* zb = zbuf[it & 1];
        if (phase == 0) {
            float cm = -3.0e38f;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (act[t]) {
                    f32x16_t s = C::tile(a[t], zb, lane);
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        rmax[t][q] = fmaxf(rmax[t][q], s[q]);
                        cm = fmaxf(cm, s[q]);
                    }
                }
            }
            cm = fmaxf(cm, shfl_xor_f(cm, 32));
            if (lane < 32) cmg[cc * 32 + lane] = cm;
        } else {
            const float cmx = cmg[cc * 32 + (lane & 31)];
            float cs = 0.f;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (act[t]) {
                    f32x16_t s = C::tile(a[t], zb, lane);
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        rsum[t][q] += fast_exp2(s[q] - rmax[t][q]);
                        cs += fast_exp2(s[q] - cmx);
                    }
                }
            }
            cs += shfl_xor_f(cs, 32);
            if (lane < 32) {
                float M = cM[cc * 32 + lane], S = cS[cc * 32 + lane];
                lse_merge(M, S, cmx, cs);
                cM[cc * 32 + lane] = M;
                cS[cc * 32 + lane] = S;
            }
            if (cc == nch - 1) {
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    if (act[t]) {
                        float mo, so;
                        half_transpose_lse16(rmax[t], rsum[t], lane, mo, so);
                        if (!(lane & 16)) {
                            const size_t o = (size_t)cb * p.n_pad + (rchunk0 + t) * 32 + acc_row(lane & 15, lane);
                            p.rp[o] = mo;
                            p.rp2[o] = so;
                        }
                    }
                }
            }
        }
        if (has_next) st.store(zbuf[(it + 1) & 1], tid);
        __syncthreads();
    }
    for (int i = tid; i < nch * 32; i += THREADS) {
        float M = -3.0e38f, S = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) lse_merge(M, S, dyn[(1 * WAVES + w) * bcw + i], dyn[(2 * WAVES + w) * bcw + i]);
        const size_t o = (size_t)rb * p.m_pad + c0 * 32 + i;
        p.cp[o] = M;
        p.cp2[o] = S;
    }
}

template <class C, int RW>
__global__ void __launch_bounds__(THREADS) k_pass_safe(PassArgs p) {
    pass_safe_body<C, RW>(p, blockIdx.x);
}

template <class C, int RW>
__global__ void __launch_bounds__(THREADS) k_pass_safe_batch(PassBatch b) {
    const int r = batch_slot(b.start, b.n, blockIdx.x);
    pass_safe_body<C, RW>(b.req[r], blockIdx.x - b.start[r]);
}

// ---------------------------------------------------------------------------
// VALU pass for D < 16: lane = row (RV rows per lane), columns broadcast
// from LDS as records [Z_j (D), V_j, m_j].  The exponent is evaluated in the
// direct (unexpanded) form of Algorithm 1's squared distance between lifted
// points,
//   s_ij = U_i + V_j - k (|X_i - Z_j|^2 + (n_i - m_j)^2 / 4),
// with U_i = log2 a_i + k f_i, V_j = log2 b_j + k g_j, which keeps every term
// small and so loses far less to FP32 rounding than the expanded form.
// ---------------------------------------------------------------------------

constexpr int RV = 4;                       // rows per lane
constexpr int VALU_ROWS = WAVES * 64 * RV;  // rows per row group

struct ValuArgs {
    const float* X;
    const float* xn;
    const float* U;
    const float* Ul;
    const float* Z;
    const float* mm;
    const float* V;
    const float* Vl;
    float kappa;
    float* rp;
    float* rp2;
    float* cp;
    float* cp2;
    const int* ctl;
    int run_if;
    int token;
    int n_pad, m_pad;
    int n_chunks_c;
    int rg, bc_chunks, n_mt_r, n_mt_c;
};

template <int D>
__device__ __forceinline__ void valu_load_chunk(float* dst, const ValuArgs& p, int c, int tid) {
    constexpr int R = D + 3;  // [Z (D), Vh, m/2, Vl]
    for (int u = tid; u < 32 * R; u += THREADS) {
        const int j = u / R, k = u - j * R;
        const int col = c * 32 + j;
        float v;
        if (k < D) v = p.Z[(size_t)col * D + k];
        else if (k == D) v = p.V[col];
        else if (k == D + 1) v = 0.5f * p.mm[col];
        else v = p.Vl[col];
        dst[u] = v;
    }
}

template <int D, int SAFE>
__global__ void __launch_bounds__(THREADS) k_pass_valu(ValuArgs p) {
    if (!should_run(p.ctl, p.run_if, p.token)) return;
    constexpr int R = D + 3;
    __shared__ float zc[2][32 * R];
    extern __shared__ float dyn[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int rb, cb;
    tile_coords(blockIdx.x, p.n_mt_r, p.n_mt_c, rb, cb);
    const int c0 = cb * p.bc_chunks;
    const int nch = min(p.bc_chunks, p.n_chunks_c - c0);
    const int bcw = p.bc_chunks * 32;
    float* cacc = dyn + wave * bcw;              // stab sums / safe cM
    float* cS = dyn + (WAVES + wave) * bcw;      // safe sums
    float* cmg = dyn + (2 * WAVES + wave) * bcw; // safe group maxima
    for (int i = lane; i < nch * 32; i += 64) {
        cacc[i] = SAFE ? -3.0e38f : 0.f;
        if (SAFE) cS[i] = 0.f;
    }
    valu_load_chunk<D>(zc[0], p, c0, tid);
    __syncthreads();

    float xr[RV][D], ur[RV], ul[RV], nr[RV], racc[RV], rmax[RV];
    int row0 = 0;
    const int phases = SAFE ? 2 : 1;
    const int per_g = phases * nch;
    const int total = p.rg * per_g;
    for (int it = 0; it < total; ++it) {
        const int g = it / per_g, rem = it - g * per_g;
        const int phase = rem >= nch ? 1 : 0;
        const int cc = rem - phase * nch;
        if (rem == 0) {
            row0 = (rb * p.rg + g) * VALU_ROWS + wave * 64 * RV;
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                const int row = row0 + r * 64 + lane;
                const bool ok = row < p.n_pad;
#pragma unroll
                for (int d = 0; d < D; ++d) xr[r][d] = ok ? p.X[(size_t)row * D + d] : 0.f;
                ur[r] = ok ? p.U[row] : -INFINITY;
                ul[r] = ok ? p.Ul[row] : 0.f;
                nr[r] = ok ? 0.5f * p.xn[row] : 0.f;
                racc[r] = 0.f;
                rmax[r] = -3.0e38f;
            }
        }
        const float* zb = zc[it & 1];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            float cv[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const float* zr = zb + (half * 16 + jj) * R;
                float acc_c = SAFE && phase == 0 ? -3.0e38f : 0.f;
                const float cmx = (SAFE && phase == 1) ? cmg[cc * 32 + half * 16 + jj] : 0.f;
#pragma unroll
                for (int r = 0; r < RV; ++r) {
                    const float dl = nr[r] - zr[D + 1];
                    float dist = dl * dl;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const float df = xr[r][d] - zr[d];
                        dist = fmaf(df, df, dist);
                    }
                    const float s = assemble_exponent(ur[r], ul[r], zr[D], zr[D + 2], p.kappa * dist);
                    if (!SAFE) {
                        const float e = fast_exp2(s);
                        racc[r] += e;
                        acc_c += e;
                    } else if (phase == 0) {
                        rmax[r] = fmaxf(rmax[r], s);
                        acc_c = fmaxf(acc_c, s);
                    } else {
                        racc[r] += fast_exp2(s - rmax[r]);
                        acc_c += fast_exp2(s - cmx);
                    }
                }
                cv[jj] = acc_c;
            }
            if (SAFE && phase == 0) {
                float m = half_transpose_reduce16(cv, lane, OpMax());
                m = fmaxf(m, shfl_xor_f(m, 32));
                if (lane < 16) cmg[cc * 32 + half * 16 + lane] = m;
            } else {
                float tot = half_transpose_sum16(cv, lane);
                tot += shfl_xor_f(tot, 32);
                if (lane < 16) {
                    const int ci = cc * 32 + half * 16 + lane;
                    if (!SAFE) {
                        cacc[ci] += tot;
                    } else {
                        float M = cacc[ci], S = cS[ci];
                        lse_merge(M, S, cmg[ci], tot);
                        cacc[ci] = M;
                        cS[ci] = S;
                    }
                }
            }
        }
        const bool last_of_group = SAFE ? (phase == 1 && cc == nch - 1) : (cc == nch - 1);
        if (last_of_group) {
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                const int row = row0 + r * 64 + lane;
                if (row < p.n_pad) {
                    const size_t o = (size_t)cb * p.n_pad + row;
                    if (!SAFE) {
                        p.rp[o] = racc[r];
                    } else {
                        p.rp[o] = rmax[r];
                        p.rp2[o] = racc[r];
                    }
                }
            }
        }
        if (it + 1 < total) {
            const int nrem = (it + 1) % per_g;
            valu_load_chunk<D>(zc[(it + 1) & 1], p, c0 + nrem % nch, tid);
        }
        __syncthreads();
    }
    for (int i = tid; i < nch * 32; i += THREADS) {
        const size_t o = (size_t)rb * p.m_pad + c0 * 32 + i;
        if (!SAFE) {
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) s += dyn[w * bcw + i];
            p.cp[o] = s;
        } else {
            float M = -3.0e38f, S = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) lse_merge(M, S, dyn[w * bcw + i], dyn[(WAVES + w) * bcw + i]);
            p.cp[o] = M;
            p.cp2[o] = S;
        }
    }
}

// ---------------------------------------------------------------------------
// Geometry and dispatch
// ---------------------------------------------------------------------------

static int rows_per_wave_tiles(int prec, int d) {
    const int units = pack_units(prec, d);
    return units <= 9 ? 2 : 1;  // RW: row tiles per wave
}

Geometry pass_geometry(int prec, int d, int64_t n, int64_t m, int multiplier) {
    Geometry g{};
    g.n_pad = (int)((n + 31) / 32 * 32);
    g.m_pad = (int)((m + 31) / 32 * 32);
    const int n_chunks_c = g.m_pad / 32;
    if (d <= VALU_MAX_DIM) {
        g.path = 1;
        g.rows_per_group = VALU_ROWS;
    } else {
        g.path = 0;
        g.rows_per_group = WAVES * rows_per_wave_tiles(prec, d) * 32;
    }
    g.bc_chunks = n_chunks_c < 32 ? n_chunks_c : 32;
    if (g.path == 1) {
        // small problems on the VALU path: narrower column tiles (even chunk
        // counts, at least 2) until the grid has ~1024 workgroups, so that a
        // few thousand rows still fill the 256 CUs
        const int64_t nmr_min = (g.n_pad + g.rows_per_group - 1) / g.rows_per_group;
        while (g.bc_chunks > 2 && (g.bc_chunks & 1) == 0 &&
               nmr_min * ((n_chunks_c + g.bc_chunks - 1) / g.bc_chunks) < 1024)
            g.bc_chunks >>= 1;
    }
    g.n_mt_c = (n_chunks_c + g.bc_chunks - 1) / g.bc_chunks;
    // as many row groups per macro tile as keeps >= ~2048 workgroups
    const int target = 2048 * (multiplier > 0 ? multiplier : 1);
    int rg = 8;
    while (rg > 1) {
        const int64_t rows = (int64_t)rg * g.rows_per_group;
        const int64_t nmr = (g.n_pad + rows - 1) / rows;
        if (nmr * g.n_mt_c >= target) break;
        rg >>= 1;
    }
    g.rg = rg;
    const int64_t rows = (int64_t)rg * g.rows_per_group;
    g.n_mt_r = (int)((g.n_pad + rows - 1) / rows);
    return g;
}

static PassArgs make_pass_args(const Operands& op, const Geometry& g, const Partials& pp, int* ctl, int run_if) {
    PassArgs a;
    a.A = (const uint4*)op.A;
    a.B = (const uint4*)op.B;
    a.rp = pp.row;
    a.rp2 = pp.row2;
    a.cp = pp.col;
    a.cp2 = pp.col2;
    a.ctl = ctl;
    a.run_if = run_if;
    a.token = op.token;
    a.n_chunks_r = g.n_pad / 32;
    a.n_chunks_c = g.m_pad / 32;
    a.rg = g.rg;
    a.bc_chunks = g.bc_chunks;
    a.n_mt_r = g.n_mt_r;
    a.n_mt_c = g.n_mt_c;
    a.n_pad = g.n_pad;
    a.m_pad = g.m_pad;
    return a;
}

// Dynamic LDS of a pass launch: per-wave column accumulators (three arrays in
// the safe pass), plus the macro tile's row partials in the stabilised pass.
static size_t pass_lds_bytes(const Geometry& g, int safe) {
    const size_t cols = (size_t)WAVES * g.bc_chunks * 32;
    return (safe ? 3 * cols : cols + (size_t)g.rg * g.rows_per_group) * sizeof(float);
}

template <class C, int RW>
static hipError_t launch_mfma_batch(const PassBatch& b, size_t lds, int safe, hipStream_t stream) {
    if (safe)
        hipLaunchKernelGGL((k_pass_safe_batch<C, RW>), dim3(b.start[b.n]), dim3(THREADS), lds, stream, b);
    else
        hipLaunchKernelGGL((k_pass_stab_batch<C, RW>), dim3(b.start[b.n]), dim3(THREADS), lds, stream, b);
    return hipGetLastError();
}

static hipError_t dispatch_batch(int prec, int units, const PassBatch& b, size_t lds, int safe, hipStream_t stream) {
    if (prec == PREC_F32) {
        switch (units) {
            case 3: return launch_mfma_batch<CoreF32<3>, 2>(b, lds, safe, stream);
            case 5: return launch_mfma_batch<CoreF32<5>, 2>(b, lds, safe, stream);
            case 7: return launch_mfma_batch<CoreF32<7>, 2>(b, lds, safe, stream);
            case 9: return launch_mfma_batch<CoreF32<9>, 2>(b, lds, safe, stream);
            case 13: return launch_mfma_batch<CoreF32<13>, 1>(b, lds, safe, stream);
            case 17: return launch_mfma_batch<CoreF32<17>, 1>(b, lds, safe, stream);
            case 25: return launch_mfma_batch<CoreF32<25>, 1>(b, lds, safe, stream);
            case 33: return launch_mfma_batch<CoreF32<33>, 1>(b, lds, safe, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (units) {
        case 2: return launch_mfma_batch<CoreBF16<2>, 2>(b, lds, safe, stream);
        case 3: return launch_mfma_batch<CoreBF16<3>, 2>(b, lds, safe, stream);
        case 4: return launch_mfma_batch<CoreBF16<4>, 2>(b, lds, safe, stream);
        case 5: return launch_mfma_batch<CoreBF16<5>, 2>(b, lds, safe, stream);
        case 7: return launch_mfma_batch<CoreBF16<7>, 2>(b, lds, safe, stream);
        case 9: return launch_mfma_batch<CoreBF16<9>, 2>(b, lds, safe, stream);
        case 10: return launch_mfma_batch<CoreBF16<10>, 1>(b, lds, safe, stream);
        case 13: return launch_mfma_batch<CoreBF16<13>, 1>(b, lds, safe, stream);
        case 17: return launch_mfma_batch<CoreBF16<17>, 1>(b, lds, safe, stream);
        case 19: return launch_mfma_batch<CoreBF16<19>, 1>(b, lds, safe, stream);
        case 25: return launch_mfma_batch<CoreBF16<25>, 1>(b, lds, safe, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass_batch(const PassItem* items, int n, int run_if, int safe, hipStream_t stream) {
    // consecutive items sharing one kernel instantiation go into one launch
    int g0 = 0;
    while (g0 < n) {
        const int prec = items[g0].op.prec == PREC_F32 ? PREC_F32 : PREC_BF16;
        const int units = pack_units(items[g0].op.prec, items[g0].op.d);
        PassBatch b{};
        b.n = 0;
        b.start[0] = 0;
        size_t lds = 0;
        while (g0 < n && b.n < BATCH_MAX) {
            const PassItem& it = items[g0];
            if (it.g.path != 0) return hipErrorInvalidValue;
            const int p2 = it.op.prec == PREC_F32 ? PREC_F32 : PREC_BF16;
            if (p2 != prec || pack_units(it.op.prec, it.op.d) != units) break;
            b.req[b.n] = make_pass_args(it.op, it.g, it.pp, it.ctl, run_if);
            b.start[b.n + 1] = b.start[b.n] + it.g.n_mt_r * it.g.n_mt_c;
            const size_t l = pass_lds_bytes(it.g, safe);
            lds = l > lds ? l : lds;
            ++b.n;
            ++g0;
        }
        const hipError_t e = dispatch_batch(prec, units, b, lds, safe, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class C, int RW>
static hipError_t launch_mfma(const Operands& op, const Geometry& g, const Partials& pp, int* ctl, int run_if,
                              int safe, hipStream_t stream) {
    PassArgs a;
    a.A = (const uint4*)op.A;
    a.B = (const uint4*)op.B;
    a.rp = pp.row;
    a.rp2 = pp.row2;
    a.cp = pp.col;
    a.cp2 = pp.col2;
    a.ctl = ctl;
    a.run_if = run_if;
    a.token = op.token;
    a.n_chunks_r = g.n_pad / 32;
    a.n_chunks_c = g.m_pad / 32;
    a.rg = g.rg;
    a.bc_chunks = g.bc_chunks;
    a.n_mt_r = g.n_mt_r;
    a.n_mt_c = g.n_mt_c;
    a.n_pad = g.n_pad;
    a.m_pad = g.m_pad;
    const int grid = g.n_mt_r * g.n_mt_c;
    const size_t lds = pass_lds_bytes(g, safe);
    if (safe)
        hipLaunchKernelGGL((k_pass_safe<C, RW>), dim3(grid), dim3(THREADS), lds, stream, a);
    else
        hipLaunchKernelGGL((k_pass_stab<C, RW>), dim3(grid), dim3(THREADS), lds, stream, a);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_valu_d(const Operands& op, const Geometry& g, const Partials& pp, int* ctl, int run_if,
                                int safe, hipStream_t stream) {
    ValuArgs a;
    a.X = op.X;
    a.xn = op.xn;
    a.U = op.U;
    a.Ul = op.Ul;
    a.Z = op.Zs;
    a.mm = op.ms;
    a.V = op.V;
    a.Vl = op.Vl;
    a.kappa = op.kappa;
    a.rp = pp.row;
    a.rp2 = pp.row2;
    a.cp = pp.col;
    a.cp2 = pp.col2;
    a.ctl = ctl;
    a.run_if = run_if;
    a.token = op.token;
    a.n_pad = g.n_pad;
    a.m_pad = g.m_pad;
    a.n_chunks_c = g.m_pad / 32;
    a.rg = g.rg;
    a.bc_chunks = g.bc_chunks;
    a.n_mt_r = g.n_mt_r;
    a.n_mt_c = g.n_mt_c;
    const int grid = g.n_mt_r * g.n_mt_c;
    const size_t lds = pass_lds_bytes(g, safe);
    if (safe)
        hipLaunchKernelGGL((k_pass_valu<D, 1>), dim3(grid), dim3(THREADS), lds, stream, a);
    else
        hipLaunchKernelGGL((k_pass_valu<D, 0>), dim3(grid), dim3(THREADS), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_pass(const Operands& op, const Geometry& g, const Partials& pp, int* ctl, int run_if, int safe,
                       hipStream_t stream) {
    if (g.path == 1) {
        switch (op.d) {
#define GW_VALU_CASE(DD) \
    case DD:             \
        return launch_valu_d<DD>(op, g, pp, ctl, run_if, safe, stream);
            GW_VALU_CASE(1) GW_VALU_CASE(2) GW_VALU_CASE(3) GW_VALU_CASE(4) GW_VALU_CASE(5)
            GW_VALU_CASE(6) GW_VALU_CASE(7) GW_VALU_CASE(8) GW_VALU_CASE(9) GW_VALU_CASE(10)
            GW_VALU_CASE(11) GW_VALU_CASE(12) GW_VALU_CASE(13) GW_VALU_CASE(14) GW_VALU_CASE(15)
#undef GW_VALU_CASE
            default:
                return hipErrorInvalidValue;
        }
    }
    const int units = pack_units(op.prec, op.d);
    if (op.prec == PREC_F32) {
        switch (units) {
            case 3: return launch_mfma<CoreF32<3>, 2>(op, g, pp, ctl, run_if, safe, stream);
            case 5: return launch_mfma<CoreF32<5>, 2>(op, g, pp, ctl, run_if, safe, stream);
            case 7: return launch_mfma<CoreF32<7>, 2>(op, g, pp, ctl, run_if, safe, stream);
            case 9: return launch_mfma<CoreF32<9>, 2>(op, g, pp, ctl, run_if, safe, stream);
            case 13: return launch_mfma<CoreF32<13>, 1>(op, g, pp, ctl, run_if, safe, stream);
            case 17: return launch_mfma<CoreF32<17>, 1>(op, g, pp, ctl, run_if, safe, stream);
            case 25: return launch_mfma<CoreF32<25>, 1>(op, g, pp, ctl, run_if, safe, stream);
            case 33: return launch_mfma<CoreF32<33>, 1>(op, g, pp, ctl, run_if, safe, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (units) {  // BF16 and split-BF16 share the core
        case 2: return launch_mfma<CoreBF16<2>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 3: return launch_mfma<CoreBF16<3>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 4: return launch_mfma<CoreBF16<4>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 5: return launch_mfma<CoreBF16<5>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 7: return launch_mfma<CoreBF16<7>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 9: return launch_mfma<CoreBF16<9>, 2>(op, g, pp, ctl, run_if, safe, stream);
        case 10: return launch_mfma<CoreBF16<10>, 1>(op, g, pp, ctl, run_if, safe, stream);
        case 13: return launch_mfma<CoreBF16<13>, 1>(op, g, pp, ctl, run_if, safe, stream);
        case 17: return launch_mfma<CoreBF16<17>, 1>(op, g, pp, ctl, run_if, safe, stream);
        case 19: return launch_mfma<CoreBF16<19>, 1>(op, g, pp, ctl, run_if, safe, stream);
        case 25: return launch_mfma<CoreBF16<25>, 1>(op, g, pp, ctl, run_if, safe, stream);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Combine: deterministic fixed-order reduction of the partials, potential
// update, bias-slot refresh, range checks and the device-side mode decision.
// ---------------------------------------------------------------------------

struct CombineDev {
    CombineArgs a;
    int kb;       // first bias slot
    int units;    // pack units per chunk
};

// blk / nblk: this block's index among the problem's nblk blocks (the last
// one to finish takes the mode decision)
constexpr int COMBINE_UNROLL = 16;

__device__ __forceinline__ void combine_body(const CombineDev& cd, int* ctl, int run_if, int blk, int nblk) {
    const CombineArgs& a = cd.a;
    if (!should_run(ctl, run_if, a.token)) return;
    const int mode = ctl[CTL_MODE];
    const int user = ctl[CTL_USER];
    const bool safe_parts = a.is_retry || mode == MODE_SAFE;
    const bool check_stab = !a.is_retry && mode == MODE_STAB && user != 2;
    // each thread merges four consecutive rows (or columns): one 16-byte
    // load per partial tile; the partials are merged in tile order and their
    // loads issued a block at a time so that many are in flight
    const int nrow4 = a.do_rows ? (a.n + 3) / 4 : 0;
    const int ncol4 = a.do_cols ? (a.m + 3) / 4 : 0;
    const int idx = blk * blockDim.x + threadIdx.x;
    int bad = 0, unsafe = 0, numeric = 0;
    if (idx < nrow4 + ncol4) {
        const bool is_row = idx < nrow4;
        const int i0 = 4 * (is_row ? idx : idx - nrow4);
        const int cnt = min(4, (is_row ? a.n : a.m) - i0);
        const int npart = is_row ? a.n_mt_c : a.n_mt_r;
        const size_t stride4 = (size_t)(is_row ? a.n_pad : a.m_pad) / 4;
        const float4* q1 = reinterpret_cast<const float4*>((is_row ? a.rp : a.cp) + i0);
        const float4* q2 = reinterpret_cast<const float4*>((is_row ? a.rp2 : a.cp2) + i0);
        double l2d[4];
        int k = 0;
        if (!safe_parts) {
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            for (; k + COMBINE_UNROLL <= npart; k += COMBINE_UNROLL) {
                float4 v[COMBINE_UNROLL];
#pragma unroll
                for (int u = 0; u < COMBINE_UNROLL; ++u) v[u] = q1[(k + u) * stride4];
#pragma unroll
                for (int u = 0; u < COMBINE_UNROLL; ++u) {
                    acc.x += v[u].x;
                    acc.y += v[u].y;
                    acc.z += v[u].z;
                    acc.w += v[u].w;
                }
            }
            for (; k < npart; ++k) {
                const float4 v = q1[k * stride4];
                acc.x += v.x;
                acc.y += v.y;
                acc.z += v.z;
                acc.w += v.w;
            }
            l2d[0] = log2((double)acc.x);
            l2d[1] = log2((double)acc.y);
            l2d[2] = log2((double)acc.z);
            l2d[3] = log2((double)acc.w);
        } else {
            float M[4] = {-3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f}, S[4] = {0.f, 0.f, 0.f, 0.f};
            constexpr int U2 = COMBINE_UNROLL / 2;
            auto merge4 = [&](const float4& vm, const float4& vs) {
                lse_merge(M[0], S[0], vm.x, vs.x);
                lse_merge(M[1], S[1], vm.y, vs.y);
                lse_merge(M[2], S[2], vm.z, vs.z);
                lse_merge(M[3], S[3], vm.w, vs.w);
            };
            for (; k + U2 <= npart; k += U2) {
                float4 vm[U2], vs[U2];
#pragma unroll
                for (int u = 0; u < U2; ++u) {
                    vm[u] = q1[(k + u) * stride4];
                    vs[u] = q2[(k + u) * stride4];
                }
#pragma unroll
                for (int u = 0; u < U2; ++u) merge4(vm[u], vs[u]);
            }
            for (; k < npart; ++k) merge4(q1[k * stride4], q2[k * stride4]);
#pragma unroll
            for (int c = 0; c < 4; ++c) l2d[c] = (double)M[c] + log2((double)S[c]);
        }
        void* pack = is_row ? a.packA_next : a.packB_next;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= cnt) break;
            const int i = i0 + c;
            const float l2 = (float)l2d[c];
            const float lw = is_row ? a.la2[i] : a.lb2[i];
            const float lr = l2 - lw;
            const bool fin = isfinite(lr);
            if (check_stab && (!fin || fabsf(lr) > STAB_LIMIT)) bad = 1;
            if (!fin && !check_stab) numeric = 1;
            if (!fin || fabsf(lr) > COMFORT_LIMIT) unsafe = 1;
            // potentials are FP32 (hi, lo) pairs; the update itself runs in FP64
            const double cur = is_row ? join_df(a.U_cur[i], a.Ul_cur[i]) : join_df(a.V_cur[i], a.Vl_cur[i]);
            const double lr64 = l2d[c] - (double)lw;
            const double nxt = fin ? cur - (double)a.step * lr64 : cur;
            float nh, nl;
            split_df(nxt, nh, nl);
            if (is_row) {
                a.U_next[i] = nh;
                a.Ul_next[i] = nl;
            } else {
                a.V_next[i] = nh;
                a.Vl_next[i] = nl;
            }
            if (pack) {
                if (a.prec == PREC_F32) {
                    if (is_row) write_pot_a_f32((float*)pack, i, cd.kb, cd.units, nh, nl);
                    else write_pot_b_f32((float*)pack, i, cd.kb, cd.units, nh, nl);
                } else {
                    if (is_row) write_pot_a_bf16((uint16_t*)pack, i, cd.kb, cd.units, nh, nl);
                    else write_pot_b_bf16((uint16_t*)pack, i, cd.kb, cd.units, nh, nl);
                }
            }
        }
    }
    bad = __syncthreads_or(bad);
    unsafe = __syncthreads_or(unsafe);
    numeric = __syncthreads_or(numeric);
    __shared__ int last;
    if (threadIdx.x == 0) {
        if (bad) atomicOr(&ctl[CTL_BAD], 1);
        if (unsafe) atomicOr(&ctl[CTL_UNSAFE], 1);
        if (numeric) atomicOr(&ctl[CTL_NUMERIC], 1);
        __threadfence();
        const int prev = atomicAdd(&ctl[CTL_COUNT], 1);
        last = prev == nblk - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const int any_bad = atomicOr(&ctl[CTL_BAD], 0);
        const int any_unsafe = atomicOr(&ctl[CTL_UNSAFE], 0);
        if (check_stab && any_bad) {
            // the retry pass and combine run next and decide the mode
        } else {
            const int next = user == 1 ? MODE_SAFE : (user == 2 ? MODE_STAB : (any_unsafe ? MODE_SAFE : MODE_STAB));
            if (safe_parts) atomicAdd(&ctl[CTL_SAFE_ITERS], 1);
            atomicExch(&ctl[CTL_MODE], next);
            atomicExch(&ctl[CTL_DONE], a.token);
            atomicExch(&ctl[CTL_BAD], 0);
            atomicExch(&ctl[CTL_UNSAFE], 0);
        }
        atomicExch(&ctl[CTL_COUNT], 0);
    }
}

__global__ void __launch_bounds__(256) k_combine(CombineDev cd, int* ctl, int run_if) {
    combine_body(cd, ctl, run_if, blockIdx.x, gridDim.x);
}

struct CombineBatch {
    int n;
    int start[BATCH_MAX + 1];
    int* ctl[BATCH_MAX];
    CombineDev req[BATCH_MAX];
};
static_assert(sizeof(CombineBatch) <= 4000, "batch table must fit the kernel argument space");
static_assert(sizeof(PassBatch) <= 4000, "batch table must fit the kernel argument space");

__global__ void __launch_bounds__(256) k_combine_batch(CombineBatch b, int run_if) {
    const int r = batch_slot(b.start, b.n, blockIdx.x);
    combine_body(b.req[r], b.ctl[r], run_if, blockIdx.x - b.start[r], b.start[r + 1] - b.start[r]);
}

static CombineDev make_combine_dev(const CombineArgs& a) {
    CombineDev cd;
    cd.a = a;
    cd.kb = 0;
    cd.units = 0;
    if (a.packA_next || a.packB_next) {
        const int dp = feat_pad(a.d);
        cd.kb = a.prec == PREC_BF16X3 ? 3 * dp : dp;
        cd.units = pack_units(a.prec, a.d);
    }
    return cd;
}

static int combine_blocks(const CombineArgs& a) {
    const int total = (a.do_rows ? (a.n + 3) / 4 : 0) + (a.do_cols ? (a.m + 3) / 4 : 0);
    return (total + 255) / 256;
}

hipError_t launch_combine(const CombineArgs& a, int* ctl, int run_if, hipStream_t stream) {
    const CombineDev cd = make_combine_dev(a);
    hipLaunchKernelGGL(k_combine, dim3(combine_blocks(a)), dim3(256), 0, stream, cd, ctl, run_if);
    return hipGetLastError();
}

hipError_t launch_combine_batch(const CombineArgs* items, int* const* ctls, int n, int run_if, hipStream_t stream) {
    for (int g0 = 0; g0 < n; g0 += BATCH_MAX) {
        CombineBatch b{};
        b.n = n - g0 < BATCH_MAX ? n - g0 : BATCH_MAX;
        b.start[0] = 0;
        for (int r = 0; r < b.n; ++r) {
            b.req[r] = make_combine_dev(items[g0 + r]);
            b.ctl[r] = ctls[g0 + r];
            b.start[r + 1] = b.start[r] + combine_blocks(items[g0 + r]);
        }
        hipLaunchKernelGGL(k_combine_batch, dim3(b.start[b.n]), dim3(256), 0, stream, b, run_if);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ void k_ctl_init(int* ctl, int user) {
    if (threadIdx.x == 0) {
        for (int w = 0; w < CTL_WORDS; ++w) ctl[w] = 0;
        ctl[CTL_USER] = user;
        ctl[CTL_MODE] = user == 2 ? MODE_STAB : MODE_SAFE;
    }
}

hipError_t launch_ctl_init(int* ctl, int user_mode, hipStream_t stream) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, ctl, user_mode);
    return hipGetLastError();
}

}  // namespace gwk
