// Device-side helpers shared by the gfx950 kernels: vector types, the packed
// MFMA operand layouts, the bias-slot encoding of the exponent, and
// wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gw_layout.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

#define GW_LDS_ALIGN __attribute__((aligned(16)))

// ---------------------------------------------------------------------------
// Scalar helpers
// ---------------------------------------------------------------------------

// 2^x on the transcendental unit (v_exp_f32).
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// s_waitcnt vmcnt(0) with expcnt and lgkmcnt left at their maxima (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// Work-group barrier without the memory fence of __syncthreads(), for
// callers that have already waited for what the other waves must see.  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void barrier_only() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

// Round-to-nearest-even float -> bf16 bits (finite inputs; +-inf kept).
__device__ __host__ __forceinline__ uint16_t f32_to_bf16_bits(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __host__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ float bf16_round(float v) { return bf16_bits_to_f32(f32_to_bf16_bits(v)); }

// Device copy of gwl::feat_pad.
__device__ __forceinline__ int feat_pad_dev(int d) {
    return d <= 16 ? 16 : d <= 32 ? 32 : d <= 48 ? 48 : d <= 64 ? 64 : d <= 96 ? 96 : d <= 128 ? 128 : d <= 192 ? 192 : 256;
}

// ---------------------------------------------------------------------------
// Packed operand layouts (see gw_layout.h for the host-visible description)
// ---------------------------------------------------------------------------

// BF16 pack: [chunk][slab s][lane 64][8]; lane l <-> row 32*chunk + (l & 31),
// k = 16 s + 8 (l >> 5) + e.  Returns the bf16-element offset.
__device__ __host__ __forceinline__ size_t bf16_pack_off(int row, int k, int slabs) {
    int chunk = row >> 5, r = row & 31;
    int s = k >> 4, h = (k >> 3) & 1, e = k & 7;
    int lane = r + 32 * h;
    return (((size_t)chunk * slabs + s) * 64 + lane) * 8 + e;
}

// F32 pack for v_mfma_f32_32x32x2f32: [chunk][group G][lane 64][4]; element
// e of group G is slab s = 4G + e, k = 2 s + (l >> 5), row 32*chunk + (l&31).
__device__ __host__ __forceinline__ size_t f32_pack_off(int row, int k, int groups) {
    int chunk = row >> 5, r = row & 31;
    int s = k >> 1, h = k & 1;
    int G = s >> 2, e = s & 3;
    int lane = r + 32 * h;
    return (((size_t)chunk * groups + G) * 64 + lane) * 4 + e;
}

// Split a float into three bf16 parts whose exact sum is the float (8
// significant bits per part covers the 24-bit significand).
__device__ __forceinline__ void split3_bf16(float v, uint16_t& h, uint16_t& m, uint16_t& l) {
    if (!(v > -3.0e38f)) {  // -inf or NaN marker: padded row/column
        h = f32_to_bf16_bits(v);
        m = 0;
        l = 0;
        return;
    }
    h = f32_to_bf16_bits(v);
    float r1 = v - bf16_bits_to_f32(h);
    m = f32_to_bf16_bits(r1);
    float r2 = r1 - bf16_bits_to_f32(m);
    l = f32_to_bf16_bits(r2);
}
__device__ __forceinline__ void split2_bf16(float v, uint16_t& h, uint16_t& l) {
    h = f32_to_bf16_bits(v);
    l = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
}

// Bias slots of a BF16 pack.  The exponent terms are carried as exact bf16
// splits so that sum_k A_k B_k = X.Zs + (Uh + Ul) + (Vh + Vl) + n ms, with
// the potentials as FP32 (hi, lo) pairs (compensated FP32) and n ms from
// three-part splits n = n1 + n2 + n3, ms = m1 + m2 + m3 keeping the six
// cross terms of weight >= 2^-24:
//   A: [U1, U2, U3, 1, 1, 1, n1, n1, n2, Ul1, Ul2, 1, 1, n1, n2, n3]
//   B: [1, 1, 1, V1, V2, V3, m1, m2, m1, 1, 1, Vl1, Vl2, m3, m2, m1]
__device__ __forceinline__ void write_bias_a_bf16(uint16_t* pack, int row, int kb, int slabs, float Uh, float Ul,
                                                  float n) {
    uint16_t u1, u2, u3, l1, l2, n1, n2, n3;
    split3_bf16(Uh, u1, u2, u3);
    split2_bf16(Ul, l1, l2);
    split3_bf16(n, n1, n2, n3);
    const uint16_t one = 0x3f80;
    uint16_t v[16] = {u1, u2, u3, one, one, one, n1, n1, n2, l1, l2, one, one, n1, n2, n3};
#pragma unroll
    for (int t = 0; t < 16; ++t) pack[bf16_pack_off(row, kb + t, slabs)] = v[t];
}
__device__ __forceinline__ void write_bias_b_bf16(uint16_t* pack, int col, int kb, int slabs, float Vh, float Vl,
                                                  float ms) {
    uint16_t v1, v2, v3, l1, l2, m1, m2, m3;
    split3_bf16(Vh, v1, v2, v3);
    split2_bf16(Vl, l1, l2);
    split3_bf16(ms, m1, m2, m3);
    const uint16_t one = 0x3f80;
    uint16_t v[16] = {one, one, one, v1, v2, v3, m1, m2, m1, one, one, l1, l2, m3, m2, m1};
#pragma unroll
    for (int t = 0; t < 16; ++t) pack[bf16_pack_off(col, kb + t, slabs)] = v[t];
}
// Only the potential slots change between Sinkhorn iterations.
__device__ __forceinline__ void write_pot_a_bf16(uint16_t* pack, int row, int kb, int slabs, float Uh, float Ul) {
    uint16_t u1, u2, u3, l1, l2;
    split3_bf16(Uh, u1, u2, u3);
    split2_bf16(Ul, l1, l2);
    pack[bf16_pack_off(row, kb + 0, slabs)] = u1;
    pack[bf16_pack_off(row, kb + 1, slabs)] = u2;
    pack[bf16_pack_off(row, kb + 2, slabs)] = u3;
    pack[bf16_pack_off(row, kb + 9, slabs)] = l1;
    pack[bf16_pack_off(row, kb + 10, slabs)] = l2;
}
__device__ __forceinline__ void write_pot_b_bf16(uint16_t* pack, int col, int kb, int slabs, float Vh, float Vl) {
    uint16_t v1, v2, v3, l1, l2;
    split3_bf16(Vh, v1, v2, v3);
    split2_bf16(Vl, l1, l2);
    pack[bf16_pack_off(col, kb + 3, slabs)] = v1;
    pack[bf16_pack_off(col, kb + 4, slabs)] = v2;
    pack[bf16_pack_off(col, kb + 5, slabs)] = v3;
    pack[bf16_pack_off(col, kb + 11, slabs)] = l1;
    pack[bf16_pack_off(col, kb + 12, slabs)] = l2;
}

// F32 bias slots: A: [Uh, 1, n, Ul, 1, 0, 0, 0], B: [1, Vh, ms, 1, Vl, 0, 0, 0].
// FP32 bias slots: k slots 5 to 7 stay zero (the pass cores skip the MFMA of
// slots 6 and 7)
__device__ __forceinline__ void write_bias_a_f32(float* pack, int row, int kb, int groups, float Uh, float Ul,
                                                 float n) {
    float v[8] = {Uh, 1.f, n, Ul, 1.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 8; ++t) pack[f32_pack_off(row, kb + t, groups)] = v[t];
}
__device__ __forceinline__ void write_bias_b_f32(float* pack, int col, int kb, int groups, float Vh, float Vl,
                                                 float ms) {
    float v[8] = {1.f, Vh, ms, 1.f, Vl, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 8; ++t) pack[f32_pack_off(col, kb + t, groups)] = v[t];
}
__device__ __forceinline__ void write_pot_a_f32(float* pack, int row, int kb, int groups, float Uh, float Ul) {
    pack[f32_pack_off(row, kb + 0, groups)] = Uh;
    pack[f32_pack_off(row, kb + 3, groups)] = Ul;
}
__device__ __forceinline__ void write_pot_b_f32(float* pack, int col, int kb, int groups, float Vh, float Vl) {
    pack[f32_pack_off(col, kb + 1, groups)] = Vh;
    pack[f32_pack_off(col, kb + 4, groups)] = Vl;
}

// A double as an FP32 (hi, lo) pair and back.
__device__ __forceinline__ void split_df(double v, float& h, float& l) {
    h = (float)v;
    l = isfinite(h) ? (float)(v - (double)h) : 0.f;
}
__device__ __forceinline__ double join_df(float h, float l) { return (double)h + (double)l; }

// Exponent assembly s = (Uh + Ul) + (Vh + Vl) - p with one rounding at the
// magnitude of s: Uh + Vh is formed exactly by a two-sum, and (th - p) is
// exact when th and p agree to a factor of two (every entry that matters).
// Padded rows and columns carry -inf potentials; the guard keeps them at
// -inf instead of the NaN the two-sum would produce.
__device__ __forceinline__ float assemble_exponent(float uh, float ul, float vh, float vl, float p) {
    const float th = uh + vh;
    const float bb = th - uh;
    const float tl = (uh - (th - bb)) + (vh - bb);
    const float s = (th - p) + (tl + (ul + vl));
    return th > -3.0e38f ? s : -INFINITY;
}

// ---------------------------------------------------------------------------
// Wavefront reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ float shfl_xor_f(float v, int mask) { return __shfl_xor(v, mask, 64); }

// Reduce 16 per-lane values over the 32 lanes of each wave half (lanes with
// the same l >> 5) with an associative, commutative operation.  On return,
// lane l holds the result for value index q = (l & 15) of its half (lanes l
// and l ^ 16 hold the same q).  Butterfly transpose-reduce: 8 + 4 + 2 + 1
// exchanges, then one full exchange across bit 4.
struct OpSum {
    __device__ float operator()(float a, float b) const { return a + b; }
};
struct OpMax {
    __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};

template <class Op>
__device__ __forceinline__ float half_transpose_reduce16(const float (&v)[16], int lane, Op op) {
    float a8[8];
    {
        const bool up = (lane & 8) != 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float send = up ? v[i] : v[i + 8];
            float keep = up ? v[i + 8] : v[i];
            a8[i] = op(keep, shfl_xor_f(send, 8));
        }
    }
    float a4[4];
    {
        const bool up = (lane & 4) != 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float send = up ? a8[i] : a8[i + 4];
            float keep = up ? a8[i + 4] : a8[i];
            a4[i] = op(keep, shfl_xor_f(send, 4));
        }
    }
    float a2[2];
    {
        const bool up = (lane & 2) != 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float send = up ? a4[i] : a4[i + 2];
            float keep = up ? a4[i + 2] : a4[i];
            a2[i] = op(keep, shfl_xor_f(send, 2));
        }
    }
    float a1;
    {
        const bool up = (lane & 1) != 0;
        float send = up ? a2[0] : a2[1];
        float keep = up ? a2[1] : a2[0];
        a1 = op(keep, shfl_xor_f(send, 1));
    }
    return op(a1, shfl_xor_f(a1, 16));
}

__device__ __forceinline__ float half_transpose_sum16(const float (&v)[16], int lane) {
    return half_transpose_reduce16(v, lane, OpSum());
}

// (max, sum of 2^(s - max)) pairs in log2 units.
__device__ __forceinline__ void lse_merge(float& m, float& s, float m2, float s2) {
    float M = fmaxf(m, m2);
    s = s * fast_exp2(m - M) + s2 * fast_exp2(m2 - M);
    m = M;
}

// Same butterfly for (max, sum) pairs.
__device__ __forceinline__ void half_transpose_lse16(const float (&m)[16], const float (&s)[16], int lane,
                                                     float& mo, float& so) {
    float m8[8], s8[8];
    {
        const bool up = (lane & 8) != 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float sm = up ? m[i] : m[i + 8], ss = up ? s[i] : s[i + 8];
            float km = up ? m[i + 8] : m[i], ks = up ? s[i + 8] : s[i];
            float rm = shfl_xor_f(sm, 8), rs = shfl_xor_f(ss, 8);
            lse_merge(km, ks, rm, rs);
            m8[i] = km;
            s8[i] = ks;
        }
    }
    float m4[4], s4[4];
    {
        const bool up = (lane & 4) != 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float sm = up ? m8[i] : m8[i + 4], ss = up ? s8[i] : s8[i + 4];
            float km = up ? m8[i + 4] : m8[i], ks = up ? s8[i + 4] : s8[i];
            float rm = shfl_xor_f(sm, 4), rs = shfl_xor_f(ss, 4);
            lse_merge(km, ks, rm, rs);
            m4[i] = km;
            s4[i] = ks;
        }
    }
    float m2[2], s2[2];
    {
        const bool up = (lane & 2) != 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float sm = up ? m4[i] : m4[i + 2], ss = up ? s4[i] : s4[i + 2];
            float km = up ? m4[i + 2] : m4[i], ks = up ? s4[i + 2] : s4[i];
            float rm = shfl_xor_f(sm, 2), rs = shfl_xor_f(ss, 2);
            lse_merge(km, ks, rm, rs);
            m2[i] = km;
            s2[i] = ks;
        }
    }
    float m1, s1;
    {
        const bool up = (lane & 1) != 0;
        float sm = up ? m2[0] : m2[1], ss = up ? s2[0] : s2[1];
        m1 = up ? m2[1] : m2[0];
        s1 = up ? s2[1] : s2[0];
        float rm = shfl_xor_f(sm, 1), rs = shfl_xor_f(ss, 1);
        lse_merge(m1, s1, rm, rs);
    }
    float rm = shfl_xor_f(m1, 16), rs = shfl_xor_f(s1, 16);
    lse_merge(m1, s1, rm, rs);
    mo = m1;
    so = s1;
}

// Row index within a 32x32 MFMA output tile for accumulator register q of
// lane l: rows 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32.
__device__ __forceinline__ int acc_row(int q, int lane) { return 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3); }

// Map a linear workgroup id to a tile id so that workgroups resident on the
// same XCD (dispatched round-robin, id % 8) take consecutive tiles.
__device__ __forceinline__ int xcd_remap(int wg, int ntiles) {
    const int X = 8;
    int per = ntiles / X;              // full share per XCD
    int full = per * X;
    if (wg >= full) return wg;         // ragged tail keeps identity order
    return (wg % X) * per + wg / X;
}

// Work-group -> (row tile, column tile).  After the XCD remap each XCD walks
// a contiguous range of a grouped raster: TILE_GROUP row tiles side by side,
// then the next column tile, so the work-groups resident on one XCD at a time
// share a few row and column operand blocks in that XCD's L2 instead of each
// streaming its own row block from HBM.
constexpr int TILE_GROUP = 8;
__device__ __forceinline__ void tile_coords(int wg, int n_mt_r, int n_mt_c, int& rb, int& cb) {
    const int t = xcd_remap(wg, n_mt_r * n_mt_c);
    const int per_group = TILE_GROUP * n_mt_c;
    const int grp = t / per_group;
    const int gsize = min(TILE_GROUP, n_mt_r - grp * TILE_GROUP);
    const int w = t - grp * per_group;
    cb = w / gsize;
    rb = grp * TILE_GROUP + (w - cb * gsize);
}
