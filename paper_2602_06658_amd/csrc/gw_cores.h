// MFMA tile cores, LDS chunk staging and the mode gate shared by the pass,
// covariance and gradient kernels.
#pragma once

#include "gw_device.h"

namespace gwk {

using namespace gwl;

// ---------------------------------------------------------------------------
// MFMA cores: a 32x32 tile of s from packed operands.
// ---------------------------------------------------------------------------

template <int KS>
struct CoreBF16 {
    static constexpr int UNITS = KS;  // 16-byte units per lane per chunk
    struct A {
        bf16x8_t v[KS];
    };
    __device__ static void load(A& a, const uint4* pack, int chunk, int lane) {
        const uint4* p = pack + (size_t)chunk * KS * 64 + lane;
#pragma unroll
        for (int s = 0; s < KS; ++s) a.v[s] = __builtin_bit_cast(bf16x8_t, p[s * 64]);
    }
    struct B {
        bf16x8_t v[KS];
    };
    __device__ static void load_b(B& b, const uint4* lds, int lane) {
#pragma unroll
        for (int s = 0; s < KS; ++s) b.v[s] = __builtin_bit_cast(bf16x8_t, lds[s * 64 + lane]);
    }
    // s = X Zs^T from register fragments of both operands.
    __device__ static f32x16_t tile_ab(const A& a, const B& b) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[s], b.v[s], acc, 0, 0, 0);
        return acc;
    }
    // s = X Zs^T: lane l gets column l % 32, rows acc_row(q, l).
    __device__ static f32x16_t tile(const A& a, const uint4* lds, int lane) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[s], __builtin_bit_cast(bf16x8_t, lds[s * 64 + lane]),
                                                          acc, 0, 0, 0);
        return acc;
    }
    // s^T = Zs X^T: lane l gets row l % 32, columns acc_row(q, l).
    __device__ static f32x16_t tileT(const A& a, const uint4* lds, int lane) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, lds[s * 64 + lane]), a.v[s],
                                                          acc, 0, 0, 0);
        return acc;
    }
};

// The last group is the bias unit; its k slots 6 and 7 are zero in both
// operands (write_bias_a_f32 / write_bias_b_f32), so its fourth slab is not
// issued: 4 KG - 1 MFMAs per tile, and the sums are the same bit for bit.
template <int KG>
struct CoreF32 {
    static constexpr int UNITS = KG;  // groups of four 32x32x2 slabs
    __device__ static constexpr bool issued(int g, int e) { return !(g == KG - 1 && e == 3); }
    struct A {
        f32x4_t v[KG];
    };
    __device__ static void load(A& a, const uint4* pack, int chunk, int lane) {
        const uint4* p = pack + (size_t)chunk * KG * 64 + lane;
#pragma unroll
        for (int g = 0; g < KG; ++g) a.v[g] = __builtin_bit_cast(f32x4_t, p[g * 64]);
    }
    struct B {
        f32x4_t v[KG];
    };
    __device__ static void load_b(B& b, const uint4* lds, int lane) {
#pragma unroll
        for (int g = 0; g < KG; ++g) b.v[g] = __builtin_bit_cast(f32x4_t, lds[g * 64 + lane]);
    }
    __device__ static f32x16_t tile_ab(const A& a, const B& b) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (issued(g, e)) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[g][e], b.v[g][e], acc, 0, 0, 0);
        return acc;
    }
    __device__ static f32x16_t tile(const A& a, const uint4* lds, int lane) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            f32x4_t b = __builtin_bit_cast(f32x4_t, lds[g * 64 + lane]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (issued(g, e)) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[g][e], b[e], acc, 0, 0, 0);
        }
        return acc;
    }
    __device__ static f32x16_t tileT(const A& a, const uint4* lds, int lane) {
        f32x16_t acc = (f32x16_t)0.0f;
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            f32x4_t b = __builtin_bit_cast(f32x4_t, lds[g * 64 + lane]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (issued(g, e)) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b[e], a.v[g][e], acc, 0, 0, 0);
        }
        return acc;
    }
};

// token: the half-step's number (never 0), which a successful combine stores
// in CTL_DONE so that the safe kernels of the same half-step skip
__device__ __forceinline__ bool should_run(const int* ctl, int run_if, int token) {
    if (run_if == RUN_ALWAYS) return true;
    const int mode = ctl[CTL_MODE];
    if (run_if == RUN_STAB) return mode == MODE_STAB;
    return ctl[CTL_DONE] != token && (mode == MODE_SAFE || ctl[CTL_BAD] != 0);  // RUN_SAFE_OR_RETRY
}

// Cooperative copy of one 32-column chunk of the B pack into LDS, staged
// through registers so the load of chunk c+1 overlaps the compute of c.
// Every thread moves FULL units; the first REM threads move one more.  The
// registers are separate scalars so none of them is demoted to scratch.
template <int NU>
struct ChunkStage {
    using v4 = unsigned __attribute__((ext_vector_type(4)));
    static constexpr int FULL = NU / THREADS, REM = NU % THREADS;
    v4 r[FULL > 0 ? FULL : 1];
    v4 t;
    __device__ __forceinline__ void load(const uint4* src_, int tid) {
        const v4* src = reinterpret_cast<const v4*>(src_);
#pragma unroll
        for (int k = 0; k < FULL; ++k) r[k] = src[tid + k * THREADS];
        if (REM > 0 && tid < REM) t = src[FULL * THREADS + tid];
    }
    __device__ __forceinline__ void store(uint4* dst_, int tid) const {
        v4* dst = reinterpret_cast<v4*>(dst_);
#pragma unroll
        for (int k = 0; k < FULL; ++k) dst[tid + k * THREADS] = r[k];
        if (REM > 0 && tid < REM) dst[FULL * THREADS + tid] = t;
    }
};

}  // namespace gwk
