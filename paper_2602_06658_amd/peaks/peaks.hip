// Instruction-rate microbenchmark for gfx950: the unit rates the roofline of
// the Sinkhorn pass is derived from.  Built as its own library
// (libgwpeaks.so), not part of libgwmi.so.
//
// Each probe is a register-only kernel: 8192 work-groups of 256 threads
// (4 waves), every wave runs independent dependency chains so that issue,
// not latency, limits the rate.  The host times each probe with HIP events
// after one warm-up launch and reports operations per second:
//   fma      v_fma_f32 (non-packed; packed FP32 is disabled in this build)
//   exp_sub  v_exp_f32 followed by one v_sub_f32 (x <- 2^x - 1.5, which
//            stays near its fixed point -1.05)
//   entry    the stabilised pass's per-entry VALU work: one 2^x and two
//            adds (a row and a column sum) per value
//   mfma_bf16  v_mfma_f32_32x32x16_bf16 (32768 flops each)
//   mfma_f32   v_mfma_f32_32x32x2f32   (4096 flops each)
// and the shader clock over the fma probe (s_memtime cycles against the
// 100 MHz s_memrealtime counter).
//
// gwp_overlap times whether the matrix unit and the VALU of a SIMD work at
// the same time, on the stabilised BF16 pass's instruction mix per wave and
// step: two dependent chains of five v_mfma_f32_32x32x16_bf16 and 32 entries
// of one 2^x and two adds.  Four forms at two waves per SIMD (64 KiB of
// dynamic LDS per work-group): MFMA work alone, VALU work alone, both in
// every wave, and half the work-groups doing twice the MFMA work while the
// other half do twice the VALU work.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int BLOCKS = 8192;
constexpr int THREADS = 256;

typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(THREADS) void k_fma(int iters, float* sink, unsigned long long* clk) {
    float v[8];
    const float s = 1.0f + 1e-7f * (float)threadIdx.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (float)k * 0.1f;
    unsigned long long c0 = 0, w0 = 0;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = __builtin_fmaf(v[k], s, -0.5f);
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - w0;
    }
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
    if (acc == 12345.0f) sink[threadIdx.x] = acc;
}

__global__ __launch_bounds__(THREADS) void k_exp_sub(int iters, float* sink) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = -1.0f - 0.01f * (float)k - 1e-6f * (float)threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_exp2f(v[k]) - 1.5f;
    }
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
    if (acc == 12345.0f) sink[threadIdx.x] = acc;
}

// 16 values per lane stand for one lane's share of a 32x32 tile; each is
// exponentiated and added into a row sum and a column sum, as in the pass.
// The exponent of the next value is minus the column sum (a free source
// modifier), so the chains stay finite (they grow like log2 of the count)
// and nothing is loop-invariant.
__global__ __launch_bounds__(THREADS) void k_entry(int iters, float* sink) {
    float rs[4] = {0.f, 0.f, 0.f, 0.f}, cs[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) cs[k] = 1.0f + 0.03f * (float)k + 1e-6f * (float)threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float e = __builtin_amdgcn_exp2f(-cs[k]);
            rs[k & 3] += e;
            cs[k] += e;
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += cs[k];
    acc += rs[0] + rs[1] + rs[2] + rs[3];
    if (acc == 12345.0f) sink[threadIdx.x] = acc;
}

__global__ __launch_bounds__(THREADS) void k_mfma_bf16(int iters, float* sink) {
    bf16x8_t a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(0.001f * (float)(threadIdx.x + k));
        b[k] = (__bf16)(0.002f * (float)(k + 1));
    }
    f32x16_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (f32x16_t)0.0f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[q], 0, 0, 0);
    }
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) t += acc[q][e];
    if (t == 12345.0f) sink[threadIdx.x] = t;
}

__global__ __launch_bounds__(THREADS) void k_mfma_f32(int iters, float* sink) {
    const float a = 0.001f * (float)threadIdx.x, b = 0.5f;
    f32x16_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (f32x16_t)0.0f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[q], 0, 0, 0);
    }
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) t += acc[q][e];
    if (t == 12345.0f) sink[threadIdx.x] = t;
}

// MODE 0: MFMA only; 1: VALU only; 2: both in every wave; 3: even work-groups
// MFMA (twice), odd ones VALU (twice)
template <int MODE>
__global__ __launch_bounds__(THREADS) void k_mix(int iters, float* sink) {
    bf16x8_t a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(0.001f * (float)(threadIdx.x + k));
        b[k] = (__bf16)(0.002f * (float)(k + 1));
    }
    f32x16_t acc[2];
    acc[0] = (f32x16_t)0.0f;
    acc[1] = (f32x16_t)0.0f;
    float rs[4] = {0.f, 0.f, 0.f, 0.f}, cs[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) cs[k] = 1.0f + 0.03f * (float)k + 1e-6f * (float)threadIdx.x;
    const bool do_m = MODE == 0 || MODE == 2 || (MODE == 3 && !(blockIdx.x & 1));
    const bool do_v = MODE == 1 || MODE == 2 || (MODE == 3 && (blockIdx.x & 1));
    const int reps = MODE == 3 ? 2 : 1;
    for (int i = 0; i < iters * reps; ++i) {
        if (do_m) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int s = 0; s < 5; ++s) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
        }
        if (do_v) {
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const float e = __builtin_amdgcn_exp2f(-cs[k]);
                rs[k & 3] += e;
                cs[k] += e;
            }
        }
    }
    float t = rs[0] + rs[1] + rs[2] + rs[3];
#pragma unroll
    for (int k = 0; k < 32; ++k) t += cs[k];
#pragma unroll
    for (int q = 0; q < 16; ++q) t += acc[0][q] + acc[1][q];
    if (t == 12345.0f) sink[threadIdx.x] = t;
}

template <class F>
int timed(F launch, float* ms_out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    launch();  // warm-up
    if (hipEventRecord(e0, nullptr) != hipSuccess) return -1;
    launch();
    if (hipEventRecord(e1, nullptr) != hipSuccess) return -1;
    if (hipEventSynchronize(e1) != hipSuccess) return -1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" {

// out[0] fma/s, out[1] (exp2 + sub)/s, out[2] entries/s of the pass's VALU
// mix, out[3] BF16 MFMA flop/s, out[4] FP32 MFMA flop/s, out[5] shader
// clock in Hz.  Runs on the current device's null stream; returns 0, or -1
// on a HIP error.
int gwp_measure(double* out) {
    float* sink = nullptr;
    unsigned long long* clk = nullptr;
    if (hipMalloc(&sink, THREADS * sizeof(float)) != hipSuccess) return -1;
    if (hipMalloc(&clk, 2 * sizeof(unsigned long long)) != hipSuccess) return -1;
    const double threads = (double)BLOCKS * THREADS;
    float ms = 0.f;
    int rc = 0;
    const int it_fma = 2048;
    rc |= timed([&] { k_fma<<<BLOCKS, THREADS>>>(it_fma, sink, clk); }, &ms);
    out[0] = threads * it_fma * 16 * 8 / (ms * 1e-3);
    unsigned long long hc[2] = {0, 0};
    rc |= hipMemcpy(hc, clk, sizeof(hc), hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
    out[5] = hc[1] ? (double)hc[0] / (double)hc[1] * 1e8 : 0.0;
    const int it_exp = 512;
    rc |= timed([&] { k_exp_sub<<<BLOCKS, THREADS>>>(it_exp, sink); }, &ms);
    out[1] = threads * it_exp * 16 * 8 / (ms * 1e-3);
    const int it_ent = 4096;
    rc |= timed([&] { k_entry<<<BLOCKS, THREADS>>>(it_ent, sink); }, &ms);
    out[2] = threads * it_ent * 16 / (ms * 1e-3);
    const int it_mm = 256;
    rc |= timed([&] { k_mfma_bf16<<<BLOCKS, THREADS>>>(it_mm, sink); }, &ms);
    out[3] = (double)BLOCKS * (THREADS / 64) * it_mm * 4 * 32768.0 / (ms * 1e-3);
    rc |= timed([&] { k_mfma_f32<<<BLOCKS, THREADS>>>(it_mm, sink); }, &ms);
    out[4] = (double)BLOCKS * (THREADS / 64) * it_mm * 4 * 4096.0 / (ms * 1e-3);
    (void)hipFree(sink);
    (void)hipFree(clk);
    return rc ? -1 : 0;
}

// out[0..3]: milliseconds of the four k_mix forms (MFMA alone, VALU alone,
// both in every wave, split across work-groups), 4096 work-groups of 256
// threads, 512 steps each.  Returns 0, or -1 on a HIP error.
int gwp_overlap(double* out) {
    float* sink = nullptr;
    if (hipMalloc(&sink, THREADS * sizeof(float)) != hipSuccess) return -1;
    constexpr int MIX_BLOCKS = 4096, MIX_ITERS = 512;
    constexpr size_t LDS = 64 * 1024;  // two work-groups (two waves per SIMD) per CU
    int rc = 0;
    rc |= hipFuncSetAttribute((const void*)k_mix<0>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS) == hipSuccess ? 0 : -1;
    rc |= hipFuncSetAttribute((const void*)k_mix<1>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS) == hipSuccess ? 0 : -1;
    rc |= hipFuncSetAttribute((const void*)k_mix<2>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS) == hipSuccess ? 0 : -1;
    rc |= hipFuncSetAttribute((const void*)k_mix<3>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS) == hipSuccess ? 0 : -1;
    float ms = 0.f;
    rc |= timed([&] { k_mix<0><<<MIX_BLOCKS, THREADS, LDS>>>(MIX_ITERS, sink); }, &ms);
    out[0] = ms;
    rc |= timed([&] { k_mix<1><<<MIX_BLOCKS, THREADS, LDS>>>(MIX_ITERS, sink); }, &ms);
    out[1] = ms;
    rc |= timed([&] { k_mix<2><<<MIX_BLOCKS, THREADS, LDS>>>(MIX_ITERS, sink); }, &ms);
    out[2] = ms;
    rc |= timed([&] { k_mix<3><<<MIX_BLOCKS, THREADS, LDS>>>(MIX_ITERS, sink); }, &ms);
    out[3] = ms;
    (void)hipFree(sink);
    return rc ? -1 : 0;
}

}  // extern "C"
