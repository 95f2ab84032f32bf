// Host- and device-visible constants of the operand layouts and the
// per-iteration control block.
#pragma once

#include <stdint.h>

namespace gwl {

enum Prec { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

// Bias slots appended to the feature part of a packed operand.
constexpr int BIAS_BF16 = 16;
constexpr int BIAS_F32 = 8;

// Rows of one MFMA tile / pack chunk.
constexpr int TILE = 32;
constexpr int WAVES = 4;           // waves per workgroup in the pass kernels
constexpr int THREADS = 64 * WAVES;

// Control block words (device int array, one per solve slot).
enum Ctl {
    CTL_MODE = 0,        // mode of the current iteration: MODE_STAB / MODE_SAFE
    CTL_BAD = 1,         // stabilised pass out of range -> retry safe
    CTL_UNSAFE = 2,      // some ratio outside the comfort band -> next safe
    CTL_COUNT = 3,       // last-block counter of a combine
    CTL_NUMERIC = 4,     // sticky: non-finite values seen
    CTL_SAFE_ITERS = 5,  // iterations that ran the safe pass
    CTL_USER = 6,        // user mode: 0 auto, 1 safe, 2 stabilised
    CTL_DONE = 7,        // token of the last half-step whose combine succeeded
    CTL_WORDS = 8
};
enum Mode { MODE_STAB = 0, MODE_SAFE = 1 };
// Launch gates of a half-step: the stabilised pass and its combine run in
// stabilised mode; the safe pass and its combine run after them unless the
// half-step is already done, i.e. in safe mode or after a flagged
// stabilised combine.
enum RunIf { RUN_ALWAYS = 0, RUN_STAB = 1, RUN_SAFE_OR_RETRY = 2 };

// |log2 (marginal / weight)| above which a stabilised pass is redone safely,
// and above which the next iteration runs safely.
constexpr float STAB_LIMIT = 40.0f;
constexpr float COMFORT_LIMIT = 30.0f;

inline int pad_to(int v, int m) { return (v + m - 1) / m * m; }

// Feature dimension as stored in a pack: the next instantiated size.
inline int feat_pad(int d) {
    const int sizes[] = {16, 32, 48, 64, 96, 128, 192, 256};
    for (int s : sizes)
        if (d <= s) return s;
    return -1;
}
constexpr int MAX_DIM = 256;        // FP32 / BF16 packs
constexpr int MAX_DIM_BF16X3 = 128; // split-BF16 packs
constexpr int VALU_MAX_DIM = 15;    // D below this runs on the VALU path

// K of a packed operand.
inline int pack_k(int prec, int d) {
    int dp = feat_pad(d);
    if (prec == PREC_F32) return dp + BIAS_F32;
    if (prec == PREC_BF16) return dp + BIAS_BF16;
    return 3 * dp + BIAS_BF16;
}
// Number of 16-byte units per lane per 32-row chunk (bf16: slabs of 16 k;
// f32: groups of 4 slabs of 2 k).
inline int pack_units(int prec, int d) {
    int k = pack_k(prec, d);
    return prec == PREC_F32 ? k / 8 : k / 16;
}
// Bytes of a pack holding `rows` rows (padded to 32).
inline size_t pack_bytes(int prec, int d, int64_t rows) {
    int64_t chunks = (rows + TILE - 1) / TILE;
    return (size_t)chunks * pack_units(prec, d) * 64 * 16;
}

}  // namespace gwl
