// Host-visible launch interface of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gw_layout.h"

namespace gwk {

// Work decomposition of an N x M pass: macro tiles of
// (rg * rows_per_group) rows x (bc_chunks * 32) columns.
struct Geometry {
    int path;            // 0: MFMA pack path, 1: VALU path (D < 16)
    int rows_per_group;  // rows one workgroup covers per row group
    int rg;              // row groups per macro tile
    int bc_chunks;       // 32-column chunks per macro tile
    int n_mt_r, n_mt_c;  // macro tiles along rows / columns
    int n_pad, m_pad;    // sizes padded to 32
};

// Operands of the passes.  MFMA path: packs A (rows) and B (columns) of
// the current parity.  VALU path: row-major features and the exponent terms.
struct Operands {
    int prec;            // gwl::Prec of the packs
    int d;               // feature dimension D (unpadded)
    const void* A;
    const void* B;
    // VALU path (direct form): s = U + V - kappa (|X - Z|^2 + (n - m)^2 / 4)
    const float* X;      // n_pad x d
    const float* xn;     // |X_i|^2, n_pad
    const float* U;      // row potentials log2 a_i + kappa f_i, FP32 hi part
    const float* Ul;     // ... and lo part
    const float* Zs;     // m_pad x d, Z_j = Gamma Y_j (unscaled)
    const float* ms;     // |Y_j|^2, m_pad
    const float* V;      // column potentials log2 b_j + kappa g_j, hi
    const float* Vl;     // ... lo
    float kappa;         // log2(e) * 8 / eps
    int token;           // half-step number, never 0 (launch gates)
};

struct Partials {
    float* row;          // [n_mt_c][n_pad]   (stabilised sums / safe maxima)
    float* row2;         // [n_mt_c][n_pad]   (safe sums)
    float* col;          // [n_mt_r][m_pad]
    float* col2;
};

Geometry pass_geometry(int prec, int d, int64_t n, int64_t m, int multiplier);

// One Sinkhorn pass: per-macro-tile row and column partial sums of
// pi_ij = 2^{s_ij}.  safe = 0: one exponential per entry; 1: max-shifted.
hipError_t launch_pass(const Operands& op, const Geometry& g, const Partials& p, int* ctl,
                       int run_if, int safe, hipStream_t stream);

// The same pass for several independent problems (MFMA path only), one
// launch per run of consecutive items that share a kernel instantiation
// (precision class and pack width), at most 16 problems per launch.
struct PassItem {
    Operands op;
    Geometry g;
    Partials pp;
    int* ctl;
};
hipError_t launch_pass_batch(const PassItem* items, int n, int run_if, int safe, hipStream_t stream);

struct CombineArgs {
    const float* rp;
    const float* rp2;
    const float* cp;
    const float* cp2;
    int n_mt_c, n_mt_r;
    int n, m, n_pad, m_pad;
    const float* la2;    // log2 a_i
    const float* lb2;    // log2 b_j
    const float* U_cur;   // potentials as FP32 (hi, lo) pairs
    const float* Ul_cur;
    const float* V_cur;
    const float* Vl_cur;
    float* U_next;
    float* Ul_next;
    float* V_next;
    float* Vl_next;
    void* packA_next;    // MFMA path: bias slots to refresh (nullptr on VALU path)
    void* packB_next;
    int prec, d;
    int do_rows, do_cols;
    float step;          // 0.5 (Algorithm 3) or 1.0 (Algorithm 2)
    int is_retry;
    int token;           // the half-step's number, as in Operands
};
hipError_t launch_combine(const CombineArgs& a, int* ctl, int run_if, hipStream_t stream);
// Combines of several independent problems, 16 per launch; ctls[r] is the
// control block of problem r.
hipError_t launch_combine_batch(const CombineArgs* items, int* const* ctls, int n, int run_if, hipStream_t stream);

// Control block initialisation for a solve: mode, user mode.
hipError_t launch_ctl_init(int* ctl, int user_mode, hipStream_t stream);

}  // namespace gwk
