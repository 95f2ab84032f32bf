// Host runtime of the CNT-GW library: context, workspace and the solver
// state machine (one Algorithm 1 solve).  Shared by the C ABI and the
// serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gw.h"
#include "gw_kernels.h"
#include "gw_layout.h"
#include "gw_prep.h"

namespace gwr {

struct Status {
    gw_status code = GW_OK;
    std::string msg;
    static Status ok() { return Status(); }
    bool good() const { return code == GW_OK; }
};
Status fail(gw_status c, const std::string& m);
Status hip_fail(hipError_t e, const char* where);

#define GW_HIP(call)                                      \
    do {                                                  \
        hipError_t e__ = (call);                          \
        if (e__ != hipSuccess) return hip_fail(e__, #call); \
    } while (0)
#define GW_TRY(expr)                     \
    do {                                 \
        Status s__ = (expr);             \
        if (!s__.good()) return s__;     \
    } while (0)

// Grow-only device buffers addressed by name, with a byte limit.
class Workspace {
   public:
    explicit Workspace(size_t limit = 0) : limit_(limit) {}
    ~Workspace();
    // Returns nullptr (and sets status) when the limit would be exceeded or
    // the allocation fails.
    void* get(const std::string& name, size_t bytes, Status* st);
    template <class T>
    T* get_t(const std::string& name, size_t count, Status* st) {
        return (T*)get(name, count * sizeof(T), st);
    }
    void release_all();
    void release_prefix(const std::string& prefix);
    size_t total() const { return total_; }
    size_t limit() const { return limit_; }
    void set_limit(size_t l) { limit_ = l; }
    // Arena mode: buffers are carved from the caller's [base, base + bytes)
    // in request order (256-byte aligned) instead of allocated, and never
    // freed; get() fails with GW_ENOMEM when the arena is exhausted.
    void use_arena(void* base, size_t bytes) {
        arena_ = (char*)base;
        arena_bytes_ = bytes;
        arena_used_ = 0;
    }
    size_t arena_used() const { return arena_used_; }

   private:
    struct Buf {
        void* p = nullptr;
        size_t bytes = 0;
        bool owned = true;
    };
    std::map<std::string, Buf> bufs_;
    size_t total_ = 0;
    size_t limit_ = 0;
    char* arena_ = nullptr;
    size_t arena_bytes_ = 0, arena_used_ = 0;
};

// Frozen landmark kernel PCA of one side (GW_PEN_POWER).
struct Landmarks {
    bool fitted = false;
    int n_l = 0;       // landmarks
    int d_in = 0;      // input dimension
    int dim = 0;       // lifted dimension D
    float* pts = nullptr;   // n_l x d_in (device)
    float* W = nullptr;     // n_l x D: -V_ld / (2 sqrt(lambda_d)), 0 for dropped
    float* chat = nullptr;  // n_l: landmark column means of the cost
    float* sumW = nullptr;  // D: sum_l W_ld
    double cbarbar = 0.0;   // grand mean of the landmark cost
    std::vector<double> lambda;  // eigenvalues kept (host copy, diagnostics)
};

struct SideCfg {
    int kind = GW_PEN_SQEUCLID;
    double p = 1.0;
    int lifted_dim = 0;
    int n_landmarks = 0;
    uint64_t seed = 0;
    std::vector<int64_t> explicit_idx;
    Landmarks lm;
};

// Event pairs around kernel launches, resolved on demand.
class Profiler {
   public:
    bool on = false;
    void begin(int cls, hipStream_t s);
    void end(hipStream_t s);
    // resolves recorded pairs into the totals (synchronises the stream)
    Status collect(hipStream_t s);
    void reset();
    ~Profiler();
    int64_t launches[GW_PROF_CLASSES] = {};
    double ms[GW_PROF_CLASSES] = {};
    // intervals under IDLE_MS (mode-gated launches at large sizes)
    static constexpr float IDLE_MS = 0.02f;
    int64_t idle_launches[GW_PROF_CLASSES] = {};
    double idle_ms[GW_PROF_CLASSES] = {};
    int64_t entries = 0;

   private:
    struct Pair {
        hipEvent_t a, b;
        int cls;
    };
    hipEvent_t take();
    std::vector<Pair> pairs_;
    std::vector<hipEvent_t> pool_;
    Pair cur_{};
};

class Solve;

struct Ctx {
    Profiler prof;
    int device = 0;
    hipStream_t stream = nullptr;
    Workspace ws;
    std::string err;
    SideCfg side[2];
    void* rocblas = nullptr;  // rocblas_handle, created on first eigensolve
    std::mutex mu;
    // The solve of the stepwise entry points (gw_solve_begin / advance /
    // end), kept between calls; its buffers carry their own name prefix.
    std::unique_ptr<Solve> stepped;
    // Pinned host staging for result readback, grown on demand; bytes = 0
    // returns the current buffer.
    void* host_stage(size_t bytes, Status* st);
    // Use the caller's host buffer for readback instead (never grown or
    // freed; a request beyond it fails).
    void set_host_stage(void* p, size_t bytes) {
        stage_ = p;
        stage_bytes_ = bytes;
        stage_owned_ = false;
    }
    // The first k (at most SIDE_STREAMS) streams on which one call runs
    // independent solves side by side; created on first use, default
    // priority, destroyed with the context.
    static constexpr int SIDE_STREAMS = 3;
    Status side_streams(int k, hipStream_t* out);
    ~Ctx();

   private:
    hipStream_t side_[SIDE_STREAMS] = {};
    void* stage_ = nullptr;
    size_t stage_bytes_ = 0;
    bool stage_owned_ = true;
};

int feature_dim(const SideCfg& s, int d);

// Lift points of one side into centred features X (n_pad x D, padded rows
// zero).  Fits landmarks on first use for GW_PEN_POWER.
Status lift_side(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                 const std::string& tag);

// Device check of nx values of x (finite) and nw weights (finite, > 0,
// summing to 1 within 1e-6, FP64 sum); waits for the result.
Status check_points(Ctx& c, const float* x, int64_t nx, const float* w, int64_t nw, const std::string& tag,
                    const char* what);

// Host-side validation of a problem; launches the device checks and waits.
Status validate_inputs(Ctx& c, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                       const float* b, const gw_params* prm, const std::string& tag);

// One Algorithm 1 solve as a resumable state machine.
class Solve {
   public:
    Solve(Ctx& c, const std::string& tag) : c_(c), tag_(tag) {}
    Status setup(const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                 const float* b, const gw_params& prm, const float* gamma0, const float* f0, const float* g0,
                 int pen_src, int pen_tgt, hipStream_t stream);
    // Enqueue outer step t (prologue, n_inner Sinkhorn iterations,
    // covariance).  Returns false when the solve has finished.
    Status outer_step();
    bool done() const { return done_; }
    int outer_done() const { return t_; }
    // FP64 final check and result readback (blocks on the stream) =
    // finish_enqueue, a wait for the stream, finish_collect.  The split form
    // lets a caller wait on an event instead (serving loop).
    Status finish(gw_result* out);
    Status finish_enqueue(gw_result* out);
    Status finish_collect(gw_result* out);
    // Move the solve's later work to another stream (after an event on the
    // old one has been made a dependency of the new one).
    void set_stream(hipStream_t s) { st_ = s; }
    // Gradients of the final state (after finish).
    Status gradients(float* grad_x, float* grad_a, float* grad_y, float* grad_b);

    // Stepwise control (serving loop): outer_step() is begin_outer(),
    // n_inner inner_iteration() calls, end_outer().
    Status begin_outer();
    // Before inner iteration k of the current outer step (the annealing of
    // the last step re-tempers the operands here); then inner_iteration(k).
    Status before_inner(int k);
    Status inner_iteration(int k);
    Status end_outer();
    // Symmetric MFMA-path solves can run their Sinkhorn iterations in the
    // batched kernels: the arguments of the current iteration, then
    // advance_parity() once it is enqueued.
    bool batchable() const { return geo_.path == 0 && prm_.symmetric != 0; }
    void iteration_items(gwk::PassItem& item, gwk::CombineArgs& main, gwk::CombineArgs& retry, int** ctl);
    void advance_parity() {
        pa_ ^= 1;
        pb_ ^= 1;
    }
    int n_inner() const { return n_inner_cur_; }
    // Device bytes of the solve's buffers for these sizes (nothing allocated);
    // 0 if the sizes are rejected.
    static size_t plan_bytes(Ctx& c, int64_t n, int dx, int64_t m, int dy, const gw_params& prm);
    size_t footprint() const { return footprint_; }
    int64_t n() const { return n_; }
    int64_t m() const { return m_; }
    double entries_per_outer() const { return (double)n_ * (double)m_ * prm_.n_inner; }

   private:
    Status prologue(int first);
    Status enqueue_check();
    Status adaptive_step();
    Status configure(int64_t n, int dx, int64_t m, int dy, const gw_params& prm);
    Status buffers(bool dry = false);
    void make_half(int do_rows, int do_cols, float step, gwk::Operands& op, gwk::CombineArgs& ca);
    Status covariance(int rows_side, float* T_out, float* r_out, float* rm_out);
    Status side_gradient(int side, float* grad_pos, float* grad_w);

    Ctx& c_;
    std::string tag_;
    hipStream_t st_ = nullptr;
    gw_params prm_{};
    int64_t n_ = 0, m_ = 0, n_pad_ = 0, m_pad_ = 0;
    int dx_ = 0, dy_ = 0, D_ = 0, E_ = 0;
    int prec_ = 0;
    int pen_[2] = {0, 0};
    const float* x_ = nullptr;
    const float* y_ = nullptr;
    const float* a_ = nullptr;
    const float* b_ = nullptr;
    gwk::Geometry geo_{};
    int cov_rg_ = 1, cov_bc_ = 1, cov_mtr_ = 1, cov_mtc_ = 1;
    // covariance with the target as the row operand (gradient of the target)
    int cov2_rg_ = 1, cov2_bc_ = 1, cov2_mtr_ = 1, cov2_mtc_ = 1, cov2_tw_ = 0;
    int t_ = 0;
    bool done_ = false;
    int pa_ = 0, pb_ = 0;      // pack / potential parities
    int half_token_ = 0;       // number of the last half-step issued (launch gates)
    double eps_t_ = 0.0, kappa_ = 0.0;
    double asum_ = 1.0, bsum_ = 1.0;
    size_t footprint_ = 0;
    std::vector<double> eps_sched_;
    // device buffers
    float *X_ = nullptr, *Y_ = nullptr, *xn_ = nullptr, *ym_ = nullptr, *la2_ = nullptr, *lb2_ = nullptr;
    void* packA_[2] = {nullptr, nullptr};
    void* packB_[2] = {nullptr, nullptr};
    // BF16 form: covariance payload packs (Y for source rows, X for target rows)
    void* pwY_ = nullptr;
    void* pwX_ = nullptr;
    // potentials in log2 units as FP32 (hi, lo) pairs, two parities
    float *U_[2] = {nullptr, nullptr}, *V_[2] = {nullptr, nullptr};
    float *Ul_[2] = {nullptr, nullptr}, *Vl_[2] = {nullptr, nullptr};
    float *Zs_ = nullptr, *ms_ = nullptr;
    double* beta_ = nullptr;
    float *f_ = nullptr, *g_ = nullptr;  // warm-start input / output staging
    bool have_init_ = false;
    double kappa_old_ = 0.0;
    float *gam_[2] = {nullptr, nullptr};
    int gcur_ = 0;
    double* gam64_ = nullptr;
    float *rp_ = nullptr, *rp2_ = nullptr, *cp_ = nullptr, *cp2_ = nullptr;
    float *Tp_ = nullptr, *crp_ = nullptr, *crmp_ = nullptr;
    float *T_ = nullptr, *rsum_ = nullptr, *rm_ = nullptr;
    double* part_ = nullptr;
    double* scal_ = nullptr;
    int* ctl_ = nullptr;
    double *momx_ = nullptr, *momy_ = nullptr, *mompart_ = nullptr;
    double* chk_ = nullptr;  // FP64 check partials (MFMA path)
    double *r64_ = nullptr, *kl64_ = nullptr, *c64_ = nullptr;  // FP64 check sums
    int cov_tw_ = 0;
    // adaptive Sinkhorn counts (Algorithm 6)
    int n_inner_cur_ = 0, doublings_ = 0;
    bool gamma0_given_ = false, have_prev_ = false, have_c_ = false;
    double prev_loss_ = 0.0, prev_kl_ = 0.0, c_const_ = 0.0;
};

// The constant C(alpha, beta) of Lemma C.1 from the FP64 moments of both sides.
double lemma_c1_constant(const double* mx, int D, const double* my, int E);

}  // namespace gwr

// The opaque handle of the C ABI.
struct gw_ctx {
    gwr::Ctx c;
};

namespace gwr {
void release_landmarks(Ctx& c);
// Free one landmark map's device data and mark it unfitted.
void free_landmarks(Landmarks& lm);
Status lift_nystrom(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                    const std::string& tag);
// Fit both sides' landmark maps with one batched eigensolve when both use the
// power penalty unfitted with equal landmark counts; otherwise does nothing.
Status fit_landmarks_pair(Ctx& c, const float* x, int64_t n, int dx, const float* y, int64_t m, int dy,
                          const std::string& tag);
}  // namespace gwr

namespace gwr {
std::vector<int64_t> seeded_landmarks(int64_t n, int nl, uint64_t seed);
}  // namespace gwr

namespace gwr {
// One side's penalty (with its fitted landmark map) used on the other side
// too, for the self terms GW(alpha, alpha) and GW(beta, beta) of the
// divergence; restored on every exit path.  The copy shares the fitted
// landmark data, which only release_landmarks and a refit free, and a
// fitted copy is never refitted.
struct SideShare {
    Ctx& c;
    int dst;
    SideCfg saved;
    SideShare(Ctx& ctx, int src, int dst_) : c(ctx), dst(dst_) {
        saved = std::move(c.side[dst]);
        c.side[dst] = c.side[src];
    }
    ~SideShare() { c.side[dst] = std::move(saved); }
};

// The context's penalties replaced by "features" for solves that run on
// features lifted beforehand; restored on every exit path.  (SideCfg holds
// plain handles, so moving it out and back leaves fitted landmarks alone.)
struct FeatureSides {
    Ctx& c;
    SideCfg saved[2];
    explicit FeatureSides(Ctx& ctx) : c(ctx) {
        for (int s = 0; s < 2; ++s) {
            saved[s] = std::move(c.side[s]);
            c.side[s] = SideCfg{};
            c.side[s].kind = GW_PEN_FEATURES;
        }
    }
    ~FeatureSides() {
        for (int s = 0; s < 2; ++s) c.side[s] = std::move(saved[s]);
    }
};
}  // namespace gwr
