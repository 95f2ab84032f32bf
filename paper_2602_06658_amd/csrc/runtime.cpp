// Host runtime: workspace, validation, lifting dispatch and the Algorithm 1
// state machine (Section 5).  All device work is ordered on one HIP stream;
// the host blocks only at validation and at the final scalar readback (and
// once per outer step when a Gamma tolerance is set).
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace gwr {

using namespace gwl;

Status fail(gw_status c, const std::string& m) {
    Status s;
    s.code = c;
    s.msg = m;
    return s;
}

Status hip_fail(hipError_t e, const char* where) {
    return fail(e == hipErrorOutOfMemory ? GW_ENOMEM : GW_EDEVICE,
                std::string(where) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Workspace
// ---------------------------------------------------------------------------

Workspace::~Workspace() { release_all(); }

void* Workspace::get(const std::string& name, size_t bytes, Status* st) {
    if (bytes == 0) bytes = 16;
    auto it = bufs_.find(name);
    if (it != bufs_.end() && it->second.bytes >= bytes) return it->second.p;
    if (arena_) {
        const size_t off = (arena_used_ + 255) / 256 * 256;
        if (off > arena_bytes_ || bytes > arena_bytes_ - off) {
            *st = fail(GW_ENOMEM, "scratch array of " + std::to_string(arena_bytes_) + " bytes exhausted at '" +
                                      name + "' (" + std::to_string(bytes) + " more bytes after " +
                                      std::to_string(off) + ")");
            return nullptr;
        }
        void* p = arena_ + off;
        if (it != bufs_.end()) {
            total_ -= it->second.bytes;
            bufs_.erase(it);
        }
        bufs_[name] = Buf{p, bytes, false};
        total_ += bytes;
        arena_used_ = off + bytes;
        return p;
    }
    size_t old = 0;
    if (it != bufs_.end()) old = it->second.bytes;
    if (limit_ && total_ - old + bytes > limit_) {
        *st = fail(GW_ENOMEM, "workspace limit exceeded allocating '" + name + "' (" + std::to_string(bytes) +
                                  " bytes, in use " + std::to_string(total_) + ", limit " + std::to_string(limit_) +
                                  ")");
        return nullptr;
    }
    if (it != bufs_.end()) {
        if (it->second.owned) (void)hipFree(it->second.p);
        total_ -= it->second.bytes;
        bufs_.erase(it);
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        *st = hip_fail(e, ("hipMalloc " + name).c_str());
        return nullptr;
    }
    bufs_[name] = Buf{p, bytes};
    total_ += bytes;
    return p;
}

void Workspace::release_all() {
    for (auto& kv : bufs_)
        if (kv.second.owned) (void)hipFree(kv.second.p);
    bufs_.clear();
    total_ = 0;
    arena_used_ = 0;
}

void Workspace::release_prefix(const std::string& prefix) {
    for (auto it = bufs_.begin(); it != bufs_.end();) {
        if (it->first.compare(0, prefix.size(), prefix) == 0) {
            if (it->second.owned) (void)hipFree(it->second.p);
            total_ -= it->second.bytes;
            it = bufs_.erase(it);
        } else {
            ++it;
        }
    }
}

// ---------------------------------------------------------------------------
// Profiler
// ---------------------------------------------------------------------------

void* Ctx::host_stage(size_t bytes, Status* st) {
    if (bytes > stage_bytes_ && !stage_owned_) {
        *st = fail(GW_ENOMEM, "host staging of " + std::to_string(stage_bytes_) + " bytes is too small");
        return nullptr;
    }
    if (bytes > stage_bytes_) {
        if (stage_) (void)hipHostFree(stage_);
        stage_ = nullptr;
        stage_bytes_ = 0;
        if (hipHostMalloc(&stage_, bytes, hipHostMallocDefault) != hipSuccess) {
            stage_ = nullptr;
            *st = fail(GW_ENOMEM, "pinned host staging");
            return nullptr;
        }
        stage_bytes_ = bytes;
    }
    return stage_;
}

Status Ctx::side_streams(int k, hipStream_t* out) {
    if (k < 1 || k > SIDE_STREAMS) return fail(GW_EINVAL, "side-by-side solves: 1 to 3 streams");
    for (int i = 0; i < k; ++i) {
        if (!side_[i]) GW_HIP(hipStreamCreateWithFlags(&side_[i], hipStreamNonBlocking));
        out[i] = side_[i];
    }
    return Status::ok();
}

Ctx::~Ctx() {
    stepped.reset();
    if (stage_ && stage_owned_) (void)hipHostFree(stage_);
    for (hipStream_t s : side_)
        if (s) (void)hipStreamDestroy(s);
}

hipEvent_t Profiler::take() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void Profiler::begin(int cls, hipStream_t s) {
    if (!on) return;
    cur_.a = take();
    cur_.b = take();
    cur_.cls = cls;
    (void)hipEventRecord(cur_.a, s);
}

void Profiler::end(hipStream_t s) {
    if (!on) return;
    (void)hipEventRecord(cur_.b, s);
    pairs_.push_back(cur_);
}

Status Profiler::collect(hipStream_t s) {
    GW_HIP(hipStreamSynchronize(s));
    for (auto& p : pairs_) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            ms[p.cls] += t;
            launches[p.cls] += 1;
            if (t < IDLE_MS) {
                idle_ms[p.cls] += t;
                idle_launches[p.cls] += 1;
            }
        }
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    pairs_.clear();
    return Status::ok();
}

void Profiler::reset() {
    for (auto& p : pairs_) {
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    pairs_.clear();
    for (int k = 0; k < GW_PROF_CLASSES; ++k) {
        launches[k] = 0;
        ms[k] = 0.0;
        idle_launches[k] = 0;
        idle_ms[k] = 0.0;
    }
}

Profiler::~Profiler() {
    reset();
    for (auto e : pool_) (void)hipEventDestroy(e);
}

#define GW_PROF(cls, call)               \
    do {                                 \
        c_.prof.begin((cls), st_);       \
        hipError_t pe__ = (call);        \
        c_.prof.end(st_);                \
        if (pe__ != hipSuccess) return hip_fail(pe__, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------

int feature_dim(const SideCfg& s, int d) {
    if (s.kind == GW_PEN_POWER) return s.lifted_dim;
    return d;
}

static Status check_params(const gw_params* prm) {
    if (!prm) return fail(GW_EINVAL, "params is NULL");
    if (!(prm->eps_start > 0.0) || !(prm->eps_end > 0.0) || !std::isfinite(prm->eps_start) ||
        !std::isfinite(prm->eps_end))
        return fail(GW_EINVAL, "eps must be finite and > 0");
    if (prm->n_outer < 1 || prm->n_inner < 1) return fail(GW_EINVAL, "n_outer and n_inner must be >= 1");
    if (prm->precision < 0 || prm->precision > 2) return fail(GW_EINVAL, "unknown precision");
    if (prm->mode < 0 || prm->mode > 2) return fail(GW_EINVAL, "unknown mode");
    if (prm->symmetric != 0 && prm->symmetric != 1) return fail(GW_EINVAL, "symmetric must be 0 or 1");
    if (!(prm->tol_gamma >= 0.0)) return fail(GW_EINVAL, "tol_gamma must be >= 0");
    if (prm->anneal_final != 0 && prm->anneal_final != 1) return fail(GW_EINVAL, "anneal_final must be 0 or 1");
    if (prm->adaptive_inner != 0 && prm->adaptive_inner != 1)
        return fail(GW_EINVAL, "adaptive_inner must be 0 or 1");
    return Status::ok();
}

static Status device_check(Ctx& c, const float* x, int64_t nx, const float* w, int64_t nw, const std::string& tag,
                           double* wsum, const char* what) {
    Status st;
    const int blocks = 64;
    int* flags = c.ws.get_t<int>(tag + "vflags", 4, &st);
    double* part = c.ws.get_t<double>(tag + "vpart", blocks, &st);
    if (!st.good()) return st;
    GW_HIP(hipMemsetAsync(flags, 0, sizeof(int), c.stream));
    GW_HIP(gwk::launch_validate(x, nx, w, nw, flags, part, blocks, c.stream));
    int hf = 0;
    std::vector<double> hp(blocks);
    GW_HIP(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipMemcpyAsync(hp.data(), part, blocks * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    GW_HIP(hipStreamSynchronize(c.stream));
    if (hf & 1) return fail(GW_EINVAL, std::string("non-finite value in ") + what);
    if (hf & 2) return fail(GW_EINVAL, std::string("weights of ") + what + " must be > 0");
    double s = 0.0;
    for (double v : hp) s += v;
    if (std::fabs(s - 1.0) > 1e-6)
        return fail(GW_EINVAL, std::string("weights of ") + what + " must sum to 1 within 1e-6");
    *wsum = s;
    return Status::ok();
}

Status check_points(Ctx& c, const float* x, int64_t nx, const float* w, int64_t nw, const std::string& tag,
                    const char* what) {
    double wsum = 0.0;
    return device_check(c, x, nx, w, nw, tag, &wsum, what);
}

Status validate_inputs(Ctx& c, const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                       const float* b, const gw_params* prm, const std::string& tag) {
    GW_TRY(check_params(prm));
    if (!x || !a || !y || !b) return fail(GW_EINVAL, "NULL input pointer");
    if (n < 1 || m < 1) return fail(GW_EINVAL, "n and m must be >= 1");
    if (n > (int64_t)1 << 30 || m > (int64_t)1 << 30) return fail(GW_EINVAL, "n or m too large");
    if (dx < 1 || dy < 1 || dx > MAX_DIM || dy > MAX_DIM) return fail(GW_EINVAL, "dimensions must be in [1, 256]");
    (void)tag;
    return Status::ok();
}

// ---------------------------------------------------------------------------
// Lifting (Section 3 squared-norm example / Section 5 CNT embeddings)
// ---------------------------------------------------------------------------

Status lift_nystrom(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                    const std::string& tag);

Status lift_side(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                 const std::string& tag) {
    const SideCfg& s = c.side[side];
    if (s.kind == GW_PEN_POWER) return lift_nystrom(c, side, x, n, d, w, X, n_pad, tag);
    Status st;
    double* part = c.ws.get_t<double>(tag + "cpart" + std::to_string(side), gwk::centre_part_doubles(n, d), &st);
    double* mean = c.ws.get_t<double>(tag + "cmean" + std::to_string(side), d, &st);
    if (!st.good()) return st;
    GW_HIP(gwk::launch_centre(x, n, n_pad, d, d, w, part, mean, X, c.stream));
    return Status::ok();
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------

static constexpr double LOG2E = 1.4426950408889634;

Status Solve::configure(int64_t n, int dx, int64_t m, int dy, const gw_params& prm) {
    n_ = n;
    m_ = m;
    D_ = feature_dim(c_.side[0], dx);
    E_ = feature_dim(c_.side[1], dy);
    if (D_ < 1 || E_ < 1 || D_ > MAX_DIM || E_ > MAX_DIM) return fail(GW_EINVAL, "lifted dimension out of range");
    prec_ = prm.precision;
    if (D_ <= VALU_MAX_DIM) prec_ = PREC_F32;  // no contraction worth MFMA
    if (prec_ == PREC_BF16X3 && D_ > MAX_DIM_BF16X3)
        return fail(GW_EUNSUPPORTED, "split-BF16 supports D <= 128");
    n_pad_ = (n + 31) / 32 * 32;
    m_pad_ = (m + 31) / 32 * 32;
    geo_ = gwk::pass_geometry(prec_, D_, n, m, 1);
    if (geo_.path == 1 && E_ > 16)
        return fail(GW_EUNSUPPORTED, "source dimension below 16 needs a target dimension of at most 16");

    // covariance geometry: one row group per macro tile, few column tiles
    // (about 2048 work-groups, each at least 1024 columns wide: every column
    // tile adds a partial per row that the reduction reads back); forward
    // (source rows, payload Y) and swapped (target rows, payload X)
    {
        const int path = geo_.path;
        auto geom = [&](int64_t rows_pad, int64_t cols_pad, int dw, int& rg, int& bc, int& mtr, int& mtc, int& tw) {
            const int rpg = gwk::cov_rows_per_group(path, prec_, D_, dw);
            rg = 1;
            mtr = (int)((rows_pad + rpg - 1) / rpg);
            const int nchc = (int)(cols_pad / 32);
            tw = gwk::cov_tw(path, dw);
            int want = std::max(1, (2048 + mtr - 1) / mtr);
            const size_t per_tile = (size_t)rows_pad * (tw + 2) * sizeof(float);
            const int mem_cap = (int)std::max<size_t>(1, ((size_t)1 << 30) / per_tile);
            // the VALU form (D < 16) has 512-row groups and a payload of at
            // most 16 columns, so its partials stay small: there the column
            // tile narrows to one 32-column chunk if the grid needs it (a
            // 3,000-row problem would otherwise run on a dozen work-groups)
            const int min_cols = path == 1 ? 1 : 32;
            want = std::min(want, std::min(mem_cap, std::max(1, nchc / min_cols)));
            bc = (nchc + want - 1) / want;
            mtc = (nchc + bc - 1) / bc;
        };
        geom(n_pad_, m_pad_, E_, cov_rg_, cov_bc_, cov_mtr_, cov_mtc_, cov_tw_);
        geom(m_pad_, n_pad_, D_, cov2_rg_, cov2_bc_, cov2_mtr_, cov2_mtc_, cov2_tw_);
    }
    return Status::ok();
}

size_t Solve::plan_bytes(Ctx& c, int64_t n, int dx, int64_t m, int dy, const gw_params& prm) {
    Solve s(c, "plan.");
    s.prm_ = prm;
    if (!s.configure(n, dx, m, dy, prm).good()) return 0;
    if (!s.buffers(true).good()) return 0;
    return s.footprint_;
}

Status Solve::setup(const float* x, int64_t n, int dx, const float* a, const float* y, int64_t m, int dy,
                    const float* b, const gw_params& prm, const float* gamma0, const float* f0, const float* g0,
                    int pen_src, int pen_tgt, hipStream_t stream) {
    st_ = stream;
    prm_ = prm;
    n_ = n;
    m_ = m;
    n_inner_cur_ = prm.n_inner;
    doublings_ = 0;
    gamma0_given_ = gamma0 != nullptr;
    have_prev_ = have_c_ = false;
    dx_ = dx;
    dy_ = dy;
    x_ = x;
    y_ = y;
    a_ = a;
    b_ = b;
    pen_[0] = pen_src;
    pen_[1] = pen_tgt;
    GW_TRY(configure(n, dx, m, dy, prm));
    GW_TRY(buffers());

    // weights: validation also gives their FP64 sums
    double asum = 1.0, bsum = 1.0;
    {
        Status s1 = device_check(c_, x, n * (int64_t)dx, a, n, tag_ + "va", &asum, "source");
        if (!s1.good()) return s1;
        Status s2 = device_check(c_, y, m * (int64_t)dy, b, m, tag_ + "vb", &bsum, "target");
        if (!s2.good()) return s2;
    }
    asum_ = asum;
    bsum_ = bsum;

    // lifting
    c_.prof.begin(GW_PROF_LIFT, st_);
    GW_TRY(fit_landmarks_pair(c_, x, n, dx, y, m, dy, tag_));
    GW_TRY(lift_side(c_, 0, x, n, dx, a, X_, n_pad_, tag_));
    GW_TRY(lift_side(c_, 1, y, m, dy, b, Y_, m_pad_, tag_));
    c_.prof.end(st_);
    GW_HIP(gwk::launch_norms_logw(X_, n, n_pad_, D_, a, asum, xn_, la2_, st_));
    GW_HIP(gwk::launch_norms_logw(Y_, m, m_pad_, E_, b, bsum, ym_, lb2_, st_));
    if (pwY_) GW_HIP(gwk::launch_pack_payload(Y_, m, m_pad_, E_, pwY_, st_));
    // moments of the features for C(alpha, beta) of Lemma C.1 (and the
    // gradients); they depend on X, Y and the weights only
    GW_HIP(gwk::launch_moments(X_, n, D_, a, mompart_, momx_, st_));
    GW_HIP(gwk::launch_moments(Y_, m, E_, b, mompart_, momy_, st_));

    // initial state
    if (gamma0) {
        GW_HIP(hipMemcpyAsync(gam_[0], gamma0, (size_t)D_ * E_ * sizeof(float), hipMemcpyDeviceToDevice, st_));
    } else {
        GW_HIP(hipMemsetAsync(gam_[0], 0, (size_t)D_ * E_ * sizeof(float), st_));
    }
    gcur_ = 0;
    have_init_ = f0 && g0;
    if (have_init_) {
        GW_HIP(hipMemcpyAsync(f_, f0, n * sizeof(float), hipMemcpyDeviceToDevice, st_));
        GW_HIP(hipMemcpyAsync(g_, g0, m * sizeof(float), hipMemcpyDeviceToDevice, st_));
    }
    GW_HIP(gwk::launch_ctl_init(ctl_, prm.mode, st_));
    // padded rows and columns keep -inf potentials in both parities (the
    // combines only ever write real rows and columns)
    for (int p = 0; p < 2; ++p) {
        GW_HIP(gwk::launch_fill(U_[p], n_pad_, -INFINITY, st_));
        GW_HIP(gwk::launch_fill(V_[p], m_pad_, -INFINITY, st_));
        GW_HIP(gwk::launch_fill(Ul_[p], n_pad_, 0.f, st_));
        GW_HIP(gwk::launch_fill(Vl_[p], m_pad_, 0.f, st_));
    }

    // row operand packs: features and |X|^2 slots once (potential slots are
    // refreshed by the prologue and the combines)
    if (geo_.path == 0) {
        for (int p = 0; p < 2; ++p)
            GW_HIP(gwk::launch_pack(X_, n, n_pad_, D_, 1.0f, prec_, 0, U_[p], Ul_[p], xn_, packA_[p], st_));
    }
    eps_sched_.resize(prm.n_outer);
    for (int t = 0; t < prm.n_outer; ++t) {
        if (prm.n_outer == 1 || prm.eps_start == prm.eps_end)
            eps_sched_[t] = prm.eps_start;
        else
            eps_sched_[t] = prm.eps_start * std::pow(prm.eps_end / prm.eps_start, (double)t / (prm.n_outer - 1));
    }
    t_ = 0;
    done_ = false;
    pa_ = pb_ = 0;
    return Status::ok();
}

Status Solve::buffers(bool dry) {
    Status st;
    auto& ws = c_.ws;
    const std::string& T = tag_;
    footprint_ = 0;
    auto getf = [&](const char* nm, size_t cnt) -> float* {
        footprint_ += cnt * 4;
        return dry ? nullptr : ws.get_t<float>(T + nm, cnt, &st);
    };
    auto getd = [&](const char* nm, size_t cnt) -> double* {
        footprint_ += cnt * 8;
        return dry ? nullptr : ws.get_t<double>(T + nm, cnt, &st);
    };
    X_ = getf("X", (size_t)n_pad_ * D_);
    Y_ = getf("Y", (size_t)m_pad_ * E_);
    xn_ = getf("xn", n_pad_);
    ym_ = getf("ym", m_pad_);
    la2_ = getf("la2", n_pad_);
    lb2_ = getf("lb2", m_pad_);
    for (int p = 0; p < 2; ++p) {
        U_[p] = getf(p ? "U1" : "U0", n_pad_);
        V_[p] = getf(p ? "V1" : "V0", m_pad_);
        Ul_[p] = getf(p ? "Ul1" : "Ul0", n_pad_);
        Vl_[p] = getf(p ? "Vl1" : "Vl0", m_pad_);
    }
    if (geo_.path == 0) {
        const size_t ba = pack_bytes(prec_, D_, n_pad_), bb = pack_bytes(prec_, D_, m_pad_);
        packA_[0] = getf("pA0", ba / 4);
        packA_[1] = getf("pA1", ba / 4);
        packB_[0] = getf("pB0", bb / 4);
        packB_[1] = getf("pB1", bb / 4);
    }
    pwY_ = gwk::cov_bf16_form(geo_.path, prec_, D_, E_) ? (void*)getf("pwY", gwk::payload_pack_bytes(m_pad_, E_) / 4)
                                                         : nullptr;
    Zs_ = getf("Zs", (size_t)m_pad_ * D_);
    beta_ = getd("beta", m_pad_);
    ms_ = getf("ms", m_pad_);
    f_ = getf("f", n_pad_);
    g_ = getf("g", m_pad_);
    gam_[0] = getf("gam0", (size_t)D_ * E_);
    gam_[1] = getf("gam1", (size_t)D_ * E_);
    gam64_ = getd("gam64", (size_t)D_ * E_);
    rp_ = getf("rp", (size_t)geo_.n_mt_c * n_pad_);
    rp2_ = getf("rp2", (size_t)geo_.n_mt_c * n_pad_);
    cp_ = getf("cp", (size_t)geo_.n_mt_r * m_pad_);
    cp2_ = getf("cp2", (size_t)geo_.n_mt_r * m_pad_);
    // partial sums of the covariance pass in either direction
    const size_t tp_n = std::max((size_t)cov_mtc_ * n_pad_ * cov_tw_, (size_t)cov2_mtc_ * m_pad_ * cov2_tw_);
    const size_t cr_n = std::max((size_t)cov_mtc_ * n_pad_, (size_t)cov2_mtc_ * m_pad_);
    const int64_t np_max = std::max(n_pad_, m_pad_);
    Tp_ = getf("Tp", tp_n);
    crp_ = getf("crp", cr_n);
    crmp_ = getf("crmp", cr_n);
    rsum_ = getf("rsum", np_max);
    rm_ = getf("rm", np_max);
    part_ = getd("part", std::max(gwk::cov_reduce_part_doubles(n_, D_, E_), gwk::cov_reduce_part_doubles(m_, E_, D_)));
    scal_ = getd("scal", 16);
    ctl_ = (int*)getf("ctl", CTL_WORDS);
    momx_ = getd("momx", 2 + D_ * D_ + D_);
    momy_ = getd("momy", 2 + E_ * E_ + E_);
    mompart_ = getd("mompart", std::max(gwk::moments_part_doubles(n_, D_), gwk::moments_part_doubles(m_, E_)));
    chk_ = geo_.path == 0 ? getd("chk", gwk::check64_part_doubles(n_, m_)) : nullptr;
    // per-row and per-column FP64 sums of the final check
    r64_ = getd("r64", n_);
    kl64_ = getd("kl64", n_);
    c64_ = getd("c64", m_);
    return st;
}

void Solve::make_half(int do_rows, int do_cols, float step, gwk::Operands& op, gwk::CombineArgs& ca) {
    // a new number per half-step, cycling through [1, 2^30 - 1]: the control
    // block starts at 0 and only the previous half-step's number can be there
    half_token_ = half_token_ % 0x3fffffff + 1;
    op = gwk::Operands{};
    op.token = half_token_;
    op.prec = prec_;
    op.d = D_;
    if (geo_.path == 0) {
        op.A = packA_[pa_];
        op.B = packB_[pb_];
    } else {
        op.X = X_;
        op.xn = xn_;
        op.U = U_[pa_];
        op.Ul = Ul_[pa_];
        op.Zs = Zs_;
        op.ms = ym_;
        op.V = V_[pb_];
        op.Vl = Vl_[pb_];
        op.kappa = (float)kappa_;
    }
    ca = gwk::CombineArgs{};
    ca.token = half_token_;
    ca.rp = rp_;
    ca.rp2 = rp2_;
    ca.cp = cp_;
    ca.cp2 = cp2_;
    ca.n_mt_c = geo_.n_mt_c;
    ca.n_mt_r = geo_.n_mt_r;
    ca.n = (int)n_;
    ca.m = (int)m_;
    ca.n_pad = (int)n_pad_;
    ca.m_pad = (int)m_pad_;
    ca.la2 = la2_;
    ca.lb2 = lb2_;
    ca.U_cur = U_[pa_];
    ca.Ul_cur = Ul_[pa_];
    ca.V_cur = V_[pb_];
    ca.Vl_cur = Vl_[pb_];
    ca.U_next = U_[1 - pa_];
    ca.Ul_next = Ul_[1 - pa_];
    ca.V_next = V_[1 - pb_];
    ca.Vl_next = Vl_[1 - pb_];
    ca.packA_next = geo_.path == 0 && do_rows ? packA_[1 - pa_] : nullptr;
    ca.packB_next = geo_.path == 0 && do_cols ? packB_[1 - pb_] : nullptr;
    ca.prec = prec_;
    ca.d = D_;
    ca.do_rows = do_rows;
    ca.do_cols = do_cols;
    ca.step = step;
    ca.is_retry = 0;
}

Status Solve::inner_iteration(int k) {
    (void)k;
    gwk::Partials pp{rp_, rp2_, cp_, cp2_};
    // one half-step: stabilised pass and its combine (run in stabilised
    // mode); then the safe pass and its combine, which run in safe mode and
    // as the retry when the first combine flagged the stabilised sums
    auto half = [&](int do_rows, int do_cols, float step) -> Status {
        gwk::Operands op;
        gwk::CombineArgs ca;
        make_half(do_rows, do_cols, step, op, ca);
        GW_PROF(GW_PROF_PASS_STAB, gwk::launch_pass(op, geo_, pp, ctl_, RUN_STAB, 0, st_));
        GW_PROF(GW_PROF_COMBINE, gwk::launch_combine(ca, ctl_, RUN_STAB, st_));
        GW_PROF(GW_PROF_PASS_SAFE, gwk::launch_pass(op, geo_, pp, ctl_, RUN_SAFE_OR_RETRY, 1, st_));
        ca.is_retry = 1;
        GW_PROF(GW_PROF_COMBINE, gwk::launch_combine(ca, ctl_, RUN_SAFE_OR_RETRY, st_));
        return Status::ok();
    };
    if (prm_.symmetric) {
        GW_TRY(half(1, 1, 0.5f));
        pa_ ^= 1;
        pb_ ^= 1;
    } else {
        GW_TRY(half(1, 0, 1.0f));
        // the row half-step wrote U into the other parity; columns read it
        pa_ ^= 1;
        GW_TRY(half(0, 1, 1.0f));
        pb_ ^= 1;
    }
    return Status::ok();
}

void Solve::iteration_items(gwk::PassItem& item, gwk::CombineArgs& main, gwk::CombineArgs& retry, int** ctl) {
    make_half(1, 1, 0.5f, item.op, main);
    item.g = geo_;
    item.pp = gwk::Partials{rp_, rp2_, cp_, cp2_};
    item.ctl = ctl_;
    retry = main;
    retry.is_retry = 1;
    *ctl = ctl_;
}

Status Solve::covariance(int rows_side, float* T_out, float* r_out, float* rm_out) {
    gwk::CovOut out{Tp_, crp_, crmp_, 0};
    if (rows_side == 0) {
        out.tw = cov_tw_;
        GW_HIP(gwk::launch_cov(geo_.path, prec_, D_, packA_[pa_], packB_[pb_], pwY_, X_, xn_, U_[pa_], Ul_[pa_], Zs_,
                               geo_.path == 1 ? ym_ : ms_, V_[pb_], Vl_[pb_], (float)kappa_, Y_, ym_, E_, n_pad_,
                               m_pad_, cov_rg_, cov_bc_, cov_mtr_, cov_mtc_, out, st_));
        GW_HIP(gwk::launch_cov_reduce(out, cov_mtc_, n_, n_pad_, X_, D_, xn_, E_, T_out, r_out, rm_out, part_, st_));
        return Status::ok();
    }
    // target rows, source columns: the exponent is symmetric in the two
    // operands (s_ij = sum_k A_ik B_jk, or the direct form with X <-> Z,
    // n <-> m, U <-> V), so the same kernels run with the packs swapped and
    // X as the payload; gives T'_j = sum_i pi_ij X_i and sum_i pi_ij |X_i|^2
    out.tw = cov2_tw_;
    if (gwk::cov_bf16_form(geo_.path, prec_, D_, D_) && !pwX_) {
        Status st;
        pwX_ = c_.ws.get(tag_ + "pwX", gwk::payload_pack_bytes(n_pad_, D_), &st);
        if (!st.good()) return st;
        GW_HIP(gwk::launch_pack_payload(X_, n_, n_pad_, D_, pwX_, st_));
    }
    GW_HIP(gwk::launch_cov(geo_.path, prec_, D_, packB_[pb_], packA_[pa_], pwX_, Zs_, ym_, V_[pb_], Vl_[pb_], X_, xn_,
                           U_[pa_], Ul_[pa_], (float)kappa_, X_, xn_, D_, m_pad_, n_pad_, cov2_rg_, cov2_bc_,
                           cov2_mtr_, cov2_mtc_, out, st_));
    GW_HIP(gwk::launch_cov_reduce(out, cov2_mtc_, m_, m_pad_, Y_, E_, ym_, D_, T_out, r_out, rm_out, part_, st_));
    return Status::ok();
}

Status Solve::outer_step() {
    if (done_) return Status::ok();
    GW_TRY(begin_outer());
    // Sinkhorn at eps_t / 8 (Algorithm 3 or 2), warm-started
    for (int k = 0; k < n_inner_cur_; ++k) {
        GW_TRY(before_inner(k));
        GW_TRY(inner_iteration(k));
    }
    GW_TRY(end_outer());
    if (prm_.adaptive_inner && !done_) GW_TRY(adaptive_step());
    return Status::ok();
}

// Algorithm 6 (adaptive Sinkhorn iterations) for CNT-GW: the EGW objective
// L_lift + eps KL of the new coupling against that of the previous one, both
// at this step's eps; an increase means the inner solve was too short, and
// the count doubles.  The paper doubles on any increase.  Here an increase
// counts only above 1e-6 max(|EGW|, C) (C of Lemma C.1, the scale of the
// terms L_lift is a difference of): L_lift comes from single-precision
// passes, and smaller changes are within their rounding.  This tolerance,
// and the cap of 64 n_inner, are implementation limits, not the paper's
// rule.  L_lift = C - 8 |Gamma_{t+1}|^2 - 4 sum pi n m comes from the
// covariance pass, KL from the FP64 check of the same coupling.
Status Solve::adaptive_step() {
    GW_TRY(enqueue_check());
    const size_t nmx = 2 + (size_t)D_ * D_ + D_, nmy = 2 + (size_t)E_ * E_ + E_;
    std::vector<double> hs(16), mx, my;
    GW_HIP(hipMemcpyAsync(hs.data(), scal_, 16 * sizeof(double), hipMemcpyDeviceToHost, st_));
    if (!have_c_) {
        mx.resize(nmx);
        my.resize(nmy);
        GW_HIP(hipMemcpyAsync(mx.data(), momx_, nmx * sizeof(double), hipMemcpyDeviceToHost, st_));
        GW_HIP(hipMemcpyAsync(my.data(), momy_, nmy * sizeof(double), hipMemcpyDeviceToHost, st_));
    }
    GW_HIP(hipStreamSynchronize(st_));
    if (!have_c_) {
        c_const_ = lemma_c1_constant(mx.data(), D_, my.data(), E_);
        have_c_ = true;
        if (!gamma0_given_) {
            // pi^0 = a x b: Gamma_0 = 0 for centred features, KL = 0
            prev_loss_ = c_const_ - 4.0 * mx[0] * my[0];
            prev_kl_ = 0.0;
            have_prev_ = true;
        }
    }
    const double loss = c_const_ - 8.0 * hs[2] - 4.0 * hs[1];
    const double kl = hs[5];
    if (!std::isfinite(loss) || !std::isfinite(kl)) return fail(GW_ENUMERIC, "non-finite EGW objective");
    if (have_prev_) {
        const double e_new = loss + eps_t_ * kl, e_old = prev_loss_ + eps_t_ * prev_kl_;
        if (e_new - e_old > 1e-6 * std::max(std::fabs(e_old), c_const_) && n_inner_cur_ < 64 * prm_.n_inner) {
            n_inner_cur_ = std::min(2 * n_inner_cur_, 64 * prm_.n_inner);
            ++doublings_;
        }
    }
    prev_loss_ = loss;
    prev_kl_ = kl;
    have_prev_ = true;
    return Status::ok();
}

Status Solve::before_inner(int k) {
    // Sinkhorn annealing in the scheduled last outer step (Appendix B.1):
    // iteration n = k + 1 runs at eps_T / sqrt(n); the column operand and the
    // potentials are re-expressed at the new temperature with the same Gamma
    if (!prm_.anneal_final || t_ != prm_.n_outer - 1 || k == 0) return Status::ok();
    eps_t_ = eps_sched_[t_] / std::sqrt((double)(k + 1));
    kappa_ = LOG2E * 8.0 / eps_t_;
    return prologue(0);
}

Status Solve::begin_outer() {
    eps_t_ = eps_sched_[t_];
    kappa_ = LOG2E * 8.0 / eps_t_;
    return prologue(t_ == 0 ? 1 : 0);
}

Status Solve::prologue(int first) {
    // Algorithm 1: Zbar_j = [Gamma_t Y_j, |Y_j|^2 / 2]; potentials rebased
    // from kappa_old_ to kappa_ and to Gamma in FP64
    const int expanded = geo_.path == 0 ? 1 : 0;
    c_.prof.begin(GW_PROF_PROLOGUE, st_);
    GW_HIP(gwk::launch_prologue_cols(Y_, m_, m_pad_, E_, D_, gam_[gcur_], ym_, lb2_, have_init_ ? g_ : nullptr, first,
                                     expanded, kappa_, kappa_old_, Zs_, beta_, V_[pb_], Vl_[pb_], ms_, st_));
    GW_HIP(gwk::launch_prologue_rows(n_, n_pad_, xn_, la2_, have_init_ ? f_ : nullptr, first, expanded, kappa_,
                                     kappa_old_, U_[pa_], Ul_[pa_], st_));
    if (geo_.path == 0) {
        for (int p = 0; p < 2; ++p)
            GW_HIP(gwk::launch_pack(Zs_, m_, m_pad_, D_, 1.0f, prec_, 1, V_[pb_], Vl_[pb_], ms_, packB_[p], st_));
        GW_HIP(gwk::launch_pack_pot(U_[pa_], Ul_[pa_], n_pad_, D_, prec_, 0, packA_[pa_], st_));
    }
    kappa_old_ = kappa_;
    c_.prof.end(st_);
    return Status::ok();
}

Status Solve::end_outer() {
    // covariance: Gamma_{t+1} = sum_ij pi_ij X_i Y_j^T
    c_.prof.begin(GW_PROF_COVARIANCE, st_);
    GW_TRY(covariance(0, nullptr, rsum_, rm_));
    GW_HIP(gwk::launch_gamma_final(part_, n_, D_, E_, gam_[gcur_], gam64_, gam_[1 - gcur_], scal_, st_));
    c_.prof.end(st_);
    gcur_ ^= 1;
    ++t_;
    if (t_ >= prm_.n_outer) done_ = true;
    if (!done_ && prm_.tol_gamma > 0.0) {
        double d2 = 0.0;
        GW_HIP(hipMemcpyAsync(&d2, scal_ + 3, sizeof(double), hipMemcpyDeviceToHost, st_));
        GW_HIP(hipStreamSynchronize(st_));
        if (std::sqrt(d2) <= prm_.tol_gamma) done_ = true;
    }
    return Status::ok();
}

Status Solve::finish(gw_result* out) {
    GW_TRY(finish_enqueue(out));
    GW_HIP(hipStreamSynchronize(st_));
    return finish_collect(out);
}

Status Solve::finish_enqueue(gw_result* out) {
    Status st;
    GW_TRY(enqueue_check());
    // outputs: potentials back in Algorithm 1's convention (cost units)
    if (geo_.path == 1) {
        if (out->f) GW_HIP(gwk::launch_epilogue(n_, U_[pa_], Ul_[pa_], la2_, nullptr, nullptr, 0, kappa_, out->f, st_));
        if (out->g) GW_HIP(gwk::launch_epilogue(m_, V_[pb_], Vl_[pb_], lb2_, nullptr, nullptr, 0, kappa_, out->g, st_));
    } else {
        if (out->f) GW_HIP(gwk::launch_epilogue(n_, U_[pa_], Ul_[pa_], la2_, xn_, nullptr, 1, kappa_, out->f, st_));
        if (out->g) GW_HIP(gwk::launch_epilogue(m_, V_[pb_], Vl_[pb_], lb2_, nullptr, beta_, 2, kappa_, out->g, st_));
    }
    if (out->gamma)
        GW_HIP(hipMemcpyAsync(out->gamma, gam_[gcur_], (size_t)D_ * E_ * sizeof(float), hipMemcpyDeviceToDevice,
                              st_));
    // scalars, moments and control words to pinned host memory
    const size_t nmx = 2 + (size_t)D_ * D_ + D_, nmy = 2 + (size_t)E_ * E_ + E_;
    const size_t bytes = (16 + nmx + nmy) * sizeof(double) + CTL_WORDS * sizeof(int);
    double* h = (double*)c_.host_stage(bytes, &st);
    if (!st.good()) return st;
    GW_HIP(hipMemcpyAsync(h, scal_, 16 * sizeof(double), hipMemcpyDeviceToHost, st_));
    GW_HIP(hipMemcpyAsync(h + 16, momx_, nmx * sizeof(double), hipMemcpyDeviceToHost, st_));
    GW_HIP(hipMemcpyAsync(h + 16 + nmx, momy_, nmy * sizeof(double), hipMemcpyDeviceToHost, st_));
    GW_HIP(hipMemcpyAsync(h + 16 + nmx + nmy, ctl_, CTL_WORDS * sizeof(int), hipMemcpyDeviceToHost, st_));
    return Status::ok();
}

// FP64 check of the current coupling (f_t, g_t, Gamma_{t-1}): row sums, KL
// and column sums, reduced into scal_[4] (Err) and scal_[5] (KL).
Status Solve::enqueue_check() {
    double* r64 = r64_;
    double* kl64 = kl64_;
    double* c64 = c64_;
    c_.prof.begin(GW_PROF_CHECK, st_);
    if (geo_.path == 1) {
        const float kap = (float)kappa_;
        GW_HIP(gwk::launch_check64_direct(D_, X_, xn_, U_[pa_], Ul_[pa_], Zs_, ym_, V_[pb_], Vl_[pb_], kap, n_, m_,
                                          la2_, lb2_, r64, kl64, st_));
        GW_HIP(gwk::launch_check64_direct(D_, Zs_, ym_, V_[pb_], Vl_[pb_], X_, xn_, U_[pa_], Ul_[pa_], kap, m_, n_,
                                          lb2_, nullptr, c64, nullptr, st_));
    } else {
        GW_HIP(gwk::launch_check64(prec_, D_, packA_[pa_], packB_[pb_], n_, m_, la2_, lb2_, chk_, r64, kl64, c64,
                                   st_));
    }
    GW_HIP(gwk::launch_check_final(r64, kl64, n_, a_, c64, m_, b_, asum_, bsum_, scal_, st_));
    c_.prof.end(st_);
    c_.prof.entries = n_ * m_;
    return Status::ok();
}

// Lemma C.1: C = iint|x-x'|^4 + iint|y-y'|^4 - 4 s_x s_y; for centred
// measures iint |x - x'|^4 = 2 m4 + 4 |Sigma|^2 + 2 s^2 (moments: s, m4, Sigma).
double lemma_c1_constant(const double* mx, int D, const double* my, int E) {
    auto cpart = [](const double* mo, int d) {
        double s = mo[0], m4 = mo[1], sig2 = 0.0;
        for (int k = 0; k < d * d; ++k) sig2 += mo[2 + k] * mo[2 + k];
        return 2.0 * m4 + 4.0 * sig2 + 2.0 * s * s;
    };
    return cpart(mx, D) + cpart(my, E) - 4.0 * mx[0] * my[0];
}

Status Solve::finish_collect(gw_result* out) {
    const size_t nmx = 2 + (size_t)D_ * D_ + D_, nmy = 2 + (size_t)E_ * E_ + E_;
    Status st;
    const double* hs = (const double*)c_.host_stage(0, &st);
    if (!hs) return fail(GW_ESTATE, "finish_collect without finish_enqueue");
    const double* mx = hs + 16;
    const double* my = hs + 16 + nmx;
    const int* hctl = (const int*)(hs + 16 + nmx + nmy);
    const double C = lemma_c1_constant(mx, D_, my, E_);
    out->constant_c = C;
    out->sum_pi_nm = hs[1];
    out->loss_lift = C - 8.0 * hs[2] - 4.0 * hs[1];
    out->kl = hs[5];
    out->marginal_err = hs[4];
    out->egw_objective = out->loss_lift + eps_t_ * hs[5];
    out->gamma_step = std::sqrt(hs[3]);
    out->eps_final = eps_t_;
    out->outer_done = t_;
    out->dim_x = D_;
    out->dim_y = E_;
    out->safe_iters = hctl[CTL_SAFE_ITERS];
    out->n_inner_final = n_inner_cur_;
    out->inner_doublings = doublings_;
    if (hctl[CTL_NUMERIC] || !std::isfinite(out->loss_lift) || !std::isfinite(out->kl))
        return fail(GW_ENUMERIC, "non-finite values in the Sinkhorn iteration");
    return Status::ok();
}

}  // namespace gwr
