/*
 * gw.h - C ABI of the MI355X (gfx950) CNT-GW hot-path library (libgwmi.so).
 *
 * Problem (Section 5, "Notations"): two discrete measures
 *   alpha = sum_i a_i delta_{x_i}  (N points in R^dx),
 *   beta  = sum_j b_j delta_{y_j}  (M points in R^dy),
 * positive weights summing to 1, a distortion penalty per side that is
 * conditionally of negative type (Section 2, "Embeddable Costs"), and a
 * temperature eps.  The library lifts both sides into centred features
 * X (N x D), Y (M x E) (Section 3, Definition of GW-embeddings; Section 5,
 * "CNT Embeddings") and runs Algorithm 1 (CNT-GW): per outer step the
 * squared-norm EOT problem between [X_i, |X_i|^2/2] and [Gamma Y_j, |Y_j|^2/2]
 * at temperature eps/8 is solved by log-domain Sinkhorn (Algorithm 3, or
 * Algorithm 2), then Gamma <- sum_ij pi_ij X_i Y_j^T.  The N x M cost and
 * coupling are never stored.
 *
 * Conventions for every entry point below:
 *   - Array arguments named x, y, a, b, f, g, gamma, gamma0, grad_* and
 *     features are DEVICE pointers (HIP global memory of the context's
 *     device), float32, row-major, owned by the caller.  The library never
 *     frees them and never keeps them after the call returns (the serving
 *     API is the exception and says so).
 *   - All GPU work is ordered on the context's HIP stream.  gw_solve and
 *     gw_loss_and_grad block until their scalar results are on the host.
 *   - Errors are returned as gw_status; nothing aborts or throws across the
 *     ABI.  gw_last_error() gives a message for the last failing call on the
 *     context.  On error, output buffers may hold partial results.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef GWMI_GW_H
#define GWMI_GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gw_ctx gw_ctx;
typedef struct gw_server gw_server;

typedef enum {
    GW_OK = 0,
    GW_EINVAL = 1,        /* invalid argument (sizes, weights, eps, NULL) */
    GW_ENOMEM = 2,        /* device allocation or workspace limit */
    GW_EDEVICE = 3,       /* HIP runtime error */
    GW_ENUMERIC = 4,      /* non-finite value detected in the iteration */
    GW_ESTATE = 5,        /* call not valid in the context's current state */
    GW_EUNSUPPORTED = 6,  /* valid request the library does not implement */
    GW_EBUSY = 7,         /* serving: result not ready yet */
    GW_ECANCELLED = 8     /* serving: request was cancelled */
} gw_status;

/* Distortion penalty of one side (Section 2, "Embeddable Costs"). */
typedef enum {
    /* c(x, x') = |x - x'|^2: features are the centred points, D = dx
       (Section 3, "Example").  */
    GW_PEN_SQEUCLID = 0,
    /* c(x, x') = |x - x'|^p, 0 < p < 2: landmark kernel PCA (Algorithm 4 and
       the Kernel PCA paragraph of Appendix B.2) with the Nystrom map of
       Algorithm 13 for every point, re-centred with the weights; D =
       lifted_dim.  Landmarks are fitted on the first solve after
       gw_set_penalty and stay frozen until the next gw_set_penalty. */
    GW_PEN_POWER = 1,
    /* the caller passes features directly (x is N x D); they are re-centred
       with the weights, as Section 5 requires. */
    GW_PEN_FEATURES = 2
} gw_penalty;

/* Arithmetic of the feature contraction X_i . Z_j in the Sinkhorn and
   covariance passes.  Log-sum-exp, potentials and marginals are FP32 in
   every form; the final marginal check is FP64. */
typedef enum {
    GW_FP32 = 0,    /* FP32: MFMA f32 for D >= 16, VALU for D < 16 */
    GW_BF16 = 1,    /* BF16 x BF16 -> FP32 MFMA (D >= 16; D < 16 runs FP32) */
    GW_BF16X3 = 2   /* split BF16 (hi*hi + hi*lo + lo*hi) on MFMA */
} gw_precision;

typedef enum {
    GW_MODE_AUTO = 0,        /* device-side choice per iteration */
    GW_MODE_SAFE = 1,        /* max-shifted row and column log-sum-exp */
    GW_MODE_STABILISED = 2   /* one exponential per entry feeds both sums */
} gw_mode;

typedef struct {
    double eps_start;          /* temperature of outer step 0, > 0 */
    double eps_end;            /* of the last outer step; geometric in between */
    int32_t n_outer;           /* outer CNT-GW steps, >= 1 */
    int32_t n_inner;           /* Sinkhorn iterations per outer step, >= 1 */
    int32_t symmetric;         /* 1: Algorithm 3 (default), 0: Algorithm 2 */
    int32_t precision;         /* gw_precision */
    int32_t mode;              /* gw_mode */
    int32_t use_init_potentials; /* 1: read result->f, result->g as warm start */
    double tol_gamma;          /* > 0: stop when |Gamma_t - Gamma_{t+1}|_F <= tol
                                  (Algorithm 1's loop condition; one 8-byte
                                  readback per outer step) */
    int32_t anneal_final;      /* 1: Sinkhorn annealing in the scheduled last
                                  outer step (Appendix B.1): its iteration
                                  n = 1..n_inner runs at eps_T / sqrt(n), and
                                  the plan, Gamma_T and the reported eps use the
                                  last of them; 0: off.  Not applied when
                                  tol_gamma stops the loop earlier. */
    int32_t adaptive_inner;    /* 1: Algorithm 6's adaptive Sinkhorn counts:
                                  n_inner is the first step's count, and it
                                  doubles after a step whose coupling has a
                                  larger EGW objective (at that step's eps)
                                  than the previous coupling (the previous
                                  coupling of step 0 is a x b when gamma0 is
                                  NULL, none otherwise).  Two implementation
                                  limits depart from the paper's rule, which
                                  doubles on any increase without bound: an
                                  increase counts only above 1e-6 max(|EGW|,
                                  C), C the constant of Lemma C.1, since the
                                  objective is evaluated from single-precision
                                  passes; and the count is capped at
                                  64 x n_inner.  Each
                                  outer step then runs the FP64 check (one
                                  extra N x M evaluation and a readback).
                                  gw_solve only (the server rejects it).
                                  0: fixed counts. */
} gw_params;

typedef struct {
    /* caller-allocated device outputs (in/out for warm starts) */
    float* f;                  /* N, Algorithm 1 convention, cost units */
    float* g;                  /* M */
    float* gamma;              /* D x E row-major: Gamma_T */
    /* host scalars written by the library */
    double loss_lift;          /* Lemma C.1 lifted GW loss of the final coupling */
    double egw_objective;      /* loss_lift + eps_T * KL */
    double kl;                 /* KL(pi | a x b) of the final coupling (FP64) */
    double marginal_err;       /* Err(pi) = |pi 1 - a|_1 + |pi^T 1 - b|_1, FP64 */
    double constant_c;         /* C(alpha, beta) of Lemma C.1 (FP64 moments) */
    double sum_pi_nm;          /* sum_ij pi_ij |X_i|^2 |Y_j|^2 */
    double gamma_step;         /* |Gamma_T - Gamma_{T-1}|_F */
    double eps_final;          /* eps_T */
    int32_t outer_done;        /* outer steps run */
    int32_t dim_x;             /* D, lifted source dimension */
    int32_t dim_y;             /* E */
    int32_t safe_iters;        /* Sinkhorn iterations that ran max-shifted */
    int32_t n_inner_final;     /* Sinkhorn count of the last outer step */
    int32_t inner_doublings;   /* adaptive_inner: doublings made */
} gw_result;

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
   (a hipStream_t; NULL = the null stream).  workspace_limit_bytes bounds the
   library's own device memory (0 = no limit).  *out is set on success. */
gw_status gw_create(gw_ctx** out, int device, void* hip_stream,
                    size_t workspace_limit_bytes);

/* Select the penalty of a side (0 source, 1 target, 2 both).  p is the
   exponent for GW_PEN_POWER (0 < p < 2); lifted_dim is D (resp. E) for
   GW_PEN_POWER (1..256); n_landmarks (>= lifted_dim + 1) and seed choose the
   landmark subset as the first n_landmarks entries of a seeded permutation
   (SplitMix64-driven Fisher-Yates, fixed by the library).  Clears fitted
   landmarks of that side. */
gw_status gw_set_penalty(gw_ctx* ctx, int side, int kind, double p,
                         int lifted_dim, int n_landmarks, uint64_t seed);

/* The landmark subset the seeded choice gives (host only, no GPU work):
   writes min(n_landmarks, n) sorted indices into idx_host (caller
   allocated): the first entries of a Fisher-Yates shuffle of 0..n-1 driven
   by SplitMix64 (Steele, Lea, Flood 2014) started at seed.  The source side
   of a served request uses seed, the target side seed + 1.  Returns
   GW_EINVAL for n < 1, n_landmarks < 1 or a null pointer. */
gw_status gw_seeded_landmarks(int64_t n, int n_landmarks, uint64_t seed, int64_t* idx_host);

/* Use explicit landmark indices (host array of n_landmarks distinct indices
   into the next solve's points of that side) instead of the seeded choice.
   For GW_PEN_POWER only; clears fitted landmarks of that side. */
gw_status gw_set_landmarks(gw_ctx* ctx, int side, const int64_t* idx_host,
                           int n_landmarks);

/* Lift one side into centred features (the setup step of Algorithm 1's
   inputs, Eq. embedding_X / embedding_Y): features (n x D, device, caller
   allocated; D from gw_feature_dim).  Fits landmarks if needed. */
gw_status gw_lift(gw_ctx* ctx, int side, const float* x, int64_t n, int d,
                  const float* w, float* features);

/* Lifted dimension of a side for input dimension d under its penalty. */
int gw_feature_dim(const gw_ctx* ctx, int side, int d);

/* Solve the entropic GW problem with Algorithm 1.  gamma0 (D x E, device)
   initialises Gamma (NULL: Gamma_0 = 0, the product coupling).  Potentials
   start at 0 unless params->use_init_potentials.  Inputs: x (n x dx), a (n),
   y (m x dy), b (m).  Errors: GW_EINVAL for n or m < 1, dims out of range,
   non-finite inputs, weights <= 0 or |sum - 1| > 1e-6 (sum taken in FP64),
   eps <= 0, counts < 1;
   GW_ENUMERIC if the iteration produced non-finite values. */
gw_status gw_solve(gw_ctx* ctx,
                   const float* x, int64_t n, int dx, const float* a,
                   const float* y, int64_t m, int dy, const float* b,
                   const gw_params* params, const float* gamma0,
                   gw_result* out);

/* gw_solve for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation):
   the same solve, bit for bit, with every device buffer carved from a fixed
   scratch array of 256 MiB per GPU that the library holds until the process
   ends, so the call makes no hipMalloc, hipFree or other allocating call
   (host bookkeeping uses the C++ heap).  Inputs, outputs and errors as
   gw_solve, with these limits: both sides must use GW_PEN_SQEUCLID or
   GW_PEN_FEATURES (lifting allocates; GW_EUNSUPPORTED otherwise);
   adaptive_inner is not run (GW_EUNSUPPORTED); a problem whose buffers
   exceed the array is refused with GW_ENOMEM before any work (square
   problems up to about 159,000 points per side at D = 3, 67,000 at D = 32
   and 29,000 at D = 64).
   Profiling is not recorded.  Calls in one process are serialised (they
   share the array and a host staging buffer), and the array is only in use
   during a call (which waits for its results): its contents are left from
   the previous call and nothing in it needs to start at zero.  Calls from
   different processes use their own copies. */
gw_status gw_solve_noalloc(gw_ctx* ctx,
                           const float* x, int64_t n, int dx, const float* a,
                           const float* y, int64_t m, int dy, const float* b,
                           const gw_params* params, const float* gamma0,
                           gw_result* out);

/* ---- Stepwise solve: Algorithm 1 one outer step at a time ----
   The state of Algorithm 1 between outer steps is (f, g, Gamma_t, t, eps_t)
   (Algorithm 1; warm starts as in Appendix B.1).  These three calls keep it
   inside the context, so a caller can run a solve in pieces and synchronise,
   time or inspect between them:
     gw_solve_begin   validation and setup exactly as gw_solve (same
                      inputs, errors and warm start: out->f, out->g are read
                      when params->use_init_potentials); no outer step yet.
     gw_solve_advance enqueues up to n_steps further outer steps (prologue,
                      the step's Sinkhorn iterations, covariance) on the
                      context's stream and returns without waiting, except
                      where tol_gamma or adaptive_inner read back one scalar
                      per step.  *outer_done (host, nullable) receives the
                      outer steps enqueued so far; once it equals n_outer
                      (or tol_gamma stopped the loop), further calls do
                      nothing.  n_steps >= 0.
     gw_solve_end     the FP64 final check and the outputs of gw_solve
                      (out->f, out->g, out->gamma and the scalars), then
                      releases the stepwise solve.  Valid after any number
                      of outer steps >= 1; the result then describes the
                      coupling after those steps.
   begin, advance(k1), advance(k2), ..., end with k1 + k2 + ... = n_outer is
   the same computation as gw_solve, bit for bit.  One stepwise solve per
   context: a new gw_solve_begin replaces an unfinished one.  Its device
   inputs (x, a, y, b, gamma0) must stay valid and unchanged until
   gw_solve_end.  Other entry points may run on the context in between; the
   stepwise solve's buffers are its own.  Errors: as gw_solve; GW_ESTATE for
   advance or end without an active stepwise solve, or end before the first
   outer step; GW_EINVAL for n_steps < 0. */
gw_status gw_solve_begin(gw_ctx* ctx,
                         const float* x, int64_t n, int dx, const float* a,
                         const float* y, int64_t m, int dy, const float* b,
                         const gw_params* params, const float* gamma0,
                         const gw_result* warm);
gw_status gw_solve_advance(gw_ctx* ctx, int n_steps, int32_t* outer_done);
gw_status gw_solve_end(gw_ctx* ctx, gw_result* out);

/* Result of gw_sgw. */
typedef struct {
    double sgw;                /* GW_eps(a, b) - (GW_eps(a, a) + GW_eps(b, b)) / 2 */
    double gw_xy;              /* EGW objective of each of the three solves */
    double gw_xx;
    double gw_yy;
    double marginal_err;       /* largest FP64 marginal error of the three */
    int32_t dim_x, dim_y;      /* lifted dimensions D, E */
} gw_sgw_result;

/* Sinkhorn-GW divergence (Section 4, "Entropic Bias"; zero between
   isometric measures and non-negative for CNT costs, Theorem 4.3): both
   sides are lifted once with their penalties, then Algorithm 1 runs three
   times on the lifted features, (x, y), (x, x) and (y, y), from Gamma_0 = 0
   with the same params; each GW_eps is the EGW objective at the schedule's
   last eps.  Same inputs and errors as gw_solve; params->use_init_potentials
   is rejected (GW_EINVAL).  When no problem has more than 1e9 entries, the
   three solves run side by side, each on a stream the context creates once
   (default priority) and on device buffers of its own; the results are
   those of the solves run one after another, bit for bit, and the call
   returns once all three have finished. */
gw_status gw_sgw(gw_ctx* ctx,
                 const float* x, int64_t n, int dx, const float* a,
                 const float* y, int64_t m, int dy, const float* b,
                 const gw_params* params, gw_sgw_result* out);

/* Position and weight gradients of the Sinkhorn-GW divergence (Section 4;
   envelope gradients of Appendix B.6): the three solves of gw_sgw on the
   raw points, then
   grad_x = dGW(x, y)/dx - (dGW(x, x)/dx_source + dGW(x, x)/dx_target) / 2
   and the same for y (device, caller allocated, n x dx and m x dy).  The
   envelope gradient is exact at converged solves.  Each measure keeps its
   side's penalty in every term: with GW_PEN_POWER the pair solve fits the
   landmark maps (source on x, target on y, or keeps maps fitted before), the
   self term of x uses x's frozen map on both of its sides and that of y
   uses y's, and every gradient chains through its side's frozen map
   (Algorithm 12 with Algorithm 13), as gw_sgw embeds the three problems.
   grad_a and grad_b (device, n and m floats, each nullable) receive the
   weight gradients in the same composition (the self term's source and
   target weight gradients summed, since it carries the measure's weights in
   both marginals), each as gw_loss_and_grad gives them: along the simplex,
   centred so that sum_i a_i grad_a_i = 0.  Other inputs, outputs and errors
   as gw_sgw. */
gw_status gw_sgw_grad(gw_ctx* ctx,
                      const float* x, int64_t n, int dx, const float* a,
                      const float* y, int64_t m, int dy, const float* b,
                      const gw_params* params, gw_sgw_result* out,
                      float* grad_x, float* grad_y,
                      float* grad_a, float* grad_b);

/* GW barycentre flow (Section 6, "GW Barycenters"): gradient descent on the
   points z (k x d, device, in/out) of gamma_z = sum_i w_i delta_{z_i} (w:
   k device weights, > 0, sum 1) for the objective
   (1 - lambda) SGW_eps(gamma_z, alpha) + lambda SGW_eps(gamma_z, beta), with
   alpha = (x, a) (n x d) and beta = (y, b) (m x d) on the device.  Each of
   the n_steps steps runs Algorithm 1 on (z, x), (z, y) and (z, z) with params,
   takes the divergence's position gradient (gw_sgw_grad) and moves
   z_i -= step / w_i * gradient_i; GW_eps(alpha, alpha) and GW_eps(beta, beta)
   are solved once.  The solves of a step run side by side as in gw_sgw.  objective (host, n_steps + 1 values, nullable) receives
   the objective before each step and after the last.  Penalties: the same
   GW_PEN_SQEUCLID or GW_PEN_FEATURES on both sides, or GW_PEN_POWER on both
   sides, where z is embedded by a landmark map with side 0's settings
   fitted on z as passed in (its landmark points stay there while z moves),
   and alpha and beta by maps with side 1's settings fitted on x and on y
   (landmark seeds s and s + 1, or side 1's explicit indices into both); all
   solves then run on the embedded features and z's gradients chain through
   its frozen map (GW_EUNSUPPORTED for other combinations).  Errors as
   gw_sgw_grad; GW_EINVAL for lambda outside [0, 1], step < 0 or n_steps
   outside [0, 100000]. */
gw_status gw_sgw_barycenter(gw_ctx* ctx,
                            const float* x, int64_t n, const float* a,
                            const float* y, int64_t m, const float* b, int d,
                            float* z, int64_t k, const float* w,
                            double lambda, double step, int n_steps,
                            const gw_params* params, double* objective);

/* Full-N kernel PCA (Appendix B, "Kernel PCA"; the paper's KeOps + eigsh
   route for all points): features X (n x D, device, row-major, caller
   allocated) with X_i = V_i sqrt(Lambda) for the D largest eigenpairs of
   Algorithm 4's kernel of c(x, x') = |x - x'|^p over all n points, weighted
   double centring with w (device, > 0, sum 1).  x: n x d device points,
   1 <= d <= 8, 0 < p <= 2, 1 <= D <= min(256, n - 1).  Matrix-free
   randomized subspace iteration (Halko, Martinsson, Tropp 2011) with D + 32
   vectors, n_iter (0..100) power steps and a Rayleigh-Ritz step, in FP64;
   the start block is SplitMix64 noise of seed.  Eigenvalues at or below
   1e-12 of the largest give zero columns.  lambda (host, D, nullable)
   receives the eigenvalues, descending.  Features are centred with w (w
   spans the kernel's null space).  Eigenvectors are defined up to sign (and
   rotation inside repeated eigenvalues).  GW_EUNSUPPORTED for d > 8 or
   n (D + 32) >= 2^31; GW_EINVAL for other sizes out of range, null
   pointers or invalid inputs; GW_ENUMERIC if the iteration loses rank. */
gw_status gw_kpca_full(gw_ctx* ctx, const float* x, int64_t n, int d, const float* w,
                       double p, int D, int n_iter, uint64_t seed,
                       float* X, double* lambda);

/* ---- Multiscale-GW (Appendix B, "Implementation of Multiscale-GW") ---- */

/* Coarsen of Multiscale-GW: weighted K-Means of the rows of X (n x D,
   device, row-major; 1 <= D <= 256) with weights w (n, device, > 0, summing
   to 1), k = number of clusters (1 <= k <= n) started at the rows
   gw_seeded_landmarks(n, k, seed) gives, n_lloyd (1..10000) Lloyd
   iterations.  Each iteration assigns every row to its nearest centroid
   (squared distance summed over the coordinates in order in single
   precision without fused multiply-add, ties to the lowest index), then
   moves each centroid to the weighted mean of its cluster; the cluster sums
   are exact integer sums of rint(w_i X_id 2^S), S the largest exponent with
   max|X| 2^S <= 2^61, and of rint(w_i 2^61); the mean is one FP64 division
   rounded to single precision; an empty cluster keeps its centroid.
   Outputs (device, caller allocated): Xc (k x D) and wc (k) receive the
   non-empty clusters of the last assignment in index order, their
   centroids and aggregated weights; assign (n, nullable) the cluster index
   (0..k-1) of every row; *kc (host) their count.  GW_EINVAL on sizes out of
   range, null pointers, non-finite X or invalid weights. */
gw_status gw_kmeans(gw_ctx* ctx, const float* X, int64_t n, int D, const float* w,
                    int64_t k, int n_lloyd, uint64_t seed,
                    float* Xc, float* wc, int32_t* assign, int64_t* kc);

/* Interpolate (Algorithm 8), in the potentials' convention of Algorithm 1:
   out_q = -eps' ln sum_r w_r exp((h_r - |Pbar_q - Qbar_r|^2) / eps'),
   eps' = eps / 8, over lifted features.  side 0: P (nq x D) are source
   features, Q (nr x E) target features, Pbar = [P, |P|^2/2],
   Qbar = [Gamma Q, |Q|^2/2], h = g of the coarse target, out = f.  side 1:
   P (nq x E) target features, Q (nr x D) source features,
   Pbar = [Gamma P, |P|^2/2], Qbar = [Q, |Q|^2/2], h = f, out = g.  gamma is
   D x E row-major; every array is device memory; w > 0.  GW_EINVAL on
   sizes out of range (D, E in 1..256), null pointers or eps <= 0. */
gw_status gw_interpolate(gw_ctx* ctx, int side, const float* h,
                         const float* P, int64_t nq, const float* Q, int64_t nr,
                         const float* w, const float* gamma, int D, int E,
                         double eps, float* out);

/* Options of gw_msgw. */
typedef struct {
    double rho;        /* coarsening ratio in (0, 1]: ceil(rho n) and ceil(rho m) clusters */
    int32_t n_lloyd;   /* Lloyd iterations of each K-Means, >= 1 */
    int32_t reserved;  /* must be 0 */
    uint64_t seed;     /* K-Means starts: gw_seeded_landmarks with seed (source), seed + 1 (target) */
} gw_msgw_opts;

/* Coarse-scale figures of gw_msgw. */
typedef struct {
    int64_t n_coarse, m_coarse;     /* non-empty clusters per side */
    double coarse_loss_lift;        /* gw_result fields of the coarse solve */
    double coarse_egw_objective;
    double coarse_marginal_err;
    double ms_coarsen;              /* wall-clock milliseconds per phase (the */
    double ms_coarse_solve;         /* stream is synchronised between phases) */
    double ms_interpolate;
    double ms_fine_solve;
} gw_msgw_info;

/* Multiscale-GW (Algorithm 7): both sides are lifted once with their
   penalties (features X, Y, centred), coarsened with gw_kmeans' procedure,
   the coarse features re-centred with their weights; Algorithm 1 runs on
   the coarse measures with params `coarse` from gamma0 (NULL: 0); f and g
   of the fine points are interpolated (gw_interpolate) from the coarse
   potentials with the coarse Gamma at fine->eps_start; then Algorithm 1
   runs on the fine features with params `fine`, starting from the coarse
   Gamma and the interpolated potentials.  out (f, g, gamma and the scalars)
   is the fine solve's result; info (nullable) the coarse figures.  Inputs
   and errors as gw_solve; use_init_potentials must be 0 in both params. */
gw_status gw_msgw(gw_ctx* ctx,
                  const float* x, int64_t n, int dx, const float* a,
                  const float* y, int64_t m, int dy, const float* b,
                  const gw_params* coarse, const gw_params* fine,
                  const gw_msgw_opts* opts, const float* gamma0,
                  gw_result* out, gw_msgw_info* info);

/* Solve, then the envelope gradient of GW_eps (Appendix B.6, "EGW Gradient
   Computations"; Algorithm 12 through the frozen Nystrom map of Algorithm 13
   for GW_PEN_POWER) with respect to the positions and weights.  Any grad_*
   may be NULL.  grad_x: n x dx, grad_a: n (projected so sum_i a_i g_i = 0),
   grad_y: m x dy, grad_b: m.  The loss is out->egw_objective. */
gw_status gw_loss_and_grad(gw_ctx* ctx,
                           const float* x, int64_t n, int dx, const float* a,
                           const float* y, int64_t m, int dy, const float* b,
                           const gw_params* params, const float* gamma0,
                           gw_result* out,
                           float* grad_x, float* grad_a,
                           float* grad_y, float* grad_b);

/* Free the context and its device memory; waits for queued work.
   NULL-safe. */
void gw_destroy(gw_ctx* ctx);

/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char* gw_last_error(const gw_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* Profiling: HIP events around each kernel class on the context stream.   */
/* ---------------------------------------------------------------------- */

typedef enum {
    GW_PROF_PASS_STAB = 0,   /* stabilised Sinkhorn pass launches */
    GW_PROF_PASS_SAFE = 1,   /* safe / retry pass launches (may be no-ops) */
    GW_PROF_COMBINE = 2,     /* partial combines + potential updates */
    GW_PROF_COVARIANCE = 3,  /* covariance pass and Gamma reduction */
    GW_PROF_PROLOGUE = 4,    /* per-outer-step prologue and packing */
    GW_PROF_CHECK = 5,       /* FP64 final check */
    GW_PROF_LIFT = 6,        /* feature lifting */
    GW_PROF_GRAD = 7,        /* backward pass */
    GW_PROF_CLASSES = 8
} gw_prof_class;

typedef struct {
    int64_t launches[GW_PROF_CLASSES];
    double milliseconds[GW_PROF_CLASSES];   /* summed event intervals */
    int64_t entries_per_pass;               /* N * M of the last solve */
    /* the part of launches / milliseconds from intervals under 20
       microseconds: at large sizes these are the launches the device-side
       mode gate turned into no-ops (a stabilised pass in a safe iteration,
       a retry that was not needed), so (milliseconds - idle) / (launches -
       idle) is the mean duration of the launches that did the work */
    int64_t idle_launches[GW_PROF_CLASSES];
    double idle_milliseconds[GW_PROF_CLASSES];
} gw_profile;

/* Enable (1) or disable (0) event timing; either call resets the counters.
   Timing adds an event pair per recorded launch. */
gw_status gw_set_profiling(gw_ctx* ctx, int enable);

/* Synchronise the context stream and return the counters accumulated since
   the last gw_set_profiling. */
gw_status gw_get_profile(gw_ctx* ctx, gw_profile* out);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of independent solves on one GPU.         */
/* ---------------------------------------------------------------------- */

typedef struct {
    const float* x; int64_t n; int32_t dx; const float* a;   /* device */
    const float* y; int64_t m; int32_t dy; const float* b;   /* device */
    gw_params params;
    int32_t penalty;           /* gw_penalty, both sides */
    double p;                  /* exponent for GW_PEN_POWER */
    int32_t lifted_dim;        /* D = E for GW_PEN_POWER */
    int32_t n_landmarks;
    uint64_t seed;
    float* f; float* g; float* gamma;  /* device outputs, caller allocated */
    const float* gamma0;       /* device, D x E row-major initial Gamma, or
                                  NULL for Gamma_0 = 0 (read at setup) */
} gw_request;

typedef struct {
    uint64_t submitted, completed, cancelled, rejected;
    int32_t active, queued;
    double busy_seconds;       /* wall time with at least one active request */
    uint64_t device_bytes;     /* device memory the server's request slots
                                  hold now (workspaces and landmark data) */
    uint64_t peak_device_bytes;/* the largest device_bytes seen */
} gw_server_stats;

/* Create a server on ctx's device and stream.  max_slots bounds the number
   of requests resident on the GPU at once.  hbm_budget_bytes (0 = no bound)
   bounds the device memory of the resident requests: a request is admitted
   when its planned footprint (every buffer of its solve, its FP64 check and
   its lifting) fits beside those of the requests already admitted, and a
   finished request's slot then gives its memory back (without a budget,
   slots keep their buffers for the next request).  Memory the rocBLAS /
   rocSOLVER handle of the landmark eigensolve keeps is not counted.  The
   server runs its own host threads. */
gw_status gw_server_create(gw_ctx* ctx, int max_slots, size_t hbm_budget_bytes,
                           gw_server** out);

/* Queue a request.  The caller keeps every array of *req alive and
   unmodified until the request completes or is cancelled.  A request whose
   footprint alone exceeds the budget is rejected with GW_ENOMEM. */
gw_status gw_server_submit(gw_server* s, const gw_request* req, uint64_t* ticket);

/* GW_OK with *out filled when done; GW_EBUSY while queued or running;
   GW_ECANCELLED; GW_EINVAL for an unknown ticket.  latency_s (may be NULL)
   receives submit-to-completion wall time. */
gw_status gw_server_poll(gw_server* s, uint64_t ticket, gw_result* out,
                         double* latency_s);

/* Block until the ticket completes (or is cancelled). */
gw_status gw_server_wait(gw_server* s, uint64_t ticket, gw_result* out,
                         double* latency_s);

/* Cancel a queued or running request; its outputs are unspecified. */
gw_status gw_server_cancel(gw_server* s, uint64_t ticket);

gw_status gw_server_get_stats(gw_server* s, gw_server_stats* out);

/* Stop the server thread (cancelling unfinished requests) and free it. */
void gw_server_destroy(gw_server* s);

#ifdef __cplusplus
}
#endif
#endif /* GWMI_GW_H */
