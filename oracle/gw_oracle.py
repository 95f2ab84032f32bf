"""FP64 CPU oracle for the CNT-GW hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call it.  It shares no code, constant or helper
with the HIP library.

It is the plain, slow, materialised form of what the paper computes:

* every N x M cost is materialised in float64, directly as a sum of squared
  coordinate differences (never through the expanded dot product the GPU
  uses);
* every log-sum-exp is a max-shifted reduction over a full row or column;
* the algorithms run in the paper's order and notation.

Readings of passages where the paper is silent or garbled are listed in the
design notes; each function states the passage it follows.

Parity status per function (what pins it, in ``tests/test_oracle_*.py``):
    centre, lifted_loss, constant_c, quartic_loss  - brute force / closed form
    sinkhorn (NumPy and C loops)                  - unique EOT optimum, textbook
                                                    scaling iteration, separable
                                                    costs, N = 1; the C loop
                                                    (sinkhorn.c) also equals the
                                                    NumPy loop to float64 rounding
    cnt_gw                                        - Entropic-GW and Kernel-GW
                                                    agreement, permutation
                                                    enumeration, rigid motion,
                                                    monotone objective, Thm 4.5
    sgw_divergence                                - Thm 4.3: zero between isometric
                                                    measures, non-negative; symmetric
                                                    in its two arguments
    sgw_barycenter                                - descent, first-order decrease
                                                    matching the step's scaling
    sgw_grad_positions                            - central differences of the
                                                    converged divergence; zero at
                                                    isometric measures (a minimum
                                                    by Thm 4.3)
    landmark_lift, kernel_from_cost, kernel_pca   - full-rank exact embedding
    full_kpca_features                            - full-rank exact embedding for
                                                    p = 1/2, 1, 2; p = 2 equals
                                                    weighted PCA (numpy SVD)
    grad_positions, grad_weights                  - quartic-form envelope,
                                                    central finite differences,
                                                    translation / rotation
                                                    invariants
    coarsen, nearest_centroid                     - Lloyd step worked by hand,
                                                    scikit-learn K-Means, one
                                                    point per cluster, weight /
                                                    mean conservation, ties
    interpolate                                   - one coarse point (closed
                                                    form), the paper's bilinear
                                                    form via scipy logsumexp,
                                                    Sinkhorn fixed point
    msgw                                          - fixed point of Algorithm 1
                                                    kept from coarse to fine,
                                                    rotation invariance
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------


def centre(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Centred embedding phi(x) = x - x_alpha of the squared-norm example
    (Section 3, "Example": GW-embeddings for squared Euclidean costs), with
    x_alpha = sum_i w_i x_i.  Also used to re-centre any embedding so that
    sum_i a_i X_i = 0 as Section 5 requires of the inputs to CNT-GW."""
    x = np.asarray(x, dtype=np.float64)
    return x - (w[:, None] * x).sum(axis=0)[None, :]


def sqdist(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Pairwise squared Euclidean distances, summed coordinate by
    coordinate (no expansion into norms and dot products)."""
    out = np.zeros((x.shape[0], y.shape[0]))
    for k in range(x.shape[1]):
        diff = x[:, k][:, None] - y[:, k][None, :]
        out += diff * diff
    return out


def power_cost(x: np.ndarray, y: np.ndarray, p: float) -> np.ndarray:
    """c(x, y) = |x - y|^p, conditionally of negative type for 0 < p <= 2
    (Section 2, "Embeddable Costs")."""
    d2 = sqdist(x, y)
    if p == 2.0:
        return d2
    return np.power(d2, 0.5 * p)


def cnt_kernel(c_xy: np.ndarray, c_x0: np.ndarray, c_0y: np.ndarray) -> np.ndarray:
    """k(x, x') = (c(x, x0) + c(x0, x') - c(x, x')) / 2
    (Section 2, Proposition on CNT costs inducing positive kernels)."""
    return 0.5 * (c_x0[:, None] + c_0y[None, :] - c_xy)


def kernel_from_cost(c: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Algorithm 4 (Kernel), Appendix B.2: kernel from a CNT cost matrix with
    base index 1, then weighted double centring.  The centring step's indices
    are garbled in the paper; it is read as K <- (I - 1 w^T) K (I - w 1^T)."""
    k = cnt_kernel(c, c[:, 0], c[0, :])
    col = w @ k                      # sum_i w_i K_ij
    row = k @ w                      # sum_j w_j K_ij
    tot = w @ k @ w
    return k - col[None, :] - row[:, None] + tot


def kernel_pca(k: np.ndarray, dim: int, rel_floor: float = 1e-12):
    """Kernel PCA (Appendix B.2): top-D eigenpairs of the centred kernel,
    X = V sqrt(Lambda).  Eigenvalues below rel_floor * lambda_max are
    dropped (their feature columns are zero)."""
    lam, vec = np.linalg.eigh(k)
    order = np.argsort(lam)[::-1][:dim]
    lam, vec = lam[order], vec[:, order]
    keep = lam > rel_floor * max(lam[0], 0.0)
    lam = np.where(keep, lam, 0.0)
    vec = np.where(keep[None, :], vec, 0.0)
    return lam, vec


def full_kpca_features(x: np.ndarray, a: np.ndarray, p: float, dim: int):
    """Kernel PCA of all n points (Appendix B, "Kernel PCA"): Algorithm 4's
    kernel of c = |x - x'|^p with weighted double centring by a, its top
    dim eigenpairs, X_i = V_i sqrt(Lambda).  Returns (X n x dim, Lambda)."""
    x = np.asarray(x, np.float64)
    k = kernel_from_cost(power_cost(x, x, p), np.asarray(a, np.float64))
    lam, vec = kernel_pca(k, dim)
    return vec * np.sqrt(lam)[None, :], lam


@dataclass
class Landmarks:
    """Frozen landmark kernel PCA: positions, weights, eigenpairs."""

    pts: np.ndarray      # (L, d)
    w: np.ndarray        # (L,)
    lam: np.ndarray      # (D,)
    vec: np.ndarray      # (L, D)
    p: float


def fit_landmarks(pts: np.ndarray, p: float, dim: int) -> Landmarks:
    """Landmark kernel PCA: Algorithm 4 on the landmark cost matrix with
    uniform landmark weights, then the top-D eigenpairs."""
    w = np.full(pts.shape[0], 1.0 / pts.shape[0])
    k = kernel_from_cost(power_cost(pts, pts, p), w)
    lam, vec = kernel_pca(k, dim)
    return Landmarks(np.array(pts, dtype=np.float64), w, lam, vec, p)


def kernel_proj(x: np.ndarray, lm: Landmarks) -> np.ndarray:
    """Algorithm 13 (Kernel-Proj): Pi(x)_d = Lambda_d^{-1/2} sum_l k(x, x_l)
    V_ld, with k the landmark-centred CNT kernel (the kernel of the CNT
    proposition, centred against the landmark measure as in Algorithm 4)."""
    c_xl = power_cost(x, lm.pts, lm.p)               # (N, L)
    c_ll = power_cost(lm.pts, lm.pts, lm.p)          # (L, L)
    x0 = lm.pts[0:1]
    c_x0 = power_cost(x, x0, lm.p)[:, 0]
    c_l0 = power_cost(lm.pts, x0, lm.p)[:, 0]
    k_xl = cnt_kernel(c_xl, c_x0, c_l0)              # (N, L)
    k_ll = cnt_kernel(c_ll, c_l0, c_l0)              # (L, L)
    w = lm.w
    kc = (k_xl - (k_xl @ w)[:, None] - (w @ k_ll)[None, :] + w @ k_ll @ w)
    inv = np.where(lm.lam > 0, 1.0 / np.sqrt(np.where(lm.lam > 0, lm.lam, 1.0)), 0.0)
    return (kc @ lm.vec) * inv[None, :]


def kernel_proj_jacobian(x: np.ndarray, lm: Landmarks) -> np.ndarray:
    """Gradient of Algorithm 13's map (Appendix B.6, "Approximation with
    Kernel PCA"): J[n, d, :] = Lambda_d^{-1/2} sum_l grad_x k(x_n, x_l) V_ld.
    For c = |x - x'|^p, grad_x c = p |x - x'|^{p-2} (x - x'), taken as 0 at
    x = x' (the subgradient that central differences return for p = 1)."""
    n, dim_in = x.shape
    diff = x[:, None, :] - lm.pts[None, :, :]                 # (N, L, d)
    r2 = (diff * diff).sum(-1)
    if lm.p == 2.0:
        coef = np.full_like(r2, 2.0)
    else:
        safe = np.where(r2 > 0, r2, 1.0)
        coef = np.where(r2 > 0, lm.p * np.power(safe, 0.5 * lm.p - 1.0), 0.0)
    grad_c = coef[:, :, None] * diff                          # (N, L, d)
    # centred kernel: k~ = -1/2 [c(x, x_l) - sum_m w_m c(x, x_m)] + const(x_l)
    mean_grad = np.einsum("m,nmk->nk", lm.w, grad_c)
    grad_k = -0.5 * (grad_c - mean_grad[:, None, :])          # (N, L, d)
    inv = np.where(lm.lam > 0, 1.0 / np.sqrt(np.where(lm.lam > 0, lm.lam, 1.0)), 0.0)
    return np.einsum("nlk,ld->ndk", grad_k, lm.vec) * inv[None, :, None]


def landmark_features(x: np.ndarray, a: np.ndarray, lm: Landmarks) -> np.ndarray:
    """Lifted features of all points: Nystrom map through the frozen
    landmarks, then re-centred with the weights a (Section 5 requires
    sum_i a_i X_i = 0)."""
    return centre(kernel_proj(x, lm), a)


# --------------------------------------------------------------------------
# Entropic OT
# --------------------------------------------------------------------------


def lse(v: np.ndarray, axis: int) -> np.ndarray:
    """Max-shifted log-sum-exp along one axis."""
    mx = np.max(v, axis=axis, keepdims=True)
    mx = np.where(np.isfinite(mx), mx, 0.0)
    return (mx + np.log(np.sum(np.exp(v - mx), axis=axis, keepdims=True))).squeeze(axis)


def softmin_rows(b: np.ndarray, g: np.ndarray, c: np.ndarray, eps: float) -> np.ndarray:
    """Sinkhorn operator over j (Appendix A.1, Eq. sinkhorn_operators):
    -eps log sum_j exp(log b_j + (g_j - C_ij) / eps)."""
    return -eps * lse(np.log(b)[None, :] + (g[None, :] - c) / eps, axis=1)


def softmin_cols(a: np.ndarray, f: np.ndarray, c: np.ndarray, eps: float) -> np.ndarray:
    """Sinkhorn operator over i: -eps log sum_i exp(log a_i + (f_i - C_ij)/eps)."""
    return -eps * lse(np.log(a)[:, None] + (f[:, None] - c) / eps, axis=0)


_CLIB = None


def _c_sinkhorn_lib():
    """The oracle's compiled Sinkhorn loop (sinkhorn.c), built with gcc on
    first use if it is missing."""
    global _CLIB
    if _CLIB is None:
        import ctypes
        import os

        from . import build_c
        if not os.path.exists(build_c.OUT):
            build_c.build()
        lib = ctypes.CDLL(build_c.OUT)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_sinkhorn.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_sinkhorn.restype = ctypes.c_int
        _CLIB = lib
    return _CLIB


def _sinkhorn_c(a, b, c, eps, n_iter, f, g, symmetric, ct=None):
    """The same iterations as the NumPy loop of sinkhorn(), in plain C over
    rows (and rows of C^T for the columns), threads over rows."""
    import ctypes

    lib = _c_sinkhorn_lib()
    dp = ctypes.POINTER(ctypes.c_double)
    c = np.ascontiguousarray(c, dtype=np.float64)
    ct = np.ascontiguousarray(c.T) if ct is None else ct
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    g = np.ascontiguousarray(g, dtype=np.float64).copy()
    ptr = lambda v: v.ctypes.data_as(dp)  # noqa: E731
    rc = lib.oracle_sinkhorn(ptr(c), ptr(ct), c.shape[0], c.shape[1], ptr(a), ptr(b), float(eps), int(n_iter),
                             1 if symmetric else 0, ptr(f), ptr(g))
    if rc != 0:
        raise MemoryError("oracle C Sinkhorn: allocation failed")
    return f, g


def sinkhorn(a, b, c, eps, n_iter, f0=None, g0=None, symmetric=True, backend="numpy", ct=None):
    """Algorithm 2 (Sinkhorn) or Algorithm 3 (Sinkhorn-symm), Appendix B.1,
    in the log domain.  Symmetric: both half-steps read iterate n.
    Alternating: the g update reads the new f.  backend "c" runs the same
    iterations in the oracle's C loop (sinkhorn.c; ct may pass C^T)."""
    f = np.zeros(len(a)) if f0 is None else np.array(f0, dtype=np.float64)
    g = np.zeros(len(b)) if g0 is None else np.array(g0, dtype=np.float64)
    if backend == "c":
        return _sinkhorn_c(a, b, c, eps, n_iter, f, g, symmetric, ct)
    if backend != "numpy":
        raise ValueError(f"unknown backend {backend!r}")
    for _ in range(n_iter):
        if symmetric:
            tf = softmin_rows(b, g, c, eps)
            tg = softmin_cols(a, f, c, eps)
            f, g = 0.5 * (f + tf), 0.5 * (g + tg)
        else:
            f = softmin_rows(b, g, c, eps)
            g = softmin_cols(a, f, c, eps)
    return f, g


def plan(a, b, f, g, c, eps):
    """Coupling from dual potentials (Section 2, Eq. sinkhorn_pi):
    pi_ij = a_i b_j exp((f_i + g_j - C_ij) / eps)."""
    return a[:, None] * b[None, :] * np.exp((f[:, None] + g[None, :] - c) / eps)


def marginal_error(pi, a, b) -> float:
    """Err(pi) = |pi 1 - a|_1 + |pi^T 1 - b|_1 (Appendix A.1)."""
    return float(np.abs(pi.sum(1) - a).sum() + np.abs(pi.sum(0) - b).sum())


def kl_divergence(pi, a, b) -> float:
    """KL(pi | a x b) = sum pi log(pi / (a b)) (Section 2, EOT problem)."""
    ab = a[:, None] * b[None, :]
    mask = pi > 0
    return float(np.sum(pi[mask] * np.log(pi[mask] / ab[mask])))


# --------------------------------------------------------------------------
# CNT-GW (Algorithm 1)
# --------------------------------------------------------------------------


# Algorithm 6 doubles the count when the EGW objective increases.  An
# increase is taken to be one above the float64 rounding of the two values
# compared (relative to the scale of the terms they are differences of).
ADAPTIVE_TIE = 1e-12


def eps_schedule(eps_start: float, eps_end: float, n_outer: int) -> np.ndarray:
    """Outer temperature schedule.  The paper fixes eps; an annealed
    schedule is read as geometric, eps_t = eps_0 (eps_end/eps_0)^(t/(T-1))."""
    if n_outer <= 1 or eps_start == eps_end:
        return np.full(max(n_outer, 1), float(eps_start))
    t = np.arange(n_outer) / (n_outer - 1)
    return eps_start * np.power(eps_end / eps_start, t)


def lift(v: np.ndarray) -> np.ndarray:
    """[v, |v|^2 / 2] (Algorithm 1, lifted features)."""
    return np.concatenate([v, 0.5 * np.sum(v * v, axis=1, keepdims=True)], axis=1)


@dataclass
class GWResult:
    f: np.ndarray            # final potentials, Algorithm 1 convention
    g: np.ndarray
    gamma: np.ndarray        # Gamma_T = X^T pi Y
    gamma_prev: np.ndarray   # Gamma_{T-1}, the map the final pi was built with
    pi: np.ndarray           # final coupling
    eps: float               # last outer temperature
    history: list = field(default_factory=list)
    n_inner_final: int = 0   # Sinkhorn count of the last outer step
    doublings: int = 0       # adaptive counts: doublings made
    adaptive_log: list = field(default_factory=list)   # (t, e_new, e_old, scale, doubled)


def cnt_gw(a, b, X, Y, eps_start, eps_end, n_outer, n_inner, gamma0=None,
           f0=None, g0=None, symmetric=True, record=False, inner_tol=None,
           anneal_final=False, adaptive=False, backend="numpy") -> GWResult:
    """Algorithm 1 (CNT-GW), Section 5, with a fixed number of outer steps.

    Per outer step t: Zbar_j = [Gamma_t Y_j, |Y_j|^2/2]; the squared-norm
    cost between lifted features is materialised; Sinkhorn runs at eps_t/8
    warm-started from the previous potentials (Appendix B.1, warm start);
    then X~_j = sum_i a_i X_i exp(8/eps (f_i + g_j - |Xbar_i - Zbar_j|^2)) and
    Gamma_{t+1} = sum_j b_j X~_j Y_j^T.  With inner_tol set, each inner solve
    runs to that marginal error instead of n_inner iterations.

    anneal_final: Sinkhorn annealing in the last outer step only (Appendix
    B.1, "Sinkhorn Annealing"): iteration n = 1..n_inner of that step runs
    at eps_n = eps_T / sqrt(n); the plan, Gamma_T and the returned eps use
    the last eps_n.  Potentials are in cost units, so nothing is rebased.

    adaptive: Algorithm 6's adaptive counts applied to CNT-GW (Appendix B,
    "Adaptive Sinkhorn Iterations", with the lifted squared-norm loss as the
    base cost): after each outer step the EGW objective L_lift + eps KL of
    the new plan is compared with that of the previous plan at the same
    eps, and the count doubles when the new value is larger.  "Larger" is
    read as larger by more than the float64 rounding of the comparison,
    1e-12 max(|EGW|, C) (C the constant of Lemma C.1, the scale of the terms
    the loss is a difference of), so that an exact tie never fires; there
    is no cap.  The previous plan of step 0 is a x b when gamma0 is None;
    with a given gamma0 the first comparison is after step 1.  Each
    comparison is recorded in GWResult.adaptive_log as (t, e_new, e_old,
    scale, doubled).

    backend: "numpy", or "c" for the fixed-count Sinkhorn iterations in the
    oracle's C loop (large problems)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    gamma = np.zeros((X.shape[1], Y.shape[1])) if gamma0 is None else np.array(gamma0, np.float64)
    xbar = lift(X)
    f = np.zeros(len(a)) if f0 is None else np.array(f0, np.float64)
    g = np.zeros(len(b)) if g0 is None else np.array(g0, np.float64)
    hist = []
    gamma_prev = gamma
    pi = None
    eps_list = list(eps_schedule(eps_start, eps_end, n_outer))
    n_in, doublings = int(n_inner), 0
    adaptive_log = []
    prev = None
    c_scale = constant_c(X, Y, a, b) if adaptive else 0.0
    if adaptive and gamma0 is None:
        prev = (lifted_loss(X, Y, a, b, a[:, None] * b[None, :]), 0.0)
    for t, eps in enumerate(eps_list):
        zbar = np.concatenate([Y @ gamma.T, 0.5 * np.sum(Y * Y, axis=1, keepdims=True)], axis=1)
        cbar = sqdist(xbar, zbar)
        cbar_t = np.ascontiguousarray(cbar.T) if backend == "c" else None
        if anneal_final and t == n_outer - 1:
            for it in range(1, n_in + 1):
                f, g = sinkhorn(a, b, cbar, eps / np.sqrt(it) / 8.0, 1, f, g, symmetric, backend, cbar_t)
            eps = eps / np.sqrt(max(n_in, 1))
            eps_list[-1] = eps
        elif inner_tol is None:
            f, g = sinkhorn(a, b, cbar, eps / 8.0, n_in, f, g, symmetric, backend, cbar_t)
        else:
            f, g = sinkhorn_converged(a, b, cbar, eps / 8.0, f, g, tol=inner_tol)
        epsp = eps / 8.0
        expo = np.exp((f[:, None] + g[None, :] - cbar) / epsp)
        del cbar_t
        xt = expo.T @ (a[:, None] * X)          # X~_j = sum_i a_i X_i expo_ij
        new_gamma = (b[:, None] * xt).T @ Y
        pi = a[:, None] * b[None, :] * expo
        if record:
            hist.append({"eps": float(eps), "gamma": new_gamma.copy(),
                         "pi": pi.copy(), "f": f.copy(), "g": g.copy()})
        gamma_prev, gamma = gamma, new_gamma
        if adaptive and t < n_outer - 1:
            cur = (lifted_loss(X, Y, a, b, pi), kl_divergence(pi, a, b))
            if prev is not None:
                e_new, e_old = cur[0] + eps * cur[1], prev[0] + eps * prev[1]
                scale = max(abs(e_old), c_scale)
                doubled = e_new - e_old > ADAPTIVE_TIE * scale
                if doubled:
                    n_in *= 2
                    doublings += 1
                adaptive_log.append((t, e_new, e_old, scale, doubled))
            prev = cur
    return GWResult(f, g, gamma, gamma_prev, pi, float(eps_list[-1]), hist, n_in, doublings, adaptive_log)


# --------------------------------------------------------------------------
# Losses
# --------------------------------------------------------------------------


def constant_c(X, Y, a, b) -> float:
    """C(alpha, beta) of Lemma C.1 by its O(N^2) definition:
    sum a a |x - x'|^4 + sum b b |y - y'|^4 - 4 (sum a |x|^2)(sum b |y|^2)."""
    dx = sqdist(X, X)
    dy = sqdist(Y, Y)
    return float(a @ (dx * dx) @ a + b @ (dy * dy) @ b
                 - 4.0 * (a @ np.sum(X * X, 1)) * (b @ np.sum(Y * Y, 1)))


def lifted_loss(X, Y, a, b, pi) -> float:
    """Lemma C.1: L(pi) = C - 8 |sum pi x y^T|^2 - 4 sum pi |x|^2 |y|^2, for
    centred features.  Equals the GW loss for any pi in Pi(a, b)."""
    gam = X.T @ pi @ Y
    nm = np.sum(X * X, 1)[:, None] * np.sum(Y * Y, 1)[None, :]
    return constant_c(X, Y, a, b) - 8.0 * float(np.sum(gam * gam)) - 4.0 * float(np.sum(pi * nm))


def quartic_loss_literal(cx, cy, pi) -> float:
    """Eq. GW_loss by its definition, sum_ijkl (cX_ik - cY_jl)^2 pi_ij pi_kl
    (small inputs only: N^2 M^2 terms)."""
    diff = cx[:, None, :, None] - cy[None, :, None, :]        # (i, j, k, l)
    return float(np.einsum("ijkl,ij,kl->", diff * diff, pi, pi))


def quartic_loss(cx, cy, pi) -> float:
    """Eq. GW_loss, exactly rearranged for any pi (no feasibility used):
    r^T cX^2 r + c^T cY^2 c - 2 sum_ij pi_ij (cX pi cY)_ij with r, c the
    marginals of pi itself."""
    r = pi.sum(1)
    c = pi.sum(0)
    return float(r @ (cx * cx) @ r + c @ (cy * cy) @ c - 2.0 * np.sum(pi * (cx @ pi @ cy)))


def egw_objective(X, Y, a, b, pi, eps) -> float:
    """EGW objective L(pi) + eps KL(pi | a x b) (Section 2, Eq. entropic GW),
    with L in the lifted form."""
    return lifted_loss(X, Y, a, b, pi) + eps * kl_divergence(pi, a, b)


def dual_function(X, Y, a, b, gamma, eps, tol=1e-15) -> float:
    """Phi_eps(Gamma) = |Gamma|^2 + OT^Gamma_eps / 8 (proof of the dual-descent
    proposition), with OT^Gamma_eps the EOT value for the bilinear cost
    c_Gamma = -16 <Gamma, x y^T> - 4 |x|^2 |y|^2 (Remark C.2) at eps."""
    c = -16.0 * (X @ gamma @ Y.T) - 4.0 * np.sum(X * X, 1)[:, None] * np.sum(Y * Y, 1)[None, :]
    f, g = sinkhorn_converged(a, b, c, eps, tol=tol)
    pi = plan(a, b, f, g, c, eps)
    ot = float(np.sum(pi * c)) + eps * kl_divergence(pi, a, b)
    return float(np.sum(gamma * gamma)) + ot / 8.0


# --------------------------------------------------------------------------
# Comparison algorithms used as pins
# --------------------------------------------------------------------------


def full_linearisation(cx, cy, pi):
    """grad L(pi)_ij = 2 sum_kl (cX_ik - cY_jl)^2 pi_kl (primal-descent proof,
    Appendix C), exactly rearranged for any pi."""
    r = pi.sum(1)
    c = pi.sum(0)
    return 2.0 * ((cx * cx) @ r[:, None] + ((cy * cy) @ c)[None, :] - 2.0 * (cx @ pi @ cy))


def entropic_gw(a, b, cx, cy, eps, n_outer, n_inner, pi0=None, inner_tol=None):
    """Entropic-GW (Section 4.2, Eq. entropic_cgd_sequence): pi_{t+1} is the
    EOT plan at eps for the cost grad L(pi_t), starting from a x b."""
    pi = np.outer(a, b) if pi0 is None else pi0
    out = []
    for _ in range(n_outer):
        c = full_linearisation(cx, cy, pi)
        if inner_tol is None:
            f, g = sinkhorn(a, b, c, eps, n_inner)
        else:
            f, g = sinkhorn_converged(a, b, c, eps, tol=inner_tol)
        pi = plan(a, b, f, g, c, eps)
        out.append(pi)
    return out


def kernel_gw(a, b, cx, cy, eps, n_outer, n_inner, inner_tol=None):
    """Algorithm 5 (Kernel-GW), Appendix B.3: cost -4 K^X_ii K^Y_jj
    - 16 sum_kl K^X_ik K^Y_jl pi_kl, symmetric Sinkhorn at eps."""
    kx = kernel_from_cost(cx, a)
    ky = kernel_from_cost(cy, b)
    pi = np.outer(a, b)
    out = []
    for _ in range(n_outer):
        c = -4.0 * np.diag(kx)[:, None] * np.diag(ky)[None, :] - 16.0 * (kx @ pi @ ky.T)
        if inner_tol is None:
            f, g = sinkhorn(a, b, c, eps, n_inner, symmetric=True)
        else:
            f, g = sinkhorn_converged(a, b, c, eps, tol=inner_tol, symmetric=True)
        pi = plan(a, b, f, g, c, eps)
        out.append(pi)
    return out


# --------------------------------------------------------------------------
# Gradients (Appendix B.6)
# --------------------------------------------------------------------------


def grad_features(X, Y, a, b, pi, gamma):
    """Envelope gradient of GW_eps with respect to the lifted source
    features (Appendix B.6): d/dX_i of the constant C of Lemma C.1 plus
    sum_j pi_ij d/dX_i c_Gamma(X_i, Y_j), with c_Gamma of Remark C.2 and
    Gamma, pi held at the optimum.  Derivative of C written from its double
    sum: 8 a_i sum_k a_k |X_i - X_k|^2 (X_i - X_k) - 8 a_i s_y X_i."""
    n2 = np.sum(X * X, 1)
    m2 = np.sum(Y * Y, 1)
    s_y = float(b @ m2)
    dx = sqdist(X, X)
    wk = a[None, :] * dx                                      # a_k |X_i - X_k|^2
    dc = 8.0 * a[:, None] * (wk.sum(1)[:, None] * X - wk @ X) - 8.0 * a[:, None] * s_y * X
    dot = -16.0 * (pi @ Y) @ gamma.T - 8.0 * X * (pi @ m2)[:, None]
    return dc + dot


def grad_features_target(X, Y, a, b, pi, gamma):
    """Same envelope gradient for the target features (roles swapped)."""
    return grad_features(Y, X, b, a, pi.T, gamma.T)


def chain_centre(gx_feat, w):
    """Chain rule through re-centring X = P - sum_k w_k P_k:
    dL/dP_i = G_i - w_i sum_k G_k."""
    return gx_feat - w[:, None] * gx_feat.sum(0)[None, :]


def grad_positions_sqeuclid(X, Y, a, b, pi, gamma):
    """Position gradient for the squared Euclidean penalty (features are the
    centred points, Section 3 example)."""
    return chain_centre(grad_features(X, Y, a, b, pi, gamma), a)


def grad_positions_power(x, X, Y, a, b, pi, gamma, lm: Landmarks):
    """Position gradient through the frozen Nystrom map (Algorithm 12 with
    Algorithm 13), including re-centring."""
    gf = chain_centre(grad_features(X, Y, a, b, pi, gamma), a)   # (N, D)
    jac = kernel_proj_jacobian(x, lm)                            # (N, D, d)
    return np.einsum("nd,ndk->nk", gf, jac)


def grad_positions_quartic(x, a, pi, cy, p=2.0):
    """Independent pin: envelope gradient of Eq. GW_loss itself at fixed pi,
    d/dx_i sum_ijkl (cX_ik - cY_jl)^2 pi_ij pi_kl
      = 4 sum_k [cX_ik r_i r_k - (pi cY pi^T)_ik] grad_1 cX(x_i, x_k)."""
    cx = power_cost(x, x, p)
    r = pi.sum(1)
    w = cx * r[:, None] * r[None, :] - pi @ cy @ pi.T
    diff = x[:, None, :] - x[None, :, :]
    r2 = (diff * diff).sum(-1)
    if p == 2.0:
        coef = np.full_like(r2, 2.0)
    else:
        safe = np.where(r2 > 0, r2, 1.0)
        coef = np.where(r2 > 0, p * np.power(safe, 0.5 * p - 1.0), 0.0)
    return 4.0 * np.einsum("ik,ik,ikd->id", w, coef, diff)


def grad_weights(cx, cy, a, b, pi, eps, max_iter=200000):
    """Weight gradient of GW_eps: by the Lagrangian of the EGW problem the
    derivative along sum(da) = 0 is <F, da>, with F the EOT potential at eps
    for the linearised cost grad L(pi*) = 2 sum_kl (cX - cY)^2 pi*_kl (the
    potential of the converged problem: Sinkhorn runs to the FP64 floor).
    Returned centred (sum a_i F_i = 0); constants do not matter on the
    simplex."""
    c = full_linearisation(cx, cy, pi)
    f, g = sinkhorn_converged(a, b, c, eps, tol=1e-13, max_iter=max_iter)
    return f - a @ f


# --------------------------------------------------------------------------
# Converged solves (for finite differences and pins)
# --------------------------------------------------------------------------


def sinkhorn_converged(a, b, c, eps, f0=None, g0=None, tol=1e-14, max_iter=100000,
                       symmetric=False):
    """Run Sinkhorn until the marginal error of the plan is below tol, or
    until it stops decreasing (the float64 rounding floor)."""
    f = np.zeros(len(a)) if f0 is None else f0.copy()
    g = np.zeros(len(b)) if g0 is None else g0.copy()
    it = 0
    best = np.inf
    stall = 0
    while it < max_iter:
        f, g = sinkhorn(a, b, c, eps, 20, f, g, symmetric)
        it += 20
        err = marginal_error(plan(a, b, f, g, c, eps), a, b)
        if err < tol:
            break
        if err < 0.5 * best:
            best = err
            stall = 0
        else:
            stall += 1
            if stall >= 10 and err < 1e-12:
                break
    return f, g


def sgw_divergence(a, b, X, Y, eps_start, eps_end, n_outer, n_inner, inner_tol=None) -> dict:
    """Sinkhorn-GW divergence (Section 4, "Entropic Bias"): the EGW value of
    the pair minus half the EGW values of each measure with itself,
        SGW = GW_eps(alpha, beta) - (GW_eps(alpha, alpha) + GW_eps(beta, beta)) / 2,
    each GW_eps the EGW objective L(pi) + eps KL(pi | a x b) of Algorithm 1
    run from Gamma_0 = 0 with the same schedule (eps the last temperature;
    inner_tol as in cnt_gw)."""
    def one(p, P, q, Q):
        res = cnt_gw(p, q, P, Q, eps_start, eps_end, n_outer, n_inner, inner_tol=inner_tol)
        return egw_objective(P, Q, p, q, res.pi, res.eps)

    xy = one(a, X, b, Y)
    xx = one(a, X, a, X)
    yy = one(b, Y, b, Y)
    return {"sgw": xy - 0.5 * (xx + yy), "gw_xy": xy, "gw_xx": xx, "gw_yy": yy}


def sgw_grad_positions(a, b, x, y, eps, tol=1e-13):
    """Position gradient of the Sinkhorn-GW divergence (Section 4, "Entropic
    Bias") for the squared Euclidean penalty, by the envelope theorem
    (Appendix B.6) at solves converged at a fixed eps: the gradient of
    GW_eps(alpha, beta) minus half that of GW_eps(alpha, alpha), in which x
    is both the source and the target (the two envelope gradients summed);
    the same for y.  tol: the outer and inner tolerances of the converged
    solves (tol and tol / 10).  Returns (grad_x, grad_y)."""
    def parts(p, P, q, Q):
        PP, QQ = centre(P, p), centre(Q, q)
        gam, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        gs = chain_centre(grad_features(PP, QQ, p, q, pi, gam), p)
        gt = chain_centre(grad_features_target(PP, QQ, p, q, pi, gam), q)
        return gs, gt

    gx, gy = parts(a, x, b, y)
    sx, tx = parts(a, x, a, x)
    sy, ty = parts(b, y, b, y)
    return gx - 0.5 * (sx + tx), gy - 0.5 * (sy + ty)


def sgw_grad_weights(a, b, x, y, eps, tol=1e-13):
    """Weight gradient of the Sinkhorn-GW divergence (Section 4, "Entropic
    Bias") for the squared Euclidean penalty.  GW_eps(alpha, beta) depends on
    a through its source marginal and on b through its target marginal; by
    the Lagrangian of the EGW problem (as in grad_weights) each derivative
    along the simplex is the EOT potential of the linearised cost
    2 sum_kl (cX - cY)^2 pi*_kl on that side.  GW_eps(alpha, alpha) has a in
    both marginals, so its derivative is the sum of its two potentials.
    Solves converged at eps (tol and tol / 10); returns (grad_a, grad_b),
    each centred (sum a_i grad_a_i = 0), since constants do not matter on
    the simplex."""
    def pots(p, P, q, Q):
        PP, QQ = centre(P, p), centre(Q, q)
        gam, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        c = full_linearisation(sqdist(PP, PP), sqdist(QQ, QQ), pi)
        return sinkhorn_converged(p, q, c, eps, tol=tol, max_iter=200000)

    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fxy, gxy = pots(a, x, b, y)
    fxx, gxx = pots(a, x, a, x)
    fyy, gyy = pots(b, y, b, y)
    ga = fxy - 0.5 * (fxx + gxx)
    gb = gxy - 0.5 * (fyy + gyy)
    return ga - a @ ga, gb - b @ gb


def sgw_grad_weights_lifted(a, b, x, y, eps, lmx: Landmarks, lmy: Landmarks, tol=1e-13):
    """sgw_grad_weights for a penalty lifted by frozen landmark maps (as in
    sgw_grad_positions_lifted): each problem's cost matrices are the squared
    distances of the embedded, re-centred features.  Returns (grad_a,
    grad_b), centred."""
    def pots(p, P, lmP, q, Q, lmQ):
        PP, QQ = landmark_features(P, p, lmP), landmark_features(Q, q, lmQ)
        gam, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        c = full_linearisation(sqdist(PP, PP), sqdist(QQ, QQ), pi)
        return sinkhorn_converged(p, q, c, eps, tol=tol, max_iter=200000)

    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fxy, gxy = pots(a, x, lmx, b, y, lmy)
    fxx, gxx = pots(a, x, lmx, a, x, lmx)
    fyy, gyy = pots(b, y, lmy, b, y, lmy)
    ga = fxy - 0.5 * (fxx + gxx)
    gb = gxy - 0.5 * (fyy + gyy)
    return ga - a @ ga, gb - b @ gb


def sgw_grad_positions_lifted(a, b, x, y, eps, lmx: Landmarks, lmy: Landmarks, tol=1e-13):
    """Position gradient of the Sinkhorn-GW divergence for a penalty lifted
    by frozen landmark maps (|x - x'|^p through kernel PCA, Section 5,
    Algorithm 4 and Algorithm 13): alpha's points are embedded by Pi_x and
    beta's by Pi_y in every term, so GW_eps(alpha, alpha) compares
    Pi_x(x) with itself and GW_eps(beta, beta) compares Pi_y(y) with itself.
    Each envelope gradient (Appendix B.6) is taken with respect to the
    re-centred features and chained through the centring and the frozen
    map's Jacobian (Algorithm 12).  Returns (grad_x, grad_y)."""
    def parts(p, P, lmP, q, Q, lmQ):
        PP, QQ = landmark_features(P, p, lmP), landmark_features(Q, q, lmQ)
        gam, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        gs = chain_centre(grad_features(PP, QQ, p, q, pi, gam), p)
        gt = chain_centre(grad_features_target(PP, QQ, p, q, pi, gam), q)
        return (np.einsum("nd,ndk->nk", gs, kernel_proj_jacobian(P, lmP)),
                np.einsum("nd,ndk->nk", gt, kernel_proj_jacobian(Q, lmQ)))

    gx, gy = parts(a, x, lmx, b, y, lmy)
    sx, tx = parts(a, x, lmx, a, x, lmx)
    sy, ty = parts(b, y, lmy, b, y, lmy)
    return gx - 0.5 * (sx + tx), gy - 0.5 * (sy + ty)


def sgw_value_converged_lifted(a, b, x, y, eps, lmx: Landmarks, lmy: Landmarks, tol=1e-13) -> float:
    """SGW_eps of the measures embedded by the frozen maps Pi_x and Pi_y
    (as in sgw_grad_positions_lifted), every EGW problem converged at eps."""
    def one(p, P, lmP, q, Q, lmQ):
        PP, QQ = landmark_features(P, p, lmP), landmark_features(Q, q, lmQ)
        _, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        return egw_objective(PP, QQ, p, q, pi, eps)
    return one(a, x, lmx, b, y, lmy) - 0.5 * (one(a, x, lmx, a, x, lmx) + one(b, y, lmy, b, y, lmy))


def sgw_value_converged(a, b, x, y, eps, tol=1e-13) -> float:
    """SGW_eps with every EGW problem solved by cnt_gw_converged at eps."""
    def one(p, P, q, Q):
        PP, QQ = centre(P, p), centre(Q, q)
        _, pi, _, _ = cnt_gw_converged(p, q, PP, QQ, eps, tol=tol, sink_tol=tol / 10)
        return egw_objective(PP, QQ, p, q, pi, eps)
    return one(a, x, b, y) - 0.5 * (one(a, x, a, x) + one(b, y, b, y))


def sgw_barycenter(a, b, x, y, z0, w, lam, step, n_steps, eps, tol=1e-13):
    """GW barycentre flow (Section 6, "GW Barycenters"): gradient descent on
    the points z of gamma_z = sum_i w_i delta_{z_i} for
    (1 - lam) SGW_eps(gamma_z, alpha) + lam SGW_eps(gamma_z, beta), squared
    Euclidean penalty, converged solves; each point moves by -step / w_i
    times its gradient (the gradient per unit of mass).  Returns z after
    n_steps and the objective before each step and after the last."""
    z = np.array(z0, np.float64)
    w = np.asarray(w, np.float64)
    obj = []
    for s in range(n_steps + 1):
        obj.append((1 - lam) * sgw_value_converged(w, a, z, x, eps, tol)
                   + lam * sgw_value_converged(w, b, z, y, eps, tol))
        if s == n_steps:
            break
        gzx, _ = sgw_grad_positions(w, a, z, x, eps, tol)
        gzy, _ = sgw_grad_positions(w, b, z, y, eps, tol)
        z = z - step / w[:, None] * ((1 - lam) * gzx + lam * gzy)
    return z, obj


def sgw_barycenter_lifted(a, b, x, y, z0, w, lam, step, n_steps, eps, lmz: Landmarks, lma: Landmarks,
                          lmb: Landmarks, tol=1e-13):
    """The barycentre flow of sgw_barycenter for a penalty lifted by frozen
    landmark maps: z is embedded by Pi_z (its landmark points stay where
    they were fitted while z moves), alpha by Pi_a and beta by Pi_b, in every
    term (sgw_grad_positions_lifted).  Returns z after n_steps and the
    objective before each step and after the last."""
    z = np.array(z0, np.float64)
    w = np.asarray(w, np.float64)
    obj = []
    for s in range(n_steps + 1):
        obj.append((1 - lam) * sgw_value_converged_lifted(w, a, z, x, eps, lmz, lma, tol)
                   + lam * sgw_value_converged_lifted(w, b, z, y, eps, lmz, lmb, tol))
        if s == n_steps:
            break
        gzx, _ = sgw_grad_positions_lifted(w, a, z, x, eps, lmz, lma, tol)
        gzy, _ = sgw_grad_positions_lifted(w, b, z, y, eps, lmz, lmb, tol)
        z = z - step / w[:, None] * ((1 - lam) * gzx + lam * gzy)
    return z, obj


def cnt_gw_converged(a, b, X, Y, eps, gamma0=None, tol=1e-13, max_outer=5000,
                     sink_tol=1e-14):
    """Algorithm 1 with the paper's stopping rule |Gamma_t - Gamma_{t+1}| <= tol
    and Sinkhorn solved to sink_tol at every outer step."""
    gamma = np.zeros((X.shape[1], Y.shape[1])) if gamma0 is None else gamma0.copy()
    xbar = lift(X)
    f = np.zeros(len(a))
    g = np.zeros(len(b))
    epsp = eps / 8.0
    pi = None
    for _ in range(max_outer):
        zbar = np.concatenate([Y @ gamma.T, 0.5 * np.sum(Y * Y, 1, keepdims=True)], 1)
        cbar = sqdist(xbar, zbar)
        f, g = sinkhorn_converged(a, b, cbar, epsp, f, g, tol=sink_tol)
        pi = plan(a, b, f, g, cbar, epsp)
        new_gamma = X.T @ pi @ Y
        step = float(np.linalg.norm(new_gamma - gamma))
        gamma = new_gamma
        if step <= tol:
            break
    return gamma, pi, f, g


# --------------------------------------------------------------------------
# Multiscale-GW (Appendix B, "Implementation of Multiscale-GW":
# Algorithm 7 with Coarsen and Algorithm 8, Interpolate)
# --------------------------------------------------------------------------

# Cluster sums are taken in exact integer arithmetic: every term a_i X_id is
# rounded once to a multiple of 2^-S, so the sums do not depend on the order
# of the additions.  S is the largest exponent with max|X| 2^S <= 2^61 (a
# cluster sum is at most sum(a) max|X|, which stays below 2^63); weights use
# 2^-61.
WEIGHT_SCALE_EXP = 61


def coarsen_scale_exp(X32: np.ndarray) -> int:
    """Exponent S of the fixed-point grid 2^-S of the cluster sums a_i X_id."""
    mx = float(np.max(np.abs(X32))) if X32.size else 0.0
    if mx == 0.0:
        return WEIGHT_SCALE_EXP
    _, e = np.frexp(mx)            # mx = m 2^e with 1/2 <= m < 1
    return WEIGHT_SCALE_EXP - int(e)


def nearest_centroid(X32: np.ndarray, C32: np.ndarray, block: int = 256) -> np.ndarray:
    """Index of the nearest centroid of every row, ties to the lowest index.
    The squared distance is accumulated in single precision over the
    coordinates in their order, each subtraction, square and addition
    rounded on its own: the assignment is an integer decided by floating
    point, and this fixes the precision and the order in which it is
    decided."""
    n, k = X32.shape[0], C32.shape[0]
    best = np.full(n, np.inf, dtype=np.float32)
    arg = np.zeros(n, dtype=np.int64)
    for j0 in range(0, k, block):
        cj = C32[j0:j0 + block]
        dist = np.zeros((n, cj.shape[0]), dtype=np.float32)
        for d in range(X32.shape[1]):
            t = X32[:, d][:, None] - cj[:, d][None, :]
            dist = dist + t * t
        jb = np.argmin(dist, axis=1)                  # first minimum in the block
        db = dist[np.arange(n), jb]
        upd = db < best                               # earlier blocks win ties
        best[upd] = db[upd]
        arg[upd] = j0 + jb[upd]
    return arg


def coarsen(X, a, init_idx, n_lloyd: int):
    """Coarsen (Appendix B, Multiscale-GW): weighted K-Means of the rows of
    X with k = len(init_idx) centroids started at the rows init_idx, run for
    n_lloyd Lloyd iterations (assignment to the nearest centroid, then each
    centroid moved to the a-weighted mean of its cluster; an empty cluster
    keeps its centroid).  The coarse weights are the aggregated weights of
    the clusters of the last assignment, the coarse points the centroids of
    the last update, and empty clusters are dropped (index order kept).

    X and a are taken as the single-precision values a device receives;
    centroids are held in single precision between iterations.
    Returns (Xc float32 kc x D, ac float32 kc, assign int64 n, kept int64 kc)."""
    if n_lloyd < 1:
        raise ValueError("n_lloyd >= 1")
    X32 = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
    a32 = np.asarray(a, dtype=np.float32)
    n, dim = X32.shape
    idx = np.asarray(init_idx, dtype=np.int64)
    k = len(idx)
    S = coarsen_scale_exp(X32)
    ax = np.rint(a32.astype(np.float64)[:, None] * X32.astype(np.float64) * 2.0 ** S).astype(np.int64)
    aw = np.rint(a32.astype(np.float64) * 2.0 ** WEIGHT_SCALE_EXP).astype(np.int64)
    C32 = X32[idx].copy()
    assign = np.zeros(n, dtype=np.int64)
    w = np.zeros(k, dtype=np.int64)
    for _ in range(n_lloyd):
        assign = nearest_centroid(X32, C32)
        sums = np.zeros((k, dim), dtype=np.int64)
        np.add.at(sums, assign, ax)
        w = np.zeros(k, dtype=np.int64)
        np.add.at(w, assign, aw)
        nz = w > 0
        mean = (sums[nz].astype(np.float64) * 2.0 ** -S) / (w[nz].astype(np.float64)[:, None]
                                                            * 2.0 ** -WEIGHT_SCALE_EXP)
        C32[nz] = mean.astype(np.float32)
    kept = np.nonzero(w > 0)[0]
    ac = (w[kept].astype(np.float64) * 2.0 ** -WEIGHT_SCALE_EXP).astype(np.float32)
    return C32[kept].copy(), ac, assign, kept


def kmeans_plain(X, a, init_idx, n_lloyd: int):
    """Weighted K-Means as the textbook states it (Coarsen, Appendix B,
    Multiscale-GW), in float64 throughout: n_lloyd Lloyd iterations from the
    rows init_idx, each assigning every row to its nearest centroid (ties to
    the lowest index) and moving each centroid to the a-weighted mean of its
    cluster (an empty cluster keeps its centroid).  No rounding is imposed:
    coarsen is this algorithm with its sums on a fixed-point grid and its
    distances in single precision, and the two agree wherever no assignment
    is decided within single-precision rounding of a tie.
    Returns (centroids k x D, cluster weights k, assignment n)."""
    X = np.asarray(X, np.float64)
    a = np.asarray(a, np.float64)
    C = X[np.asarray(init_idx, dtype=np.int64)].copy()
    k = C.shape[0]
    assign = np.zeros(X.shape[0], dtype=np.int64)
    w = np.zeros(k)
    for _ in range(n_lloyd):
        d2 = np.sum((X[:, None, :] - C[None, :, :]) ** 2, axis=2)
        assign = np.argmin(d2, axis=1)
        w = np.bincount(assign, weights=a, minlength=k)
        sums = np.zeros_like(C)
        np.add.at(sums, assign, a[:, None] * X)
        nz = w > 0
        C[nz] = sums[nz] / w[nz][:, None]
    return C, w, assign


def target_lift(Y, gamma) -> np.ndarray:
    """Zbar_j = [Gamma Y_j, |Y_j|^2 / 2] (Algorithm 1, lifted target)."""
    Y = np.asarray(Y, np.float64)
    return np.concatenate([Y @ np.asarray(gamma, np.float64).T, 0.5 * np.sum(Y * Y, axis=1, keepdims=True)],
                          axis=1)


def interpolate(h, P, Q, w, gamma, eps, side: int) -> np.ndarray:
    """Interpolate (Algorithm 8): the potential of fine points from the
    coarse potential h of the other side, one Sinkhorn operator against the
    coarse measure with the coarse map Gamma, in the convention of
    Algorithm 1 (squared distances between lifted features at eps/8).

    side 0: P are fine source features (N x D), Q coarse target features
            (Mc x E) with weights w and potential h = g^c; returns f (N).
    side 1: P are fine target features (M x E), Q coarse source features
            (Nc x D) with weights w and potential h = f^c; returns g (M)."""
    if side == 0:
        pbar, qbar = lift(np.asarray(P, np.float64)), target_lift(Q, gamma)
    else:
        pbar, qbar = target_lift(P, gamma), lift(np.asarray(Q, np.float64))
    c = sqdist(pbar, qbar)
    return softmin_rows(np.asarray(w, np.float64), np.asarray(h, np.float64), c, eps / 8.0)


@dataclass
class MsGWResult:
    fine: GWResult
    coarse: GWResult
    Xc: np.ndarray           # centred coarse source features
    ac: np.ndarray
    Yc: np.ndarray
    bc: np.ndarray
    f0: np.ndarray           # interpolated potentials the fine solve starts from
    g0: np.ndarray


def msgw(a, b, X, Y, init_x, init_y, n_lloyd, coarse: dict, fine: dict, gamma0=None) -> MsGWResult:
    """Multiscale-GW (Algorithm 7).  X, Y: features of the fine measures
    (centred with a, b); init_x, init_y: the rows that start each K-Means
    (k = ceil(rho N) of them); coarse, fine: keyword schedules of cnt_gw
    (eps_start, eps_end, n_outer, n_inner, ...).

    The coarse features are re-centred with their weights, as Algorithm 1
    requires of its inputs.  The coarse solve starts from gamma0 (zero by
    default); the potentials are interpolated with the coarse Gamma at the
    fine solve's first temperature, which then starts from Gamma^c and the
    interpolated (f, g)."""
    a64 = np.asarray(a, np.float64)
    b64 = np.asarray(b, np.float64)
    X = centre(X, a64)
    Y = centre(Y, b64)
    Xc, ac, _, _ = coarsen(X, a, init_x, n_lloyd)
    Yc, bc, _, _ = coarsen(Y, b, init_y, n_lloyd)
    ac64, bc64 = ac.astype(np.float64), bc.astype(np.float64)
    Xc = centre(Xc, ac64)
    Yc = centre(Yc, bc64)
    rc = cnt_gw(ac64, bc64, Xc, Yc, gamma0=gamma0, **coarse)
    eps_f = float(fine["eps_start"])
    f0 = interpolate(rc.g, X, Yc, bc64, rc.gamma, eps_f, side=0)
    g0 = interpolate(rc.f, Y, Xc, ac64, rc.gamma, eps_f, side=1)
    rf = cnt_gw(a64, b64, X, Y, gamma0=rc.gamma, f0=f0, g0=g0, **fine)
    return MsGWResult(rf, rc, Xc, ac64, Yc, bc64, f0, g0)
