"""Thin Python binding over include/gw.h: argument marshalling only.

PyTorch provides device memory and the HIP stream; every step of the solve
runs in libgwmi.so.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_PREC = {"fp32": L.FP32, "bf16": L.BF16, "bf16x3": L.BF16X3}
_MODE = {"auto": L.MODE_AUTO, "safe": L.MODE_SAFE, "stabilised": L.MODE_STABILISED}
_PEN = {"sqeuclid": L.PEN_SQEUCLID, "power": L.PEN_POWER, "features": L.PEN_FEATURES}


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.contiguous()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_params(eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True, precision="fp32",
                mode="auto", use_init_potentials=False, tol_gamma=0.0, anneal_final=False,
                adaptive_inner=False) -> L.GwParams:
    p = L.GwParams()
    p.eps_start = float(eps_start)
    p.eps_end = float(eps_start if eps_end is None else eps_end)
    p.n_outer = int(n_outer)
    p.n_inner = int(n_inner)
    p.symmetric = 1 if symmetric else 0
    p.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    p.mode = _MODE[mode] if isinstance(mode, str) else int(mode)
    p.use_init_potentials = 1 if use_init_potentials else 0
    p.tol_gamma = float(tol_gamma)
    p.anneal_final = 1 if anneal_final else 0
    p.adaptive_inner = 1 if adaptive_inner else 0
    return p


def _result_dict(r: L.GwResult, f, g, gamma) -> dict:
    return {
        "f": f, "g": g, "gamma": gamma,
        "loss_lift": r.loss_lift, "egw_objective": r.egw_objective, "kl": r.kl,
        "marginal_err": r.marginal_err, "constant_c": r.constant_c, "sum_pi_nm": r.sum_pi_nm,
        "gamma_step": r.gamma_step, "eps_final": r.eps_final, "outer_done": r.outer_done,
        "dim_x": r.dim_x, "dim_y": r.dim_y, "safe_iters": r.safe_iters,
        "n_inner_final": r.n_inner_final, "inner_doublings": r.inner_doublings,
    }


class Context:
    """Owns a gw_ctx on one device, ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, workspace_limit: int = 0):
        self.lib = L.load()
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = ctypes.c_void_p()
        rc = self.lib.gw_create(ctypes.byref(h), device, ctypes.c_void_p(s.cuda_stream), workspace_limit)
        if rc != L.GW_OK:
            raise L.GWError(rc, "gw_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.gw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != L.GW_OK:
            raise L.GWError(rc, self.lib.gw_last_error(self.h).decode())

    def set_profiling(self, enable: bool = True):
        self._check(self.lib.gw_set_profiling(self.h, 1 if enable else 0))

    def profile(self) -> dict:
        pr = L.GwProfile()
        self._check(self.lib.gw_get_profile(self.h, ctypes.byref(pr)))
        out = {name: {"launches": int(pr.launches[k]), "ms": float(pr.milliseconds[k]),
                      "idle_launches": int(pr.idle_launches[k]), "idle_ms": float(pr.idle_milliseconds[k])}
               for k, name in enumerate(L.PROF_NAMES)}
        out["entries_per_pass"] = int(pr.entries_per_pass)
        return out

    def set_penalty(self, side: int, kind="sqeuclid", p: float = 1.0, lifted_dim: int = 0,
                    n_landmarks: int = 0, seed: int = 0):
        k = _PEN[kind] if isinstance(kind, str) else int(kind)
        self._check(self.lib.gw_set_penalty(self.h, side, k, float(p), int(lifted_dim), int(n_landmarks),
                                            ctypes.c_uint64(seed)))

    def set_landmarks(self, side: int, idx):
        arr = (ctypes.c_int64 * len(idx))(*[int(v) for v in idx])
        self._check(self.lib.gw_set_landmarks(self.h, side, arr, len(idx)))

    def feature_dim(self, side: int, d: int) -> int:
        return self.lib.gw_feature_dim(self.h, side, d)

    def lift(self, side: int, x: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
        x = _dev_f32(x, "x")
        w = _dev_f32(w, "w")
        n, d = x.shape
        D = self.feature_dim(side, d)
        out = torch.empty((n, D), dtype=torch.float32, device=x.device)
        self._check(self.lib.gw_lift(self.h, side, _ptr(x), n, d, _ptr(w), _ptr(out)))
        return out

    def _prep(self, x, a, y, b):
        x = _dev_f32(x, "x")
        a = _dev_f32(a, "a")
        y = _dev_f32(y, "y")
        b = _dev_f32(b, "b")
        if x.dim() != 2 or y.dim() != 2 or a.shape != (x.shape[0],) or b.shape != (y.shape[0],):
            raise ValueError("x: (N, dx), a: (N,), y: (M, dy), b: (M,)")
        return x, a, y, b

    def solve(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
              precision="fp32", mode="auto", gamma0=None, f0=None, g0=None, tol_gamma=0.0,
              anneal_final=False, adaptive_inner=False) -> dict:
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        D, E = self.feature_dim(0, dx), self.feature_dim(1, dy)
        f = torch.empty(n, dtype=torch.float32, device=x.device) if f0 is None else _dev_f32(f0, "f0").clone()
        g = torch.empty(m, dtype=torch.float32, device=x.device) if g0 is None else _dev_f32(g0, "g0").clone()
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        g0t = None if gamma0 is None else _dev_f32(gamma0, "gamma0")
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode,
                          f0 is not None and g0 is not None, tol_gamma, anneal_final, adaptive_inner)
        r = L.GwResult()
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        self._check(self.lib.gw_solve(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                      ctypes.byref(prm), _ptr(g0t), ctypes.byref(r)))
        return _result_dict(r, f, g, gamma)

    def solve_noalloc(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
                      precision="fp32", mode="auto", gamma0=None, f0=None, g0=None, tol_gamma=0.0,
                      anneal_final=False) -> dict:
        """solve() through gw_solve_noalloc: the library allocates no device
        memory (its buffers come from a fixed scratch array); the outputs are
        allocated here, by torch."""
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        D, E = self.feature_dim(0, dx), self.feature_dim(1, dy)
        f = torch.empty(n, dtype=torch.float32, device=x.device) if f0 is None else _dev_f32(f0, "f0").clone()
        g = torch.empty(m, dtype=torch.float32, device=x.device) if g0 is None else _dev_f32(g0, "g0").clone()
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        g0t = None if gamma0 is None else _dev_f32(gamma0, "gamma0")
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode,
                          f0 is not None and g0 is not None, tol_gamma, anneal_final, False)
        r = L.GwResult()
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        self._check(self.lib.gw_solve_noalloc(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                              ctypes.byref(prm), _ptr(g0t), ctypes.byref(r)))
        return _result_dict(r, f, g, gamma)

    def solve_begin(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
                    precision="fp32", mode="auto", gamma0=None, f0=None, g0=None, tol_gamma=0.0,
                    anneal_final=False, adaptive_inner=False):
        """Set up a stepwise solve (gw_solve_begin): same arguments as
        solve().  The inputs are held until solve_end()."""
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        g0t = None if gamma0 is None else _dev_f32(gamma0, "gamma0")
        warm = L.GwResult()
        f0t = g0t_ = None
        if f0 is not None and g0 is not None:
            f0t, g0t_ = _dev_f32(f0, "f0"), _dev_f32(g0, "g0")
            warm.f, warm.g = f0t.data_ptr(), g0t_.data_ptr()
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode,
                          f0t is not None, tol_gamma, anneal_final, adaptive_inner)
        self._stepped = (x, a, y, b, g0t)  # kept alive for the library
        self._check(self.lib.gw_solve_begin(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                            ctypes.byref(prm), _ptr(g0t), ctypes.byref(warm)))

    def solve_advance(self, n_steps: int = 1) -> int:
        """Enqueue up to n_steps outer steps of the stepwise solve
        (gw_solve_advance); returns the outer steps enqueued so far."""
        done = ctypes.c_int32()
        self._check(self.lib.gw_solve_advance(self.h, int(n_steps), ctypes.byref(done)))
        return int(done.value)

    def solve_end(self) -> dict:
        """Final check and outputs of the stepwise solve (gw_solve_end)."""
        x, _, y, _, _ = self._stepped
        n, m = x.shape[0], y.shape[0]
        D, E = self.feature_dim(0, x.shape[1]), self.feature_dim(1, y.shape[1])
        f = torch.empty(n, dtype=torch.float32, device=x.device)
        g = torch.empty(m, dtype=torch.float32, device=x.device)
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        r = L.GwResult()
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        try:
            self._check(self.lib.gw_solve_end(self.h, ctypes.byref(r)))
        finally:
            self._stepped = None
        return _result_dict(r, f, g, gamma)

    def sgw(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
            precision="fp32", mode="auto") -> dict:
        """Sinkhorn-GW divergence GW(x, y) - (GW(x, x) + GW(y, y)) / 2
        (gw_sgw): three solves on the lifted features."""
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode, False, 0.0)
        r = L.GwSgwResult()
        self._check(self.lib.gw_sgw(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                    ctypes.byref(prm), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in L.GwSgwResult._fields_}

    def kpca_full(self, x, w, p: float = 1.0, D: int = 64, n_iter: int = 10, seed: int = 0):
        """Full-N kernel PCA of |x - x'|^p (gw_kpca_full): features (n, D)
        and the D eigenvalues, descending."""
        x = _dev_f32(x, "x")
        w = _dev_f32(w, "w")
        n, d = x.shape
        X = torch.empty((n, D), dtype=torch.float32, device=x.device)
        lam = (ctypes.c_double * D)()
        self._check(self.lib.gw_kpca_full(self.h, _ptr(x), n, d, _ptr(w), float(p), int(D), int(n_iter),
                                          ctypes.c_uint64(seed), _ptr(X), lam))
        return X, [float(v) for v in lam]

    def kmeans(self, X, w, k: int, n_lloyd: int = 10, seed: int = 0) -> dict:
        """Coarsen of Multiscale-GW (gw_kmeans): weighted K-Means of the rows
        of X (n, D) with weights w (n,).  Returns the non-empty clusters
        (Xc, wc) in index order, the cluster of every row and their count."""
        X = _dev_f32(X, "X")
        w = _dev_f32(w, "w")
        n, D = X.shape
        Xc = torch.empty((k, D), dtype=torch.float32, device=X.device)
        wc = torch.empty(k, dtype=torch.float32, device=X.device)
        assign = torch.empty(n, dtype=torch.int32, device=X.device)
        kc = ctypes.c_int64()
        self._check(self.lib.gw_kmeans(self.h, _ptr(X), n, D, _ptr(w), int(k), int(n_lloyd), ctypes.c_uint64(seed),
                                       _ptr(Xc), _ptr(wc), _ptr(assign), ctypes.byref(kc)))
        kc = int(kc.value)
        return {"Xc": Xc[:kc], "wc": wc[:kc], "assign": assign, "kc": kc}

    def interpolate(self, side: int, h, P, Q, w, gamma, eps: float) -> torch.Tensor:
        """Algorithm 8 (gw_interpolate): side 0 gives f of the source points P
        from the coarse target (Q, w, h = g); side 1 gives g of the target
        points P from the coarse source (Q, w, h = f).  gamma: (D, E)."""
        h, P, Q, w, gamma = (_dev_f32(t, nm) for t, nm in ((h, "h"), (P, "P"), (Q, "Q"), (w, "w"),
                                                            (gamma, "gamma")))
        D, E = gamma.shape
        out = torch.empty(P.shape[0], dtype=torch.float32, device=P.device)
        self._check(self.lib.gw_interpolate(self.h, int(side), _ptr(h), _ptr(P), P.shape[0], _ptr(Q), Q.shape[0],
                                            _ptr(w), _ptr(gamma), D, E, float(eps), _ptr(out)))
        return out

    def msgw(self, x, a, y, b, coarse: dict, fine: dict, rho: float = 0.1, n_lloyd: int = 10, seed: int = 0,
             gamma0=None) -> dict:
        """Multiscale-GW (gw_msgw, Algorithm 7).  coarse / fine: keyword
        arguments of make_params (eps_start, eps_end, n_outer, n_inner,
        symmetric, precision, mode, ...).  Returns the fine result with the
        coarse figures under "info"."""
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        D, E = self.feature_dim(0, dx), self.feature_dim(1, dy)
        f = torch.empty(n, dtype=torch.float32, device=x.device)
        g = torch.empty(m, dtype=torch.float32, device=x.device)
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        pc = make_params(**coarse)
        pf = make_params(**fine)
        o = L.GwMsgwOpts()
        o.rho, o.n_lloyd, o.reserved, o.seed = float(rho), int(n_lloyd), 0, int(seed)
        g0t = None if gamma0 is None else _dev_f32(gamma0, "gamma0")
        r = L.GwResult()
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        info = L.GwMsgwInfo()
        self._check(self.lib.gw_msgw(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b), ctypes.byref(pc),
                                     ctypes.byref(pf), ctypes.byref(o), _ptr(g0t), ctypes.byref(r),
                                     ctypes.byref(info)))
        out = _result_dict(r, f, g, gamma)
        out["info"] = {k: getattr(info, k) for k, _ in L.GwMsgwInfo._fields_}
        return out

    def sgw_grad(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
                 precision="fp32", mode="auto", weights=False) -> dict:
        """The divergence (gw_sgw fields) and its position gradients
        (gw_sgw_grad); with weights=True also its weight gradients grad_a,
        grad_b (centred along the simplex)."""
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode, False, 0.0)
        r = L.GwSgwResult()
        gx, gy = torch.empty_like(x), torch.empty_like(y)
        ga = torch.empty_like(a) if weights else None
        gb = torch.empty_like(b) if weights else None
        self._check(self.lib.gw_sgw_grad(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                         ctypes.byref(prm), ctypes.byref(r), _ptr(gx), _ptr(gy), _ptr(ga),
                                         _ptr(gb)))
        out = {k: getattr(r, k) for k, _ in L.GwSgwResult._fields_}
        out.update({"grad_x": gx, "grad_y": gy})
        if weights:
            out.update({"grad_a": ga, "grad_b": gb})
        return out

    def sgw_barycenter(self, x, a, y, b, z0, w, lam: float, step: float, n_steps: int, eps_start, eps_end=None,
                       n_outer=20, n_inner=50, symmetric=True, precision="fp32", mode="auto"):
        """GW barycentre flow (gw_sgw_barycenter): returns the moved points z
        and the objective before each step and after the last."""
        x, a, y, b = self._prep(x, a, y, b)
        z = _dev_f32(z0, "z0").clone()
        w = _dev_f32(w, "w")
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode, False, 0.0)
        obj = (ctypes.c_double * (n_steps + 1))()
        self._check(self.lib.gw_sgw_barycenter(self.h, _ptr(x), x.shape[0], _ptr(a), _ptr(y), y.shape[0], _ptr(b),
                                               x.shape[1], _ptr(z), z.shape[0], _ptr(w), float(lam), float(step),
                                               int(n_steps), ctypes.byref(prm), obj))
        return z, [float(v) for v in obj]

    def loss_and_grad(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
                      precision="fp32", mode="auto", gamma0=None, f0=None, g0=None, want=("x", "a", "y", "b")):
        x, a, y, b = self._prep(x, a, y, b)
        n, dx = x.shape
        m, dy = y.shape
        D, E = self.feature_dim(0, dx), self.feature_dim(1, dy)
        f = torch.empty(n, dtype=torch.float32, device=x.device) if f0 is None else _dev_f32(f0, "f0").clone()
        g = torch.empty(m, dtype=torch.float32, device=x.device) if g0 is None else _dev_f32(g0, "g0").clone()
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        gx = torch.empty_like(x) if "x" in want else None
        ga = torch.empty_like(a) if "a" in want else None
        gy = torch.empty_like(y) if "y" in want else None
        gb = torch.empty_like(b) if "b" in want else None
        g0t = None if gamma0 is None else _dev_f32(gamma0, "gamma0")
        prm = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode,
                          f0 is not None and g0 is not None, 0.0)
        r = L.GwResult()
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        self._check(self.lib.gw_loss_and_grad(self.h, _ptr(x), n, dx, _ptr(a), _ptr(y), m, dy, _ptr(b),
                                              ctypes.byref(prm), _ptr(g0t), ctypes.byref(r),
                                              _ptr(gx), _ptr(ga), _ptr(gy), _ptr(gb)))
        out = _result_dict(r, f, g, gamma)
        out.update({"grad_x": gx, "grad_a": ga, "grad_y": gy, "grad_b": gb})
        return out
