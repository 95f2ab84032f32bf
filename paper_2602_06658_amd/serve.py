"""Serving loop binding (gw_server_* of include/gw.h): continuous batching of
independent GW solves on one GPU.  Argument marshalling only; admission,
batching and the solves run in libgwmi.so's server thread."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import Context, _PEN, _dev_f32, _result_dict, make_params


class Server:
    def __init__(self, context: Context, max_slots: int = 16, hbm_budget_bytes: int = 0):
        self.ctx = context
        self.lib = context.lib
        h = ctypes.c_void_p()
        rc = self.lib.gw_server_create(context.h, int(max_slots), int(hbm_budget_bytes), ctypes.byref(h))
        if rc != L.GW_OK:
            raise L.GWError(rc, "gw_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, x, a, y, b, eps_start, eps_end=None, n_outer=20, n_inner=50, symmetric=True,
               precision="fp32", mode="auto", penalty="sqeuclid", p=1.0, lifted_dim=0, n_landmarks=0,
               seed=0, anneal_final=False, gamma0=None, adaptive_inner=False) -> int:
        """Queue one solve; returns its ticket.  The tensors stay referenced
        until the result is collected.  Landmarks of the |x - x'|^p penalty
        use seed for the source and seed + 1 for the target."""
        x, a, y, b = (_dev_f32(t, nm) for t, nm in ((x, "x"), (a, "a"), (y, "y"), (b, "b")))
        n, dx = x.shape
        m, dy = y.shape
        pen = _PEN[penalty] if isinstance(penalty, str) else int(penalty)
        D = lifted_dim if pen == L.PEN_POWER else dx
        E = lifted_dim if pen == L.PEN_POWER else dy
        f = torch.empty(n, dtype=torch.float32, device=x.device)
        g = torch.empty(m, dtype=torch.float32, device=x.device)
        gamma = torch.empty((D, E), dtype=torch.float32, device=x.device)
        r = L.GwRequest()
        r.x, r.n, r.dx, r.a = x.data_ptr(), n, dx, a.data_ptr()
        r.y, r.m, r.dy, r.b = y.data_ptr(), m, dy, b.data_ptr()
        r.params = make_params(eps_start, eps_end, n_outer, n_inner, symmetric, precision, mode,
                               anneal_final=anneal_final, adaptive_inner=adaptive_inner)
        r.penalty, r.p, r.lifted_dim, r.n_landmarks, r.seed = pen, float(p), int(lifted_dim), int(n_landmarks), seed
        r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
        g0 = None
        if gamma0 is not None:
            g0 = _dev_f32(gamma0, "gamma0")
            if tuple(g0.shape) != (D, E):
                raise ValueError(f"gamma0 must be {D} x {E}")
            r.gamma0 = g0.data_ptr()
        t = ctypes.c_uint64()
        rc = self.lib.gw_server_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        if rc != L.GW_OK:
            raise L.GWError(rc, "gw_server_submit rejected the request")
        self._keep[t.value] = (x, a, y, b, f, g, gamma, g0)
        return t.value

    def _collect(self, ticket, rc, res, lat):
        if rc == L.GW_EBUSY:
            return None
        keep = self._keep.pop(ticket, None)
        if rc != L.GW_OK:
            raise L.GWError(rc, f"request {ticket} did not complete")
        f, g, gamma = keep[4:7]
        out = _result_dict(res, f, g, gamma)
        out["latency_s"] = lat.value
        return out

    def poll(self, ticket: int):
        """The result dict if done, None while queued or running."""
        res, lat = L.GwResult(), ctypes.c_double()
        rc = self.lib.gw_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res), ctypes.byref(lat))
        return self._collect(ticket, rc, res, lat)

    def wait(self, ticket: int) -> dict:
        res, lat = L.GwResult(), ctypes.c_double()
        rc = self.lib.gw_server_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(res), ctypes.byref(lat))
        return self._collect(ticket, rc, res, lat)

    def cancel(self, ticket: int):
        rc = self.lib.gw_server_cancel(self.h, ctypes.c_uint64(ticket))
        if rc != L.GW_OK:
            raise L.GWError(rc, f"cannot cancel {ticket}")

    def stats(self) -> dict:
        st = L.GwServerStats()
        rc = self.lib.gw_server_get_stats(self.h, ctypes.byref(st))
        if rc != L.GW_OK:
            raise L.GWError(rc, "gw_server_get_stats")
        return {k: getattr(st, k) for k, _ in L.GwServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.gw_server_destroy(self.h)
            self.h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
