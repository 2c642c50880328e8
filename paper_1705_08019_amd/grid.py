"""Python handle for one FIT grid (thin wrapper over the C ABI in include/fit.h).

PyTorch supplies the device memory -- both field buffer sets, the per-cell
material arrays and the adjoint state are torch tensors the library borrows
(fit_bind_fields, fit_bind_materials, fit_adjoint_bind) -- and the stream the
library enqueues on; every step of the method runs in libfit's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import call, dptr

_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64}
_NP_DTYPE = {"f32": np.float32, "f64": np.float64}


def current_stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class FitGrid:
    """nx x ny x nz cell grid with PEC walls, fields in the slot layout
    (3, nz, ny, nx): slot [a, k, j, i] = edge/facet of direction a at node (i, j, k)."""

    def __init__(self, nx: int, ny: int, nz: int, dtype: str = "f32",
                 spacing=(1.0, 1.0, 1.0), eps0: float = 1.0, mu0: float = 1.0,
                 allow_unstable: bool = False, stream=None):
        if dtype not in _TORCH_DTYPE:
            raise ValueError("dtype must be 'f32' or 'f64'")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dtype = dtype
        self.tdtype = _TORCH_DTYPE[dtype]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = current_stream_handle() if stream is None else int(stream)
        # three scalars: uniform spacing; any per-axis array: a tensor grid
        widths = [np.asarray(s, dtype=np.float64) for s in spacing]
        tensor = any(w.ndim > 0 for w in widths)
        uni = (1.0, 1.0, 1.0) if tensor else tuple(float(w) for w in widths)
        desc = _lib.GridDesc(self.nx, self.ny, self.nz, *uni,
                             float(eps0), float(mu0),
                             _lib.FIT_F64 if dtype == "f64" else _lib.FIT_F32,
                             _lib.FIT_ALLOW_UNSTABLE if allow_unstable else 0)
        h = C.c_void_p()
        call("fit_grid_create", C.byref(desc), C.c_void_p(self._stream), C.byref(h))
        self._h = h
        # device storage owned by PyTorch and borrowed by the library
        f = dict(dtype=self.tdtype, device=self.device)
        self._fields = [torch.zeros(self.shape, **f) for _ in range(4)]
        self._cells = [torch.zeros((self.nz, self.ny, self.nx), **f) for _ in range(3)]
        self._adj_bufs = None
        call("fit_bind_fields", self._h, *(C.c_void_p(t.data_ptr()) for t in self._fields))
        call("fit_bind_materials", self._h, *(C.c_void_p(t.data_ptr()) for t in self._cells))
        if tensor:
            self.set_spacing(*widths)

    # ------------------------------------------------------------------ lifecycle
    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().fit_grid_destroy(self._h)
            self._h = None
        # the bound storage outlives the handle
        self._fields = self._cells = self._adj_bufs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (3, self.nz, self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    # ------------------------------------------------------------------ setup
    def set_materials(self, eps_r, mu_r=None, sigma=None):
        def prep(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.size != self.cells:
                raise ValueError("per-cell arrays need nx*ny*nz values")
            return a
        e, m, s = prep(eps_r), prep(mu_r), prep(sigma)
        call("fit_set_materials", self._h, dptr(e), dptr(m), dptr(s))

    def set_spacing(self, dx=None, dy=None, dz=None):
        """Per-axis cell widths (arrays of nx, ny, nz values; scalars are
        broadcast); all None returns to the descriptor's uniform spacing."""
        if dx is None and dy is None and dz is None:
            call("fit_set_spacing", self._h, None, None, None)
            return
        ws = [np.ascontiguousarray(np.broadcast_to(np.asarray(w, dtype=np.float64), (n,)))
              for w, n in zip((dx, dy, dz), (self.nx, self.ny, self.nz))]
        call("fit_set_spacing", self._h, *(dptr(w) for w in ws))

    def set_source(self, axis: int, i: int, j: int, k: int, i_max: float, sigma_t: float):
        call("fit_set_source", self._h, axis, i, j, k, float(i_max), float(sigma_t))

    def clear_source(self):
        call("fit_set_source", self._h, -1, 0, 0, 0, 0.0, 1.0)

    def step_dt(self, dt: float) -> float:
        """The step the grid takes when asked for dt (FP32 grids: dt rounded
        down to FP32)."""
        v = C.c_double()
        call("fit_step_dt", self._h, float(dt), C.byref(v))
        return v.value

    def cfl_dt(self) -> float:
        v = C.c_double()
        call("fit_cfl_dt", self._h, C.byref(v))
        return v.value

    # ------------------------------------------------------------------ state
    def _as_arg(self, x):
        """(pointer, on_device, keepalive) for a field given as tensor/ndarray/None."""
        if x is None:
            return None, 1, None
        if isinstance(x, torch.Tensor):
            if tuple(x.shape) != self.shape and x.numel() != 3 * self.cells:
                raise ValueError(f"field must have {3 * self.cells} values")
            if x.is_cuda:
                x = x.to(self.tdtype).contiguous()
                return C.c_void_p(x.data_ptr()), 1, x
            x = x.detach().numpy()
        a = np.ascontiguousarray(x, dtype=_NP_DTYPE[self.dtype])
        if a.size != 3 * self.cells:
            raise ValueError(f"field must have {3 * self.cells} values")
        return C.c_void_p(a.ctypes.data), 0, a

    def set_fields(self, e=None, h=None, step: int = 0):
        pe, de, ke = self._as_arg(e)
        ph, dh, kh = self._as_arg(h)
        if pe is not None and ph is not None and de != dh:
            # mixed host/device: go through the device for both
            e = torch.as_tensor(np.asarray(e)).to(self.device) if de == 0 else e
            h = torch.as_tensor(np.asarray(h)).to(self.device) if dh == 0 else h
            return self.set_fields(e, h, step)
        on_dev = de if pe is not None else dh
        call("fit_set_fields", self._h, pe, ph, int(step), on_dev)
        torch.cuda.current_stream().synchronize() if on_dev else None
        del ke, kh

    def get_fields(self):
        """(e, h) as new device tensors of shape (3, nz, ny, nx)."""
        e = torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        h = torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        call("fit_get_fields", self._h, C.c_void_p(e.data_ptr()), C.c_void_p(h.data_ptr()), 1)
        return e, h

    def state(self):
        """The bound tensors holding the current state (e^m, h^(m+1/2)): views,
        not copies; valid until the next call that steps the grid."""
        pe, ph = C.c_void_p(), C.c_void_p()
        call("fit_get_state", self._h, C.byref(pe), C.byref(ph))
        by_ptr = {t.data_ptr(): t for t in self._fields}
        return by_ptr[pe.value], by_ptr[ph.value]

    def get_fields_host(self):
        e = np.empty(self.shape, dtype=_NP_DTYPE[self.dtype])
        h = np.empty(self.shape, dtype=_NP_DTYPE[self.dtype])
        call("fit_get_fields", self._h, C.c_void_p(e.ctypes.data), C.c_void_p(h.ctypes.data), 0)
        return e, h

    @property
    def step_index(self) -> int:
        v = C.c_int64()
        call("fit_get_step", self._h, C.byref(v))
        return v.value

    # ------------------------------------------------------------------ operators
    def apply_curl(self, x: torch.Tensor, which: int) -> torch.Tensor:
        """which = 0: C (edges -> facets); which = 1: C~ (facets -> edges)."""
        if x.numel() != 3 * self.cells:
            raise ValueError(f"input must have {3 * self.cells} values")
        x = x.to(device=self.device, dtype=self.tdtype).contiguous()
        out = torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        call("fit_apply_curl", self._h, int(which), C.c_void_p(x.data_ptr()),
             C.c_void_p(out.data_ptr()))
        return out

    def _dev(self, *xs):
        for x in xs:
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.tdtype
                    and x.is_contiguous() and x.numel() == 3 * self.cells):
                raise ValueError("fields must be contiguous device tensors of the grid dtype "
                                 f"with {3 * self.cells} values")
        return [C.c_void_p(x.data_ptr()) for x in xs]

    def new_field(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=self.tdtype, device=self.device)

    def op_apply(self, e: torch.Tensor, h: torch.Tensor, alpha: float = 1.0):
        """alpha B (e, h) = alpha (M_eps^{-1} C~ h, -M_mu^{-1} C e) as new tensors."""
        eo, ho = self.new_field(), self.new_field()
        call("fit_op_apply", self._h, float(alpha), *self._dev(e, h, eo, ho))
        return eo, ho

    def op_norm(self, iters: int = 100, seed: int = 1) -> float:
        """||A||_2 of eq. FIT_ode_2 by power iteration (approaches from below)."""
        v = C.c_double()
        call("fit_op_norm", self._h, int(iters), C.c_uint64(seed), C.byref(v))
        return v.value

    def expm(self, t: float, e: torch.Tensor, h: torch.Tensor, rho: float, tol: float = 1e-12,
             out=None, method: str = "taylor"):
        """exp(t B) (e, h); returns (e_out, h_out, params): params (m, s) of
        the scaled Taylor recurrence, or (K, s) of the K-pair Leja
        interpolant (method "leja")."""
        if method not in ("taylor", "leja"):
            raise ValueError("method must be 'taylor' or 'leja'")
        eo, ho = (self.new_field(), self.new_field()) if out is None else out
        m, s_ = C.c_int(), C.c_int64()
        call("fit_expm" if method == "taylor" else "fit_expm_leja", self._h, float(t), float(tol),
             float(rho), *self._dev(e, h, eo, ho), C.byref(m), C.byref(s_))
        return eo, ho, (m.value, s_.value)

    def shift_h(self, c: float, e: torch.Tensor, h_in: torch.Tensor, h_out=None):
        """h_in - c M_mu^{-1} C e (c = -dt/2: collocate h^(m+1/2) at t_m)."""
        ho = self.new_field() if h_out is None else h_out
        call("fit_shift_h", self._h, float(c), *self._dev(e, h_in, ho))
        return ho

    def axpy(self, a: float, xe, xh, ye, yh):
        """(ye, yh) += a (xe, xh) in place."""
        call("fit_axpy", self._h, float(a), *self._dev(xe, xh, ye, yh))

    UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}

    @staticmethod
    def expm_params(theta: float, tol: float, unit_roundoff: float = 2.0 ** -53):
        m, s_ = C.c_int(), C.c_int64()
        call("fit_expm_params", float(theta), float(tol), float(unit_roundoff), C.byref(m),
             C.byref(s_))
        return m.value, s_.value

    @staticmethod
    def leja_params(theta: float, tol: float, unit_roundoff: float = 2.0 ** -53):
        K, s_ = C.c_int(), C.c_int64()
        call("fit_leja_params", float(theta), float(tol), float(unit_roundoff), C.byref(K),
             C.byref(s_))
        return K.value, s_.value

    @staticmethod
    def leja_coefficients(K: int, c: float):
        """(alpha, beta, a2, g2) of the scaled K-pair basis on i[-c, c]."""
        al, be, a2 = (np.empty(K) for _ in range(3))
        g2 = C.c_double()
        call("fit_leja_coefficients", int(K), float(c), dptr(al), dptr(be), dptr(a2), C.byref(g2))
        return al, be, a2, g2.value

    @staticmethod
    def expm_tolerance(beta: float, dt: float, rho: float) -> float:
        """beta dt^2 / ||A||_2 (eq. tolerance_leja_2)."""
        v = C.c_double()
        call("fit_expm_tolerance", float(beta), float(dt), float(rho), C.byref(v))
        return v.value

    def step(self, nsteps: int, dt: float):
        call("fit_step", self._h, int(nsteps), float(dt))

    def energy(self):
        """(<e^m,e^m>_eps, <h^(m+1/2),h^(m+1/2)>_mu) of the current state."""
        out = self.energies()
        return out["ee"], out["hh"]

    def energies(self) -> dict:
        """eq. energy at the current state: ee = <e,e>_eps, hh = <h,h>_mu, the
        conserved W, Q and dQ = Q^(m+1) - Q^m (NaN before the first step)."""
        out = (C.c_double * 5)()
        call("fit_energy", self._h, out)
        return dict(zip(("ee", "hh", "W", "Q", "dQ"), out))

    # ------------------------------------------------------------------ diagnostics
    def trace_config(self, every: int, capacity: int):
        call("fit_trace_config", self._h, int(every), int(capacity))
        self._trace_cap = int(capacity)

    def trace_read(self, max_rows: int = None):
        cap = int(getattr(self, "_trace_cap", 0) if max_rows is None else max_rows)
        out = np.empty((max(cap, 1), _lib.FIT_TRACE_COLS), dtype=np.float64)
        n, dropped = C.c_int64(), C.c_int64()
        call("fit_trace_read", self._h, dptr(out), cap, C.byref(n), C.byref(dropped))
        return out[: n.value].copy(), dropped.value

    def set_probe(self, lo, hi):
        lo_a = (C.c_int32 * 3)(*map(int, lo))
        hi_a = (C.c_int32 * 3)(*map(int, hi))
        call("fit_set_probe", self._h, lo_a, hi_a)

    def clear_probe(self):
        call("fit_set_probe", self._h, None, None)

    def probe_value(self) -> float:
        v = C.c_double()
        call("fit_probe_value", self._h, C.byref(v))
        return v.value

    def probe_reset(self):
        call("fit_probe_reset", self._h)

    # ------------------------------------------------------------------ timing
    def profile_begin(self, max_launches: int):
        call("fit_profile_begin", self._h, int(max_launches))

    def profile_end(self) -> dict:
        """{kind: (total_ms, launches)} over the launches since profile_begin."""
        n = len(_lib.PROF_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        call("fit_profile_end", self._h, ms, cnt)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.PROF_KINDS)}

    def smvp_count(self) -> int:
        v = C.c_int64()
        call("fit_smvp_count", self._h, C.byref(v))
        return v.value

    # ------------------------------------------------------------------ tuning
    PATHS = {"auto": 0, "split": 1, "fused": 2}

    def set_tuning(self, path: str = "auto", ty: int = 0, kc: int = 0, tw: int = None):
        """Kernel path and tile (tw x ty columns, kc planes); zeros = defaults.
        tw defaults to 64 when ty/kc are given."""
        if tw is None:
            tw = 64 if (ty or kc) else 0
        call("fit_set_tuning", self._h, self.PATHS[path], int(tw), int(ty), int(kc))

    def set_pair(self, enable: bool = True, tw: int = 0, ty: int = 0, kc: int = 0):
        """Two steps per launch (temporal blocking) where eligible; tile tw x ty,
        kc planes per chunk (zeros: defaults)."""
        call("fit_set_pair_tuning", self._h, int(bool(enable)), int(tw), int(ty), int(kc))

    def get_pair(self):
        """(enabled, tw, ty, kc)."""
        e, w, t, k = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        call("fit_get_pair_tuning", self._h, C.byref(e), C.byref(w), C.byref(t), C.byref(k))
        return bool(e.value), w.value, t.value, k.value

    def get_tuning(self):
        """(path, ty, kc, tw)."""
        p, w, t, k = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        call("fit_get_tuning", self._h, C.byref(p), C.byref(w), C.byref(t), C.byref(k))
        return {1: "split", 2: "fused"}[p.value], t.value, k.value, w.value

    def autotune(self, dt: float, reps: int = 10):
        """Time candidate paths/tiles on the current state (unchanged) and keep
        the fastest; returns (path, ty, kc, ms_per_step, tw)."""
        p, w, t, k, ms = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_float()
        call("fit_autotune", self._h, float(dt), int(reps), C.byref(p), C.byref(w), C.byref(t),
             C.byref(k), C.byref(ms))
        return {1: "split", 2: "fused"}[p.value], t.value, k.value, ms.value, w.value

    # ------------------------------------------------------------------ Gram
    def gram(self, X: torch.Tensor, which: int = 0) -> np.ndarray:
        """G = X^T diag(M) X for K snapshots X of shape (K, 3, nz, ny, nx) (or
        (K, 3 nx ny nz)) on the device; which 0: e with M_eps, 1: h with M_mu."""
        if not (isinstance(X, torch.Tensor) and X.is_cuda):
            raise ValueError("X must be a device tensor")
        K = X.shape[0]
        Xc = X.to(self.tdtype).reshape(K, int(np.prod(X.shape[1:]))).contiguous()
        if Xc.shape[1] != 3 * self.cells:
            raise ValueError("each snapshot must have 3 * nx * ny * nz values")
        G = np.empty((K, K), dtype=np.float64)
        call("fit_gram", self._h, C.c_void_p(Xc.data_ptr()), Xc.stride(0), int(K), int(which),
             dptr(G))
        return G

    # ------------------------------------------------------------------ adjoint
    def step_record(self, nsteps: int, dt: float, e_rec: torch.Tensor, h_rec: torch.Tensor):
        """Advance nsteps, writing e^(m0+s) to e_rec[s] and h^(m0+s+1/2) to
        h_rec[s] (device tensors with >= nsteps+1 leading entries)."""
        for r in (e_rec, h_rec):
            if not (r.is_cuda and r.dtype == self.tdtype and r.is_contiguous()
                    and r.numel() >= (nsteps + 1) * 3 * self.cells):
                raise ValueError("record buffers: contiguous device tensors of the grid dtype "
                                 "with (nsteps+1) * 3 * cells values")
        call("fit_step_record", self._h, int(nsteps), float(dt), C.c_void_p(e_rec.data_ptr()),
             C.c_void_p(h_rec.data_ptr()))

    def adjoint_set_tuning(self, tw: int = 0, ty: int = 0, kc: int = 0):
        """Reverse-step tile (tw x ty columns, kc planes) from the next
        adjoint_begin; zeros select the defaults."""
        call("fit_adjoint_set_tuning", self._h, int(tw), int(ty), int(kc))

    def adjoint_get_tuning(self):
        """(tw, ty, kc) of the reverse-step tile the next adjoint_begin uses."""
        w, t, k = C.c_int(), C.c_int(), C.c_int()
        call("fit_adjoint_get_tuning", self._h, C.byref(w), C.byref(t), C.byref(k))
        return w.value, t.value, k.value

    def adjoint_begin(self, nsteps: int, dt: float):
        if self._adj_bufs is None:   # lambda, mu ping-pong pairs and the cell gradients
            f = dict(dtype=self.tdtype, device=self.device)
            self._adj_bufs = [torch.zeros(self.shape, **f) for _ in range(4)] + [
                torch.zeros((2, self.nz, self.ny, self.nx), dtype=torch.float64,
                            device=self.device)]
            call("fit_adjoint_bind", self._h,
                 *(C.c_void_p(t.data_ptr()) for t in self._adj_bufs))
        call("fit_adjoint_begin", self._h, int(nsteps), float(dt))

    def adjoint_step(self, m: int, e_m: torch.Tensor, e_m1: torch.Tensor, h_mh: torch.Tensor):
        for x in (e_m, e_m1, h_mh):
            if not (x.is_cuda and x.dtype == self.tdtype and x.is_contiguous()
                    and x.numel() == 3 * self.cells):
                raise ValueError("states must be contiguous device tensors of the grid dtype")
        call("fit_adjoint_step", self._h, int(m), C.c_void_p(e_m.data_ptr()),
             C.c_void_p(e_m1.data_ptr()), C.c_void_p(h_mh.data_ptr()))

    def adjoint_segment(self, m0: int, nsteps: int, e_rec: torch.Tensor, h_rec: torch.Tensor):
        for r in (e_rec, h_rec):
            if not (r.is_cuda and r.dtype == self.tdtype and r.is_contiguous()
                    and r.numel() >= (nsteps + 1) * 3 * self.cells):
                raise ValueError("record buffers too small")
        call("fit_adjoint_segment", self._h, int(m0), int(nsteps), C.c_void_p(e_rec.data_ptr()),
             C.c_void_p(h_rec.data_ptr()))

    def adjoint_grad(self):
        """(dJ/deps_r, dJ/dsigma) as FP64 device tensors of shape (nz, ny, nx)."""
        de = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        ds = torch.empty_like(de)
        call("fit_adjoint_grad", self._h, C.c_void_p(de.data_ptr()), C.c_void_p(ds.data_ptr()), 1)
        return de, ds
