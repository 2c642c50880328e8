"""Python handle for a batch of grids advanced together, one launch per step
of all grids (thin wrapper over fit_batch_* in include/fit.h)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import call, dptr
from .grid import FitGrid, current_stream_handle


class FitBatch:
    TW_ROWS = -1     # row-packed tiles (ty = threads per workgroup)

    def __init__(self, grids, stream=None):
        self.grids = list(grids)
        if not all(isinstance(g, FitGrid) for g in self.grids):
            raise TypeError("FitBatch takes FitGrid objects")
        arr = (C.c_void_p * len(self.grids))(*[g.handle.value for g in self.grids])
        h = C.c_void_p()
        st = current_stream_handle() if stream is None else int(stream)
        call("fit_batch_create", arr, len(self.grids), C.c_void_p(st), C.byref(h))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().fit_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dt(self, dt):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64),
                                                 (len(self.grids),)))
        return a

    def set_tuning(self, ty: int = 0, kc: int = 0, steps_per_graph: int = 0, tw: int = 0):
        """tw x ty tiles (tw = TW_ROWS: row-packed, ty threads per workgroup),
        kc planes per item (0: whole columns); zeros keep."""
        call("fit_batch_set_tuning", self._h, int(tw), int(ty), int(kc), int(steps_per_graph))

    def get_tuning(self):
        """(ty, kc, steps_per_graph, workgroups per step, tw)."""
        v = [C.c_int() for _ in range(5)]
        call("fit_batch_get_tuning", self._h, *[C.byref(x) for x in v])
        tw, ty, kc, spg, nwg = (x.value for x in v)
        return ty, kc, spg, nwg, tw

    def set_pair(self, enable: bool = True, kc: int = 0):
        """Two steps of every grid per launch (each grid in the pair tile shape
        that suits its extent, columns cut into even z-chunks of at most kc
        planes, 0: whole columns)."""
        call("fit_batch_set_pair", self._h, int(bool(enable)), int(kc))

    def set_persistent(self, enable: bool = True):
        """S steps of every grid per cooperative launch with a grid-wide barrier
        between the steps (S = steps_per_graph), captured in a hipGraph."""
        call("fit_batch_set_persistent", self._h, int(bool(enable)))

    def get_persistent(self):
        """(enabled, workgroups of the launch, captured in a graph, a barrier of
        the last step call gave up); synchronises."""
        e, w, c, f = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        call("fit_batch_get_persistent", self._h, C.byref(e), C.byref(w), C.byref(c), C.byref(f))
        return bool(e.value), w.value, bool(c.value), bool(f.value)

    def get_pair(self):
        """(enabled, kc)."""
        e, k = C.c_int(), C.c_int()
        call("fit_batch_get_pair", self._h, C.byref(e), C.byref(k))
        return bool(e.value), k.value

    def get_pair_tile(self, g: int):
        """(tw, ty, kc) of grid g's pair tiles in the current layout."""
        w, t, k = C.c_int(), C.c_int(), C.c_int()
        call("fit_batch_get_pair_tile", self._h, int(g), C.byref(w), C.byref(t), C.byref(k))
        return w.value, t.value, k.value

    def autotune(self, dt, reps: int = 5):
        """Returns (ty, kc, ms_per_step, tw)."""
        a = self._dt(dt)
        w, t, k, ms = C.c_int(), C.c_int(), C.c_int(), C.c_float()
        call("fit_batch_autotune", self._h, dptr(a), int(reps), C.byref(w), C.byref(t),
             C.byref(k), C.byref(ms))
        return t.value, k.value, ms.value, w.value

    def step(self, nsteps: int, dt, use_graph: bool = True):
        a = self._dt(dt)
        call("fit_batch_step", self._h, int(nsteps), dptr(a), 1 if use_graph else 0)
