"""Leapfrog time stepping and discrete energies (oracle; test infrastructure only).

Paper: Sec. II-A (Leapfrog).  Given e^(0) and h^(1/2), for m = 0 .. n_t - 1

    (M_eps + dt/2 M_sigma) e^(m+1) = (M_eps - dt/2 M_sigma) e^(m) + dt (C~ h^(m+1/2) - j_s(t_{m+1/2}))
    h^(m+3/2) = h^(m+1/2) - dt M_mu^{-1} C e^(m+1)

Readings taken (the text is silent, garbled or self-inconsistent here):

* The h-update applies the PRIMAL curl C to e (Faraday, eq. maxwell_grid1;
  the first row [0, C] of K in eq. fit_matrices).  The printed update shows
  the dual curl, which cannot act on edge voltages.
* The excitation enters with a minus sign: row 2 of M du/dt + K u = g reads
  M_eps de/dt - C~ h = -j, as in the cylindrical-wave section.
* The paper sets sigma = 0.  With conduction the current at the half step
  is j^(m+1/2) = M_sigma (e^m + e^(m+1))/2 + j_s(t_{m+1/2}), using the
  paper's own interpolation e^(m+1/2) := (e^m + e^(m+1))/2; for sigma = 0 it
  is the printed update exactly.
* PEC walls (the only boundary in the paper): e on boundary-tangential edges
  and h on boundary-normal facets are held at zero, i.e. the operators are
  restricted to interior edges and facets.

Energies (eq. energy): <x, y>_eps := x^T M_eps y, <x, y>_mu := x^T M_mu y.
With no loss and no source the following are conserved exactly by the
recurrence (derived from the two updates and C~ = C^T):

    W^m = <e^m, e^(m+1/2)>_eps + <h^m, h^(m+1/2)>_mu    (the paper's form,
          e^(m+1/2) = (e^m + e^(m+1))/2,  h^m = (h^(m-1/2) + h^(m+1/2))/2)
    Q^m = <e^m, e^m>_eps + <h^(m-1/2), h^(m+1/2)>_mu
    R^m = <e^m, e^(m+1)>_eps + <h^(m+1/2), h^(m+1/2)>_mu,   W = (Q + R)/2,

and with loss/source  Q^(m+1) - Q^m = -2 dt ebar . (M_sigma ebar + j_s),
ebar = (e^m + e^(m+1))/2.
"""
from __future__ import annotations

import math

import numpy as np

from .topology import Topology
from .materials import Materials

__all__ = ["gaussian_current", "Operators", "TRACE_COLS", "run", "trace_derived"]

# One row per step m: the inner products the step makes available.
TRACE_COLS = ("m", "ee_mm", "ee_m_m1", "ee_m1_m1", "hh_prev_cur", "hh_cur_cur",
              "hh_cur_next", "hh_next_next", "loss", "src")


def gaussian_current(t, i_max: float, sigma_t: float):
    """Line-current waveform of the cylindrical-wave example (eq. line_current):
    i(t) = i_max exp(-4 ((t - sigma_t) / sigma_t)^2)."""
    return i_max * np.exp(-4.0 * ((np.asarray(t, dtype=np.float64) - sigma_t) / sigma_t) ** 2)


class Operators:
    """PEC-restricted operators and material diagonals for one grid."""

    def __init__(self, top: Topology, mats: Materials):
        self.top = top
        self.mats = mats
        self.ie = np.flatnonzero(top.interior_edges())     # kept edges (global ids)
        self.if_ = np.flatnonzero(top.interior_facets())   # kept facets
        C = top.curl()
        Ct = top.dual_curl()
        self.C = C[self.if_][:, self.ie].tocsr()           # kept edges -> kept facets
        self.Ct = Ct[self.ie][:, self.if_].tocsr()         # kept facets -> kept edges
        self.M_eps = mats.M_eps[self.ie]
        self.M_sigma = mats.M_sigma[self.ie]
        self.M_mu_inv = mats.M_mu_inv[self.if_]
        self.M_mu = 1.0 / self.M_mu_inv
        self._edge_pos = np.full(top.n_edges, -1, dtype=np.int64)
        self._edge_pos[self.ie] = np.arange(self.ie.size)

    @property
    def n_e(self):
        return self.ie.size

    @property
    def n_h(self):
        return self.if_.size

    def edge_slot(self, axis: int, i: int, j: int, k: int) -> int:
        """Position (in the kept-edge vector) of the a-edge at node (i, j, k)."""
        g = int(self.top.edge(axis, np.array([[i], [j], [k]]))[0])
        pos = int(self._edge_pos[g])
        if pos < 0:
            raise ValueError("source edge lies on a PEC wall")
        return pos


def run(ops: Operators, e0, h0, dt: float, nsteps: int, source=None, record=False,
        step0: int = 0):
    """Advance (e^m0, h^(m0+1/2)) by ``nsteps`` leapfrog steps, m0 = ``step0``
    (the global index of the first step; it only sets the source time).

    ``source``: None or dict(axis, i, j, k, i_max, sigma_t) with sigma_t in
    time units; the current i(t_{m+1/2}) flows on that one edge.
    Returns (e^N, h^(N+1/2), trace) where trace has one row per step with the
    columns TRACE_COLS; ``hh_prev_cur`` of step 0 is NaN (h^(-1/2) does not
    exist).  With ``record`` also returns the lists of all e^m and h^(m+1/2).
    """
    e = np.array(e0, dtype=np.float64, copy=True)
    h = np.array(h0, dtype=np.float64, copy=True)
    Me, Ms, Mmi, Mm = ops.M_eps, ops.M_sigma, ops.M_mu_inv, ops.M_mu
    lhs = Me + 0.5 * dt * Ms
    rhs = Me - 0.5 * dt * Ms
    src_pos = None
    if source is not None:
        src_pos = ops.edge_slot(source["axis"], source["i"], source["j"], source["k"])
    trace = np.zeros((nsteps, len(TRACE_COLS)))
    hh_prev_cur = math.nan
    es, hs = ([e.copy()], [h.copy()]) if record else (None, None)
    for m in range(nsteps):
        js = np.zeros_like(e)
        if src_pos is not None:
            js[src_pos] = gaussian_current((step0 + m + 0.5) * dt, source["i_max"],
                                           source["sigma_t"])
        e1 = (rhs * e + dt * (ops.Ct @ h - js)) / lhs
        h1 = h - dt * Mmi * (ops.C @ e1)
        ebar = 0.5 * (e + e1)
        trace[m] = (m, e @ (Me * e), e @ (Me * e1), e1 @ (Me * e1), hh_prev_cur,
                    h @ (Mm * h), h @ (Mm * h1), h1 @ (Mm * h1),
                    ebar @ (Ms * ebar), ebar @ js)
        hh_prev_cur = trace[m, 6]
        e, h = e1, h1
        if record:
            es.append(e.copy())
            hs.append(h.copy())
    if record:
        return e, h, trace, es, hs
    return e, h, trace


def trace_derived(trace: np.ndarray) -> dict:
    """W^m, Q^m, R^m and Q^(m+1) per row (W and Q^m are NaN where the
    previous step's h cross term is missing)."""
    t = trace
    Q_m = t[:, 1] + t[:, 4]
    R_m = t[:, 2] + t[:, 5]
    Q_m1 = t[:, 3] + t[:, 6]
    return dict(W=0.5 * (Q_m + R_m), Q=Q_m, R=R_m, Q_next=Q_m1,
                ee=t[:, 1], hh=t[:, 5])
