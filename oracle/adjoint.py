"""Discrete adjoint of the leapfrog recurrence (oracle; test infrastructure only).

Not in the paper: it differentiates the leapfrog of Sec. II-A (with the loss
reading documented in ``oracle.leapfrog``).  Written as one step

    e^(m+1)   = a * e^m + b * s^m,           s^m = C~ h^(m+1/2) - j_s(t_{m+1/2})
    h^(m+3/2) = h^(m+1/2) - d * (C e^(m+1))

with a = (M_eps - dt/2 M_sigma) / (M_eps + dt/2 M_sigma),
b = dt / (M_eps + dt/2 M_sigma), d = dt M_mu^{-1} (all diagonal), and the
probe objective

    J = dt * sum_{m=1..N} sum_i w_i M_eps,i (e_i^m)^2          (w = probe mask).

Reverse recursion (lambda = dJ/de, mu = dJ/dh; mu^(N+1/2) = 0):

    lambda^(m+1) = [m+1 < N] a * lambda^(m+2) - C~ (d * mu^(m+3/2)) + 2 dt w M_eps e^(m+1)
    mu^(m+1/2)   = mu^(m+3/2) + C (b * lambda^(m+1))

accumulating dJ/da += lambda^(m+1) e^m and dJ/db += lambda^(m+1) s^m, then the
chain rule through a(M_eps, M_sigma), b(M_eps, M_sigma), the direct term
dJ/dM_eps += dt sum_m w (e^m)^2, and M_eps = eps0 W_e eps_r, M_sigma = W_e sigma.
dt is held fixed (not differentiated through the CFL bound).
"""
from __future__ import annotations

import numpy as np

from .leapfrog import Operators, gaussian_current

__all__ = ["coefficients", "step_map", "step_map_adjoint", "probe_weights",
           "objective", "gradient"]


def coefficients(ops: Operators, dt: float):
    D = ops.M_eps + 0.5 * dt * ops.M_sigma
    a = (ops.M_eps - 0.5 * dt * ops.M_sigma) / D
    b = dt / D
    d = dt * ops.M_mu_inv
    return a, b, d, D


def step_map(ops: Operators, dt: float, e, h):
    """The source-free step as a linear map (e^m, h^(m+1/2)) -> (e^(m+1), h^(m+3/2))."""
    a, b, d, _ = coefficients(ops, dt)
    e1 = a * e + b * (ops.Ct @ h)
    return e1, h - d * (ops.C @ e1)


def step_map_adjoint(ops: Operators, dt: float, lam1, mu1):
    """Transpose of ``step_map``: cotangents of (e^(m+1), h^(m+3/2)) ->
    cotangents of (e^m, h^(m+1/2))."""
    a, b, d, _ = coefficients(ops, dt)
    lam_tot = lam1 - ops.Ct @ (d * mu1)
    return a * lam_tot, mu1 + ops.C @ (b * lam_tot)


def probe_weights(ops: Operators, box) -> np.ndarray:
    """1 on kept edges whose midpoint lies in the closed node-coordinate box
    ((lo_x, hi_x), (lo_y, hi_y), (lo_z, hi_z)), else 0."""
    top = ops.top
    w = np.zeros(top.n_edges)
    for a in range(3):
        p = top.edge_coords(a).astype(np.float64)
        mid = p.copy()
        mid[a] += 0.5
        ok = np.ones(p.shape[1], dtype=bool)
        for ax in range(3):
            ok &= (mid[ax] >= box[ax][0]) & (mid[ax] <= box[ax][1])
        w[top.edge(a, top.edge_coords(a))] = ok
    return w[ops.ie]


def _forward(ops, e0, h0, dt, nsteps, source):
    a, b, d, _ = coefficients(ops, dt)
    e = np.array(e0, dtype=np.float64, copy=True)
    h = np.array(h0, dtype=np.float64, copy=True)
    src_pos = None
    if source is not None:
        src_pos = ops.edge_slot(source["axis"], source["i"], source["j"], source["k"])
    es, ss = [e.copy()], []
    for m in range(nsteps):
        s = ops.Ct @ h
        if src_pos is not None:
            s[src_pos] -= gaussian_current((m + 0.5) * dt, source["i_max"], source["sigma_t"])
        e = a * e + b * s
        h = h - d * (ops.C @ e)
        es.append(e.copy())
        ss.append(s)
    return es, ss


def objective(ops: Operators, e0, h0, dt: float, nsteps: int, source, w) -> float:
    es, _ = _forward(ops, e0, h0, dt, nsteps, source)
    return float(dt * sum(np.sum(w * ops.M_eps * e * e) for e in es[1:]))


def gradient(ops: Operators, e0, h0, dt: float, nsteps: int, source, w):
    """Returns (J, dJ/deps_r per cell, dJ/dsigma per cell, per-edge dJ/dM_eps,
    per-edge dJ/dM_sigma).  Per-cell arrays are in cell numbering (x fastest)."""
    es, ss = _forward(ops, e0, h0, dt, nsteps, source)
    Me, Ms = ops.M_eps, ops.M_sigma
    a, b, d, D = coefficients(ops, dt)
    J = float(dt * sum(np.sum(w * Me * e * e) for e in es[1:]))
    da_dMe, db_dMe = dt * Ms / D ** 2, -dt / D ** 2
    da_dMs, db_dMs = -dt * Me / D ** 2, -0.5 * dt * dt / D ** 2
    lam_next = np.zeros_like(Me)      # a * lambda^(m+2) once multiplied
    mu = np.zeros(ops.n_h)            # mu^(N+1/2)
    g_a = np.zeros_like(Me)
    g_b = np.zeros_like(Me)
    direct = np.zeros_like(Me)
    for m in range(nsteps - 1, -1, -1):
        lam = 2.0 * dt * w * Me * es[m + 1] - ops.Ct @ (d * mu)
        if m + 1 < nsteps:
            lam = lam + a * lam_next
        mu = mu + ops.C @ (b * lam)
        g_a += lam * es[m]
        g_b += lam * ss[m]
        direct += w * es[m + 1] ** 2
        lam_next = lam
    g_Me = g_a * da_dMe + g_b * db_dMe + dt * direct
    g_Ms = g_a * da_dMs + g_b * db_dMs
    W = ops.mats.W_e[ops.ie]
    g_eps = ops.mats.eps0 * (W.T @ g_Me)
    g_sig = W.T @ g_Ms
    return J, np.asarray(g_eps).ravel(), np.asarray(g_sig).ravel(), g_Me, g_Ms
