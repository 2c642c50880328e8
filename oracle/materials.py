"""Diagonal material matrices (oracle; test infrastructure only).

Paper: Sec. II, eq. maxwell_grid3 -- d = M_eps e, j = M_sigma e + j_s,
b = M_mu h with M_eps, M_mu diagonal and positive definite.  The paper gives
no construction; the reading used here is the standard FIT one on a tensor
grid with per-axis cell widths (dx_i, dy_j, dz_k; three scalars for a uniform
grid, Sec. II-A eq. cfl indexes the widths by cell) and per-cell eps_r,
sigma, mu_r:

* M_eps[i] = eps0 * sum_{cells c around edge i} eps_r[c] * At[c, i] / L[i]
  where L is the primal edge length (the width of the cells around the edge
  along its axis) and At[c, i] the part of the dual facet of edge i that lies
  inside cell c (a quarter of that cell's d_b * d_c);
* M_sigma identical with sigma in place of eps0 * eps_r;
* M_mu^{-1}[f] = sum_{cells c on the dual edge of facet f} (Lt[c, f] / (mu0 mu_r[c])) / A[f]
  where A is the primal facet area (d_b * d_c of the two cells it separates)
  and Lt[c, f] = d_a[c] / 2 the part of the dual edge inside cell c.

Both reduce to the identity for eps_r = mu_r = 1 and unit cells.  Pins: a
uniform field's discrete energy equals the continuum energy integral for any
per-cell eps_r (resp. 1/mu_r), and a single-cell perturbation touches exactly
that cell's 12 edges (resp. 6 facets) with weight 1/4 (resp. 1/2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .topology import Topology, _succ

__all__ = ["cell_widths", "edge_cell_weights", "facet_cell_weights", "Materials"]


def cell_widths(top: Topology, spacing=(1.0, 1.0, 1.0)) -> list:
    """Per-axis cell widths [w_x (nx), w_y (ny), w_z (nz)] from three scalars
    (uniform grid) or three arrays."""
    out = []
    for a in range(3):
        s = np.asarray(spacing[a], dtype=np.float64)
        w = np.full(top.n[a], float(s)) if s.ndim == 0 else s.copy()
        if w.shape != (top.n[a],) or np.any(~np.isfinite(w)) or np.any(w <= 0):
            raise ValueError("cell widths must be positive, one per cell along each axis")
        out.append(w)
    return out


def edge_cell_weights(top: Topology, spacing=(1.0, 1.0, 1.0)) -> sp.csr_matrix:
    """W_e (edges x cells): W_e[i, c] = At[c, i] / L[i], so that
    M_eps = eps0 * W_e @ eps_r and M_sigma = W_e @ sigma."""
    wd = cell_widths(top, spacing)
    rows, cols, vals = [], [], []
    for a in range(3):
        b, c = _succ(a)
        p = top.edge_coords(a)
        r = top.edge(a, p)
        for db in (-1, 0):
            for dc in (-1, 0):
                q = p.copy()
                q[b] += db
                q[c] += dc
                ok = top._inside(top.cell_box, q)
                qa, qb, qc = q[a, ok], q[b, ok], q[c, ok]
                rows.append(r[ok])
                cols.append(top.cell(q[:, ok]))
                vals.append((wd[b][qb] / 2.0) * (wd[c][qc] / 2.0) / wd[a][qa])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(top.n_edges, top.n_cells))


def facet_cell_weights(top: Topology, spacing=(1.0, 1.0, 1.0)) -> sp.csr_matrix:
    """W_f (facets x cells): W_f[f, c] = Lt[c, f] / A[f], so that
    M_mu^{-1} = W_f @ (1 / (mu0 * mu_r))."""
    wd = cell_widths(top, spacing)
    rows, cols, vals = [], [], []
    for a in range(3):
        b, c = _succ(a)
        p = top.facet_coords(a)
        r = top.facet(a, p)
        for da in (-1, 0):
            q = p.copy()
            q[a] += da
            ok = top._inside(top.cell_box, q)
            qa, qb, qc = q[a, ok], q[b, ok], q[c, ok]
            rows.append(r[ok])
            cols.append(top.cell(q[:, ok]))
            vals.append((wd[a][qa] / 2.0) / (wd[b][qb] * wd[c][qc]))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(top.n_facets, top.n_cells))


class Materials:
    """Diagonals of M_eps, M_sigma and M_mu^{-1} over ALL edges / facets.

    ``eps_r``, ``sigma`` and ``mu_r`` are per-cell arrays of shape
    (nz, ny, nx); ``sigma``/``mu_r`` may be None (0 / 1).  Entries of
    boundary edges/facets are kept (they are simply not used under PEC).
    """

    def __init__(self, top: Topology, eps_r, sigma=None, mu_r=None,
                 spacing=(1.0, 1.0, 1.0), eps0: float = 1.0, mu0: float = 1.0):
        nz, ny, nx = top.n[2], top.n[1], top.n[0]
        eps_r = np.asarray(eps_r, dtype=np.float64).reshape(nz, ny, nx)
        sig = np.zeros_like(eps_r) if sigma is None else \
            np.asarray(sigma, dtype=np.float64).reshape(nz, ny, nx)
        mu = np.ones_like(eps_r) if mu_r is None else \
            np.asarray(mu_r, dtype=np.float64).reshape(nz, ny, nx)
        if np.any(eps_r <= 0) or np.any(mu <= 0) or np.any(sig < 0):
            raise ValueError("need eps_r > 0, mu_r > 0, sigma >= 0 (M_eps, M_mu SPD)")
        self.top = top
        self.eps0, self.mu0 = float(eps0), float(mu0)
        self.W_e = edge_cell_weights(top, spacing)
        self.W_f = facet_cell_weights(top, spacing)
        # per-cell arrays flattened in cell numbering (x fastest == C order of (nz,ny,nx))
        self.eps_r = eps_r.ravel()
        self.sigma = sig.ravel()
        self.mu_r = mu.ravel()
        self.M_eps = self.eps0 * (self.W_e @ self.eps_r)
        self.M_sigma = self.W_e @ self.sigma
        self.M_mu_inv = self.W_f @ (1.0 / (self.mu0 * self.mu_r))
