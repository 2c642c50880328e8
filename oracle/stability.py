"""CFL step size, the skew-symmetric system matrix and its norm (oracle; test infrastructure only).

Paper: Sec. II, eq. FIT_ode_2 (similarity transform T = blkdiag(M_mu^{1/2},
M_eps^{1/2}) giving u = [M_mu^{1/2} h; M_eps^{1/2} e] and the skew matrix A),
and Sec. II-A, eq. cfl (the practical bound) together with the sharp bound
set by lambda_max = ||A||_2.

Reading: the CFL formula indexes materials by CELL j, so eps_j, mu_j are the
per-cell values; the sharp bound of leapfrog for u' = A u with A normal is
dt < 2 / ||A||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .leapfrog import Operators

__all__ = ["cfl_dt", "skew_matrix", "spectral_norm"]


def cfl_dt(eps_r, mu_r=None, spacing=(1.0, 1.0, 1.0), eps0: float = 1.0,
           mu0: float = 1.0) -> float:
    """dt_CFL = min over cells of sqrt(eps mu / (dx^-2 + dy^-2 + dz^-2)), the
    widths taken per cell (``spacing``: three scalars or three per-axis
    arrays of cell widths; per-cell arrays have shape (nz, ny, nx))."""
    eps = eps0 * np.asarray(eps_r, dtype=np.float64)
    mu = mu0 * (np.ones_like(eps) if mu_r is None else np.asarray(mu_r, dtype=np.float64))
    nz, ny, nx = eps.shape
    wx, wy, wz = (np.broadcast_to(np.asarray(s, dtype=np.float64), (n,))
                  for s, n in zip(spacing, (nx, ny, nz)))
    inv = (1.0 / wx[None, None, :] ** 2 + 1.0 / wy[None, :, None] ** 2 +
           1.0 / wz[:, None, None] ** 2)
    return float(np.min(np.sqrt(eps * mu / inv)))


def skew_matrix(ops: Operators) -> sp.csr_matrix:
    """A of eq. FIT_ode_2 on the PEC-restricted unknowns, ordered [h; e]."""
    Mmu_mh = sp.diags(np.sqrt(ops.M_mu_inv))            # M_mu^{-1/2}
    Meps_mh = sp.diags(1.0 / np.sqrt(ops.M_eps))        # M_eps^{-1/2}
    A12 = -(Mmu_mh @ ops.C @ Meps_mh)
    A21 = Meps_mh @ ops.Ct @ Mmu_mh
    return sp.bmat([[None, A12], [A21, None]], format="csr")


def spectral_norm(ops: Operators, iters: int = 2000, seed: int = 0, tol: float = 1e-13) -> float:
    """||A||_2 by power iteration on A^T A (symmetric positive semidefinite)."""
    A = skew_matrix(ops)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.shape[1])
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = A.T @ (A @ x)
        new = float(np.linalg.norm(y))
        x = y / new
        if abs(new - lam) <= tol * new:
            lam = new
            break
        lam = new
    return float(np.sqrt(lam))
