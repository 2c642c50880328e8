"""ParaExp with leapfrog particular solutions (oracle; test infrastructure only).

Paper: Sec. III (ParaExp, Alg. 1), Sec. III-B (reconstruction on staggered
grids, eqs. averaging1/2), Sec. III-C (cost, eq. tot_cost).

The interval (0, T] is split into p sub-intervals of L = N/p leapfrog steps.
On sub-interval j the particular solution v_j is a leapfrog run from zero
fields under the source at the global time (step counter starting at
(j-1) L).  The homogeneous solutions live in the transformed unknowns
u = [M_mu^{1/2} h; M_eps^{1/2} e] of eq. FIT_ode_2:
w_1(T) = exp(T A) u_0 and w_{j+1}(T) = exp((T - T_j) A) v_j(T_j); the total
is u(T) = v_p(T) + sum_i w_i(T).  The staggered result follows eqs.
averaging1/2: e^(N) = e_p^(N) + M_eps^{-1/2} [sum w(T)]_e and
h^(N+1/2) = h_p^(N+1/2) + M_mu^{-1/2} [sum w(T + dt/2)]_h.

Readings (the paper is silent on these):

* Leapfrog gives h at half steps; the collocated h(T_j) that enters the
  transformed initial value is the paper's interpolation
  h^(m) = (h^(m-1/2) + h^(m+1/2))/2 = h^(m+1/2) + dt/2 M_mu^{-1} C e^(m)
  (one curl application: the "two transformations" of eq. tot_cost).
  The initial value u_0 is formed the same way from e^(0), h^(1/2).
* sum w(T + dt/2) = exp(dt/2 A) sum w(T).
* Lossless grids only (A of eq. FIT_ode_2 has no loss term; the paper sets
  sigma = 0).
"""
from __future__ import annotations

import numpy as np

from . import leapfrog
from .expm import expm_action
from .leja import leja_action
from .stability import skew_matrix, spectral_norm

__all__ = ["to_u", "from_u", "collocate_h", "paraexp"]


def to_u(ops, e, h):
    """u = [M_mu^{1/2} h; M_eps^{1/2} e] (eq. FIT_ode_2)."""
    return np.concatenate([np.sqrt(ops.M_mu) * h, np.sqrt(ops.M_eps) * e])


def from_u(ops, u):
    """(e, h) from u."""
    nh = ops.n_h
    return u[nh:] / np.sqrt(ops.M_eps), u[:nh] / np.sqrt(ops.M_mu)


def collocate_h(ops, e_m, h_half, dt):
    """h(t_m) = h^(m+1/2) + dt/2 M_mu^{-1} C e^(m)."""
    return h_half + 0.5 * dt * ops.M_mu_inv * (ops.C @ e_m)


def paraexp(ops, dt: float, nsteps: int, p: int, source=None, e0=None, h0=None,
            homogeneous: str = "expm", tol: float = 1e-12, rho=None,
            unit_roundoff: float = 2.0 ** -53):
    """(e^(N), h^(N+1/2), cost) of Alg. 1 for N = ``nsteps`` (divisible by p).

    ``homogeneous``: "expm" (the paper: Taylor action of exp(tA), see
    ``expm``), "leja" (Leja interpolation, see ``leja``) or "leapfrog" (the
    homogeneous problems stepped by source-free
    leapfrog on the staggered grid, which by linearity reproduces one
    leapfrog run over (0, T]).  ``cost``: leapfrog steps per sub-interval,
    applications of A per homogeneous solution, and C_proc of eq. tot_cost
    (2 L + the largest count of A applications + 2).  ``unit_roundoff``
    enters the Taylor parameter choice (see ``expm``).
    """
    if nsteps % p:
        raise ValueError("nsteps must be divisible by p")
    if np.any(ops.M_sigma != 0.0):
        raise ValueError("ParaExp needs a lossless grid")
    L = nsteps // p
    ze, zh = np.zeros(ops.n_e), np.zeros(ops.n_h)
    e0 = ze if e0 is None else np.asarray(e0, dtype=np.float64)
    h0 = zh if h0 is None else np.asarray(h0, dtype=np.float64)
    # particular solutions: zero initial values, source at the global time
    parts = []
    for j in range(p):
        e, h, _ = leapfrog.run(ops, ze, zh, dt, L, source, step0=j * L)
        parts.append((e, h))
    cost = {"leapfrog_steps_per_interval": L, "A_applications": []}
    if homogeneous == "leapfrog":
        e_tot, h_tot = parts[-1][0].copy(), parts[-1][1].copy()
        e, h, _ = leapfrog.run(ops, e0, h0, dt, nsteps)               # w_1
        e_tot += e
        h_tot += h
        for j in range(p - 1):                                        # w_{j+2}
            e, h, _ = leapfrog.run(ops, parts[j][0], parts[j][1], dt, (p - 1 - j) * L,
                                   step0=(j + 1) * L)
            e_tot += e
            h_tot += h
        return e_tot, h_tot, cost
    if homogeneous not in ("expm", "leja"):
        raise ValueError("homogeneous must be 'expm', 'leja' or 'leapfrog'")
    action = expm_action if homogeneous == "expm" else leja_action
    applications = (lambda ms: ms[0] * ms[1]) if homogeneous == "expm" else \
        (lambda ms: (2 * ms[0] - 1) * ms[1] if ms[0] > 0 else 0)
    A = skew_matrix(ops)
    rho = spectral_norm(ops) if rho is None else rho
    T = nsteps * dt
    wsum = np.zeros(ops.n_h + ops.n_e)
    u0 = to_u(ops, e0, collocate_h(ops, e0, h0, dt))
    if np.any(u0):
        w, ms = action(A, u0, T, rho, tol, unit_roundoff=unit_roundoff)
        cost["A_applications"].append(applications(ms))
        wsum += w
    for j in range(p - 1):
        e, h = parts[j]
        vj = to_u(ops, e, collocate_h(ops, e, h, dt))              # v_j(T_j)
        w, ms = action(A, vj, T - (j + 1) * L * dt, rho, tol, unit_roundoff=unit_roundoff)
        cost["A_applications"].append(applications(ms))
        wsum += w
    w_half, ms = action(A, wsum, 0.5 * dt, rho, tol, unit_roundoff=unit_roundoff)
    cost["A_applications_half_step"] = applications(ms)
    ew, _ = from_u(ops, wsum)
    _, hw = from_u(ops, w_half)
    e_p, h_p = parts[-1]
    n_a = max(cost["A_applications"], default=0)
    cost["C_proc"] = 2 * L + n_a + 2
    return e_p + ew, h_p + hw, cost
