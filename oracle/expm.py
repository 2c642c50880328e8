"""Action of the matrix exponential of the FIT system (oracle; test infrastructure only).

Paper: Sec. III-A (approximation of the matrix exponential).  exp(tA) b is
approximated by scaling and a truncated Taylor recurrence,

    exp(tA) b = (exp(tA/s))^s b ~ (T_m(tA/s))^s b,   T_m(X) = sum_{j=0..m} X^j / j!,
    b_{i+1} = T_m(tA/s) b_i,  i = 0 .. s-1,  b_0 = b,

each term of T_m costing one application of A.  A is the skew matrix of
eq. FIT_ode_2 (normal, imaginary spectrum, ||A||_2 = rho).

Reading (the parameter selection of the cited works is not in the paper):
for a normal A with spectrum in [-i rho, i rho] the Taylor remainder on one
sub-step h = t/s is bounded by the Lagrange form on the imaginary axis,
||T_m(hA) - exp(hA)||_2 <= delta = (rho h)^(m+1) / (m+1)!, and
||T_m(hA)||_2 <= 1 + delta, so after s sub-steps the truncation error is at
most s delta (1 + delta)^(s-1) relative.  The terms of one sub-step sum to at
most e^(rho h) in norm while the result has norm 1, so rounding (unit
roundoff u of the arithmetic, each term built from <= m + 2 rounded
operations) adds at most about s (m + 2) u e^(rho h).  (m, s) are chosen to
minimise the number of applications m s subject to the sum of the two being
<= tol; a tolerance below what the arithmetic can reach is an error.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["taylor_error_bound", "taylor_parameters", "expm_action", "optimal_tolerance"]


def taylor_error_bound(theta: float, m: int, s: int, unit_roundoff: float = 2.0 ** -53) -> float:
    """Truncation plus rounding bound on ||(T_m(tA/s))^s b - exp(tA) b|| / ||b||
    for normal A with imaginary spectrum and theta = |t| ||A||_2."""
    if theta == 0.0:
        return 0.0
    log_delta = (m + 1) * math.log(theta / s) - math.lgamma(m + 2)
    if log_delta > 50.0 or theta / s > 700.0:
        return math.inf
    delta = math.exp(log_delta)
    log_trunc = math.log(s) + log_delta + (s - 1) * math.log1p(delta)
    log_round = math.log(s * (m + 2) * unit_roundoff) + theta / s
    if max(log_trunc, log_round) > 700.0:
        return math.inf
    return math.exp(log_trunc) + math.exp(log_round)


def _first_feasible_generic(bound, theta, tol):
    """Smallest s with bound(s) <= tol, or None, for a bound that falls with s
    on s <= theta: bisection there; beyond, the samples s* x (3/2)^q,
    q = 1..6 (s* = ceil(theta)), are tried and the first feasible one is
    bisected down to the previous sample."""
    s_star = max(1, math.ceil(theta))
    lo = None
    if bound(s_star) <= tol:
        lo, hi = 1, s_star
    else:
        prev = s_star
        for q in range(1, 7):
            cand = int(math.ceil(s_star * 1.5 ** q))
            if bound(cand) <= tol:
                lo, hi = prev + 1, cand
                break
            prev = cand
    if lo is None:
        return None
    while lo < hi:
        mid = (lo + hi) // 2
        if bound(mid) <= tol:
            hi = mid
        else:
            lo = mid + 1
    return lo


def _first_feasible(theta, m, tol, u):
    """Smallest s with taylor_error_bound(theta, m, s) <= tol, or None.  On
    s <= theta both parts of the bound fall with s (bisection is exact
    there)."""
    return _first_feasible_generic(lambda q: taylor_error_bound(theta, m, q, u), theta, tol)


def taylor_parameters(theta: float, tol: float, unit_roundoff: float = 2.0 ** -53,
                      m_max: int = 60) -> tuple:
    """(m, s) with the fewest applications m s whose bound is <= tol (ties:
    fewer sub-steps)."""
    if theta == 0.0:
        return 0, 1
    best = None
    for m in range(1, m_max + 1):
        s = _first_feasible(theta, m, tol, unit_roundoff)
        if s is None:
            continue
        cost = m * s
        if best is None or cost < best[0] or (cost == best[0] and s < best[2]):
            best = (cost, m, s)
    if best is None:
        raise ValueError("tolerance below the rounding floor of the arithmetic")
    return best[1], best[2]


def expm_action(A, b, t: float, rho: float, tol: float = 1e-12, params=None,
                unit_roundoff: float = 2.0 ** -53):
    """exp(tA) b by (T_m(tA/s))^s b; ``rho`` = ||A||_2 (or a bound on it);
    (m, s) from ``taylor_parameters`` for the given unit roundoff (the
    arithmetic the result is meant for).  Returns (x, (m, s))."""
    m, s = params if params is not None else taylor_parameters(abs(t) * rho, tol, unit_roundoff)
    x = np.array(b, dtype=np.float64, copy=True)
    if m == 0:
        return x, (m, s)
    h = t / s
    for _ in range(s):
        term = x.copy()
        acc = x.copy()
        for k in range(1, m + 1):
            term = (h / k) * (A @ term)
            acc += term
        x = acc
    return x, (m, s)


def optimal_tolerance(beta: float, dt: float, rho: float) -> float:
    """Sec. III-D, eq. tolerance_leja_2: with the leapfrog error of the
    particular solutions eps_B = beta dt^2, the exponential's backward-error
    tolerance that makes eps_B / eps_A equal to kappa_exp(A), and
    kappa_exp(A) = ||A||_2 = rho for the normal A of eq. FIT_ode_2."""
    if not (beta > 0 and dt > 0 and rho > 0):
        raise ValueError("beta, dt and rho must be positive")
    eps_b = beta * dt * dt
    return eps_b / rho
