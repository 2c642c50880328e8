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
||T_m(hA)||_2 <= 1 + delta, so after s sub-steps the relative error is at
most s delta (1 + delta)^(s-1).  (m, s) are chosen to minimise the number of
applications m s subject to that bound being <= tol.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["taylor_error_bound", "taylor_parameters", "expm_action"]


def taylor_error_bound(theta: float, m: int, s: int) -> float:
    """Bound on ||(T_m(tA/s))^s - exp(tA)||_2 for normal A with imaginary
    spectrum and theta = |t| ||A||_2."""
    if theta == 0.0:
        return 0.0
    log_delta = (m + 1) * math.log(theta / s) - math.lgamma(m + 2)
    if log_delta > 50.0:
        return math.inf
    delta = math.exp(log_delta)
    log_bound = math.log(s) + log_delta + (s - 1) * math.log1p(delta)
    return math.inf if log_bound > 700.0 else math.exp(log_bound)


def taylor_parameters(theta: float, tol: float, m_max: int = 60) -> tuple:
    """(m, s) with the fewest applications m s whose bound is <= tol."""
    if theta == 0.0:
        return 0, 1
    best = None
    for m in range(1, m_max + 1):
        # the bound falls monotonically in s once theta / s < 1: bisect s
        lo, hi = 1, 1
        while taylor_error_bound(theta, m, hi) > tol:
            hi *= 2
            if hi > 1 << 40:
                break
        if taylor_error_bound(theta, m, hi) > tol:
            continue
        while lo < hi:
            mid = (lo + hi) // 2
            if taylor_error_bound(theta, m, mid) <= tol:
                hi = mid
            else:
                lo = mid + 1
        cost = m * lo
        if best is None or cost < best[0] or (cost == best[0] and lo < best[2]):
            best = (cost, m, lo)
    return best[1], best[2]


def expm_action(A, b, t: float, rho: float, tol: float = 1e-12, params=None):
    """exp(tA) b by (T_m(tA/s))^s b; ``rho`` = ||A||_2 (or a bound on it).
    Returns (x, (m, s))."""
    m, s = params if params is not None else taylor_parameters(abs(t) * rho, tol)
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
