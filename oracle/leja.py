"""Leja interpolation of the exponential for the FIT system (oracle; test
infrastructure only).

Paper: Sec. III-A.  exp(tA) b = (exp(tA/s))^s b is approximated by s steps
b_{i+1} = L_{m,c}(tA/s) b_i, L_{m,c} the Newton interpolation polynomial of
exp at Leja points of an interval of the imaginary axis (the spectrum of the
skew A of eq. FIT_ode_2 is imaginary); with all points at 0 it is the Taylor
polynomial.

Readings (the point sets and parameter rules are in the cited work, not in
the paper; these are derived from the published method):

* Points come in conjugate pairs +-i c a_j, so every pair contributes the
  real factor (X^2 + c^2 a_j^2) and the whole evaluation stays real.  The
  squares x_j = a_j^2 are a Leja sequence of [0, 1]: x_0 = 1 (the interval
  end), then each x_k maximises prod_{j<k} |x - x_j| over the candidate grid
  x = (1 - cos(pi i / N)) / 2, i = 0..N, N = 4000 (ties: smallest i).  With
  K pairs the polynomial has degree m = 2K - 1 and costs m applications of A.
* In the mixed basis p(z) = sum_k (alpha_k + beta_k z) prod_{j<k} (z^2 + c^2 a_j^2)
  (unique, real for real-symmetric point sets) the coefficients follow from
  the Newton divided differences d of exp at the points in the order
  (i c a_0, -i c a_0, i c a_1, ...): alpha_k = d_2k - d_2k+1 (i c a_k),
  beta_k = d_2k+1.  The divided differences are the first column of
  exp(Z), Z lower bidiagonal with the points on the diagonal and ones below.
* Remainder on the imaginary axis: |exp(z) - p(z)| <= prod_j |z - z_j| /
  (m+1)! (Hermite-Genocchi: the divided difference of exp over imaginary
  points has modulus <= 1/(m+1)!).  For z = i y, y in [-theta_h, theta_h]
  (theta_h = rho t / s), that is delta = max_{tau in [0, theta_h^2]}
  prod_j |tau - c^2 x_j| / (2K)!, the maximum taken on 4001 Chebyshev
  points of the tau interval and raised by 0.1 %.  c = theta_h (the points
  span the spectrum).  As for Taylor, s steps err by <= s delta (1 + delta)^(s-1)
  and rounding adds about s (m + 2) u S with S = max(1, sum_k (|alpha_k| +
  theta_h |beta_k|) N_k), N_k = max_tau prod_{j<k} |tau - c^2 x_j| the bound
  on the k-th basis vector.  (K, s) minimise m s subject to the sum <= tol.
* Evaluation uses the basis divided by g^(2k), g = max(c / 2, 1) (c / 2 is
  the capacity of the interval i[-c, c]): q_0 = b, r_k = X q_k,
  q_(k+1) = (X r_k + c^2 x_k q_k) / g^2, p(X) b = sum_k alpha_k g^(2k) q_k +
  beta_k g^(2k) r_k.  The products prod (X^2 + c^2 x_j) grow like (c^2/4)^k
  and would overflow float32 unscaled; the scaled basis stays of moderate
  size.  The polynomial is the same.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .expm import _first_feasible_generic

__all__ = ["leja_squares", "pair_coefficients", "scaled_pairs", "leja_bound",
           "leja_parameters", "leja_action", "eval_pairs"]

N_CAND = 4000
_CAND = 0.5 * (1.0 - np.cos(np.pi * np.arange(N_CAND + 1) / N_CAND))


def leja_squares(K: int) -> np.ndarray:
    """The first K points x_j of the Leja sequence of [0, 1] on the candidate grid."""
    xs = [1.0]
    with np.errstate(divide="ignore"):
        logp = np.log(np.abs(_CAND - 1.0))
    while len(xs) < K:
        i = int(np.argmax(logp))          # first index of the maximum
        xs.append(float(_CAND[i]))
        with np.errstate(divide="ignore"):
            logp = logp + np.log(np.abs(_CAND - _CAND[i]))
    return np.array(xs[:K])


def _divided_differences(z: np.ndarray) -> np.ndarray:
    """f[z_0], f[z_0, z_1], ..., f[z_0..z_m] for f = exp (Opitz)."""
    m1 = z.size
    Z = np.diag(z.astype(np.complex128)) + np.diag(np.ones(m1 - 1), -1)
    return sla.expm(Z)[:, 0]


def pair_coefficients(K: int, c: float):
    """(alpha, beta, a2) of the K-pair interpolant: a2[k] = c^2 x_k."""
    x = leja_squares(K)
    a = c * np.sqrt(x)
    z = np.empty(2 * K, dtype=np.complex128)
    z[0::2] = 1j * a
    z[1::2] = -1j * a
    d = _divided_differences(z)
    alpha = d[0::2] - d[1::2] * z[0::2]
    beta = d[1::2]
    scale = np.abs(alpha).max() + np.abs(beta).max()
    assert np.abs(alpha.imag).max() <= 1e-10 * scale and np.abs(beta.imag).max() <= 1e-10 * scale
    return alpha.real.copy(), beta.real.copy(), (c * c) * x


def scaled_pairs(K: int, c: float):
    """(alpha g^2k, beta g^2k, c^2 x_k / g^2, g^2) with g = max(c / 2, 1)."""
    alpha, beta, a2 = pair_coefficients(K, c)
    g2 = max(0.5 * c, 1.0) ** 2
    w = g2 ** np.arange(K)
    return alpha * w, beta * w, a2 / g2, g2


def eval_pairs(alpha, beta, a2, z):
    """p(z) of the mixed-basis form (scalar or array z)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.zeros_like(z)
    q = np.ones_like(z)
    for k in range(len(alpha)):
        out = out + (alpha[k] + beta[k] * z) * q
        q = q * (z * z + a2[k])
    return out


def _basis_max(a2, theta_h, K):
    """N_k = max over tau in [0, theta_h^2] of prod_{j<k} |tau - a2_j|, k = 0..K."""
    tau = (theta_h * theta_h) * _CAND
    prod = np.ones_like(tau)
    out = [1.0]
    for k in range(K):
        prod = prod * np.abs(tau - a2[k])
        out.append(float(prod.max()) * 1.001)
    return out


def leja_bound(theta: float, K: int, s: int, unit_roundoff: float = 2.0 ** -53) -> float:
    """Truncation plus rounding bound of (L(tA/s))^s b against exp(tA) b
    (relative), theta = |t| ||A||_2."""
    if theta == 0.0:
        return 0.0
    th = theta / s
    if th > 700.0:
        return math.inf
    alpha, beta, a2 = pair_coefficients(K, th)
    N = _basis_max(a2, th, K)
    log_delta = math.log(N[K]) - math.lgamma(2 * K + 1) if N[K] > 0 else -math.inf
    if log_delta > 50.0:
        return math.inf
    delta = math.exp(log_delta)
    log_trunc = math.log(s) + log_delta + (s - 1) * math.log1p(delta)
    S = max(1.0, sum((abs(alpha[k]) + th * abs(beta[k])) * N[k] for k in range(K)))
    rnd = s * (2 * K + 1) * unit_roundoff * S
    if log_trunc > 700.0:
        return math.inf
    return math.exp(log_trunc) + rnd


def leja_parameters(theta: float, tol: float, unit_roundoff: float = 2.0 ** -53,
                    k_max: int = 30) -> tuple:
    """(K, s) with the fewest applications (2K - 1) s whose bound is <= tol
    (ties: fewer sub-steps); (0, 1) for theta = 0."""
    if theta == 0.0:
        return 0, 1
    best = None
    for K in range(1, k_max + 1):
        s = _first_feasible_generic(lambda q: leja_bound(theta, K, q, unit_roundoff), theta, tol)
        if s is None:
            continue
        cost = (2 * K - 1) * s
        if best is None or cost < best[0] or (cost == best[0] and s < best[2]):
            best = (cost, K, s)
    if best is None:
        raise ValueError("tolerance below the rounding floor of the arithmetic")
    return best[1], best[2]


def leja_action(A, b, t: float, rho: float, tol: float = 1e-12, params=None,
                unit_roundoff: float = 2.0 ** -53):
    """exp(tA) b by s steps of the K-pair Leja interpolant of exp(tA/s)
    (c = rho |t| / s).  Returns (x, (K, s))."""
    K, s = params if params is not None else leja_parameters(abs(t) * rho, tol, unit_roundoff)
    x = np.array(b, dtype=np.float64, copy=True)
    if K == 0:
        return x, (K, s)
    h = t / s
    alpha, beta, a2, g2 = scaled_pairs(K, abs(h) * rho)
    # the points are symmetric, so p(hA) with h < 0 is p evaluated at -|h|A:
    # p(-z) = sum (alpha - beta z) ..., i.e. beta changes sign
    sgn = 1.0 if h >= 0 else -1.0
    hA = abs(h)
    for _ in range(s):
        q = x
        acc = np.zeros_like(x)
        for k in range(K):
            r = hA * (A @ q)
            acc = acc + alpha[k] * q + sgn * beta[k] * r
            if k + 1 < K:
                q = (hA / g2) * (A @ r) + a2[k] * q
        x = acc
    return x, (K, s)
