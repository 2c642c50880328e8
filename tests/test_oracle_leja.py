"""Pins of the oracle's Leja interpolation of the exponential (Sec. III-A;
CPU only): the point sequence against potential theory, the interpolation
conditions, the Taylor limit c -> 0 the paper states, the remainder bound on
the imaginary axis, agreement with expm_multiply and with the exact TE101
rotation, the rounding term against a float32 evaluation, and the cost
advantage over Taylor for normal matrices."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators
from oracle.stability import skew_matrix, spectral_norm
from oracle import expm, leja, paraexp, layout
from fit_workloads import dielectric_blocks


def _ops(nx, ny, nz, eps=None):
    t = Topology(nx, ny, nz)
    eps = np.ones((nz, ny, nx)) if eps is None else eps
    return Operators(t, Materials(t, eps))


def test_leja_sequence_follows_the_equilibrium_measure():
    x = leja.leja_squares(60)
    assert x[0] == 1.0 and x[1] == 0.0 and abs(x[2] - 0.5) <= 1e-15
    assert np.all((x >= 0) & (x <= 1)) and np.unique(x).size == x.size
    # the k-th point's geometric mean distance to the previous ones tends to
    # the capacity of [0, 1], 1/4
    k = 59
    gm = math.exp(np.mean(np.log(np.abs(x[k] - x[:k]))))
    assert 0.2 < gm < 0.32
    # the points distribute like the arcsine law F(x) = (2/pi) asin(sqrt(x))
    for q in (0.1, 0.25, 0.5, 0.9):
        frac = np.mean(x <= q)
        assert abs(frac - 2 / math.pi * math.asin(math.sqrt(q))) <= 0.05, q


@pytest.mark.parametrize("K,c", [(1, 0.5), (3, 0.5), (8, 5.0), (15, 20.0), (30, 30.0)])
def test_interpolant_matches_exp_at_its_points(K, c):
    al, be, a2 = leja.pair_coefficients(K, c)
    a = np.sqrt(a2)
    z = np.concatenate([1j * a, -1j * a])
    np.testing.assert_allclose(leja.eval_pairs(al, be, a2, z), np.exp(z), rtol=0, atol=1e-13)


def test_scaled_basis_is_the_same_polynomial():
    for K, c in ((4, 0.7), (12, 9.0), (30, 40.0)):
        al, be, a2 = leja.pair_coefficients(K, c)
        sa, sb, sa2, g2 = leja.scaled_pairs(K, c)
        y = 1j * np.linspace(-c, c, 1001)
        ref = leja.eval_pairs(al, be, a2, y)
        # evaluate the scaled form: q_(k+1) = (z^2 + c^2 x_k) q_k / g^2
        out, q = np.zeros_like(y), np.ones_like(y)
        for k in range(K):
            out = out + (sa[k] + sb[k] * y) * q
            q = q * (y * y / g2 + sa2[k])
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)


def test_small_interval_gives_the_taylor_polynomial():
    al, be, _ = leja.pair_coefficients(6, 1e-6)
    for k in range(6):
        assert math.isclose(al[k], 1 / math.factorial(2 * k), rel_tol=1e-9)
        assert math.isclose(be[k], 1 / math.factorial(2 * k + 1), rel_tol=1e-9)


@pytest.mark.parametrize("theta,tol", [(3.0, 1e-12), (40.0, 1e-8), (300.0, 1e-6)])
def test_parameters_meet_a_true_bound(theta, tol):
    K, s = leja.leja_parameters(theta, tol)
    assert leja.leja_bound(theta, K, s) <= tol
    if s > 1:
        assert leja.leja_bound(theta, K, s - 1) > tol
    h = theta / s
    al, be, a2 = leja.pair_coefficients(K, h)
    y = np.linspace(-h, h, 100001)
    err = np.abs(leja.eval_pairs(al, be, a2, 1j * y) - np.exp(1j * y)).max()
    delta = leja._basis_max(a2, h, K)[K] / math.factorial(2 * K)
    assert err <= delta + 1e-14
    assert leja.leja_parameters(0.0, 1e-9) == (0, 1)
    with pytest.raises(ValueError):
        leja.leja_parameters(500.0, 1e-9, 2.0 ** -24)


def test_leja_is_cheaper_than_taylor_for_the_normal_fit_matrix():
    for theta, tol in ((20.0, 1e-10), (230.0, 1e-8), (1000.0, 1e-6)):
        K, s = leja.leja_parameters(theta, tol)
        m, ss = expm.taylor_parameters(theta, tol)
        assert (2 * K - 1) * s <= 0.75 * m * ss, (theta, K, s, m, ss)


def test_leja_action_matches_expm_multiply_and_inverts():
    nx, ny, nz = 6, 5, 4
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 3, 9))
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    for t in (0.05, 1.7, 23.0):
        x, (K, s) = leja.leja_action(A, b, t, rho, tol=1e-12)
        ref = spla.expm_multiply(t * A.tocsc(), b)
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(b), (t, K, s)
        back, _ = leja.leja_action(A, x, -t, rho, tol=1e-12)
        assert np.linalg.norm(back - b) <= 2e-10 * np.linalg.norm(b)


def test_leja_action_rotates_the_te101_mode():
    nx, ny, nz = 16, 12, 8
    ops = _ops(nx, ny, nz)
    arr = np.zeros((3, nz, ny, nx))
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    arr[1] = np.sin(np.pi * i / nx) * np.sin(np.pi * k / nz) * np.ones((1, ny, 1))
    phi = layout.edges_from_slots(ops, arr)
    w = math.sqrt((2 * math.sin(math.pi / 32)) ** 2 + (2 * math.sin(math.pi / 16)) ** 2)
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    u0 = paraexp.to_u(ops, phi, np.zeros(ops.n_h))
    ch = ops.M_mu_inv * (ops.C @ phi)
    for t in (0.7, 31.3):
        x, _ = leja.leja_action(A, u0, t, rho, tol=2e-12)
        e, h = paraexp.from_u(ops, x)
        np.testing.assert_allclose(e, math.cos(w * t) * phi, atol=1e-11)
        np.testing.assert_allclose(h, -math.sin(w * t) / w * ch, atol=1e-11)


def test_leja_rounding_term_tracks_a_float32_evaluation():
    nx, ny, nz = 6, 5, 4
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 3, 9))
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    b = np.random.default_rng(8).standard_normal(A.shape[0])
    A32 = A.astype(np.float32)
    u = 2.0 ** -24
    for t, tol in ((10.0, 1e-3), (40.0, 3e-3)):
        K, s = leja.leja_parameters(t * rho, tol, u)
        x64, _ = leja.leja_action(A, b, t, rho, params=(K, s))
        h = t / s
        al, be, a2, g2 = leja.scaled_pairs(K, h * rho)
        al, be, a2 = (v.astype(np.float32) for v in (al, be, a2))
        x = b.astype(np.float32)
        h32, hg = np.float32(h), np.float32(h / g2)
        for _ in range(s):
            q = x
            acc = np.zeros_like(x)
            for k in range(K):
                r = h32 * (A32 @ q)
                acc = acc + al[k] * q + be[k] * r
                if k + 1 < K:
                    q = hg * (A32 @ r) + a2[k] * q
            x = acc
        err = np.linalg.norm(x.astype(np.float64) - x64) / np.linalg.norm(b)
        assert err <= leja.leja_bound(t * rho, K, s, u), (K, s, err)
