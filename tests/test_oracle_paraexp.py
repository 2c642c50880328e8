"""Pins of the oracle's matrix-exponential action and ParaExp (CPU only).

Sec. III-A (Taylor action of exp(tA) with scaling), Sec. III / Alg. 1
(ParaExp), Sec. III-B (staggered reconstruction), eq. FIT_ode_2 (skew A).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators, run
from oracle.stability import skew_matrix, spectral_norm, cfl_dt
from oracle import expm, paraexp, layout
from fit_workloads import dielectric_blocks


def _ops(nx, ny, nz, eps=None):
    t = Topology(nx, ny, nz)
    eps = np.ones((nz, ny, nx)) if eps is None else eps
    return Operators(t, Materials(t, eps))


def _te101(ops, nx, nz):
    arr = np.zeros((3, ops.top.n[2], ops.top.n[1], ops.top.n[0]))
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    arr[1] = np.sin(np.pi * i / nx) * np.sin(np.pi * k / nz) * np.ones((1, ops.top.n[1], 1))
    return layout.edges_from_slots(ops, arr)


def test_taylor_parameters_meet_their_bound_and_are_cheapest():
    for theta, tol, u in ((0.3, 1e-12, 2.0 ** -53), (5.0, 1e-8, 2.0 ** -53),
                          (80.0, 1e-12, 2.0 ** -53), (1234.5, 1e-6, 2.0 ** -53),
                          (60.0, 1e-3, 2.0 ** -24)):
        m, s = expm.taylor_parameters(theta, tol, u)
        assert expm.taylor_error_bound(theta, m, s, u) <= tol
        # no cheaper pair meets the bound (brute force)
        for mm in range(1, 61):
            for ss in range(1, m * s // mm + 1):
                if mm * ss < m * s:
                    assert expm.taylor_error_bound(theta, mm, ss, u) > tol, (theta, mm, ss)
    assert expm.taylor_parameters(0.0, 1e-12) == (0, 1)
    with pytest.raises(ValueError):
        expm.taylor_parameters(500.0, 1e-9, 2.0 ** -24)   # below the FP32 rounding floor


def test_rounding_term_tracks_a_float32_evaluation():
    """The rounding part of the bound covers a float32 evaluation of the
    same polynomial on the skew matrix (against the float64 one)."""
    nx, ny, nz = 6, 5, 4
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 3, 9))
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(A.shape[0])
    A32 = A.astype(np.float32)
    for t, tol in ((10.0, 1e-3), (4.0, 1e-4), (15.0, 2e-3)):
        m, s = expm.taylor_parameters(t * rho, tol, 2.0 ** -24)
        x64, _ = expm.expm_action(A, b, t, rho, params=(m, s))
        x = b.astype(np.float32)
        h = np.float32(t / s)
        for _ in range(s):
            term = x.copy()
            acc = x.copy()
            for k in range(1, m + 1):
                term = (h / np.float32(k)) * (A32 @ term)
                acc += term
            x = acc
        err = np.linalg.norm(x.astype(np.float64) - x64) / np.linalg.norm(b)
        rnd = s * (m + 2) * 2.0 ** -24 * math.exp(t * rho / s)
        assert err <= rnd, (m, s, err, rnd)


def test_taylor_bound_is_a_true_bound_on_the_imaginary_axis():
    # |T_m(iy) - e^{iy}| <= |y|^(m+1)/(m+1)! for real y (Lagrange remainder)
    for m in (3, 8, 15):
        for y in np.linspace(-3.0, 3.0, 41):
            tm = sum((1j * y) ** k / math.factorial(k) for k in range(m + 1))
            # (+ rounding of the partial sum)
            assert abs(tm - np.exp(1j * y)) <= abs(y) ** (m + 1) / math.factorial(m + 1) + 1e-15


def test_expm_action_matches_scipy_expm_multiply():
    nx, ny, nz = 6, 5, 4
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 3, 9))
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    for t in (0.05, 1.7, 23.0):
        x, (m, s) = expm.expm_action(A, b, t, rho, tol=1e-12)
        ref = spla.expm_multiply(t * A.tocsc(), b)
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(b), (t, m, s)
        # skew A: exp(tA) is orthogonal
        assert abs(np.linalg.norm(x) - np.linalg.norm(b)) <= 1e-11 * np.linalg.norm(b)


def test_expm_action_rotates_the_te101_mode_at_the_discrete_frequency():
    nx, ny, nz = 16, 12, 8
    ops = _ops(nx, ny, nz)
    phi = _te101(ops, nx, nz)
    w = math.sqrt((2 * math.sin(math.pi / 32)) ** 2 + (2 * math.sin(math.pi / 16)) ** 2)
    assert abs(w - 0.436658) < 1e-6
    A = skew_matrix(ops)
    rho = spectral_norm(ops)
    u0 = paraexp.to_u(ops, phi, np.zeros(ops.n_h))
    ch = ops.M_mu_inv * (ops.C @ phi)
    for t in (0.7, 10.0, 31.3):
        x, _ = expm.expm_action(A, u0, t, rho, tol=2e-12)
        e, h = paraexp.from_u(ops, x)
        np.testing.assert_allclose(e, math.cos(w * t) * phi, atol=1e-11)
        np.testing.assert_allclose(h, -math.sin(w * t) / w * ch, atol=1e-11)


def test_paraexp_with_leapfrog_homogeneous_parts_is_one_leapfrog_run():
    nx, ny, nz = 9, 7, 6
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 4, 21))
    dt = 0.9 * cfl_dt(dielectric_blocks(nx, ny, nz, 4, 21))
    src = dict(axis=2, i=4, j=3, k=2, i_max=1.0, sigma_t=6 * dt)
    rng = np.random.default_rng(4)
    e0 = ops.Ct @ rng.uniform(-1, 1, ops.n_h)
    h0 = 0.1 * rng.standard_normal(ops.n_h)
    e_ref, h_ref, _ = run(ops, e0, h0, dt, 60, src)
    for p in (1, 2, 3, 5):
        e, h, _ = paraexp.paraexp(ops, dt, 60, p, src, e0, h0, homogeneous="leapfrog")
        scale = np.linalg.norm(e_ref)
        assert np.linalg.norm(e - e_ref) <= 1e-12 * scale, p
        assert np.linalg.norm(h - h_ref) <= 1e-12 * np.linalg.norm(h_ref), p


def test_paraexp_single_interval_propagates_the_mode_exactly():
    """p = 1, no source, e^0 = TE101 mode and h^(1/2) chosen so that the
    collocated h(0) = 0: the result is the exact semi-discrete solution,
    e at T and h at T + dt/2 (eqs. averaging1/2)."""
    nx, ny, nz = 16, 12, 8
    ops = _ops(nx, ny, nz)
    phi = _te101(ops, nx, nz)
    w = math.sqrt((2 * math.sin(math.pi / 32)) ** 2 + (2 * math.sin(math.pi / 16)) ** 2)
    dt = 0.9 / math.sqrt(3.0)
    ch = ops.M_mu_inv * (ops.C @ phi)
    h_half = -0.5 * dt * ch
    N = 40
    e, h, cost = paraexp.paraexp(ops, dt, N, 1, None, phi, h_half, tol=2e-12)
    T = N * dt
    np.testing.assert_allclose(e, math.cos(w * T) * phi, atol=1e-11)
    np.testing.assert_allclose(h, -math.sin(w * (T + 0.5 * dt)) / w * ch, atol=1e-11)
    assert cost["C_proc"] == 2 * N + cost["A_applications"][0] + 2


def test_paraexp_zero_initial_values_single_interval_is_leapfrog():
    nx, ny, nz = 8, 6, 5
    ops = _ops(nx, ny, nz)
    dt = 0.5
    src = dict(axis=1, i=3, j=2, k=2, i_max=1.0, sigma_t=5 * dt)
    e_ref, h_ref, _ = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, 30, src)
    e, h, _ = paraexp.paraexp(ops, dt, 30, 1, src)
    np.testing.assert_array_equal(e, e_ref)
    np.testing.assert_array_equal(h, h_ref)


def test_paraexp_and_leapfrog_differ_at_second_order():
    """Both approximate the same semi-discrete solution; ParaExp's error is
    leapfrog's on each sub-interval (Sec. III-D), so the gap between the two
    shrinks by ~4 when dt halves at fixed T."""
    nx, ny, nz = 8, 6, 6
    ops = _ops(nx, ny, nz, dielectric_blocks(nx, ny, nz, 3, 8))
    dt0 = 0.4 * cfl_dt(dielectric_blocks(nx, ny, nz, 3, 8))
    T = 48 * dt0
    gaps = []
    for r in (1, 2, 4):
        dt = dt0 / r
        N = 48 * r
        src = dict(axis=2, i=4, j=3, k=3, i_max=1.0, sigma_t=T / 4)
        e_lf, _, _ = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, N, src)
        e_px, _, _ = paraexp.paraexp(ops, dt, N, 4, src, tol=2e-12)
        gaps.append(np.linalg.norm(e_px - e_lf) / np.linalg.norm(e_lf))
    assert 3.5 < gaps[0] / gaps[1] < 4.5 and 3.5 < gaps[1] / gaps[2] < 4.5, gaps


def test_condition_number_of_the_fit_exponential_is_the_spectral_norm():
    """Sec. III-D uses kappa_exp(A) = ||A||_2 for normal A.  For the FIT skew
    matrix the 2-norm relative condition number of exp at tA,
    max_E ||L(tA, E)||_2 / ||E||_2 * ||tA||_2 / ||exp(tA)||_2 (L the Frechet
    derivative), is t ||A||_2: exp(tA) is orthogonal, ||L(tA, E)||_2 <=
    ||E||_2 for random E, with equality at E = I.  The optimal tolerance
    then balances eps_B / eps_A against that condition number."""
    import scipy.linalg as sla
    ops = _ops(4, 3, 3, dielectric_blocks(4, 3, 3, 2, 7))
    A = skew_matrix(ops).toarray()
    rho = spectral_norm(ops)
    t = 0.7
    X = t * A
    E_X = sla.expm(X)
    assert np.linalg.norm(E_X.T @ E_X - np.eye(len(A)), 2) <= 1e-12
    rng = np.random.default_rng(0)
    ratios = []
    for q in range(6):
        E = np.eye(len(A)) if q == 0 else rng.standard_normal(A.shape)
        _, L = sla.expm_frechet(X, E)
        ratios.append(np.linalg.norm(L, 2) / np.linalg.norm(E, 2))
    assert abs(ratios[0] - 1.0) <= 1e-10
    assert max(ratios) <= 1.0 + 1e-10
    kappa = max(ratios) * np.linalg.norm(X, 2) / np.linalg.norm(E_X, 2)
    assert abs(kappa - t * rho) <= 1e-10 * t * rho
    beta, dt = 0.3, 0.05
    tol = expm.optimal_tolerance(beta, dt, kappa / t)
    assert abs(beta * dt ** 2 / tol - kappa / t) <= 1e-12 * rho
    with pytest.raises(ValueError):
        expm.optimal_tolerance(0.0, dt, rho)
