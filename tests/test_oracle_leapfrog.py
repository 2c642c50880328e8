"""Pins of the oracle's leapfrog, energies and stability bounds (CPU only).

Sec. II-A: leapfrog updates, eq. cfl, the sharp bound via ||A||_2, eq. energy;
Sec. II eq. FIT_ode_2 (A skew, imaginary spectrum); the Yee equivalence
(closed-form discrete cavity modes); Sec. IV-A eq. line_current.
"""
import math

import numpy as np
import pytest

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators, run, trace_derived, gaussian_current
from oracle.stability import cfl_dt, skew_matrix, spectral_norm
from oracle import layout
from fit_workloads import c1, facet_potential, dielectric_blocks, lossy_slab


def _ops(nx, ny, nz, eps=None, sigma=None, mu=None, spacing=(1.0, 1.0, 1.0)):
    t = Topology(nx, ny, nz)
    eps = np.ones((nz, ny, nx)) if eps is None else eps
    return Operators(t, Materials(t, eps, sigma=sigma, mu_r=mu, spacing=spacing))


def _te101(ops, nx, nz):
    """e_y = sin(pi i / nx) sin(pi k / nz) on every kept y-edge (node coords)."""
    arr = np.zeros((3, ops.top.n[2], ops.top.n[1], ops.top.n[0]))
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    arr[1] = np.sin(np.pi * i / nx) * np.sin(np.pi * k / nz) * np.ones((1, ops.top.n[1], 1))
    return layout.edges_from_slots(ops, arr)


def test_waveform_values():
    st = 2e-8
    assert gaussian_current(st, 1.0, st) == 1.0
    assert math.isclose(float(gaussian_current(0.0, 1.0, st)), math.exp(-4.0), rel_tol=1e-15)
    assert math.isclose(float(gaussian_current(1.5 * st, 2.0, st)), 2.0 * math.exp(-1.0),
                        rel_tol=1e-15)


def test_cfl_unit_cells():
    assert math.isclose(cfl_dt(np.ones((2, 2, 2))), 1.0 / math.sqrt(3.0), rel_tol=1e-15)
    eps = np.full((2, 2, 2), 4.0)
    eps[0, 0, 0] = 2.0
    assert math.isclose(cfl_dt(eps, spacing=(1, 2, 2)), math.sqrt(2.0 / 1.5), rel_tol=1e-15)


def test_skew_and_imaginary_spectrum_matches_closed_form_modes():
    nx, ny, nz = 4, 3, 2
    ops = _ops(nx, ny, nz)
    A = skew_matrix(ops).toarray()
    assert np.array_equal(A.T, -A)
    lam = np.linalg.eigvals(A)
    assert np.max(np.abs(lam.real)) < 1e-12
    w = np.sort(lam.imag[lam.imag > 1e-8])
    # discrete PEC cavity modes: omega^2 = sum_a (2 sin(m_a pi / (2 N_a)))^2, index m_a in
    # [0, N_a - 1], at most one zero index; two polarisations when all are nonzero.
    ref = []
    for m in range(nx):
        for n in range(ny):
            for p in range(nz):
                zeros = (m == 0) + (n == 0) + (p == 0)
                if zeros > 1:
                    continue
                om = 2 * math.sqrt(math.sin(m * math.pi / (2 * nx)) ** 2 +
                                   math.sin(n * math.pi / (2 * ny)) ** 2 +
                                   math.sin(p * math.pi / (2 * nz)) ** 2)
                ref += [om] * (2 if zeros == 0 else 1)
    assert len(ref) == w.size
    np.testing.assert_allclose(w, np.sort(ref), rtol=1e-12, atol=1e-12)


def test_spectral_norm_and_sharp_bound_c1():
    ops = _ops(16, 12, 8)
    wmax = 2 * math.sqrt(math.sin(15 * math.pi / 32) ** 2 + math.sin(11 * math.pi / 24) ** 2 +
                         math.sin(7 * math.pi / 16) ** 2)
    assert abs(wmax - 3.42654) < 1e-5
    nrm = spectral_norm(ops)
    assert math.isclose(nrm, wmax, rel_tol=1e-9)
    assert cfl_dt(np.ones((8, 12, 16))) <= 2.0 / nrm          # 0.5774 <= 0.5837


def test_te101_trajectory_is_exact_discrete_recurrence():
    nx, ny, nz = 16, 12, 8
    ops = _ops(nx, ny, nz)
    phi = _te101(ops, nx, nz)
    assert math.isclose(phi @ (ops.M_eps * phi), 16 * 12 * 8 / 4.0, rel_tol=1e-13)   # 384
    dt = 0.9 / math.sqrt(3.0)
    om2 = (2 * math.sin(math.pi / 32)) ** 2 + (2 * math.sin(math.pi / 16)) ** 2
    assert abs(math.sqrt(om2) - 0.436658) < 1e-6
    theta = math.acos(1.0 - 0.5 * dt * dt * om2)
    assert abs(theta / dt - 0.437600) < 1e-6
    e, h = phi.copy(), np.zeros(ops.n_h)
    for m in range(1, 200):
        e, h, _ = run(ops, e, h, dt, 1)
        x = math.cos((m - 0.5) * theta) / math.cos(0.5 * theta)
        np.testing.assert_allclose(e, x * phi, atol=1e-12)


def test_second_order_convergence_to_analytic_te101():
    a, d = 2.0, 1.0
    w_exact = math.pi * math.sqrt(1 / a ** 2 + 1 / d ** 2)
    errs = []
    for r in (4, 8, 16):
        nx, nz, ny = int(a * r), int(d * r), 2
        h = 1.0 / r
        ops = _ops(nx, ny, nz, spacing=(h, h, h))
        phi = _te101(ops, nx, nz)
        dt = 0.9 * cfl_dt(np.ones((nz, ny, nx)), spacing=(h, h, h))
        e, hf = phi.copy(), np.zeros(ops.n_h)
        xs = [1.0]
        for _ in range(60):
            e, hf, _ = run(ops, e, hf, dt, 1)
            xs.append((e @ phi) / (phi @ phi))
        xs = np.array(xs)
        c2 = np.sum(xs[1:-1] * (xs[2:] + xs[:-2])) / np.sum(xs[1:-1] ** 2)
        errs.append(abs(math.acos(c2 / 2) / dt - w_exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 < r1 < 4.3 and 3.9 < r2 < 4.1


def _c1_initial(ops, spec):
    psi = layout.facets_from_slots(ops, facet_potential(spec.nx, spec.ny, spec.nz,
                                                        spec.init_potential_seed))
    return ops.Ct @ psi


def test_energy_conservation_c1_1000_steps():
    spec = c1()
    ops = _ops(spec.nx, spec.ny, spec.nz)
    e0 = _c1_initial(ops, spec)
    dt = spec.cfl_frac * cfl_dt(spec.eps_r)
    _, _, tr = run(ops, e0, np.zeros(ops.n_h), dt, spec.nsteps)
    der = trace_derived(tr)
    for key in ("W", "Q", "R", "Q_next"):
        v = der[key][1:]
        assert np.max(np.abs(v - v[0])) / abs(v[0]) < 1e-13, key
    # the exchange between electric and magnetic parts is real (not a trivial run)
    assert np.ptp(der["ee"]) / der["ee"][0] > 0.1


def test_charge_conservation():
    ops = _ops(6, 5, 4, eps=dielectric_blocks(6, 5, 4, 3, 9))
    rng = np.random.default_rng(3)
    e0, h0 = rng.standard_normal(ops.n_e), rng.standard_normal(ops.n_h)
    St = ops.top.dual_divergence()[ops.top.interior_nodes()][:, ops.ie]
    q0 = St @ (ops.M_eps * e0)
    e, _, _ = run(ops, e0, h0, 0.5, 300)
    np.testing.assert_allclose(St @ (ops.M_eps * e), q0, atol=1e-11)


def test_time_reversal():
    ops = _ops(6, 5, 4, eps=dielectric_blocks(6, 5, 4, 3, 9))
    rng = np.random.default_rng(4)
    e0, h0 = rng.standard_normal(ops.n_e), rng.standard_normal(ops.n_h)
    dt, n = 0.45, 400
    eN, hN, _ = run(ops, e0, h0, dt, n)
    h_prev = hN + dt * ops.M_mu_inv * (ops.C @ eN)        # undo the last h update
    eb, hb, _ = run(ops, eN, -h_prev, dt, n)
    np.testing.assert_allclose(eb, e0, atol=1e-10)
    # the reversed run ends one half step earlier in h: -h^(-1/2)
    np.testing.assert_allclose(-hb, h0 + dt * ops.M_mu_inv * (ops.C @ e0), atol=1e-10)


def test_stability_threshold():
    ops = _ops(5, 4, 3)
    dt_sharp = 2.0 / spectral_norm(ops)
    rng = np.random.default_rng(5)
    e0 = rng.standard_normal(ops.n_e)
    eS, _, _ = run(ops, e0, np.zeros(ops.n_h), 0.995 * dt_sharp, 3000)
    eU, _, _ = run(ops, e0, np.zeros(ops.n_h), 1.01 * dt_sharp, 300)
    assert np.linalg.norm(eS) < 100 * np.linalg.norm(e0)
    assert np.linalg.norm(eU) > 1e6 * np.linalg.norm(e0)


def test_lossy_source_energy_balance_and_decay():
    nx, ny, nz = 8, 7, 10
    eps = dielectric_blocks(nx, ny, nz, 4, 11)
    sig = lossy_slab(nx, ny, nz, 2)
    ops = _ops(nx, ny, nz, eps=eps, sigma=sig)
    dt = 0.9 * cfl_dt(eps)
    src = dict(axis=2, i=4, j=3, k=5, i_max=1.0, sigma_t=20 * dt)
    _, _, tr = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, 400, source=src)
    der = trace_derived(tr)
    dQ = der["Q_next"] - np.concatenate([[0.0], der["Q_next"][:-1]])   # Q^0 = 0
    expect = -2 * dt * (tr[:, 8] + tr[:, 9])
    scale = np.max(np.abs(der["Q_next"]))
    assert np.max(np.abs(dQ - expect)) < 1e-13 * scale
    assert scale > 0 and np.all(tr[:, 8] >= 0)
    late = der["Q_next"][120:]                       # source has died out (~3 sigma_t)
    assert np.all(np.diff(late) <= 1e-14 * scale)
    assert late[-1] < (1 - 1e-5) * late[0]
