"""Pins of the oracle on the paper's cylindrical wave (Sec. IV-A; CPU only).

The 20 m x 20 m x 1 m PEC box with 41 (and 121) grid points per side carries
the Gaussian line current of eq. line_current on the centre z edge.  Its
field is pinned against what physics and the scheme fix: the closed-form
field of a line current in free space (before the wall reflections arrive),
the one-cell-per-step domain of dependence of leapfrog, the box's mirror
symmetries and the energy plateau once the excitation has vanished
(Sec. II-A, eq. energy).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from fit_workloads import x1, steps_for
from oracle.leapfrog import gaussian_current, run, trace_derived
from oracle import layout
from _glue import oracle_ops, spec_dt


def _setup(points):
    spec = x1(points)
    ops = oracle_ops(spec)
    nt, dt = steps_for(spec.t_end, spec_dt(spec))
    return spec, ops, nt, dt


def _line_current_vector_potential(r, t, spec):
    """A_z(r, t) of a z-directed line current I(t) (zero before t = 0) in
    free space: the 2-D retarded potential mu0 / (2 pi) times the integral of
    I(t - tau) over tau > r / c with weight 1 / sqrt(tau^2 - r^2 / c^2);
    tau = (r / c) cosh(u) removes the weight.  E_z = -dA_z/dt."""
    c = 1.0 / math.sqrt(spec.eps0 * spec.mu0)
    s = spec.source
    if c * t <= r:
        return 0.0
    U = math.acosh(c * t / r)
    f = lambda u: float(gaussian_current(t - (r / c) * math.cosh(u), s["i_max"], s["sigma_t"])) \
        if t - (r / c) * math.cosh(u) >= 0.0 else 0.0
    return spec.mu0 / (2.0 * math.pi) * quad(f, 0.0, U, limit=200)[0]


@pytest.mark.parametrize("points,tol", [(41, 4e-3), (121, 1.5e-3)])
def test_time_integral_of_e_matches_the_free_space_line_current(points, tol):
    """-sum_m e_z dt at 4 m from the source follows A_z of the continuous
    line current up to t = 5e-8 s (the first wall reflection reaches that
    point at 16 m / c = 5.3e-8 s).  e_z is the voltage of a 1 m edge, so it
    equals E_z.  The time integral removes the front singularity that the
    jump of i(t) at t = 0 puts into E_z itself."""
    spec, ops, nt, dt = _setup(points)
    n = spec.nx
    d = spec.spacing[0]
    off = int(round(4.0 / d))
    pos = ops.edge_slot(2, n // 2 + off, n // 2, 0)
    e, h = np.zeros(ops.n_e), np.zeros(ops.n_h)
    acc, prev = 0.0, 0.0
    ts, Az = [], []
    m = 0
    while (m + 1) * dt <= 5e-8:
        e, h, _ = run(ops, e, h, dt, 1, spec.source, step0=m)
        m += 1
        acc += 0.5 * dt * (prev + e[pos])
        prev = e[pos]
        ts.append(m * dt)
        Az.append(-acc)
    sel = np.linspace(0, len(ts) - 1, 60).astype(int)
    ref = np.array([_line_current_vector_potential(off * d, ts[q], spec) for q in sel])
    got = np.array(Az)[sel]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol


def test_field_spreads_one_cell_per_step():
    """e^m is exactly zero beyond Manhattan distance m - 1 of the source node
    and not zero at that distance on the x axis."""
    spec, ops, nt, dt = _setup(41)
    n = spec.nx
    c = n // 2
    e, h = np.zeros(ops.n_e), np.zeros(ops.n_h)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    dist = np.abs(ii - c) + np.abs(jj - c)
    for m in range(1, 16):
        e, h, _ = run(ops, e, h, dt, 1, spec.source, step0=m - 1)
        ez = layout.edges_to_slots(ops, e).reshape(3, 1, n, n)[2, 0]
        assert np.all(ez[dist > m - 1] == 0.0), m
        assert ez[c, c + m - 1] != 0.0, m


def test_mirror_symmetry_of_the_cylindrical_wave():
    """Square box, centred source: e_z is symmetric under x <-> y and under
    the reflections through the centre lines (up to rounding)."""
    spec, ops, nt, dt = _setup(41)
    n = spec.nx
    e, _, _ = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, nt // 2, spec.source)
    ez = layout.edges_to_slots(ops, e).reshape(3, 1, n, n)[2, 0]
    scale = np.abs(ez).max()
    assert scale > 0
    inner = ez[1:, 1:]                      # nodes 1..n-1 (node 0 is the wall)
    assert np.abs(inner - inner.T).max() <= 1e-12 * scale
    assert np.abs(inner - inner[::-1, :]).max() <= 1e-12 * scale
    assert np.abs(inner - inner[:, ::-1]).max() <= 1e-12 * scale


@pytest.mark.parametrize("points", [41, 121])
def test_energy_plateau_after_the_excitation(points):
    """W^m of eq. energy grows while the current flows and stays constant
    (FP64 rounding) once i(t) has fallen below 1e-16 of its peak."""
    spec, ops, nt, dt = _setup(points)
    _, _, tr = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, nt, spec.source)
    W = trace_derived(tr)["W"]
    s = spec.source
    t_quiet = s["sigma_t"] * (1.0 + math.sqrt(math.log(1e16) / 4.0))
    quiet = np.array([m * dt > t_quiet for m in range(nt)])
    quiet[0] = False
    plateau = W[quiet]
    assert plateau.size > nt // 3
    assert np.abs(plateau - plateau[0]).max() <= 1e-12 * abs(plateau[0])
    early = W[1:int(0.5 * s["sigma_t"] / dt)]
    assert np.all(early < plateau[0])
    assert np.all(np.diff(early) >= -1e-12 * plateau[0])
