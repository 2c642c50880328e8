"""Pins of the oracle on tensor grids with per-axis cell widths (non-uniform
spacing; Sec. II, eq. maxwell_grid3 and eq. cfl with per-cell dimensions).
CPU only."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.topology import Topology
from oracle.materials import Materials, cell_widths
from oracle.leapfrog import Operators, run, trace_derived
from oracle.stability import cfl_dt, skew_matrix, spectral_norm


def _widths(rng, n, lo=0.3, hi=1.7):
    return [rng.uniform(lo, hi, k) for k in n]


def test_equal_widths_reproduce_the_uniform_grid():
    rng = np.random.default_rng(3)
    nx, ny, nz = 5, 4, 3
    t = Topology(nx, ny, nz)
    eps = rng.uniform(1, 10, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    sig = rng.uniform(0, 1, (nz, ny, nx))
    d = (0.7, 1.3, 0.9)
    arr = [np.full(k, v) for k, v in zip((nx, ny, nz), d)]
    a = Materials(t, eps, sig, mu, spacing=d, eps0=2.0, mu0=0.5)
    b = Materials(t, eps, sig, mu, spacing=arr, eps0=2.0, mu0=0.5)
    assert np.array_equal(a.M_eps, b.M_eps)
    assert np.array_equal(a.M_sigma, b.M_sigma)
    assert np.array_equal(a.M_mu_inv, b.M_mu_inv)
    assert cfl_dt(eps, mu, d) == cfl_dt(eps, mu, arr)


def test_widths_are_validated():
    t = Topology(3, 2, 2)
    with pytest.raises(ValueError):
        cell_widths(t, (np.ones(3), np.ones(3), np.ones(2)))
    with pytest.raises(ValueError):
        cell_widths(t, (np.ones(3), np.array([1.0, -1.0]), np.ones(2)))


def test_uniform_field_energy_on_a_graded_grid():
    """A uniform field E along axis a has e = E L on every a-edge (L = the
    edge's own length); the discrete energy over all a-edges is the integral
    of eps E^2 over the box for any widths and per-cell eps; likewise b = B A
    on every a-facet (A = the facet's own area) and the integral of B^2 / mu."""
    rng = np.random.default_rng(8)
    nx, ny, nz = 5, 4, 3
    t = Topology(nx, ny, nz)
    wd = _widths(rng, (nx, ny, nz))
    eps = rng.uniform(1, 10, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    m = Materials(t, eps, mu_r=mu, spacing=wd, eps0=2.0, mu0=0.5)
    V = wd[2][:, None, None] * wd[1][None, :, None] * wd[0][None, None, :]
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        sl = slice(t.edge_off[a], t.edge_off[a + 1])
        p = t.edge_coords(a)
        e = 1.7 * wd[a][p[a]]
        assert np.isclose(e @ (m.M_eps[sl] * e), 2.0 * (eps * V).sum() * 1.7 ** 2, rtol=1e-13)
        sf = slice(t.facet_off[a], t.facet_off[a + 1])
        q = t.facet_coords(a)
        bf = 0.3 * wd[b][q[b]] * wd[c][q[c]]
        assert np.isclose(bf @ (m.M_mu_inv[sf] * bf), (V / (0.5 * mu)).sum() * 0.3 ** 2,
                          rtol=1e-13)


def test_single_cell_perturbation_on_a_graded_grid():
    """Raising eps_r of one cell by 1 raises M_eps of exactly its 12 edges, each
    by a quarter of the cell's cross-section normal to the edge over the
    edge's length; 1/mu of one cell enters its 6 facets with half its width
    normal to the facet over the facet's area."""
    rng = np.random.default_rng(9)
    nx, ny, nz = 4, 3, 3
    t = Topology(nx, ny, nz)
    wd = _widths(rng, (nx, ny, nz))
    base = np.ones((nz, ny, nx))
    ci, cj, ck = 2, 1, 1
    pert = base.copy()
    pert[ck, cj, ci] += 1.0
    dM = Materials(t, pert, spacing=wd).M_eps - Materials(t, base, spacing=wd).M_eps
    touched = np.flatnonzero(np.abs(dM) > 1e-15)
    assert touched.size == 12
    cw = (wd[0][ci], wd[1][cj], wd[2][ck])
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for db in (0, 1):
            for dc in (0, 1):
                p = np.array([ci, cj, ck])
                p[b] += db
                p[c] += dc
                r = int(t.edge(a, p.reshape(3, 1))[0])
                assert math.isclose(dM[r], cw[b] * cw[c] / 4.0 / cw[a], rel_tol=1e-13)
    pm = base.copy()
    pm[ck, cj, ci] = 2.0                       # 1/mu changes by -1/2
    dMi = Materials(t, base, mu_r=pm, spacing=wd).M_mu_inv - Materials(t, base, spacing=wd).M_mu_inv
    tf = np.flatnonzero(np.abs(dMi) > 1e-15)
    assert tf.size == 6
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for da in (0, 1):
            p = np.array([ci, cj, ck])
            p[a] += da
            r = int(t.facet(a, p.reshape(3, 1))[0])
            assert math.isclose(dMi[r], -0.5 * (cw[a] / 2.0) / (cw[b] * cw[c]), rel_tol=1e-13)


def test_cfl_takes_each_cells_own_widths():
    eps = np.full((2, 2, 2), 4.0)
    eps[1, 1, 1] = 2.0
    wx, wy, wz = np.array([1.0, 0.5]), np.array([2.0, 1.0]), np.array([1.0, 0.25])
    # brute force over the 8 cells
    best = min(math.sqrt(eps[k, j, i] / (1 / wx[i] ** 2 + 1 / wy[j] ** 2 + 1 / wz[k] ** 2))
               for i in range(2) for j in range(2) for k in range(2))
    assert cfl_dt(eps, spacing=(wx, wy, wz)) == pytest.approx(best, rel=1e-15)
    assert cfl_dt(eps, spacing=(wx, wy, wz)) == pytest.approx(math.sqrt(2.0 / 21.0), rel=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cfl_estimate_is_stable_on_graded_grids(seed):
    """eq. cfl is a sufficient condition: dt_CFL <= 2 / ||A||_2 on random
    graded grids with random materials (the sharp bound of Sec. II-A)."""
    rng = np.random.default_rng(seed)
    n = (6, 5, 4)
    wd = _widths(rng, n, 0.1, 1.0)
    eps = rng.uniform(1, 5, n[::-1])
    mu = rng.uniform(1, 2, n[::-1])
    t = Topology(*n)
    ops = Operators(t, Materials(t, eps, mu_r=mu, spacing=wd))
    assert cfl_dt(eps, mu, wd) * spectral_norm(ops) <= 2.0


def _graded(L, cells, amp):
    """Widths of a smooth grading x(s) = L (s + amp sin(2 pi s) / (2 pi))."""
    s = np.linspace(0.0, 1.0, cells + 1)
    x = L * (s + amp * np.sin(2 * np.pi * s) / (2 * np.pi))
    return np.diff(x)


def test_cavity_frequency_converges_on_a_graded_grid():
    """The lowest TE mode of a 2 x 1 (x, z) PEC cavity (w = pi sqrt(1/4 + 1))
    on smoothly graded grids: the discrete eigenfrequency converges to it at
    second order."""
    a, d = 2.0, 1.0
    w_exact = math.pi * math.sqrt(1 / a ** 2 + 1 / d ** 2)
    errs = []
    for r in (4, 8, 16):
        nx, nz, ny = int(a * r), int(d * r), 2
        wd = [_graded(a, nx, 0.3), np.full(ny, 0.5), _graded(d, nz, 0.3)]
        t = Topology(nx, ny, nz)
        ops = Operators(t, Materials(t, np.ones((nz, ny, nx)), spacing=wd))
        A = skew_matrix(ops)
        K = (A.T @ A).tocsc()
        vals = spla.eigsh(K, k=4, sigma=0.9 * w_exact ** 2, return_eigenvectors=False)
        w = np.sqrt(np.abs(vals))
        errs.append(np.min(np.abs(w - w_exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.5 < r2 < 4.5, errs


def test_energy_is_conserved_on_a_graded_grid():
    rng = np.random.default_rng(4)
    n = (7, 6, 5)
    wd = _widths(rng, n)
    eps = rng.uniform(1, 5, n[::-1])
    t = Topology(*n)
    ops = Operators(t, Materials(t, eps, spacing=wd))
    dt = 0.95 * cfl_dt(eps, None, wd)
    e0 = ops.Ct @ rng.uniform(-1, 1, ops.n_h)
    _, _, tr = run(ops, e0, np.zeros(ops.n_h), dt, 400)
    W = trace_derived(tr)["W"][1:]
    assert np.abs(W - W[0]).max() <= 1e-13 * W[0]


@pytest.mark.parametrize("k", [1.0, 4.0, 20.0])
def test_graded_cylindrical_wave_recipe(k):
    """The k-ratio mesh of Sec. IV-A: widths sum to the 20 m box, the largest
    over the smallest is k, and the CFL step shrinks with the small cell."""
    from fit_workloads import x1, x1_graded
    from _glue import spec_dt
    s = x1_graded(41, k)
    for a in range(2):
        w = s.spacing[a]
        assert w.size == 40 and abs(w.sum() - 20.0) <= 1e-12
        assert abs(w.max() / w.min() - k) <= 1e-12 * k
    if k == 1.0:
        assert np.allclose(s.spacing[0], 0.5, rtol=1e-15)
        assert spec_dt(s) == pytest.approx(spec_dt(x1(41)), rel=1e-14)
    else:
        assert spec_dt(s) < spec_dt(x1(41))
