"""Pins of the oracle's grid topology and material matrices (CPU only).

Sec. II: the discrete curls and divergences (eqs. maxwell_grid1/2), n_dof of
the cylindrical-wave grids (Sec. IV-A), and the diagonal material matrices
(eq. maxwell_grid3).
"""
import os

import numpy as np
import pytest

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [(1, 1, 1), (2, 1, 3), (4, 3, 2), (5, 4, 3), (16, 12, 8)]


def _exact_zero(M):
    M = M.tocoo()
    M.eliminate_zeros()
    return M.nnz == 0


@pytest.mark.parametrize("shape", SHAPES)
def test_complex_identities(shape):
    t = Topology(*shape)
    G, C, S = t.gradient(), t.curl(), t.divergence()
    Ct, St = t.dual_curl(), t.dual_divergence()
    assert _exact_zero(S @ C)            # div curl = 0 on the primal grid
    assert _exact_zero(C @ G)            # curl grad = 0
    assert _exact_zero(St @ Ct)          # div curl = 0 on the dual grid
    assert _exact_zero(Ct - C.T)         # dual curl is the transposed primal curl
    assert _exact_zero(St + G.T)         # dual divergence is minus the transposed gradient
    for M in (G, C, S, Ct, St):
        assert set(np.unique(M.data)) <= {-1.0, 1.0}


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 2), (4, 3, 2), (5, 4, 3)])
def test_pec_rank_identity(shape):
    t = Topology(*shape)
    ie, if_, inn = t.interior_edges(), t.interior_facets(), t.interior_nodes()
    Cp = t.curl()[if_][:, ie].toarray()
    rank = np.linalg.matrix_rank(Cp) if Cp.size else 0
    assert rank == ie.sum() - inn.sum()
    assert rank == if_.sum() - (t.n_cells - 1)


def test_pec_counts_c1_grid():
    t = Topology(16, 12, 8)
    assert t.interior_edges().sum() == 3812
    assert t.interior_facets().sum() == 4192
    # rank of the restricted curl follows from the counts: 3812 - 1155 = 2657
    assert t.interior_edges().sum() - t.interior_nodes().sum() == 2657
    assert t.interior_facets().sum() - (t.n_cells - 1) == 2657


def test_paper_ndof_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_ndof.txt"), dtype=np.int64)
    for px, py, pz, ndof in rows:
        t = Topology(px - 1, py - 1, pz - 1)    # the paper counts points, the grid cells
        assert t.canonical_ndof() == ndof


def test_materials_identity_for_unit_vacuum():
    t = Topology(4, 3, 2)
    m = Materials(t, np.ones((2, 3, 4)))
    ops = Operators(t, m)
    assert np.array_equal(ops.M_eps, np.ones(ops.n_e))
    assert np.array_equal(ops.M_mu_inv, np.ones(ops.n_h))
    assert np.array_equal(ops.M_sigma, np.zeros(ops.n_e))


def test_uniform_field_energy_equals_continuum_energy():
    """For a uniform field E along axis a, e_i = E * L_i on every a-edge and
    the discrete energy over ALL a-edges equals the integral of eps E^2 over
    the box, for any per-cell eps; likewise for b = B * A_f and 1/mu."""
    rng = np.random.default_rng(7)
    nx, ny, nz = 5, 4, 3
    d = (0.7, 1.3, 0.9)
    eps = rng.uniform(1, 10, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    t = Topology(nx, ny, nz)
    m = Materials(t, eps, mu_r=mu, spacing=d, eps0=2.0, mu0=0.5)
    V = d[0] * d[1] * d[2]
    for a in range(3):
        sl = slice(t.edge_off[a], t.edge_off[a + 1])
        E = 1.7
        e = np.full(sl.stop - sl.start, E * d[a])
        assert np.isclose(e @ (m.M_eps[sl] * e), 2.0 * eps.sum() * V * E * E, rtol=1e-13)
        sf = slice(t.facet_off[a], t.facet_off[a + 1])
        B = 0.3
        area = d[(a + 1) % 3] * d[(a + 2) % 3]
        b = np.full(sf.stop - sf.start, B * area)
        # magnetic energy b^T M_mu^{-1} b = integral of B^2 / mu
        assert np.isclose(b @ (m.M_mu_inv[sf] * b), (1.0 / (0.5 * mu)).sum() * V * B * B,
                          rtol=1e-13)


def test_single_cell_perturbation_touches_its_edges_and_facets():
    t = Topology(4, 3, 3)
    base = np.ones((3, 3, 4))
    pert = base.copy()
    ci, cj, ck = 2, 1, 1
    pert[ck, cj, ci] += 1.0
    dM = Materials(t, pert).M_eps - Materials(t, base).M_eps
    touched = np.flatnonzero(dM)
    assert touched.size == 12 and np.allclose(dM[touched], 0.25)
    expect = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for db in (0, 1):
            for dc in (0, 1):
                p = np.array([ci, cj, ck])
                p[b] += db
                p[c] += dc
                expect.append(int(t.edge(a, p.reshape(3, 1))[0]))
    assert sorted(expect) == sorted(touched.tolist())
    pm = base.copy()
    pm[ck, cj, ci] = 2.0                       # 1/mu changes by -1/2
    dMi = Materials(t, base, mu_r=pm).M_mu_inv - Materials(t, base).M_mu_inv
    tf = np.flatnonzero(dMi)
    assert tf.size == 6 and np.allclose(dMi[tf], -0.25)


def test_materials_reject_non_spd():
    t = Topology(2, 2, 2)
    with pytest.raises(ValueError):
        Materials(t, -np.ones((2, 2, 2)))
    with pytest.raises(ValueError):
        Materials(t, np.ones((2, 2, 2)), sigma=-np.ones((2, 2, 2)))
