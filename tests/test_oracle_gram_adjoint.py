"""Pins of the oracle's Gram matrix and discrete adjoint (CPU only).

Gram: the bilinear energy form of Sec. II-A over snapshots; pinned by the
M-orthogonality of closed-form discrete cavity modes (Yee equivalence).
Adjoint: the reverse recursion of the leapfrog of Sec. II-A; pinned by the
transpose (dot-product) identity and by central finite differences of the
forward objective.
"""
import math

import numpy as np

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators, run
from oracle.gram import gram
from oracle.stability import cfl_dt
from oracle import adjoint as adj
from oracle import layout
from fit_workloads import dielectric_blocks, lossy_slab


def _ops(nx, ny, nz, eps=None, sigma=None):
    t = Topology(nx, ny, nz)
    eps = np.ones((nz, ny, nx)) if eps is None else eps
    return Operators(t, Materials(t, eps, sigma=sigma))


def test_gram_of_cavity_modes_is_closed_form_diagonal():
    nx, ny, nz = 8, 6, 5
    ops = _ops(nx, ny, nz)
    X, diag = [], []
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    for m, p in ((1, 1), (2, 1), (1, 3), (3, 2)):          # e_y modes, y-invariant
        arr = np.zeros((3, nz, ny, nx))
        arr[1] = np.sin(np.pi * m * i / nx) * np.sin(np.pi * p * k / nz) * np.ones((1, ny, 1))
        X.append(layout.edges_from_slots(ops, arr))
        diag.append(nx / 2 * nz / 2 * ny)
    for n, p in ((1, 1), (2, 3)):                           # e_x modes, x-invariant
        arr = np.zeros((3, nz, ny, nx))
        arr[0] = np.sin(np.pi * n * j / ny) * np.sin(np.pi * p * k / nz) * np.ones((1, 1, nx))
        X.append(layout.edges_from_slots(ops, arr))
        diag.append(ny / 2 * nz / 2 * nx)
    G = gram(np.array(X), ops.M_eps)
    np.testing.assert_allclose(G, np.diag(diag), atol=1e-12)


def test_gram_symmetric_psd_with_energies_on_diagonal():
    nx, ny, nz = 6, 5, 4
    ops = _ops(nx, ny, nz, eps=dielectric_blocks(nx, ny, nz, 3, 2))
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5, ops.n_e))
    X[4] = X[0] - 2 * X[1]                     # rank deficiency -> one zero eigenvalue
    G = gram(X, ops.M_eps)
    assert np.array_equal(G, G.T)
    ev = np.linalg.eigvalsh(G)
    assert ev[0] > -1e-10 * ev[-1] and ev[0] < 1e-10 * ev[-1]
    assert np.all(ev[1:] > 0)
    e, h, tr = run(ops, X[2], np.zeros(ops.n_h), 0.1, 1)
    assert math.isclose(G[2, 2], tr[0, 1], rel_tol=1e-14)


def _lossy_case():
    nx, ny, nz = 8, 7, 6
    eps = dielectric_blocks(nx, ny, nz, 4, 21)
    sig = lossy_slab(nx, ny, nz, 1) + 0.01      # conducting everywhere: central FD in sigma
    ops = _ops(nx, ny, nz, eps=eps, sigma=sig)
    dt = 0.9 * cfl_dt(eps)
    src = dict(axis=2, i=4, j=3, k=2, i_max=1.0, sigma_t=8 * dt)
    w = adj.probe_weights(ops, ((4, 7), (3, 6), (3, 5)))
    return ops, eps, sig, dt, src, w


def test_step_transpose_identity():
    ops, _, _, dt, _, _ = _lossy_case()
    rng = np.random.default_rng(2)
    e, h = rng.standard_normal(ops.n_e), rng.standard_normal(ops.n_h)
    l1, m1 = rng.standard_normal(ops.n_e), rng.standard_normal(ops.n_h)
    e1, h1 = adj.step_map(ops, dt, e, h)
    l0, m0 = adj.step_map_adjoint(ops, dt, l1, m1)
    lhs = e1 @ l1 + h1 @ m1
    rhs = e @ l0 + h @ m0
    assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + np.linalg.norm(e1) * np.linalg.norm(l1))


def test_adjoint_forward_matches_leapfrog():
    ops, _, _, dt, src, w = _lossy_case()
    e0, h0 = np.zeros(ops.n_e), np.zeros(ops.n_h)
    n = 50
    _, _, _, es, _ = run(ops, e0, h0, dt, n, source=src, record=True)
    J = dt * sum(np.sum(w * ops.M_eps * e * e) for e in es[1:])
    assert math.isclose(adj.objective(ops, e0, h0, dt, n, src, w), J, rel_tol=1e-12)
    assert J > 0


def test_adjoint_gradient_matches_central_differences():
    ops, eps, sig, dt, src, w = _lossy_case()
    nz, ny, nx = eps.shape
    n = 60
    e0, h0 = np.zeros(ops.n_e), np.zeros(ops.n_h)
    J, g_eps, g_sig, _, _ = adj.gradient(ops, e0, h0, dt, n, src, w)
    rng = np.random.default_rng(55)
    cells = rng.choice(nx * ny * nz, size=32, replace=False)
    h = 1e-3
    top = ops.top

    def J_of(eps_, sig_):
        o = Operators(top, Materials(top, eps_, sigma=sig_))
        return adj.objective(o, e0, h0, dt, n, src, w)

    scale_e = np.max(np.abs(g_eps))
    scale_s = np.max(np.abs(g_sig))
    for c in cells:
        k, j, i = np.unravel_index(c, eps.shape)
        ep, em = eps.copy(), eps.copy()
        ep[k, j, i] += h
        em[k, j, i] -= h
        fd = (J_of(ep, sig) - J_of(em, sig)) / (2 * h)
        assert abs(fd - g_eps[c]) <= 1e-5 * scale_e, (c, fd, g_eps[c])
        sp_, sm_ = sig.copy(), sig.copy()
        sp_[k, j, i] += h
        sm_[k, j, i] -= h
        fd = (J_of(eps, sp_) - J_of(eps, sm_)) / (2 * h)
        assert abs(fd - g_sig[c]) <= 1e-5 * scale_s, (c, fd, g_sig[c])
