"""GPU parity of the FP64-MFMA Gram matrix G = X^T diag(M) X against the
oracle's entry-by-entry exactly rounded sums, and against closed-form
M-orthogonal cavity modes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import dielectric_blocks
from oracle.gram import gram
from _glue import oracle_ops, edges_from_slots, facets_from_slots

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,K,which", [("f64", 24, 0), ("f64", 5, 1), ("f32", 70, 0),
                                           ("f64", 64, 0), ("f32", 1, 0), ("f32", 40, 1),
                                           ("f32", 16, 0)])
def test_gram_random_snapshots(dtype, K, which):
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = 37, 21, 13
    rng = np.random.default_rng(K + which)
    eps = dielectric_blocks(nx, ny, nz, 6, 8)
    mu = rng.uniform(1, 4, (nz, ny, nx)) if which == 1 else None
    ops = oracle_ops((nx, ny, nz), eps=eps, mu=mu)
    g = FitGrid(nx, ny, nz, dtype)
    g.set_materials(eps, mu)
    X = rng.standard_normal((K, 3, nz, ny, nx))
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
    G = g.gram(torch.tensor(X, device="cuda"), which)
    conv = edges_from_slots if which == 0 else facets_from_slots
    M = ops.M_eps if which == 0 else ops.M_mu
    Xo = np.array([conv(ops, x) for x in X])
    ref = gram(Xo, M)
    tol = 1e-13 if dtype == "f64" else 1e-6     # FP32 grid: materials rounded to FP32
    assert np.array_equal(G, G.T)
    np.testing.assert_allclose(G, ref, rtol=0, atol=tol * np.max(np.abs(ref)))


def test_gram_cavity_modes_closed_form():
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = 40, 12, 20
    g = FitGrid(nx, ny, nz, "f64")
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    X = []
    for m, p in ((1, 1), (2, 1), (1, 3), (5, 2), (7, 7)):
        arr = np.zeros((3, nz, ny, nx))
        arr[1] = np.sin(np.pi * m * i / nx) * np.sin(np.pi * p * k / nz) * np.ones((1, ny, 1))
        X.append(arr)
    G = g.gram(torch.tensor(np.array(X), device="cuda"), 0)
    np.testing.assert_allclose(G, np.eye(5) * (nx / 2) * (nz / 2) * ny, rtol=0, atol=1e-10)
