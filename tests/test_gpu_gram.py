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


@pytest.mark.parametrize("dtype,K,which", [("f32", 70, 0), ("f64", 33, 1), ("f32", 9, 1)])
def test_gram_aligned_rows_with_a_partial_round(dtype, K, which):
    """A grid whose snapshot stride is a multiple of 16 bytes takes the
    16-byte-load path of the Gram kernel (the 37 x 21 x 13 grid above takes
    the element-wise one); 3 x 28 x 12 x 10 = 10080 rows leave a last
    workgroup chunk shorter than one round of its four waves, so the partial
    round is exercised too.  Against the oracle's exactly rounded sums."""
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = 28, 12, 10
    assert (3 * nx * ny * nz * (4 if dtype == "f32" else 8)) % 16 == 0
    assert (3 * nx * ny * nz) % 128 != 0
    rng = np.random.default_rng(100 + K)
    eps = dielectric_blocks(nx, ny, nz, 4, 3)
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
    ref = gram(np.array([conv(ops, x) for x in X]), M)
    tol = 1e-13 if dtype == "f64" else 1e-6
    assert np.array_equal(G, G.T)
    np.testing.assert_allclose(G, ref, rtol=0, atol=tol * np.max(np.abs(ref)))
    g.close()


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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gram_largest_K_sampled(dtype):
    """K = 4096 snapshots (the largest accepted): entries on a sample of rows and
    columns that includes the first and the last snapshot match the oracle's
    exactly rounded sums (G restricted to a subset S of snapshots is the Gram
    matrix of S); K = 0 and K = 4097 are rejected."""
    from paper_1705_08019_amd import FitGrid, FitError
    nx, ny, nz, K = 6, 5, 4, 4096
    rng = np.random.default_rng(11)
    eps = rng.uniform(1, 5, (nz, ny, nx))
    ops = oracle_ops((nx, ny, nz), eps=eps)
    g = FitGrid(nx, ny, nz, dtype)
    g.set_materials(eps)
    X = rng.standard_normal((K, 3, nz, ny, nx))
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
    print(f"gram K={K} {dtype}", flush=True)
    G = g.gram(torch.tensor(X, device="cuda"), 0)
    assert np.array_equal(G, G.T)
    S = np.unique(np.concatenate([[0, 1, K - 2, K - 1], rng.choice(K, 60, replace=False)]))
    Xo = np.array([edges_from_slots(ops, X[s]) for s in S])
    ref = gram(Xo, ops.M_eps)
    tol = 1e-13 if dtype == "f64" else 1e-6
    np.testing.assert_allclose(G[np.ix_(S, S)], ref, rtol=0, atol=tol * np.max(np.abs(ref)))
    for bad in (0, K + 1):
        with pytest.raises(FitError, match="INVALID"):
            g.gram(torch.zeros((bad, 3, nz, ny, nx), device="cuda"), 0)
