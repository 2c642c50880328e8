"""Dead slots poisoned with NaN.  The slot layout holds an entry for every
(direction, node) pair; the entries that are not unknowns of the PEC problem
(edges tangential to a boundary plane, facets normal to one, the phantom
slots past the last node) must never be read as data by any kernel.  Each
test fills them with NaN in the state buffers (and the whole second buffer
set with NaN), steps a poisoned and a clean grid through the same path, and
requires the live entries, the energies and the trace to be bitwise those
of the clean run; dead entries of every result are 0 or untouched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import lossy_slab
from _glue import oracle_ops, edges_to_slots, facets_to_slots

pytestmark = pytest.mark.gpu

N = (37, 22, 15)


def _live_masks(n):
    ops = oracle_ops(n)
    le = edges_to_slots(ops, np.ones(ops.n_e)) != 0
    lh = facets_to_slots(ops, np.ones(ops.n_h)) != 0
    return torch.from_numpy(le).cuda(), torch.from_numpy(lh).cuda()


def _grid(dtype, rng_seed=3):
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = N
    g = FitGrid(nx, ny, nz, dtype)
    rng = np.random.default_rng(11)
    eps = 1.0 + 3.0 * rng.random((nz, ny, nx))
    g.set_materials(eps, None, lossy_slab(nx, ny, nz, 2, 0.05))
    dt = 0.9 * g.cfl_dt()
    g.set_source(2, nx // 2, ny // 2, nz // 2, 1.0, 6 * dt)
    r = np.random.default_rng(rng_seed)
    g.set_fields(r.standard_normal((3, nz, ny, nx)), r.standard_normal((3, nz, ny, nx)))
    return g, dt


def _poison(g, le, lh):
    """NaN into every dead slot of the state and into all of the other set."""
    e, h = g.state()
    state = {e.data_ptr(), h.data_ptr()}
    with torch.no_grad():
        e[~le] = float("nan")
        h[~lh] = float("nan")
        for t in g._fields:
            if t.data_ptr() not in state:
                t.fill_(float("nan"))
    torch.cuda.synchronize()


def _check(gp, gc, le, lh, tag):
    ep, hp = gp.get_fields()
    ec, hc = gc.get_fields()
    assert torch.equal(ep[le], ec[le]), f"{tag}: live e differs"
    assert torch.equal(hp[lh], hc[lh]), f"{tag}: live h differs"
    # dead entries of the result: written as 0, or never written (still NaN)
    de, dh = ep[~le], hp[~lh]
    assert bool(torch.all((de == 0) | torch.isnan(de))), f"{tag}: dead e holds data"
    assert bool(torch.all((dh == 0) | torch.isnan(dh))), f"{tag}: dead h holds data"
    return int(torch.isnan(de).sum()) + int(torch.isnan(dh).sum())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("path", ["fused", "split", "pairs"])
def test_dead_slots_are_never_read(dtype, path):
    le, lh = _live_masks(N)
    grids = []
    for _ in range(2):
        g, dt = _grid(dtype)
        if path == "split":
            g.set_tuning("split")
        elif path == "fused":
            g.set_tuning("fused")
        else:
            g.set_pair(True, 32, 16, 4)
        g.trace_config(3, 40)
        grids.append(g)
    gp, gc = grids
    _poison(gp, le, lh)
    for g in grids:
        g.step(9, dt)
    nan_left = _check(gp, gc, le, lh, f"{path} {dtype}")
    tp, _ = gp.trace_read()
    tc, _ = gc.trace_read()
    assert np.array_equal(tp, tc, equal_nan=True)
    assert not np.isnan(tp[np.isfinite(tc)]).any()
    ep, ec = gp.energies(), gc.energies()
    for k in ep:
        assert ep[k] == ec[k] or (np.isnan(ep[k]) and np.isnan(ec[k])), (k, ep[k], ec[k])
    print(f"dead slots {path} {dtype}: {nan_left} dead entries still NaN after 9 steps", flush=True)
    for g in grids:
        g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_dead_slots_batched_pairs(dtype):
    from paper_1705_08019_amd import FitBatch
    le, lh = _live_masks(N)
    gb, gc, dts = [], [], []
    for s in range(3):
        g, dt = _grid(dtype, rng_seed=s)
        gb.append(g)
        dts.append(dt)
        gc.append(_grid(dtype, rng_seed=s)[0])
    for g in gb:
        _poison(g, le, lh)
    b = FitBatch(gb)
    b.set_pair(True, 8)
    b.step(7, np.array(dts))
    for g, dt in zip(gc, dts):
        g.step(7, dt)
    for k, (p, c) in enumerate(zip(gb, gc)):
        _check(p, c, le, lh, f"batch grid {k} {dtype}")
    b.close()
    for g in gb + gc:
        g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_dead_rows_of_gram_snapshots(dtype):
    """Snapshots with NaN in their dead rows give the Gram matrix of the same
    snapshots with zeros there, bitwise (each dead row's values are selected
    away), for e- and h-snapshots and a K with a partial tile."""
    le, lh = _live_masks(N)
    g, _ = _grid(dtype)
    rng = np.random.default_rng(5)
    K = 21
    for which, live in ((0, le), (1, lh)):
        X = torch.from_numpy(rng.standard_normal((K,) + tuple(live.shape))).to(
            device="cuda", dtype=g.tdtype)
        X[:, ~live] = 0.0
        Xp = X.clone()
        Xp[:, ~live] = float("nan")
        G0, Gp = g.gram(X, which), g.gram(Xp, which)
        assert np.isfinite(G0).all()
        assert np.array_equal(G0, Gp), which
    g.close()
