"""Two fused leapfrog steps per launch (temporal blocking of the Sec. II-A
recurrence): bitwise equal to single fused steps on ragged grids, every tile
shape and z-chunk (chunk boundaries at every plane), FP32/FP64, lossy and
lossless, with a source; mixed with single steps around trace rows; and
against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import dielectric_blocks, lossy_slab
from oracle.leapfrog import run
from _glue import oracle_ops, rel_l2, to_np, edges_from_slots, facets_from_slots

pytestmark = pytest.mark.gpu


def _grid(n, dtype, lossy, seed=3):
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = n
    eps = dielectric_blocks(nx, ny, nz, 5, seed)
    sig = lossy_slab(nx, ny, nz, 1, 0.2) if lossy else None
    g = FitGrid(nx, ny, nz, dtype)
    g.set_materials(eps, None, sig)
    rng = np.random.default_rng(seed)
    g.set_fields(rng.standard_normal((3, nz, ny, nx)), rng.standard_normal((3, nz, ny, nx)), 0)
    dt = 0.9 * g.cfl_dt()
    g.set_source(2, nx // 2, ny // 2, nz // 2, 1.0, 4 * dt)
    g.set_tuning("fused")
    return g, dt, eps, sig


def _run(n, dtype, lossy, steps, pair=None):
    g, dt, _, _ = _grid(n, dtype, lossy)
    if pair is not None:
        g.set_pair(True, *pair)
    g.profile_begin(4 * steps + 8)
    g.step(steps, dt)
    prof = g.profile_end()
    e, h = g.get_fields()
    out = (e.clone(), h.clone(), g.step_index, g.smvp_count(), prof)
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,lossy", [((70, 33, 21), True), ((13, 9, 7), False), ((129, 17, 5), True),
                                     ((40, 40, 1), False), ((9, 70, 2), True), ((5, 4, 3), False)])
def test_pair_is_bitwise_two_single_steps(dtype, n, lossy):
    steps = 10
    ref = _run(n, dtype, lossy, steps)
    assert ref[4]["pair"][1] == 0
    shapes = [(64, 12, 0), (64, 8, 1), (32, 16, 2), (64, 8, 3), (32, 16, 5), (16, 8, 0),
              (128, 8, 0), (48, 10, 4), (20, 6, 0), (48, 12, 2), (32, 24, 3),
              (64, 16, 0), (64, 16, 3), (40, 24, 2)]   # the last three: two points per thread (FP32)
    from paper_1705_08019_amd import FitError
    ran = 0
    for tw, ty, kc in shapes:
        try:
            got = _run(n, dtype, lossy, steps, (tw, ty, kc))
        except FitError:
            # tiles whose LDS does not fit (FP64, wide tiles) are rejected up front
            continue
        ran += 1
        print(f"pair {dtype} {n} lossy={lossy} tile {tw}x{ty} kc={kc}", flush=True)
        assert got[4]["pair"][1] == steps // 2
        assert torch.equal(got[0], ref[0]), (tw, ty, kc)
        assert torch.equal(got[1], ref[1]), (tw, ty, kc)
        assert got[2] == ref[2] == steps and got[3] == ref[3] == 2 * steps
    assert ran >= (3 if dtype == "f64" else 5)


def test_pairs_around_trace_rows_and_odd_step_counts():
    n = (45, 26, 19)
    for dtype in ("f32", "f64"):
        g1, dt, _, _ = _grid(n, dtype, True)
        g2, _, _, _ = _grid(n, dtype, True)
        g2.set_pair(True)
        for g in (g1, g2):
            g.trace_config(7, 40)
            g.step(31, dt)
            g.step(6, dt)
        assert torch.equal(g1.get_fields()[0], g2.get_fields()[0])
        assert torch.equal(g1.get_fields()[1], g2.get_fields()[1])
        t1, _ = g1.trace_read()
        t2, _ = g2.trace_read()
        # rows recorded by energy pairs: the same per-cell FP64 terms summed
        # over the pair tiling instead of the single-step one
        assert t1.shape == t2.shape and np.array_equal(np.isnan(t1), np.isnan(t2))
        np.testing.assert_allclose(t2, t1, rtol=1e-12, atol=1e-13 * np.nanmax(np.abs(t1)),
                                   equal_nan=True)
        # a probe switches pairs off (the objective needs every step)
        g2.set_probe([2, 2, 2], [10, 10, 10])
        g1.set_probe([2, 2, 2], [10, 10, 10])
        g2.profile_begin(100)
        for g in (g1, g2):
            g.step(8, dt)
        assert g2.profile_end()["pair"][1] == 0
        assert g1.probe_value() == g2.probe_value()
        g1.close()
        g2.close()


def test_pair_matches_oracle_fp64():
    n = (70, 33, 21)
    g, dt, eps, sig = _grid(n, "f64", True)
    g.set_pair(True, 32, 16, 4)
    e0, h0 = (to_np(x) for x in g.get_fields())
    ops = oracle_ops(n, eps=eps, sigma=sig)
    nx, ny, nz = n
    src = dict(axis=2, i=nx // 2, j=ny // 2, k=nz // 2, i_max=1.0, sigma_t=4 * dt)
    g.step(24, dt)
    e, h = g.get_fields()
    eN, hN, _ = run(ops, edges_from_slots(ops, e0), facets_from_slots(ops, h0), dt, 24, src)
    assert rel_l2(edges_from_slots(ops, to_np(e)), eN) <= 1e-12
    assert rel_l2(facets_from_slots(ops, to_np(h)), hN) <= 1e-12
    g.close()


def test_pair_tuning_errors():
    from paper_1705_08019_amd import FitGrid, FitError
    g = FitGrid(16, 16, 16, "f32")
    for bad in ((64, 1, 0), (4, 8, 0), (512, 4, 0), (1024, 2, 0)):
        with pytest.raises(FitError, match="INVALID"):
            g.set_pair(True, *bad)
    with pytest.raises(FitError, match="INVALID"):
        g.set_pair(True, 64, 16, -1)
    g.set_pair(True)
    assert g.get_pair()[:3] == (True, 64, 8)
    g.close()
    g = FitGrid(16, 16, 16, "f64")
    g.set_materials(np.ones(4096), None, np.full(4096, 0.1))
    g.set_pair(True)                       # lossy FP64: 64 x 8 fits (114 KB of LDS)
    assert g.get_pair()[:3] == (True, 64, 8)
    g.close()


def test_autotune_with_pairs_keeps_the_result():
    """The autotuner may switch pairs on; the state it leaves and the steps
    taken afterwards equal plain single fused steps bitwise."""
    n = (96, 80, 64)
    g1, dt, _, _ = _grid(n, "f32", True)
    g2, _, _, _ = _grid(n, "f32", True)
    g2.autotune(dt, reps=2)
    enabled, tw, ty, kc = g2.get_pair()
    assert kc >= 1
    for g in (g1, g2):
        g.step(12, dt)
    assert torch.equal(g1.get_fields()[0], g2.get_fields()[0])
    assert torch.equal(g1.get_fields()[1], g2.get_fields()[1])
    g1.close()
    g2.close()


def test_pairs_stay_off_where_the_fused_step_does_not_run():
    """Pairs enabled on a grid whose permeability then varies per cell (the
    fused kernels take a uniform mu): stepping runs the split kernels only,
    and switching back to uniform mu runs pairs again."""
    from paper_1705_08019_amd import FitGrid
    n = (30, 20, 10)
    g = FitGrid(*n, "f64")
    g.set_materials(np.ones(6000), None, np.full(6000, 0.1))
    g.set_pair(True, 64, 8, 0)
    g.set_materials(np.ones(6000), np.random.default_rng(2).uniform(1, 2, 6000),
                    np.full(6000, 0.1))
    g.set_fields(np.random.default_rng(1).standard_normal((3, 10, 20, 30)), None, 0)
    dt = 0.9 * g.cfl_dt()
    g.profile_begin(40)
    g.step(6, dt)
    prof = g.profile_end()
    assert prof["pair"][1] == 0 and prof["step"][1] == 0 and prof["epass"][1] == 6
    g.set_materials(np.ones(6000), None, np.full(6000, 0.1))
    g.set_tuning("fused")
    g.profile_begin(40)
    g.step(6, dt)
    assert g.profile_end()["pair"][1] == 3
    g.close()


def _graded(n, dtype, lossy, seed=11):
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    wd = [rng.uniform(0.3, 1.7, k) for k in n]
    eps = dielectric_blocks(nx, ny, nz, 5, seed)
    sig = lossy_slab(nx, ny, nz, 1, 0.2) if lossy else None
    mu = np.full((nz, ny, nx), 1.3)
    g = FitGrid(nx, ny, nz, dtype, spacing=wd)
    g.set_materials(eps, mu, sig)
    g.set_fields(rng.standard_normal((3, nz, ny, nx)), rng.standard_normal((3, nz, ny, nx)), 0)
    dt = 0.9 * g.cfl_dt()
    g.set_source(2, nx // 2, ny // 2, nz // 2, 1.0, 4 * dt)
    g.set_tuning("fused")
    return g, dt, (wd, eps, mu, sig)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,lossy", [((70, 33, 21), True), ((13, 9, 7), False),
                                     ((40, 40, 1), False), ((9, 70, 2), True)])
def test_graded_pair_is_bitwise_two_single_steps(dtype, n, lossy):
    """Tensor grids: the pair kernel uses the single fused step's per-axis
    metric factors in the same arithmetic, chunk boundaries included."""
    from paper_1705_08019_amd import FitError
    steps = 10
    g, dt, _ = _graded(n, dtype, lossy)
    g.profile_begin(4 * steps + 8)
    g.step(steps, dt)
    assert g.profile_end()["pair"][1] == 0
    ref = [x.clone() for x in g.get_fields()]
    g.close()
    ran = 0
    for tw, ty, kc in [(32, 16, 0), (64, 8, 1), (32, 8, 2), (16, 8, 5), (48, 10, 3), (64, 16, 2),
                       (40, 24, 0)]:
        g, _, _ = _graded(n, dtype, lossy)
        try:
            g.set_pair(True, tw, ty, kc)
        except FitError:
            g.close()
            continue
        print(f"graded pair {dtype} {n} lossy={lossy} tile {tw}x{ty} kc={kc}", flush=True)
        g.profile_begin(4 * steps + 8)
        g.step(steps, dt)
        prof = g.profile_end()
        e, h = g.get_fields()
        assert prof["pair"][1] == steps // 2, (tw, ty, kc)
        assert torch.equal(e, ref[0]), (tw, ty, kc)
        assert torch.equal(h, ref[1]), (tw, ty, kc)
        g.close()
        ran += 1
    assert ran >= 3


def test_graded_pair_matches_oracle_fp64():
    n = (37, 22, 15)
    g, dt, (wd, eps, mu, sig) = _graded(n, "f64", True)
    g.set_pair(True, 32, 16, 4)
    e0, h0 = (to_np(x) for x in g.get_fields())
    ops = oracle_ops(n, eps=eps, sigma=sig, mu=mu, spacing=wd)
    nx, ny, nz = n
    src = dict(axis=2, i=nx // 2, j=ny // 2, k=nz // 2, i_max=1.0, sigma_t=4 * dt)
    g.profile_begin(40)
    g.step(20, dt)
    assert g.profile_end()["pair"][1] == 10
    e, h = g.get_fields()
    eN, hN, _ = run(ops, edges_from_slots(ops, e0), facets_from_slots(ops, h0), dt, 20, src)
    assert rel_l2(edges_from_slots(ops, to_np(e)), eN) <= 1e-12
    assert rel_l2(facets_from_slots(ops, to_np(h)), hN) <= 1e-12
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,lossy", [((45, 26, 19), True), ((40, 40, 1), False), ((9, 70, 2), True),
                                     ((5, 4, 3), False)])
def test_energy_pairs_record_the_rows(dtype, n, lossy):
    """A trace row whose step is the second of a pair is recorded by the pair
    (its pending h cross term by the pair's first step): the rows equal those
    of single fused steps to the summation order, the fields bitwise; rows
    past the trace's capacity are counted as dropped as on the single path;
    also on one- and two-plane grids and a grid smaller than one tile."""
    g1, dt, _, _ = _grid(n, dtype, lossy)
    g2, _, _, _ = _grid(n, dtype, lossy)
    g2.set_pair(True, 32, 16, 6)
    for g in (g1, g2):
        g.trace_config(10, 4)                   # rows at 0, 10, 20, 30; 40 and 50 dropped
    g2.profile_begin(200)
    for g in (g1, g2):
        g.step(55, dt)
    prof = g2.profile_end()
    # 0 single, then pairs (1, 2) .. (9, 10) with the row, ...: 27 pairs, 3 of
    # them recording rows 10, 20, 30 (40 and 50 do not fit), 1 single step
    assert prof["pair"][1] == 24 and prof["pair_energy"][1] == 3 and prof["step"][1] == 1, prof
    for a, b in zip(g1.get_fields(), g2.get_fields()):
        assert torch.equal(a, b)
    t1, d1 = g1.trace_read()
    t2, d2 = g2.trace_read()
    assert t1.shape == t2.shape == (4, 10) and d1 == d2 == 2
    assert np.array_equal(t1[:, 0], t2[:, 0]) and np.array_equal(np.isnan(t1), np.isnan(t2))
    np.testing.assert_allclose(t2, t1, rtol=1e-12, atol=1e-13 * np.nanmax(np.abs(t1)),
                               equal_nan=True)
    print(f"energy pairs {dtype} {n}: max rel row diff "
          f"{np.nanmax(np.abs(t2 - t1) / np.maximum(np.abs(t1), 1e-300)):.1e}", flush=True)
    g1.close()
    g2.close()


@pytest.mark.parametrize("n", [(256, 256, 160), (252, 256, 160), (128, 128, 128)])
def test_pairs_with_either_store_kind_equal_single_steps(n):
    """The pair launches write their outputs with streaming stores where rows
    and tiles are whole 128-byte lines and the state exceeds the 256 MiB
    Infinity Cache (256 x 256 x 160 FP32: 587 MB), with ordinary stores
    elsewhere (252-cell rows; the cache-resident 128^3): bitwise equal to
    single fused steps either way, across a ragged last z-chunk."""
    print(f"pairs vs single, store rule case {n}", flush=True)
    e1, h1, m1, _, prof = _run(n, "f32", True, 10, pair=(64, 8, 128))
    assert prof["pair"][1] == 5, prof
    e2, h2, m2, _, _ = _run(n, "f32", True, 10)
    assert m1 == m2 == 10
    assert torch.equal(e1, e2) and torch.equal(h1, h2)
