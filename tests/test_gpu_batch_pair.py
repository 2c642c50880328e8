"""Batched step pairs (two steps of every grid per launch, per-grid tiles):
every grid equals its plain single-grid run bitwise through direct launches,
graph replays of pairs, odd step counts (a last single step), z-chunked
items and mixed lossy / lossless grids, in FP32 and FP64."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import c4, c4_small, lossy_slab
from test_gpu_batch_step import _make, _fields, _assert_equal

pytestmark = pytest.mark.gpu


def _plain(grids, dts, n):
    for g, dt in zip(grids, dts):
        g.step(n, dt)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("which", ["small", "multi-tile"])
def test_batch_pairs_equal_plain(dtype, which):
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=7, nsteps=0) if which == "small" else c4()[:5]
    gb, dts = _make(specs, dtype, lossy_every=3)
    gp, _ = _make(specs, dtype, lossy_every=3)
    b = FitBatch(gb)
    b.set_pair(True, 0)
    assert b.get_pair() == (True, 0)
    print(f"batch pairs {dtype} {which}: direct", flush=True)
    b.step(50, dts, use_graph=False)            # 25 pair launches
    _plain(gp, dts, 50)
    _assert_equal(_fields(gb), _fields(gp))
    print(f"batch pairs {dtype} {which}: graph", flush=True)
    b.set_tuning(0, 0, 16)                      # 8 pairs per captured chunk
    b.step(37, dts)                             # 2 replays, 2 direct pairs, 1 single step
    _plain(gp, dts, 37)
    _assert_equal(_fields(gb), _fields(gp))
    print(f"batch pairs {dtype} {which}: z-chunks", flush=True)
    b.set_pair(True, 5)                         # items of 5 planes (chunk seams)
    b.step(23, dts, use_graph=False)
    _plain(gp, dts, 23)
    _assert_equal(_fields(gb), _fields(gp))
    b.set_pair(False)
    b.step(3, dts)
    _plain(gp, dts, 3)
    _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 113 for g in gb)
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_pair_tiles_per_grid(dtype):
    """Each grid takes its own pair tile shape (the one staging the fewest
    points for its x / y extent) and z-chunks of even length; the batch of
    mixed shapes, its items laid out over the XCDs, stays bitwise equal to plain
    per-grid steps through graph chunks (per-launch offsets, one counter
    advance per chunk), direct launches and a last single step."""
    import math
    from paper_1705_08019_amd import FitBatch, FitError
    specs = c4()[:12]
    gb, dts = _make(specs, dtype, lossy_every=4)
    gp, _ = _make(specs, dtype, lossy_every=4)
    b = FitBatch(gb)
    with pytest.raises(FitError, match="STATE"):
        b.get_pair_tile(0)                      # pairs are off
    b.set_pair(True, 24)
    shapes = set()
    for n, s in enumerate(specs):
        tw, ty, kc = b.get_pair_tile(n)
        shapes.add((tw, ty))
        nch = math.ceil(s.nz / 24)
        assert kc == math.ceil(s.nz / nch) and kc <= 24, (n, s.nz, kc)
    with pytest.raises(FitError, match="INVALID"):
        b.get_pair_tile(len(specs))
    print(f"pair tiles {dtype}: {sorted(shapes)}", flush=True)
    assert len(shapes) >= 2
    assert shapes <= {(32, 16), (32, 18), (40, 14), (24, 24)}
    b.set_tuning(0, 0, 8)                       # 4 pairs per captured chunk
    b.step(21, dts)                             # 2 replays, 2 direct pairs, 1 single step
    _plain(gp, dts, 21)
    _assert_equal(_fields(gb), _fields(gp))
    b.set_pair(True, 0)                         # whole columns
    b.step(18, dts, use_graph=False)
    _plain(gp, dts, 18)
    _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 39 for g in gb)
    b.close()


def _specs(sizes, seed):
    from fit_workloads.configs import WorkloadSpec, dielectric_blocks, random_source
    rng = np.random.default_rng(seed)
    return [WorkloadSpec(name=f"xcd{n}", nx=nx, ny=ny, nz=nz, dtype="f32", nsteps=0,
                         eps_r=dielectric_blocks(nx, ny, nz, 4, seed + n), sigma=None,
                         source=random_source(nx, ny, nz, rng))
            for n, (nx, ny, nz) in enumerate(sizes)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", ["one-grid", "one-tile", "uneven"])
def test_batch_pair_xcd_table_edge_cases(dtype, case):
    """The pair item table is dealt over the 8 XCDs in groups (the tiles of
    one z-chunk of one grid), cut into runs when a group exceeds a 32nd of
    the work, and padded with empty entries: a single multi-tile grid (one
    group per chunk, cut into runs), a single one-tile grid (one item, seven
    empty entries) and a large grid beside a tiny one all stay bitwise equal
    to plain per-grid steps, with whole columns and short chunks."""
    from paper_1705_08019_amd import FitBatch
    sizes = {"one-grid": [(70, 50, 30)], "one-tile": [(10, 9, 8)],
             "uneven": [(96, 80, 40), (7, 6, 5)]}[case]
    specs = _specs(sizes, 300)
    gb, dts = _make(specs, dtype, lossy_every=2)
    gp, _ = _make(specs, dtype, lossy_every=2)
    b = FitBatch(gb)
    for kc, n in ((0, 9), (7, 10), (3, 8)):
        b.set_pair(True, kc)
        print(f"xcd table {case} {dtype}: kc {kc}", flush=True)
        b.step(n, dts, use_graph=(kc == 7))
        _plain(gp, dts, n)
        _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 27 for g in gb)
    b.close()


def test_batch_pair_errors_and_autotune():
    from paper_1705_08019_amd import FitBatch, FitError
    specs = c4_small(count=4, nsteps=0)
    gb, dts = _make(specs, "f32")
    b = FitBatch(gb)
    with pytest.raises(FitError, match="INVALID"):
        b.set_pair(True, -1)
    assert b.get_pair() == (False, 0)
    b.step(10, dts)
    before = _fields(gb)
    ty, kc, ms, tw = b.autotune(dts, reps=2)    # may switch pairs on; the state is unchanged
    assert ms > 0
    _assert_equal(_fields(gb), before)
    assert all(g.step_index == 10 for g in gb)
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_zero_steps_change_nothing(dtype):
    """A step count of 0 is a valid empty call (fields, step index and SMVP count
    unchanged) for one grid and for a batch; a negative count is rejected and
    leaves the state as it was."""
    from paper_1705_08019_amd import FitBatch, FitError
    specs = c4_small(count=3, nsteps=0)
    gb, dts = _make(specs, dtype, lossy_every=2)
    b = FitBatch(gb)
    b.set_pair(True, 0)
    b.step(3, dts)
    before = _fields(gb)
    idx = [g.step_index for g in gb]
    smvp = [g.smvp_count() for g in gb]
    for n in (0, -1):
        if n < 0:
            with pytest.raises(FitError, match="INVALID"):
                b.step(n, dts)
            with pytest.raises(FitError, match="INVALID"):
                gb[0].step(n, dts[0])
        else:
            b.step(n, dts)
            b.step(n, dts, use_graph=False)
            gb[1].step(n, dts[1])
        _assert_equal(_fields(gb), before)
        assert [g.step_index for g in gb] == idx
        assert [g.smvp_count() for g in gb] == smvp
    b.step(2, dts)                                # still usable afterwards
    assert [g.step_index for g in gb] == [i + 2 for i in idx]
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("which", ["small", "c4"])
def test_batch_pairs_match_oracle(dtype, which):
    """Each grid of a batch advanced by graph-captured pair launches (Sec. III,
    Alg. 1: the p particular solutions are independent leapfrog runs) equals
    the oracle's leapfrog run of that grid: FP64 relative L2 <= 1e-12, FP32
    <= 1e-4, after >= 100 steps (odd count: a last single step)."""
    from paper_1705_08019_amd import FitBatch
    from oracle.leapfrog import run
    from _glue import oracle_ops, to_np, edges_from_slots, facets_from_slots, state_errors
    specs = c4_small(count=6, nsteps=0) if which == "small" else c4()[:3]
    gb, dts = _make(specs, dtype, lossy_every=3)
    b = FitBatch(gb)
    b.set_pair(True, 8)
    b.set_tuning(0, 0, 16)
    n = 121 if which == "small" else 101
    print(f"batch pairs vs oracle {dtype} {which}: {n} steps", flush=True)
    b.step(n, dts)
    tol = 1e-12 if dtype == "f64" else 1e-4
    for k, (s, g, dt) in enumerate(zip(specs, gb, dts)):
        sig = lossy_slab(s.nx, s.ny, s.nz, 2, 0.05) if k % 3 == 0 else None
        ops = oracle_ops((s.nx, s.ny, s.nz), eps=s.eps_r, sigma=sig)
        src = dict(s.source)
        src["sigma_t"] = src.pop("sigma_t_steps") * dt      # as _make set it
        step = g.step_dt(dt)                                # the step the grid took
        e_r, h_r, _ = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), step, n, source=src)
        e, h = g.get_fields()
        err = state_errors(ops, edges_from_slots(ops, to_np(e)), facets_from_slots(ops, to_np(h)),
                           e_r, h_r)
        print(f"  grid {k} {s.nx}x{s.ny}x{s.nz}: " +
              " ".join(f"{a} {b:.2e}" for a, b in err.items()), flush=True)
        if dtype == "f64":
            assert err["e_own"] <= tol and err["h_own"] <= tol, (k, err)
        else:   # FP32: each field in the energy norm of the state (see test_gpu_horizon)
            assert err["e_state"] <= tol and err["h_state"] <= tol and err["e_own"] <= tol, (k, err)
    b.close()


def test_batch_follows_a_grid_that_becomes_lossy():
    """A batch laid out for lossless grids, one of which is then given a
    conductivity, re-lays itself out for the lossy tile body (its LDS holds
    the sigma planes) and still equals the plain runs bitwise; a grid that
    gets a non-uniform mu is rejected."""
    from paper_1705_08019_amd import FitBatch, FitError
    specs = c4_small(count=5, nsteps=0)
    gb, dts = _make(specs, "f32")
    gp, _ = _make(specs, "f32")
    b = FitBatch(gb)
    b.set_pair(True, 0)
    b.step(10, dts)
    _plain(gp, dts, 10)
    s = specs[2]
    sig = lossy_slab(s.nx, s.ny, s.nz, 2, 0.1)
    for g in (gb[2], gp[2]):
        g.set_materials(s.eps_r, None, sig)
    b.step(31, dts)
    _plain(gp, dts, 31)
    _assert_equal(_fields(gb), _fields(gp))
    gb[1].set_materials(specs[1].eps_r, np.full(specs[1].eps_r.shape, 2.0) +
                        (np.arange(specs[1].eps_r.size) % 2).reshape(specs[1].eps_r.shape))
    with pytest.raises(FitError, match="STATE"):
        b.step(2, dts)
    b.close()
