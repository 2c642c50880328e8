"""Batched step pairs (two steps of every grid per launch, 32 x 16 tiles):
every grid equals its plain single-grid run bitwise through direct launches,
graph replays of pairs, odd step counts (a last single step), z-chunked
items and mixed lossy / lossless grids, in FP32 and FP64."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import c4, c4_small
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
