"""Tests written for the persistent work-queue form of the batched leapfrog
(one launch for S steps of all grids, per-grid completion counters).

That form's first GPU run produced no output for 180 s and was killed, and
the single run that tested a fix (bounded waits with a launch-wide abort)
did the same; its cause was not identified, so the persistent kernel was
taken out of the library.  These tests stay, skipped; the batched path that
replaced it (one launch per step of all grids) is tested in
test_gpu_batch_step.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import c4, c4_small, lossy_slab

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="persistent work-queue batch kernel removed after two "
                                      "unexplained GPU hangs; see test_gpu_batch_step.py")]


def _make(specs, dtype, lossy_every=0):
    from paper_1705_08019_amd import FitGrid
    grids, dts = [], []
    rng = np.random.default_rng(7)
    for n, s in enumerate(specs):
        g = FitGrid(s.nx, s.ny, s.nz, dtype)
        sig = lossy_slab(s.nx, s.ny, s.nz, 2, 0.05) if (lossy_every and n % lossy_every == 0) else None
        g.set_materials(s.eps_r, None, sig)
        dt = 0.9 * g.cfl_dt() * float(rng.uniform(0.8, 1.0))
        src = s.source
        g.set_source(src["axis"], src["i"], src["j"], src["k"], src["i_max"],
                     src["sigma_t_steps"] * dt)
        grids.append(g)
        dts.append(dt)
    return grids, np.array(dts)


def _fields(grids):
    return [g.get_fields() for g in grids]


def _assert_equal(fa, fb):
    for n, (a, b) in enumerate(zip(fa, fb)):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), f"grid {n} differs"


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_equals_plain(dtype):
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=7, nsteps=0)
    gb, dts = _make(specs, dtype, lossy_every=3)
    gp, _ = _make(specs, dtype, lossy_every=3)
    b = FitBatch(gb)
    b.set_tuning(0, 0, 16)
    b.step(200, dts)                        # 12 graph replays + an 8-step direct launch
    for g, dt in zip(gp, dts):
        g.step(200, dt)
    _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 200 for g in gb)
    # direct launches give the same, and tiles split in z too
    b.set_tuning(4 if dtype == "f32" else 2, 5, 0)
    b.step(37, dts, use_graph=False)
    for g, dt in zip(gp, dts):
        g.step(37, dt)
    _assert_equal(_fields(gb), _fields(gp))
    b.close()


def test_graph_replays_interleaved_with_eager_work():
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=5, nsteps=0)
    gb, dts = _make(specs, "f32")
    gp, _ = _make(specs, "f32")
    b = FitBatch(gb)
    b.set_tuning(0, 0, 8)
    for rep in range(4):
        b.step(8, dts)                      # exactly one replay of the captured graph
        for g, dt in zip(gp, dts):
            g.step(8, dt)
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        _assert_equal(_fields(gb), _fields(gp))
        assert float(junk) == float(junk)
    b.close()


def test_batch_autotune_keeps_state():
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=4, nsteps=0)
    gb, dts = _make(specs, "f32")
    b = FitBatch(gb)
    b.step(10, dts)
    before = _fields(gb)
    ty, kc, ms, tw = b.autotune(dts, reps=2)
    assert ms > 0 and b.get_tuning()[:2] == (ty, kc) and b.get_tuning()[4] == tw
    _assert_equal(_fields(gb), before)
    assert all(g.step_index == 10 for g in gb)
    b.close()


def test_batch_full_workload_equals_plain():
    """64 grids of 32..96 cells per axis, 4000 steps (the batched workload),
    graph replays of 16 steps: every grid equals its plain single-grid run."""
    from paper_1705_08019_amd import FitBatch
    specs = c4()
    gb, dts = _make(specs, "f32")
    b = FitBatch(gb)
    b.autotune(dts, reps=2)
    b.step(specs[0].nsteps, dts)
    fb = _fields(gb)
    b.close()
    for g in gb:
        g.close()
    gp, _ = _make(specs, "f32")
    for g, dt in zip(gp, dts):
        g.step(specs[0].nsteps, dt)
    _assert_equal(fb, _fields(gp))
