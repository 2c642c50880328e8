"""The persistent batched launch (S steps of every grid per cooperative
launch, grid-wide barrier between the steps, captured in a hipGraph), with
single steps and with step pairs (S / 2 pairs per launch, the pair item
table walked per XCD): every grid equals its plain single-grid run bitwise,
through graph replays, a direct launch of the remainder, a direct launch of
a whole call and an odd last step, for FP32 and FP64, mixed lossy /
lossless grids; no barrier gives up; and the batch against the oracle
(Sec. III, Alg. 1: independent leapfrog runs)."""
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
def test_persistent_equals_plain(dtype):
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=7, nsteps=0)
    gb, dts = _make(specs, dtype, lossy_every=3)
    gp, _ = _make(specs, dtype, lossy_every=3)
    b = FitBatch(gb)
    b.set_tuning(0, 0, 16)                      # 16 steps per persistent launch
    b.set_persistent(True)
    on, nwg, cap, failed = b.get_persistent()
    print(f"persistent {dtype}: {nwg} workgroups, captured {cap}", flush=True)
    assert on and nwg >= 1 and not failed
    b.step(50, dts)                             # 3 graph replays + a 2-step launch
    _plain(gp, dts, 50)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    print(f"persistent {dtype}: direct", flush=True)
    b.step(23, dts, use_graph=False)            # one launch of 23 steps
    _plain(gp, dts, 23)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    b.set_persistent(False)
    b.step(3, dts)
    _plain(gp, dts, 3)
    _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 76 for g in gb)
    b.close()


def test_persistent_c4_grids_with_several_items_per_workgroup():
    """The 64-grid workload's sizes (32-96 cells per axis): more items than
    resident workgroups, so every workgroup runs several tiles per step."""
    from paper_1705_08019_amd import FitBatch
    specs = c4()[:24]
    gb, dts = _make(specs, "f32")
    gp, _ = _make(specs, "f32")
    b = FitBatch(gb)
    b.set_tuning(0, 0, 8)
    b.set_persistent(True)
    on, nwg, cap, _ = b.get_persistent()
    ty, kc, spg, items, tw = b.get_tuning()
    print(f"persistent c4 x24: {items} items on {nwg} workgroups, captured {cap}", flush=True)
    b.step(37, dts)
    _plain(gp, dts, 37)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_persistent_pairs_equal_plain(dtype):
    from paper_1705_08019_amd import FitBatch
    specs = c4_small(count=7, nsteps=0)
    gb, dts = _make(specs, dtype, lossy_every=3)
    gp, _ = _make(specs, dtype, lossy_every=3)
    b = FitBatch(gb)
    b.set_tuning(0, 0, 16)                      # 8 pairs per persistent launch
    b.set_pair(True, 0)
    b.set_persistent(True)
    on, nwg, cap, failed = b.get_persistent()
    print(f"persistent pairs {dtype}: {nwg} workgroups, captured {cap}", flush=True)
    assert on and nwg >= 8 and nwg % 8 == 0 and not failed
    b.step(50, dts)                             # 3 graph replays + a 1-pair launch
    _plain(gp, dts, 50)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    print(f"persistent pairs {dtype}: direct, odd", flush=True)
    b.step(23, dts, use_graph=False)            # one launch of 11 pairs, one single step
    _plain(gp, dts, 23)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    print(f"persistent pairs {dtype}: z-chunks", flush=True)
    b.set_pair(True, 3)                         # items of 3 planes (chunk seams)
    b.step(9, dts)
    _plain(gp, dts, 9)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    b.set_persistent(False)
    b.step(3, dts)
    _plain(gp, dts, 3)
    _assert_equal(_fields(gb), _fields(gp))
    assert all(g.step_index == 85 for g in gb)
    b.close()


def test_persistent_pairs_c4_grids_with_several_items_per_workgroup():
    """Pairs of the 64-grid workload's sizes in 8-plane chunks: more pair
    items than resident workgroups, so each workgroup walks several tiles of
    its XCD's list per pair."""
    from paper_1705_08019_amd import FitBatch
    specs = c4()[:24]
    gb, dts = _make(specs, "f32")
    gp, _ = _make(specs, "f32")
    b = FitBatch(gb)
    b.set_tuning(0, 0, 8)                       # 4 pairs per launch
    b.set_pair(True, 8)
    b.set_persistent(True)
    on, nwg, cap, _ = b.get_persistent()
    print(f"persistent pairs c4 x24: {nwg} workgroups, captured {cap}", flush=True)
    b.step(37, dts)
    _plain(gp, dts, 37)
    assert not b.get_persistent()[3]
    _assert_equal(_fields(gb), _fields(gp))
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("pairs", [False, True])
def test_persistent_matches_oracle(dtype, pairs):
    from paper_1705_08019_amd import FitBatch
    from oracle.leapfrog import run
    from _glue import oracle_ops, to_np, edges_from_slots, facets_from_slots, state_errors
    specs = c4_small(count=4, nsteps=0)
    gb, dts = _make(specs, dtype, lossy_every=2)
    b = FitBatch(gb)
    b.set_tuning(0, 0, 16)
    if pairs:
        b.set_pair(True, 4)
    b.set_persistent(True)
    n = 101
    b.step(n, dts)
    assert not b.get_persistent()[3]
    for k, (s, g, dt) in enumerate(zip(specs, gb, dts)):
        sig = lossy_slab(s.nx, s.ny, s.nz, 2, 0.05) if k % 2 == 0 else None
        ops = oracle_ops((s.nx, s.ny, s.nz), eps=s.eps_r, sigma=sig)
        src = dict(s.source)
        src["sigma_t"] = src.pop("sigma_t_steps") * dt
        e_r, h_r, _ = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), g.step_dt(dt), n, source=src)
        e, h = g.get_fields()
        err = state_errors(ops, edges_from_slots(ops, to_np(e)), facets_from_slots(ops, to_np(h)),
                           e_r, h_r)
        print(f"  grid {k}: " + " ".join(f"{a} {v:.2e}" for a, v in err.items()), flush=True)
        if dtype == "f64":
            assert err["e_own"] <= 1e-12 and err["h_own"] <= 1e-12
        else:
            assert err["e_state"] <= 1e-4 and err["h_state"] <= 1e-4
    b.close()
