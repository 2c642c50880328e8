"""Full-size parity on the 256 x 256 x 512 bandwidth workload, in the launch
configuration the benchmark times.

The oracle cannot hold the whole grid, so one GPU step is checked on sampled
6 x 6 x 6-cell windows: the oracle, built for the window alone, advances the
window's state by one step; every e on a window-interior edge, and every h on
a facet whose boundary edges are all window-interior, depends only on data
inside the window and must match.  Along the run, the discrete energy balance
Q^(m+1) - Q^m = -2 dt (ebar M_sigma ebar + ebar j_s) is checked on the GPU's
own FP64 trace (a property that holds at any size).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import c3
from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators, run
from oracle import layout

pytestmark = pytest.mark.gpu


def _window_check(spec, e0, h0, e1, h1, dt, src, origin, step0, w=6):
    i0, j0, k0 = origin
    sl = (slice(None), slice(k0, k0 + w), slice(j0, j0 + w), slice(i0, i0 + w))
    t = Topology(w, w, w)
    eps = spec.eps_r[sl[1:]]
    sig = None if spec.sigma is None else spec.sigma[sl[1:]]
    ops = Operators(t, Materials(t, eps, sigma=sig))
    ew0 = layout.edges_from_slots(ops, e0[sl].astype(np.float64))
    hw0 = layout.facets_from_slots(ops, h0[sl].astype(np.float64))
    lsrc = None
    si, sj, sk = src["i"] - i0, src["j"] - j0, src["k"] - k0
    if 0 < si < w and 0 < sj < w and 0 <= sk < w:
        lsrc = dict(src, i=si, j=sj, k=sk)
    ew1, hw1, _ = run(ops, ew0, hw0, dt, 1, source=lsrc, step0=step0)
    eg = layout.edges_from_slots(ops, e1[sl].astype(np.float64))
    hg = layout.facets_from_slots(ops, h1[sl].astype(np.float64))
    # facets whose four boundary edges are all window-interior
    Cfull = t.curl()[ops.if_]
    kept = t.interior_edges()
    ok = np.array([kept[Cfull.indices[Cfull.indptr[r]:Cfull.indptr[r + 1]]].all()
                   for r in range(Cfull.shape[0])])
    # scale of the terms entering each update: FP32 rounding of the inputs
    # perturbs e^(m+1) by ~eps32 * (|e| + dt |C~ h| / M_eps) and h^(m+3/2) by
    # ~eps32 * (|h| + dt |C e| / M_mu); bound |C x| by 4 max |x|.
    se = max(np.max(np.abs(ew1)), np.max(np.abs(ew0)), 4 * dt * np.max(np.abs(hw0)), 1e-30)
    sh = max(np.max(np.abs(hw1[ok])), np.max(np.abs(hw0)), 4 * dt * np.max(np.abs(ew1)), 1e-30)
    de = np.max(np.abs(eg - ew1)) / se
    dh = np.max(np.abs(hg[ok] - hw1[ok])) / sh
    return de, dh, lsrc is not None


def test_c3_fullsize_sampled_windows_and_balance():
    from paper_1705_08019_amd import FitGrid
    spec = c3()
    g = FitGrid(spec.nx, spec.ny, spec.nz, "f32")
    g.set_materials(spec.eps_r, spec.mu_r, spec.sigma)
    dt = spec.cfl_frac * g.cfl_dt()
    s = spec.source
    src = dict(axis=2, i=s["i"], j=s["j"], k=s["k"], i_max=s["i_max"],
               sigma_t=s["sigma_t_steps"] * dt)
    g.set_source(2, s["i"], s["j"], s["k"], s["i_max"], src["sigma_t"])
    g.trace_config(spec.energy_every, 64)
    g.step(15, dt)
    e_a, h_a = (x.cpu().numpy() for x in g.get_fields())     # source still active here
    g.step(1, dt)
    e_b, h_b = (x.cpu().numpy() for x in g.get_fields())
    g.step(134, dt)
    tr, _ = g.trace_read()
    assert tr.shape[0] == 3
    for row in tr[1:]:
        Qm, Qm1 = row[1] + row[4], row[3] + row[6]
        assert abs((Qm1 - Qm) + 2 * dt * (row[8] + row[9])) <= 1e-5 * abs(Qm1)
    e0, h0 = (x.cpu().numpy() for x in g.get_fields())
    g.step(1, dt)
    e1, h1 = (x.cpu().numpy() for x in g.get_fields())
    rng = np.random.default_rng(2024)
    origins = [(s["i"] - 3, s["j"] - 3, s["k"] - 3)]          # the source window
    # inside the region the pulse has reached after 150 steps (|x - src| < ~50 cells)
    origins += [(int(rng.integers(s["i"] - 50, s["i"] + 45)),
                 int(rng.integers(s["j"] - 50, s["j"] + 45)),
                 int(rng.integers(s["k"] - 50, s["k"] + 45))) for _ in range(24)]
    # windows touching the walls and the tile / chunk seams
    origins += [(0, 0, 0), (spec.nx - 6, spec.ny - 6, spec.nz - 6), (61, 2, 61), (125, 61, 317)]
    for o in origins:
        de, dh, _ = _window_check(spec, e0, h0, e1, h1, dt, src, o, 150)
        assert de <= 1e-5 and dh <= 1e-5, (o, de, dh)
    # the source window while the current is near its peak (global step 15)
    de, dh, has_src = _window_check(spec, e_a, h_a, e_b, h_b, dt, src, origins[0], 15)
    assert has_src and de <= 1e-5 and dh <= 1e-5, (de, dh)
    g.close()


def _window_check_steps(spec, e0, h0, e2, h2, dt, src, origin, step0, steps, w=10, margin=3):
    """`steps` steps of a w^3 window by the oracle against the GPU's full-grid
    result on the slots `margin` cells inside the window (the window's PEC
    boundary reaches one cell further per step)."""
    i0, j0, k0 = origin
    sl = (slice(None), slice(k0, k0 + w), slice(j0, j0 + w), slice(i0, i0 + w))
    t = Topology(w, w, w)
    eps = spec.eps_r[sl[1:]]
    sig = None if spec.sigma is None else spec.sigma[sl[1:]]
    ops = Operators(t, Materials(t, eps, sigma=sig))
    ew0 = layout.edges_from_slots(ops, e0[sl].astype(np.float64))
    hw0 = layout.facets_from_slots(ops, h0[sl].astype(np.float64))
    lsrc = None
    si, sj, sk = src["i"] - i0, src["j"] - j0, src["k"] - k0
    if 0 < si < w and 0 < sj < w and 0 <= sk < w:
        lsrc = dict(src, i=si, j=sj, k=sk)
    ewN, hwN, _ = run(ops, ew0, hw0, dt, steps, source=lsrc, step0=step0)
    inner = (slice(None),) + (slice(margin, w - margin),) * 3
    eo = layout.edges_to_slots(ops, ewN)[inner]
    ho = layout.facets_to_slots(ops, hwN)[inner]
    eg = e2[sl].astype(np.float64)[inner]
    hg = h2[sl].astype(np.float64)[inner]
    se = max(np.max(np.abs(eo)), np.max(np.abs(ew0)), 4 * dt * np.max(np.abs(hw0)), 1e-30)
    sh = max(np.max(np.abs(ho)), np.max(np.abs(hw0)), 4 * dt * np.max(np.abs(ewN)), 1e-30)
    return np.max(np.abs(eg - eo)) / se, np.max(np.abs(hg - ho)) / sh


@pytest.mark.parametrize("pair", [(64, 8, 128), (32, 16, 64)])
def test_c3_fullsize_step_pairs_in_the_benchmark_configuration(pair):
    """The benchmark's launch configuration: two steps per launch on 64 x 8
    tiles with 128-plane chunks (the autotuner's choice on this grid; also
    32 x 16 with 64-plane chunks), single steps on 128 x 8 tiles around the
    trace rows every 50 steps.  47 steps bitwise equal to single fused steps;
    then one pair on sampled 10^3 windows against the oracle."""
    from paper_1705_08019_amd import FitGrid
    spec = c3()

    def make(on):
        g = FitGrid(spec.nx, spec.ny, spec.nz, "f32")
        g.set_materials(spec.eps_r, spec.mu_r, spec.sigma)
        g.set_tuning("fused", 8, 128, 128)
        if on:
            g.set_pair(True, *pair)
        g.trace_config(spec.energy_every, 64)
        return g

    g1, g2 = make(True), make(False)
    dt = spec.cfl_frac * g1.cfl_dt()
    s = spec.source
    src = dict(axis=2, i=s["i"], j=s["j"], k=s["k"], i_max=s["i_max"],
               sigma_t=s["sigma_t_steps"] * dt)
    for g in (g1, g2):
        g.set_source(2, s["i"], s["j"], s["k"], s["i_max"], src["sigma_t"])
    print(f"c3 full size: 47 steps, pairs {pair} vs single", flush=True)
    g1.profile_begin(200)
    g1.step(47, dt)
    assert g1.profile_end()["pair"][1] >= 22
    g2.step(47, dt)
    for a, b in zip(g1.get_fields(), g2.get_fields()):
        assert torch.equal(a, b)
    assert np.array_equal(g1.trace_read()[0], g2.trace_read()[0], equal_nan=True)
    g2.close()
    e0, h0 = (x.cpu().numpy() for x in g1.get_fields())
    g1.profile_begin(8)
    g1.step(2, dt)
    assert g1.profile_end()["pair"][1] == 1
    e2, h2 = (x.cpu().numpy() for x in g1.get_fields())
    rng = np.random.default_rng(7)
    origins = [(s["i"] - 5, s["j"] - 5, s["k"] - 5)]
    origins += [(int(rng.integers(s["i"] - 40, s["i"] + 30)),
                 int(rng.integers(s["j"] - 40, s["j"] + 30)),
                 int(rng.integers(s["k"] - 40, s["k"] + 30))) for _ in range(16)]
    # walls, and windows across tile seams (x 32 / 64, y 8 / 16) and chunk
    # seams (z 64 / 128)
    origins += [(0, 0, 0), (spec.nx - 10, spec.ny - 10, spec.nz - 10), (27, 11, 59),
                (123, 43, 187), (59, 5, 123)]
    print("c3 full size: pair windows vs oracle", flush=True)
    for o in origins:
        de, dh = _window_check_steps(spec, e0, h0, e2, h2, dt, src, o, 47, 2)
        assert de <= 1e-5 and dh <= 1e-5, (o, de, dh)
    g1.close()


def test_c3_fullsize_energy_pair_records_the_row():
    """The benchmark's launch configuration across a trace row: the row at
    step 50 is recorded by the pair (49, 50) -> 51 (its FP64 energy sums in
    the pair kernel's energy variant), the other steps by plain pairs and
    the single step of row 0.  Against single fused steps over the same 53
    steps: fields bitwise, both rows equal to the summation order."""
    from paper_1705_08019_amd import FitGrid
    spec = c3()

    def make(on):
        g = FitGrid(spec.nx, spec.ny, spec.nz, "f32")
        g.set_materials(spec.eps_r, spec.mu_r, spec.sigma)
        g.set_tuning("fused", 8, 128, 128)
        if on:
            g.set_pair(True, 64, 8, 128)
        g.trace_config(spec.energy_every, 64)
        return g

    g1, g2 = make(True), make(False)
    dt = spec.cfl_frac * g1.cfl_dt()
    s = spec.source
    for g in (g1, g2):
        g.set_source(2, s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
    print("c3 full size: 53 steps across the row at 50, pairs vs single", flush=True)
    g1.profile_begin(200)
    g1.step(53, dt)
    prof = g1.profile_end()
    # 0 single (row 0), pairs from 1 .. 47, the energy pair at 49, a pair at 51
    assert prof["step"][1] == 1 and prof["pair"][1] == 25 and prof["pair_energy"][1] == 1, prof
    g2.step(53, dt)
    for a, b in zip(g1.get_fields(), g2.get_fields()):
        assert torch.equal(a, b)
    t1, d1 = g1.trace_read()
    t2, d2 = g2.trace_read()
    assert t1.shape == t2.shape == (2, 10) and d1 == d2 == 0
    assert np.array_equal(t1[:, 0], t2[:, 0]) and np.array_equal(np.isnan(t1), np.isnan(t2))
    np.testing.assert_allclose(t1, t2, rtol=1e-12, atol=1e-13 * np.nanmax(np.abs(t2)),
                               equal_nan=True)
    print(f"c3 full size: row 50 max rel diff "
          f"{np.nanmax(np.abs(t1 - t2) / np.maximum(np.abs(t2), 1e-300)):.1e}", flush=True)
    g1.close()
    g2.close()
